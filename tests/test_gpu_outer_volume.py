"""HIP outer volume vs the CPU oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import raygrid

pytestmark = pytest.mark.gpu

TOL_BOX = 1e-5          # |OBV_gpu - OBV_oracle| <= TOL_BOX * V_box
Q_ONE = 2 ** 22         # per-ray inside fraction unit of the HIP path
# Per ray, each crossing's depth comes from a float32 plane y = D u + E v + F in
# units of 2^-22 of the slab: rounding gives up to 1.5 units plus 2^-24 of the
# plane's range over the face, which grows with the triangle's slope (steep
# triangles near silhouettes).  Bound: 64 units (1.5e-5 of the slab) on every
# unflagged ray, 4 units at the 99.9th percentile.
TOL_RAY_MAX = 64
TOL_RAY_P999 = 4


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def _dev(api, V, F, c, a, h):
    import torch
    Vt = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    Ft = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    B = torch.from_numpy(synth.boxes_to_array(c, a, h)).cuda()
    return Vt, Ft, B


def _oracle(V, F, c, a, h, R, seed, keys=None, rays=False):
    out = []
    for b in range(len(c)):
        key = b if keys is None else int(keys[b])
        out.append(raygrid.raygrid_obv(V, F, c[b], a[b], h[b], R, seed, key, keep_rays=rays))
    return out


def test_config1_icosphere_64_boxes_parity(api):
    """Icosphere (1,280 triangles), 64 seeded boxes, R = 32: every box within
    1e-5 V_box of the oracle, and every unflagged ray equal."""
    V, F = synth.icosphere(3)
    c, a, h = synth.random_boxes(64, seed=12)
    R, seed = 32, 13
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    res = api.outer_volume_ex(Vt, Ft, B, R, seed=seed, rays=True)
    got = res["obv"].cpu().numpy()
    q = res["ray_q"].cpu().numpy()
    ref = _oracle(V, F, c, a, h, R, seed, rays=True)
    n_flag = 0
    diffs = []
    for b in range(64):
        vb = ref[b]["v_box"]
        assert abs(got[b] - ref[b]["obv"]) <= TOL_BOX * vb, (b, got[b], ref[b]["obv"], vb)
        for w in range(3):
            ray = ref[b]["rays"][w]
            hw = float(h[b][w])
            q_ref = ray["L"] / (2 * hw) * Q_ONE
            flag = ray["near_edge"] | ray["near_slab"]
            n_flag += int(flag.sum())
            d = np.abs(q[b, w] - q_ref)
            assert d[~flag].max(initial=0) <= TOL_RAY_MAX, (b, w, d[~flag].max())
            diffs.append(d[~flag])
    diffs = np.concatenate(diffs)
    assert np.percentile(diffs, 99.9) <= TOL_RAY_P999
    print(f"flagged rays: {n_flag} of {64 * 3 * R * R}; unflagged |dq| max {diffs.max():.2f}, "
          f"p99.9 {np.percentile(diffs, 99.9):.2f} units of 2^-22")


@pytest.mark.parametrize("R", [1, 7, 20, 33])
def test_ragged_grids_and_tile_sizes(api, R):
    """Ragged tails (R not a multiple of the tile) and both tile sizes: the
    per-ray sums are exact integers, so tile 8 and tile 16 agree bitwise."""
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(6, seed=21)
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    r8 = api.outer_volume_ex(Vt, Ft, B, R, seed=5, tile=8, rays=True)
    r16 = api.outer_volume_ex(Vt, Ft, B, R, seed=5, tile=16, rays=True)
    assert np.array_equal(r8["obv"].cpu().numpy(), r16["obv"].cpu().numpy())
    assert np.array_equal(r8["ray_q"].cpu().numpy(), r16["ray_q"].cpu().numpy())
    ref = _oracle(V, F, c, a, h, R, 5)
    got = r8["obv"].cpu().numpy()
    for b in range(6):
        assert abs(got[b] - ref[b]["obv"]) <= TOL_BOX * ref[b]["v_box"]


def test_bitwise_deterministic(api):
    V, F = synth.noisy_torus(nu=64, nv=32)
    c, a, h = synth.random_boxes(32, seed=3, center_range=1.0)
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    x1 = api.outer_volume(Vt, Ft, B, 48, seed=9).cpu().numpy()
    x2 = api.outer_volume(Vt, Ft, B, 48, seed=9).cpu().numpy()
    assert np.array_equal(x1, x2)


def test_inside_disjoint_zero_and_nan_boxes(api):
    import torch
    V, F = synth.icosphere(3)
    _, a, _ = synth.random_boxes(1, seed=8)
    c = np.array([[0.05, 0.0, -0.05], [4.0, 0.3, 0.0], [0.2, 0.1, 0.0], [0.0, 0.0, 0.0], [0.1, 0.2, 0.3]],
                 np.float32)
    h = np.array([[0.3, 0.25, 0.2], [0.3, 0.4, 0.5], [0.0, 0.5, 0.5], [np.nan, 0.3, 0.3], [0.5, 0.5, 0.5]],
                 np.float32)
    ax = np.repeat(a, 5, axis=0)
    Vt, Ft, B = _dev(api, V, F, c, ax, h)
    api.status()  # clear
    got = api.outer_volume(Vt, Ft, B, 16, seed=1).cpu().numpy()
    assert got[0] == 0.0                                   # inside the solid: exactly 0
    assert got[1] == 8.0 * 0.3 * 0.4 * 0.5 or abs(got[1] - 8 * np.prod(h[1].astype(np.float64))) == 0
    assert got[2] == 0.0                                   # zero extent
    assert np.isnan(got[3])                                # NaN parameter
    assert api.status() & 0x1
    ref = _oracle(V, F, c[4:], ax[4:], h[4:], 16, 1, keys=[4])
    assert abs(got[4] - ref[0]["obv"]) <= TOL_BOX * ref[0]["v_box"]
    empty = api.outer_volume(Vt, Ft, B[:0], 16, seed=1)
    assert empty.shape == (0,)
    torch.cuda.synchronize()


def test_axis_mask_and_box_keys(api):
    import torch
    V, F = synth.noisy_cube_sphere(10)
    c, a, h = synth.random_boxes(8, seed=44, center_range=0.8)
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    keys = np.array([7, 100, 3, 9, 11, 12, 13, 4000000000], dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int32)).cuda()
    for mask in (1, 2, 4, 5, 7):
        got = api.outer_volume(Vt, Ft, B, 24, seed=77, axis_mask=mask, box_key=kt).cpu().numpy()
        for b in (0, 7):
            ref = raygrid.raygrid_obv(V, F, c[b], a[b], h[b], 24, 77, int(keys[b]), axis_mask=mask)
            assert abs(got[b] - ref["obv"]) <= TOL_BOX * ref["v_box"], (mask, b)


def test_several_meshes_in_one_call_equal_separate_calls(api):
    import torch
    meshes = [synth.icosphere(2), synth.noisy_cube_sphere(8, seed=3), synth.noisy_torus(nu=32, nv=16)]
    c, a, h = synth.random_boxes(30, seed=51, center_range=0.9)
    bm = (np.arange(30) % 3).astype(np.int32)
    dev_meshes = [(torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()) for V, F in meshes]
    B = torch.from_numpy(synth.boxes_to_array(c, a, h)).cuda()
    together = api.outer_volume_ex(None, None, B, 16, seed=2, meshes=dev_meshes,
                                   box_mesh=torch.from_numpy(bm).cuda())["obv"].cpu().numpy()
    for m in range(3):
        sel = np.nonzero(bm == m)[0]
        keys = torch.from_numpy(sel.astype(np.int32)).cuda()
        alone = api.outer_volume(dev_meshes[m][0], dev_meshes[m][1], B[torch.from_numpy(sel).cuda()], 16,
                                 seed=2, box_key=keys).cpu().numpy()
        assert np.array_equal(together[sel], alone)


def test_config2_torus_sampled_boxes_full_size(api):
    """The bench workload's mesh (noisy torus, 65,536 triangles) at R = 128 in
    the bench's launch configuration; sampled boxes checked by the oracle."""
    import torch
    V, F = synth.noisy_torus()
    c, a, h = synth.random_boxes(64, seed=22, center_range=1.1, half_range=(0.15, 0.9))
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    got = api.outer_volume(Vt, Ft, B, 128, seed=23).cpu().numpy()
    for b in (0, 17, 42):
        ref = raygrid.raygrid_obv(V, F, c[b], a[b], h[b], 128, 23, b)
        assert abs(got[b] - ref["obv"]) <= TOL_BOX * ref["v_box"], (b, got[b], ref["obv"])
    torch.cuda.synchronize()


def test_grouped_candidates_equal_plain_calls(api):
    """Boxes grouped by shared centre and axes (Lloyd candidates: a box grown in
    several ways) give bitwise the plain call's results; boxes whose group frame
    does not contain them (other axes, larger extent, bad index) fall back to
    the whole mesh and still agree."""
    import torch
    V, F = synth.noisy_torus()
    g = np.random.default_rng(12)
    c, a, h = synth.random_boxes(8, seed=61, center_range=1.0, half_range=(0.05, 0.3))
    cand, frame_of = [], []
    for k in range(8):
        for _ in range(6):
            grow = g.uniform(1.0, 1.6, size=3).astype(np.float32)
            grow[g.integers(0, 3)] = 1.0
            cand.append((c[k], a[k], (h[k] * grow).astype(np.float32)))
            frame_of.append(k)
    B = synth.boxes_to_array(np.array([x[0] for x in cand]), np.array([x[1] for x in cand]),
                             np.array([x[2] for x in cand]))
    frames = np.zeros((8, 15), np.float32)
    for k in range(8):
        sel = [i for i, f in enumerate(frame_of) if f == k]
        frames[k] = B[sel[0]]
        frames[k, 12:] = B[sel, 12:].max(axis=0)
    bf = np.array(frame_of, np.int32)
    # fallbacks: wrong frame (other axes), a box larger than its frame, an index out of range
    bf[5] = 3
    B[11, 12] = frames[1, 12] * 1.25
    bf[20] = 99
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    Bt = torch.from_numpy(B).cuda()
    keys = torch.from_numpy((np.arange(len(B)) * 7 + 3).astype(np.int32)).cuda()
    api.status()
    for R in (16, 48, 128):
        plain = api.outer_volume(Vt, Ft, Bt, R, seed=9, box_key=keys).cpu().numpy()
        grouped = api.outer_volume_grouped(Vt, Ft, Bt, R, torch.from_numpy(frames).cuda(),
                                           torch.from_numpy(bf).cuda(), seed=9, box_key=keys).cpu().numpy()
        assert np.array_equal(plain, grouped), (R, np.nonzero(plain != grouped))
    assert api.status() == 0


def test_rasterising_and_all_ray_kernels_agree(api, monkeypatch):
    """The rasterising ray test (each record against the rays of its cells) and
    the all-rays test (each record against every ray of its tile) give the same
    bits, per box and per ray, with the rasterising kernel's per-lane cell loop
    for records up to 64 cells of a tile and its wave-wide path above, and with
    either path alone (every record wide; none wide)."""
    V, F = synth.noisy_torus(nu=96, nv=48)
    c, a, h = synth.random_boxes(24, seed=71, center_range=1.0, half_range=(0.1, 0.7))
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    out = {}
    for mode, cells in (("0", "64"), ("1", "64"), ("1", "0"), ("1", "256")):
        monkeypatch.setenv("OBBV_TEST_RASTER", mode)
        monkeypatch.setenv("OBBV_RASTER_CELLS", cells)
        r = api.outer_volume_ex(Vt, Ft, B, 48, seed=5, tile=16, rays=True)
        out[(mode, cells)] = {k: r[k].cpu().numpy() for k in ("obv", "ray_q", "ray_hits")}
    ref = out[("0", "64")]
    for key in (("1", "64"), ("1", "0"), ("1", "256")):
        for k in ("obv", "ray_q", "ray_hits"):
            assert np.array_equal(out[key][k], ref[k]), (key, k)


def test_write_pass_slot_strategies_agree(api, monkeypatch):
    """Bin slots reserved per tile from LDS counts and slots taken one global
    atomic at a time fill the bins in different orders; the sums are exact
    integers, so every box and ray gets the same bits."""
    V, F = synth.noisy_torus(nu=64, nv=32)
    c, a, h = synth.random_boxes(16, seed=72, center_range=1.0, half_range=(0.1, 0.7))
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("OBBV_WRITE_LDS", mode)
        r = api.outer_volume_ex(Vt, Ft, B, 64, seed=6, tile=16, rays=True)
        out[mode] = {k: r[k].cpu().numpy() for k in ("obv", "ray_q", "ray_hits")}
    for k in ("obv", "ray_q", "ray_hits"):
        assert np.array_equal(out["1"][k], out["0"][k]), k


def test_work_item_sizes_and_record_loading_agree(api, monkeypatch):
    """Ray-test work items of 64 or 4096 records instead of the default, and the
    all-rays kernel's scalar record loads instead of LDS staging, split and
    load the same bin entries differently; every box and ray gets the same
    bits."""
    V, F = synth.noisy_torus(nu=64, nv=32)
    c, a, h = synth.random_boxes(16, seed=73, center_range=1.0, half_range=(0.1, 0.7))
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    out = {}
    for raster, chunk, stage in (("1", "384", "1"), ("1", "64", "1"), ("1", "4096", "1"), ("0", "384", "1"),
                                 ("0", "384", "0"), ("0", "64", "0")):
        monkeypatch.setenv("OBBV_TEST_RASTER", raster)
        monkeypatch.setenv("OBBV_TEST_CHUNK", chunk)
        monkeypatch.setenv("OBBV_TEST_STAGE", stage)
        r = api.outer_volume_ex(Vt, Ft, B, 64, seed=8, tile=16, rays=True)
        out[(raster, chunk, stage)] = {k: r[k].cpu().numpy() for k in ("obv", "ray_q", "ray_hits")}
    ref = out[("1", "384", "1")]
    for key, got in out.items():
        for k in ("obv", "ray_q", "ray_hits"):
            assert np.array_equal(got[k], ref[k]), (key, k)


def test_validate_mesh(api):
    import torch
    V, F = synth.icosphere(2)
    Vt = torch.from_numpy(V).cuda()
    code, rep, vol = api.validate_mesh(Vt, torch.from_numpy(F).cuda())
    assert code == 0 and rep[:3] == [0, 0, 0] and vol > 0
    code, rep, _ = api.validate_mesh(Vt, torch.from_numpy(F[1:].copy()).cuda())
    assert code == -2 and rep[0] == 3
    Fb = F.copy()
    Fb[5] = Fb[5][[0, 2, 1]]
    code, rep, _ = api.validate_mesh(Vt, torch.from_numpy(Fb).cuda())
    assert code == -3 and rep[1] > 0
    code, _, vol = api.validate_mesh(Vt, torch.from_numpy(F[:, [0, 2, 1]].copy()).cuda())
    assert code == -3 and vol < 0
