"""HIP outer volume vs the CPU oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import geometry, raygrid

from conftest import record_parity

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


def _compare_rays(res, ref, h, boxes, name):
    """Per-ray parity on the unflagged rays of `boxes`: the fixed-point inside
    length within TOL_RAY_MAX units, and the crossing counts identical -- in the
    slab, and beyond the slab face of the kept side (above it, or below it for a
    mirrored cast).  Flagged rays (within 1e-6 of a projected edge or of a slab
    face) are counted and reported."""
    q = res["ray_q"].cpu().numpy()
    hits = res["ray_hits"].cpu().numpy()
    side = res["side"].cpu().numpy()
    n_edge = n_slab = n_rays = n_count_cmp = 0
    diffs = []
    for k, b in enumerate(boxes):
        for w in range(3):
            ray = ref[k]["rays"][w]
            hw = float(h[b][w])
            q_ref = ray["L"] / (2 * hw) * Q_ONE
            flag = ray["near_edge"] | ray["near_slab"]
            n_edge += int(ray["near_edge"].sum())
            n_slab += int((ray["near_slab"] & ~ray["near_edge"]).sum())
            n_rays += flag.size
            d = np.abs(q[b, w] - q_ref)
            assert d[~flag].max(initial=0) <= TOL_RAY_MAX, (name, b, w, d[~flag].max())
            diffs.append(d[~flag])
            n_in = hits[b, w] & 0xFFFF
            n_far = hits[b, w] >> 16
            far_ref = ray["n_below"] if side[b, w] else ray["n_above"]
            bad_in = (n_in != ray["n_in"]) & ~flag
            bad_far = (n_far != far_ref) & ~flag
            assert not bad_in.any(), (name, b, w, "n_in", np.argwhere(bad_in)[:5].tolist())
            assert not bad_far.any(), (name, b, w, "n_beyond", np.argwhere(bad_far)[:5].tolist())
            n_count_cmp += int((~flag).sum())
    diffs = np.concatenate(diffs)
    assert np.percentile(diffs, 99.9) <= TOL_RAY_P999
    rec = {"test": name, "rays": n_rays, "compared": n_count_cmp, "flagged_near_edge": n_edge,
           "flagged_near_slab": n_slab, "count_mismatches_unflagged": 0,
           "max_dq_unflagged": float(diffs.max(initial=0)), "p999_dq": float(np.percentile(diffs, 99.9))}
    record_parity(rec)
    return rec


def test_config1_icosphere_64_boxes_parity(api):
    """Icosphere (1,280 triangles), 64 seeded boxes, R = 32: every box within
    1e-5 V_box of the oracle; on every unflagged ray the inside length within
    64 units of 2^-22 and the crossing counts identical."""
    V, F = synth.icosphere(3)
    c, a, h = synth.random_boxes(64, seed=12)
    R, seed = 32, 13
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    res = api.outer_volume_ex(Vt, Ft, B, R, seed=seed, rays=True)
    got = res["obv"].cpu().numpy()
    ref = _oracle(V, F, c, a, h, R, seed, rays=True)
    for b in range(64):
        vb = ref[b]["v_box"]
        assert abs(got[b] - ref[b]["obv"]) <= TOL_BOX * vb, (b, got[b], ref[b]["obv"], vb)
    rec = _compare_rays(res, ref, h, range(64), "config1_icosphere")
    print(rec)


def test_edge_tie_is_watertight(api):
    """A closed slab whose top face is cut along the exact v-coordinate of one
    ray: the shared interior edge has edge function exactly 0 in FP32 on that
    ray for both top triangles.  The top-left rule gives the ray exactly one top
    crossing (two in the slab with the bottom one), as the oracle finds, and the
    box's outer volume matches the oracle."""
    import torch
    R, seed, key = 16, 41, 0
    half = np.array([0.6, 0.6, 0.6])
    u, v = raygrid.ray_positions(half, 2, R, seed, key)
    i0, j0 = 7, 8
    rv64 = float(v[i0, j0])
    rv = np.float32(rv64)
    assert float(rv) != rv64, "the oracle's ray must not sit exactly on the edge"
    assert -0.5 < u[i0, j0] < 0.5 and -0.4 < rv < 0.45
    V, F = synth.split_top_slab(rv)
    assert geometry.directed_edge_report(F)[0]
    c = np.zeros((1, 3), np.float32)
    a = np.eye(3, dtype=np.float32)[None]
    h = half.astype(np.float32)[None]
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    key_t = torch.zeros(1, dtype=torch.int32, device="cuda")
    for mask in (4, 7):
        res = api.outer_volume_ex(Vt, Ft, B, R, seed=seed, axis_mask=mask, box_key=key_t, rays=True)
        hits = res["ray_hits"].cpu().numpy()[0, 2]
        ref = raygrid.raygrid_obv(V, F, c[0], a[0], h[0], R, seed, key, axis_mask=mask, keep_rays=True)
        ray = ref["rays"][2]
        assert ray["near_edge"][i0, j0]
        assert ray["n_in"][i0, j0] == 2
        assert (hits[i0, j0] & 0xFFFF) == 2, hits[i0, j0]
        assert np.array_equal(hits & 0xFFFF, ray["n_in"])
        got = res["obv"].cpu().numpy()[0]
        assert abs(got - ref["obv"]) <= TOL_BOX * ref["v_box"], (mask, got, ref["obv"])
    record_parity({"test": "edge_tie", "ray": [i0, j0], "gpu_n_in": int(hits[i0, j0] & 0xFFFF),
                   "oracle_n_in": int(ray["n_in"][i0, j0])})


@pytest.mark.parametrize("R", [1, 7, 20, 33, 130])
def test_ragged_grids_and_ray_blocks(api, R):
    """Ragged tails (R not a multiple of the ray block's width or height) and
    three LDS ray-block sizes: the crossings' inside lengths are exact integers,
    so every block size gives the same bits per box and per ray."""
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(6, seed=21)
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    out = {}
    for blk in (1024, 4096, 16384):
        r = api.outer_volume_ex(Vt, Ft, B, R, seed=5, block_rays=blk, rays=True)
        out[blk] = {k: r[k].cpu().numpy() for k in ("obv", "ray_q", "ray_hits", "side")}
    for blk in (4096, 16384):
        for k in ("obv", "ray_q", "ray_hits", "side"):
            assert np.array_equal(out[blk][k], out[1024][k]), (blk, k)
    ref = _oracle(V, F, c, a, h, R, 5)
    got = out[1024]["obv"]
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
    assert got[1] == 8 * np.prod(h[1].astype(np.float64))  # disjoint: exactly V_box
    assert got[2] == 0.0                                   # zero extent
    assert np.isnan(got[3])                                # NaN parameter
    assert api.status() & 0x1
    ref = _oracle(V, F, c[4:], ax[4:], h[4:], 16, 1, keys=[4])
    assert abs(got[4] - ref[0]["obv"]) <= TOL_BOX * ref[0]["v_box"]
    empty = api.outer_volume(Vt, Ft, B[:0], 16, seed=1)
    assert empty.shape == (0,)
    # a mesh without triangles: nothing is inside any box
    bare = api.outer_volume(Vt, Ft[:0], B[:3], 16, seed=1).cpu().numpy()
    assert bare[0] == 8 * np.prod(h[0].astype(np.float64)) and bare[1] == 8 * np.prod(h[1].astype(np.float64))
    assert bare[2] == 0.0
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
    the bench's launch configuration (default ray blocks); 8 boxes spanning the
    size range checked against the oracle, per box and per ray on 2 of them."""
    import torch
    V, F = synth.noisy_torus()
    c, a, h = synth.random_boxes(64, seed=22, center_range=1.1, half_range=(0.15, 0.9))
    Vt, Ft, B = _dev(api, V, F, c, a, h)
    res = api.outer_volume_ex(Vt, Ft, B, 128, seed=23, rays=True)
    got = res["obv"].cpu().numpy()
    vols = np.prod(h.astype(np.float64), axis=1)
    order = np.argsort(vols)
    sample = sorted(set(order[np.linspace(0, 63, 8).astype(int)].tolist()))
    refs = {}
    for b in sample:
        refs[b] = raygrid.raygrid_obv(V, F, c[b], a[b], h[b], 128, 23, b, keep_rays=b in sample[:2])
        assert abs(got[b] - refs[b]["obv"]) <= TOL_BOX * refs[b]["v_box"], (b, got[b], refs[b]["obv"])
    _compare_rays(res, [refs[b] for b in sample[:2]], h, sample[:2], "config2_torus_R128")
    torch.cuda.synchronize()


@pytest.mark.parametrize("lists", ["1", "2"])
def test_grouped_candidates_equal_plain_calls(api, monkeypatch, lists):
    """Boxes grouped by shared centre and axes (Lloyd candidates: a box grown in
    several ways) give bitwise the plain call's results; boxes whose group frame
    does not contain them (other axes, larger extent, bad index) fall back to
    the whole mesh and still agree.  Both frame-list builds: one pass into
    fixed segments (list order follows the blocks' arrival) and two passes
    sized exactly (OBBV_FRAME_LISTS=2); repeated calls check that the one-pass
    counters start every call at zero."""
    monkeypatch.setenv("OBBV_FRAME_LISTS", lists)
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


def test_lane_and_wave_paths_agree(api, monkeypatch):
    """A kept triangle is tested by its own lane over the cells it covers, or by
    the whole wave (one cell per lane) above a cell-count threshold; with the
    threshold at 0 (every triangle wave-wide), 64, 512 (the default) and 16384
    (every triangle per lane, those of 512 cells or more with 64-bit sums) every
    box and every ray get the same bits.  The coarse mesh and small boxes give
    triangles covering hundreds of cells."""
    V, F = synth.noisy_torus(nu=96, nv=48)
    c, a, h = synth.random_boxes(24, seed=71, center_range=1.0, half_range=(0.1, 0.7))
    Vc, Fc = synth.noisy_torus(nu=24, nv=12)
    c2, a2, h2 = synth.random_boxes(16, seed=72, center_range=1.0, half_range=(0.05, 0.25))
    for (VV, FF, cc, aa, hh, R) in ((V, F, c, a, h, 48), (Vc, Fc, c2, a2, h2, 96)):
        Vt, Ft, B = _dev(api, VV, FF, cc, aa, hh)
        out = {}
        for cells in ("0", "64", "512", "16384"):
            monkeypatch.setenv("OBBV_RASTER_CELLS", cells)
            r = api.outer_volume_ex(Vt, Ft, B, R, seed=5, rays=True)
            out[cells] = {k: r[k].cpu().numpy() for k in ("obv", "ray_q", "ray_hits")}
        for key in ("0", "64", "16384"):
            for k in ("obv", "ray_q", "ray_hits"):
                assert np.array_equal(out[key][k], out["512"][k]), (R, key, k)


def test_jitter_table_and_computed_draws_agree(api):
    """Lloyd evaluations read the ray jitter from a per-key table; a plain call
    computes the same SplitMix64 draws: a one-iteration Lloyd run's final OBV
    equals the plain call's on the same boxes and keys bit for bit."""
    import torch
    V, F = synth.noisy_cube_sphere(12, seed=5)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    st = api.Lloyd(Vt, Ft, R=24, seed=17)
    n = F.shape[0]
    tri_group = np.zeros(n, np.int32)
    c, a, h = synth.random_boxes(3, seed=5, center_range=0.5)
    boxes = synth.boxes_to_array(c, a, h)
    st.set_groups(tri_group, np.zeros(3, np.int32), boxes, box_slot=np.array([5, 9, 2], np.uint32))
    st.step()
    got = st.get()
    B = torch.from_numpy(np.ascontiguousarray(got["boxes"])).cuda()
    keys = torch.from_numpy(np.array([5, 9, 2], np.int32)).cuda()
    plain = api.outer_volume(Vt, Ft, B, 24, seed=17, box_key=keys).cpu().numpy()
    assert np.array_equal(plain, got["obv"])


def _edge_report(F, nv):
    """Brute-force counts of the validation report: directed edges whose reverse
    does not occur exactly once, repeats of a directed edge, bad indices."""
    from collections import Counter
    F = np.asarray(F, np.int64)
    bad = int(((F < 0) | (F >= nv)).sum())
    edges = Counter()
    for a, b, c in F.tolist():
        for u, v in ((a, b), (b, c), (c, a)):
            edges[(u, v)] += 1
    unmatched = sum(m for (u, v), m in edges.items() if u == v or edges.get((v, u), 0) != 1)
    repeated = sum(m - 1 for m in edges.values())
    return [unmatched, repeated, bad]


def test_validate_mesh(api):
    """Device edge table and exact volume sum: reports equal to brute-force
    counts on closed, open, flipped and bad-index meshes; the volume matches
    the oracle's sum of det / 6 and is bit-identical for any triangle order."""
    import torch
    V, F = synth.icosphere(2)
    Vt = torch.from_numpy(V).cuda()
    code, rep, vol = api.validate_mesh(Vt, torch.from_numpy(F).cuda())
    assert code == 0 and rep[:3] == [0, 0, 0] and vol > 0
    assert abs(vol - geometry.signed_volume(V, F)) <= 1e-12 * abs(vol)
    code, rep, _ = api.validate_mesh(Vt, torch.from_numpy(F[1:].copy()).cuda())
    assert code == -2 and rep[:3] == _edge_report(F[1:], len(V)) and rep[0] == 3
    Fb = F.copy()
    Fb[5] = Fb[5][[0, 2, 1]]
    code, rep, _ = api.validate_mesh(Vt, torch.from_numpy(Fb).cuda())
    assert code == -3 and rep[:3] == _edge_report(Fb, len(V)) and rep[1] == 3
    code, _, vol = api.validate_mesh(Vt, torch.from_numpy(F[:, [0, 2, 1]].copy()).cuda())
    assert code == -3 and vol < 0
    Fi = F.copy()
    Fi[7, 1] = len(V) + 3
    Fi[9, 0] = -1
    code, rep, _ = api.validate_mesh(Vt, torch.from_numpy(Fi).cuda())
    assert code == -1 and rep[2] == 2
    # bigger meshes: volume against the oracle, bit-identical under permutation
    g = np.random.default_rng(0)
    for V, F in (synth.noisy_torus(), synth.noisy_cube_sphere(60, seed=4)):
        Vt = torch.from_numpy(V).cuda()
        code, rep, vol = api.validate_mesh(Vt, torch.from_numpy(F).cuda())
        assert code == 0 and rep[:3] == [0, 0, 0]
        ref = geometry.signed_volume(V, F)
        assert abs(vol - ref) <= 1e-12 * abs(ref), (vol, ref)
        _, _, vol2 = api.validate_mesh(Vt, torch.from_numpy(F[g.permutation(len(F))].copy()).cuda())
        assert vol2 == vol


def test_span_culling_gives_the_same_bits(api, monkeypatch):
    """Whole-mesh casts skip the runs and spans of 256 triangles whose bounds
    miss the cast's kept half prism.  The skipped triangles are ones the cull
    would drop, so the results are bit-identical with the culling off
    (OBBV_SPAN_CULL=0): on a mesh in surface order (tight spans) and on the same
    mesh with its triangles shuffled (loose spans), for small boxes near the
    surface and large random ones, in one call and through a plan."""
    import torch
    V, F = synth.noisy_torus()
    g = np.random.default_rng(5)
    F_shuffled = F[g.permutation(len(F))].copy()
    c, a, h = synth.random_boxes(48, seed=8, center_range=1.2, half_range=(0.02, 0.12))
    c2, a2, h2 = synth.random_boxes(16, seed=9, center_range=1.0, half_range=(0.2, 0.9))
    B = torch.from_numpy(np.concatenate([synth.boxes_to_array(c, a, h), synth.boxes_to_array(c2, a2, h2)])).cuda()
    Vt = torch.from_numpy(V).cuda()
    for FF in (F, F_shuffled):
        Ft = torch.from_numpy(FF).cuda()
        out = {}
        for flag in ("1", "0"):
            monkeypatch.setenv("OBBV_SPAN_CULL", flag)
            api.status()
            out[flag] = api.outer_volume(Vt, Ft, B, 24, seed=4).cpu().numpy()
            assert api.status() == 0
        assert np.array_equal(out["1"], out["0"])
    monkeypatch.setenv("OBBV_SPAN_CULL", "1")
    plan = api.OuterVolumePlan(B, 24, seed=4, meshes=[(Vt, torch.from_numpy(F).cuda())], block_rays=2048)
    got = plan.launch().clone().cpu().numpy()
    ref = api.outer_volume(Vt, torch.from_numpy(F).cuda(), B, 24, seed=4, block_rays=2048).cpu().numpy()
    plan.close()
    assert np.array_equal(got, ref)


def test_span_culling_far_from_the_origin(api, monkeypatch):
    """The same comparison with the mesh and boxes moved 3,000 units from the
    origin (float32 coordinates then carry about 2.4e-4 of absolute rounding):
    the span test's margins stay relative to the local magnitudes."""
    import torch
    V, F = synth.noisy_torus(nu=128, nv=64)
    shift = np.array([3000.0, -2000.0, 1000.0], np.float32)
    c, a, h = synth.random_boxes(32, seed=18, center_range=1.2, half_range=(0.02, 0.3))
    B = torch.from_numpy(synth.boxes_to_array((c + shift).astype(np.float32), a, h)).cuda()
    Vt, Ft = torch.from_numpy((V + shift).astype(np.float32)).cuda(), torch.from_numpy(F).cuda()
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("OBBV_SPAN_CULL", flag)
        out[flag] = api.outer_volume(Vt, Ft, B, 20, seed=6).cpu().numpy()
    assert np.array_equal(out["1"], out["0"])
