"""Occupancy volume, sampled features, trained ranker and ranker-guided Lloyd
(needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import raygrid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def _frame_np(V, nb, margin=0.02):
    lo, hi = V.astype(np.float64).min(0), V.astype(np.float64).max(0)
    diag = np.linalg.norm(hi - lo)
    lo2, hi2 = lo - margin * diag, hi + margin * diag
    return np.concatenate([lo2, (hi2 - lo2) / (8 * nb), (lo + hi) / 2, [diag]])


def _trilinear(vol, fr, p):
    g = (p - fr[:3]) / fr[3:6] - 0.5
    i0 = np.floor(g).astype(int)
    f = g - i0
    N = vol.shape[0]
    acc = 0.0
    for c in range(8):
        d = np.array([c & 1, (c >> 1) & 1, c >> 2])
        idx = i0 + d
        w = np.prod(np.where(d == 1, f, 1 - f))
        if np.all(idx >= 0) and np.all(idx < N):
            acc += w * vol[idx[2], idx[1], idx[0]]
    return acc


def test_occupancy_volume_and_sampled_features_match_oracle(api):
    import torch
    V, F = synth.icosphere(2)
    nb, seed = 2, 7
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    vol, frame = api.occupancy_volume(Vt, Ft, nb=nb, seed=seed)
    fr = _frame_np(V, nb)
    assert np.allclose(frame.cpu().numpy(), fr, rtol=1e-6, atol=1e-6)
    fr32 = frame.cpu().numpy().astype(np.float64)
    N = 8 * nb
    ref = np.zeros((N, N, N))
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                idx = np.array([bx, by, bz])
                cell = 8.0 * fr32[3:6]
                c = (fr32[:3] + (idx + 0.5) * cell).astype(np.float32)
                h = (0.5 * cell).astype(np.float32)
                occ = raygrid.occupancy(V, F, c, np.eye(3, dtype=np.float32), h, seed, (bz * nb + by) * nb + bx)
                ref[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8] = occ.transpose(2, 1, 0)
    got = vol.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-4
    # sampled features of a few boxes, from the oracle volume
    c, a, h = synth.random_boxes(4, seed=3, center_range=0.8, half_range=(0.2, 0.6))
    B = synth.boxes_to_array(c, a, h)
    X = api.sample_features(vol, frame, torch.from_numpy(B).cuda()).cpu().numpy()
    for b in range(4):
        Q = a[b].astype(np.float64)
        for r in (0, 100, 311, 511):
            ix, iy, iz = r // 64, (r // 8) % 8, r % 8
            loc = (np.array([ix, iy, iz]) + 0.5) / 4.0 - 1.0
            p = c[b].astype(np.float64) + (loc * h[b]) @ Q
            assert abs(X[b, 15 + r] - _trilinear(ref, fr32, p)) <= 2e-4
        assert np.allclose(X[b, :3], (c[b] - fr32[6:9]) / fr32[9], atol=1e-5)


@pytest.fixture(scope="module")
def trained(api):
    """A ranker trained on the exact outer fractions of four noisy spheres' boxes:
    half random boxes around the surface, half boxes recorded during exact
    Lloyd iterations (the held-out mesh below is a fifth sphere)."""
    import torch
    from paper_2203_10521_amd import ranker
    meshes, boxes = [], []
    for k in range(4):
        V, F = synth.noisy_cube_sphere(12 + 4 * k, seed=100 + k)
        meshes.append((torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()))
        rec = ranker.lloyd_boxes(V, F, R=32, seed=300 + k, n_groups=8, iters=2, cap=2048)
        mixed = synth.mixed_boxes(V, 4096 - len(rec), seed=200 + k)
        boxes.append(torch.from_numpy(np.concatenate([rec, mixed])).cuda())
    X, t, _ = ranker.make_dataset(meshes, boxes, R=32, seed=1, nb=8)
    P, losses = ranker.train(X, t, steps=600, batch=2048, lr=2e-3, seed=0, log_every=100)
    return P, losses


def test_ranker_learns_and_ranks_at_least_as_well_as_the_occupancy_mean(api, trained):
    """Held-out mesh: prediction error and how often the exact best of 8
    candidate boxes is ranked first, against 1 - mean occupancy and chance."""
    import torch
    from paper_2203_10521_amd import ranker
    P, losses = trained
    assert losses[-1][1] < 0.5 * losses[0][1]
    V, F = synth.noisy_cube_sphere(14, seed=777)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    B = torch.from_numpy(synth.mixed_boxes(V, 8 * 256, seed=9)).cuda()
    X, t, _ = ranker.make_dataset([(Vt, Ft)], [B], R=32, seed=1, nb=8)
    f_nn = ranker.predict(P, X)
    f_occ = ranker.occupancy_heuristic(X)
    mae_nn = (f_nn - t).abs().mean().item()
    mae_occ = (f_occ - t).abs().mean().item()
    groups = t.reshape(256, 8)
    best = groups.argmin(dim=1)
    hit_nn = (f_nn.reshape(256, 8).argmin(dim=1) == best).float().mean().item()
    hit_occ = (f_occ.reshape(256, 8).argmin(dim=1) == best).float().mean().item()
    print(f"MAE ranker {mae_nn:.4f} occupancy-mean {mae_occ:.4f}; top-1 hit ranker {hit_nn:.3f} "
          f"occupancy-mean {hit_occ:.3f} chance 0.125")
    assert mae_nn < 0.08
    assert hit_nn > 0.3
    assert hit_nn >= hit_occ - 0.1


def test_fused_ranking_equals_features_then_forward(api, trained):
    """The ranking entry point gives the bits of features-then-network in each of
    its forms: one launch with one box per workgroup (up to 256 boxes), one
    launch with four (up to 1,024, counts that leave a partial workgroup), two
    launches (more boxes); and nothing for 0 boxes."""
    import torch
    P, _ = trained
    V, F = synth.noisy_cube_sphere(14, seed=779)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    vol, frame = api.occupancy_volume(Vt, Ft, nb=8, seed=2)
    for n in (77, 1, 32, 256, 300, 1023, 1100):
        B = torch.from_numpy(synth.mixed_boxes(V, n, seed=40 + n)).cuda()
        fused = api.mlp_rank_boxes(P, vol, frame, B).cpu().numpy()
        X = api.sample_features(vol, frame, B)
        pad = (-n) % 32
        Xp = torch.cat([X, torch.zeros((pad, X.shape[1]), dtype=X.dtype, device=X.device)])
        two = api.mlp_forward(P, Xp).cpu().numpy()[:n]
        assert np.array_equal(fused, two), (n, np.abs(fused - two).max())
    empty = api.mlp_rank_boxes(P, vol, frame, torch.zeros((0, 15), dtype=torch.float32, device="cuda"))
    assert empty.shape == (0,)


def test_ranker_guided_lloyd_close_to_exact_with_fewer_evaluations(api, trained):
    import torch
    from paper_2203_10521_amd import ranker
    P, _ = trained
    V, F = synth.noisy_cube_sphere(16, seed=778)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    vol, frame = api.occupancy_volume(Vt, Ft, nb=8, seed=1)
    centers = np.array([[0.7, 0.3, 0.0], [-0.6, 0.4, 0.2], [0.0, -0.8, 0.3], [0.1, 0.1, -0.9]], np.float32)
    axes = np.stack([np.eye(3, dtype=np.float32)] * 4)
    init = synth.boxes_to_array(centers, axes, np.zeros((4, 3), np.float32))
    out = {}
    for mode in ("exact", "ranker"):
        with api.Lloyd(Vt, Ft, R=32, seed=5, pops_per_round=32) as L:
            L.set_groups(np.zeros(len(F), np.int32), np.zeros(4, np.int32), init)
            if mode == "ranker":
                L.set_surrogate(api.Surrogate(P, vol, frame, verify_top=0, max_error=0.2, judge_every=8))
            for _ in range(3):
                L.step()
            out[mode] = L.get()
    e_x, e_r = out["exact"]["layer_error"], out["ranker"]["layer_error"]
    ev_x, ev_r = out["exact"]["counters"]["evals"], out["ranker"]["counters"]["evals"]
    print(f"layer error exact {e_x:.4f} ranker {e_r:.4f}; evaluations exact {ev_x} ranker {ev_r}; "
          f"predictions {out['ranker']['counters']['predicted']} fallbacks {out['ranker']['counters']['fallbacks']}")
    assert out["ranker"]["counters"]["predicted"] > 0
    assert ev_r < ev_x
    assert e_r <= 1.10 * e_x


def test_ranker_guided_lloyd_is_deterministic(api, trained):
    """The asynchronous judge consumes each result at a fixed later round, so
    two runs of the same ranker-guided Lloyd give identical partitions, boxes
    and counters however the device and host interleave."""
    import torch
    P, _ = trained
    V, F = synth.noisy_cube_sphere(12, seed=31)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    vol, frame = api.occupancy_volume(Vt, Ft, nb=8, seed=1)
    centers = np.array([[0.6, 0.2, 0.1], [-0.5, 0.5, 0.0], [0.1, -0.7, -0.4]], np.float32)
    init = synth.boxes_to_array(centers, np.stack([np.eye(3, dtype=np.float32)] * 3),
                                np.zeros((3, 3), np.float32))
    runs = []
    for _ in range(2):
        with api.Lloyd(Vt, Ft, R=16, seed=9, pops_per_round=16) as L:
            L.set_groups(np.zeros(len(F), np.int32), np.zeros(3, np.int32), init)
            L.set_surrogate(api.Surrogate(P, vol, frame, verify_top=0, max_error=0.2, judge_every=2))
            for _ in range(2):
                L.step()
            runs.append(L.get())
    a, b = runs
    assert a["counters"]["predicted"] > 0
    for k in ("tri_box", "boxes", "obv"):
        assert np.array_equal(a[k], b[k]), k
    assert a["layer_error"] == b["layer_error"]
    assert a["counters"] == b["counters"]
