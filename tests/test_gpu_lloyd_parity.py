"""The Lloyd step and the hierarchy sweeps on the device vs the CPU oracle, at
the shapes the builder runs (needs an MI355X).

Both sides start from the same seeded inputs and compute everything on their
own.  Where an element's two best moves differ in dOBV by less than the tie
tolerance (2e-5 of the larger grown box volume: the ray-grid estimate of the
two sides differs by float32 rounding of the ray tests), either move is
correct; the oracle then checks that the device's move is one of them, takes
it, and counts it.  The parameter update is an argmin over finite differences
of those estimates and is ill-conditioned where the gradient is small (an
estimate noise of 5e-7 of the box volume turns boxes by up to 1e-3); the
oracle takes the device's updated box when it is valid within that noise
(its own tight box for the device's axes, a line-search step along a direction
within the gradient-noise bound, a consistent outer volume: see
``oracle.lloyd.update_box``) and counts it.  Both counts are reported in the
parity records; the partition, parents and node outer volumes are compared.
"""
import numpy as np
import pytest

import synth
from conftest import record_parity
from oracle import hierarchy
from oracle import lloyd as ol
from oracle_pool import RaygridPool

pytestmark = pytest.mark.gpu

TIE = 2e-5


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def _dev(V, F):
    import torch
    return torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()


def _box_gap(a, b):
    """Largest difference between two (c, Q, h) boxes, as 15-float rows."""
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))))


def _torus_groups():
    """8k-triangle torus in 8 angular sectors, 4 boxes per sector: centres at
    the centroids of 4 seeded triangles of the sector, axes one seeded rotation
    per sector, zero extents."""
    V, F = synth.noisy_torus(nu=128, nv=32)
    cen = V[F].astype(np.float64).mean(1)
    ang = np.arctan2(cen[:, 1], cen[:, 0])
    tri_group = np.minimum(((ang + np.pi) / (2 * np.pi) * 8).astype(np.int32), 7)
    rng = np.random.default_rng(4)
    _, ax, _ = synth.random_boxes(8, seed=44)
    boxes, box_group = [], []
    for g in range(8):
        for t in rng.choice(np.nonzero(tri_group == g)[0], 4, replace=False):
            boxes.append(np.concatenate([cen[t].astype(np.float32), ax[g].reshape(-1), np.zeros(3, np.float32)]))
            box_group.append(g)
    return V, F, tri_group, np.array(boxes, np.float32), np.array(box_group, np.int32)


@pytest.mark.timeout(900)
def test_lloyd_iteration_eight_groups_k32_matches_the_oracle(api):
    """One Lloyd iteration of 8 groups x 4 boxes with 32 pops per group and
    round, R = 16: the grouped candidate frames, the containment masks and the
    jitter table of the builder's evaluator all take part.  Identical
    partition; boxes within 1e-5 (mesh units); OBV within 1e-5 of the box volume."""
    V, F, tri_group, B, box_group = _torus_groups()
    slots = (7 + 3 * np.arange(len(B))).astype(np.uint32)
    R, seed, K = 16, 9, 32
    Vt, Ft = _dev(V, F)
    with api.Lloyd(Vt, Ft, R=R, seed=seed, pops_per_round=K) as L:
        L.set_groups(tri_group, box_group, B, slots)
        L.step()
        out = L.get()
    assert out["counters"]["trivial"] > 0
    E = ol.triangle_elements(V, F)
    ties = {"ties": 0}
    ref_box = np.full(len(F), -1)
    worst_box, worst_obv = 0.0, 0.0
    with RaygridPool(V, F, R, seed) as ev:
        for g in range(8):
            bxs = np.nonzero(box_group == g)[0]
            local = {int(j): i for i, j in enumerate(bxs)}
            assign, grown, _, cnt = ol.flood(E, np.nonzero(tri_group == g)[0], B[bxs, :3],
                                             B[bxs, 3:12].reshape(-1, 3, 3), slots[bxs], ev, K,
                                             follow=lambda e: local.get(int(out["tri_box"][e])), tie=TIE)
            ties["ties"] += cnt["ties"]
            for i, j in enumerate(bxs):
                tris = sorted(e for e, k in assign.items() if k == i)
                ref_box[tris] = j
                got = out["boxes"][j]
                bx, v, _ = ol.update_box(V, F, tris, grown[i][1], int(slots[j]), ev,
                                         follow_box=(got[:3], got[3:12].reshape(3, 3), got[12:]), tie=TIE,
                                         counters=ties)
                worst_box = max(worst_box, _box_gap(np.concatenate([bx[0], bx[1].reshape(-1), bx[2]]), got))
                worst_obv = max(worst_obv, abs(out["obv"][j] - v) / ol.box_volume(bx[2]))
    record_parity({"test": "lloyd_8x4_k32_torus8k_R16", "ties": ties["ties"],
                   "update_ties": ties.get("update_ties", 0), "max_box_gap": worst_box,
                   "max_obv_gap_rel": worst_obv, "evals_device": int(out["counters"]["evals"])})
    assert np.array_equal(out["tri_box"], ref_box)
    assert worst_box <= 1e-5 and worst_obv <= 1e-5
    assert ties["ties"] <= 8


def _compare_hierarchy(got, ref, nt, L, b, tag):
    assert np.array_equal(got["tri_node"], ref["tri_node"]), tag
    assert np.array_equal(got["parent"], ref["parent"]), tag
    gap = float(np.max(np.abs(got["boxes"].astype(np.float64) - ref["boxes"].astype(np.float64))))
    vb = 8.0 * np.prod(ref["boxes"][:, 12:].astype(np.float64), axis=1)
    used = vb > 0
    rel = float(np.max(np.abs(got["obv"][used] - ref["obv"][used]) / vb[used]))
    assert gap <= 1e-5 and rel <= 1e-5, (tag, gap, rel)
    return gap, rel


@pytest.mark.timeout(900)
def test_hierarchy_top_down_and_one_sweep_match_the_oracle(api):
    """A 2k-triangle mesh, 3 layers of branching 4, one iteration per layer
    solve: the top-down build (sweeps = 0) and the build with one sweep (up pass:
    merge of layer 1 kept or undone by Eq. 7; down pass: re-solve of layer 2)
    give identical node assignments and parents, boxes within 1e-5, node OBVs
    within 1e-5 of their box volumes, and e within 1e-5 of sum(omega V_box)."""
    V, F = synth.noisy_cube_sphere(13, seed=8)
    L, b, R, seed, K = 3, 4, 8, 5, 32
    Vt, Ft = _dev(V, F)
    td = api.build_hierarchy(Vt, Ft, levels=L, branching=b, iters=1, sweeps=0, R=R, seed=seed, pops_per_round=K)
    sw = api.build_hierarchy(Vt, Ft, levels=L, branching=b, iters=1, sweeps=1, R=R, seed=seed, pops_per_round=K)
    with RaygridPool(V, F, R, seed) as ev:
        H, e, ref_td = hierarchy.build(V, F, L, b, ev, seed, iters=1, sweeps=1, K=K,
                                       follow_top_down=hierarchy.FollowArrays(td, L, b),
                                       follow_sweeps=hierarchy.FollowArrays(sw, L, b), tie=TIE)
    ref_sw = H.arrays()
    g1 = _compare_hierarchy(td, ref_td, len(F), L, b, "top-down")
    g2 = _compare_hierarchy(sw, ref_sw, len(F), L, b, "sweep")
    level = np.concatenate([[lv] * b ** lv for lv in range(L)])
    wv = float(np.sum((L - level) * 8.0 * np.prod(ref_sw["boxes"][:, 12:].astype(np.float64), axis=1)))
    assert abs(td["e"][0] - e[0]) <= 1e-5 * wv and abs(sw["e"][-1] - e[-1]) <= 1e-5 * wv
    record_parity({"test": "hierarchy_L3_b4_sweep1_R8", "triangles": int(len(F)), "ties": H.counters["ties"],
                   "update_ties": H.counters["update_ties"],
                   "trace": [[t[0], t[1], t[4]] for t in H.trace], "max_box_gap": max(g1[0], g2[0]),
                   "max_obv_gap_rel": max(g1[1], g2[1]), "e_oracle": e, "e_device": [float(x) for x in sw["e"]]})
    assert H.counters["ties"] <= 8


def _pack(centers, axes):
    n = len(centers)
    return synth.boxes_to_array(np.asarray(centers), np.asarray(axes), np.zeros((n, 3), np.float32))


def _follows(out, bxs):
    local = {int(j): i for i, j in enumerate(bxs)}
    row = out["boxes"]
    return (lambda e: local.get(int(out["tri_box"][e])),
            lambda k: (row[bxs[k], :3], row[bxs[k], 3:12].reshape(3, 3), row[bxs[k], 12:]))


def _check_group(out, bxs, clusters, boxes, obv, ref_tri, gaps):
    for i, j in enumerate(bxs):
        ref_tri[clusters[i]] = j
        c, Q, h = boxes[i]
        got = out["boxes"][j]
        gaps[0] = max(gaps[0], _box_gap(np.concatenate([c, Q.reshape(-1), h]), got))
        gaps[1] = max(gaps[1], abs(out["obv"][j] - obv[i]) / max(ol.box_volume(h), 1e-30))


@pytest.mark.timeout(900)
def test_adjustment_matches_the_oracle(api):
    """The adjustment step (Sec. 4.2.1, third step) from the same states as the
    oracle.  Stalled cuboids (two boxes in one cuboid, one over the other two):
    two adjustments kept, a third undone, the same partitions and boxes.  The
    8 x 4 torus groups after one K = 32 iteration: the same kept / undone flag
    per group, partition, boxes and outer volumes (1e-5)."""
    import torch
    counters = {"ties": 0}
    # stalled cuboids
    V, F, comp, params = synth.disjoint_cuboids(3, seed=7, spacing=3.0)
    cen = V[F].astype(np.float64).mean(1)
    t0, t1 = np.nonzero(comp == 0)[0], np.nonzero(comp == 1)[0]
    centers = np.array([cen[t0[0]], cen[t0[-1]], cen[t1[0]]], np.float32)
    axes = np.array([params[0][1], params[0][1], params[1][1]], np.float32)
    R, seed, K = 16, 3, 4
    Vt, Ft = _dev(V, F)
    outs, flags = [], []
    with api.Lloyd(Vt, Ft, R=R, seed=seed, pops_per_round=K) as L:
        L.set_groups(np.zeros(len(F), np.int32), np.zeros(3, np.int32), _pack(centers, axes), [0, 1, 2])
        L.step()
        outs.append(L.get())
        for _ in range(3):
            flags.append(int(L.adjust()[0]))
            outs.append(L.get())
    assert flags == [1, 1, 0]
    adj = ol.adjacency(F)
    group, bxs = range(len(F)), np.arange(3)
    with RaygridPool(V, F, R, seed, workers=1) as ev:
        fol, folb = _follows(outs[0], bxs)
        state = ol.lloyd_iteration(V, F, adj, group, centers, axes, [0, 1, 2], ev, K, fol, folb, TIE, counters)[:3]
        for k in range(3):
            fol, folb = _follows(outs[k + 1], bxs)
            acc, *nxt = ol.adjust(V, F, adj, group, *state, [0, 1, 2], ev, K, fol, folb, TIE, counters)
            assert int(acc) == flags[k]
            state = nxt[:3]
            ref_tri, gaps = np.full(len(F), -1), [0.0, 0.0]
            _check_group(outs[k + 1], bxs, state[0], state[1], state[2], ref_tri, gaps)
            assert np.array_equal(outs[k + 1]["tri_box"], ref_tri), k
            assert gaps[0] <= 1e-5 and gaps[1] <= 1e-5, (k, gaps)
    assert sorted(sorted(set(comp[outs[3]["tri_box"] == j])) for j in range(3)) == [[0], [1], [2]]
    # torus groups
    V, F, tri_group, B, box_group = _torus_groups()
    slots = (7 + 3 * np.arange(len(B))).astype(np.uint32)
    R, seed, K = 16, 9, 32
    Vt, Ft = _dev(V, F)
    with api.Lloyd(Vt, Ft, R=R, seed=seed, pops_per_round=K) as L:
        L.set_groups(tri_group, box_group, B, slots)
        L.step()
        pre = L.get()
        acc = L.adjust()
        post = L.get()
    E = ol.triangle_elements(V, F)
    adj = E.adj
    ref_tri, gaps = np.full(len(F), -1), [0.0, 0.0]
    with RaygridPool(V, F, R, seed) as ev:
        for g in range(8):
            bxs = np.nonzero(box_group == g)[0]
            elems = np.nonzero(tri_group == g)[0]
            fol, folb = _follows(pre, bxs)
            state = ol.lloyd_iteration(V, F, adj, elems, B[bxs, :3], B[bxs, 3:12].reshape(-1, 3, 3), slots[bxs], ev,
                                       K, fol, folb, TIE, counters)[:3]
            fol, folb = _follows(post, bxs)
            a, cl, bx, obv, _ = ol.adjust(V, F, adj, elems, *state, slots[bxs], ev, K, fol, folb, TIE, counters)
            assert int(a) == int(acc[g]), g
            _check_group(post, bxs, cl, bx, obv, ref_tri, gaps)
    record_parity({"test": "lloyd_adjustment_cuboids_and_torus_8x4", "kept": int((acc == 1).sum()),
                   "undone": int((acc == 0).sum()), "ties": counters["ties"],
                   "update_ties": counters.get("update_ties", 0), "max_box_gap": gaps[0],
                   "max_obv_gap_rel": gaps[1]})
    assert np.array_equal(post["tri_box"], ref_tri)
    assert gaps[0] <= 1e-5 and gaps[1] <= 1e-5
