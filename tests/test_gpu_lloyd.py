"""HIP-evaluated Lloyd step and hierarchy vs the CPU oracle (needs an MI355X)."""
import numpy as np
import pytest

import synth
from conftest import record_parity
from oracle import lloyd as olloyd
from oracle import raygrid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def _dev(V, F):
    import torch
    return torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()


def _raygrid_eval(V, F, R, seed):
    def ev(items):
        return [raygrid.raygrid_obv(V, F, c, Q, h, R, seed, int(slot))["obv"] for slot, c, Q, h in items]
    return ev


def _pack(centers, axes):
    n = len(centers)
    return synth.boxes_to_array(centers, axes, np.zeros((n, 3), np.float32))


@pytest.mark.parametrize("K", [1, 4])
def test_one_lloyd_iteration_matches_the_oracle(api, K):
    """Same input state, one iteration (flood + parameter update): identical
    partition and boxes, OBV within 1e-5 of the box volume."""
    V, F = synth.noisy_cube_sphere(4, seed=5)
    adj = olloyd.adjacency(F)
    centers = np.array([[0.8, 0.2, 0.1], [-0.6, 0.5, -0.2], [0.0, -0.7, 0.6]], np.float32)
    _, ax, _ = synth.random_boxes(3, seed=9)
    R, seed = 8, 3
    clusters, boxes, obv, e, _ = olloyd.lloyd_iteration(V, F, adj, range(len(F)), centers, ax, [10, 11, 12],
                                                        _raygrid_eval(V, F, R, seed), K=K)
    Vt, Ft = _dev(V, F)
    with api.Lloyd(Vt, Ft, R=R, seed=seed, pops_per_round=K) as L:
        L.set_groups(np.zeros(len(F), np.int32), np.zeros(3, np.int32), _pack(centers, ax), [10, 11, 12])
        L.step()
        out = L.get()
    ref_box = np.full(len(F), -1)
    for k, ts in enumerate(clusters):
        ref_box[ts] = k
    assert np.array_equal(out["tri_box"], ref_box)
    for k in range(3):
        c, Q, h = boxes[k]
        got = out["boxes"][k]
        assert np.allclose(got[:3], c, atol=1e-6) and np.allclose(got[3:12], Q.reshape(-1), atol=1e-6)
        assert np.allclose(got[12:], h, atol=1e-6)
        vb = 8 * np.prod(h.astype(np.float64))
        assert abs(out["obv"][k] - obv[k]) <= 1e-5 * vb
    assert out["counters"]["evals"] > 0


def test_disjoint_cuboids_reach_zero(api):
    V, F, comp, params = synth.disjoint_cuboids(3, seed=7)
    centers = np.array([p[0] for p in params], np.float32)
    axes = np.array([p[1] for p in params], np.float32)
    Vt, Ft = _dev(V, F)
    with api.Lloyd(Vt, Ft, R=16, seed=1, pops_per_round=8) as L:
        L.set_groups(np.zeros(len(F), np.int32), np.zeros(3, np.int32), _pack(centers, axes))
        L.step()
        out = L.get()
    for k in range(3):
        assert set(np.nonzero(out["tri_box"] == k)[0]) == set(np.nonzero(comp == k)[0])
    vb = sum(8 * np.prod(p[2]) for p in params)
    assert out["layer_error"] <= 1e-5 * vb


def test_hierarchy_structure_enclosure_and_error(api):
    """Small hierarchy: every triangle has a node per layer, a node's triangles
    lie in its parent's, every box encloses its triangles (F_i in O_i), the
    root covers the mesh (Definition 1), e never increases over the sweeps and
    equals Eq. 7 recomputed from the returned boxes."""
    import torch
    V, F = synth.noisy_cube_sphere(6, seed=8)
    Vt, Ft = _dev(V, F)
    L, b, R, seed = 3, 2, 8, 5
    out = api.build_hierarchy(Vt, Ft, levels=L, branching=b, iters=2, sweeps=2, R=R, seed=seed,
                              pops_per_round=8)
    boxes, obv, parent, tri_node, e = out["boxes"], out["obv"], out["parent"], out["tri_node"], out["e"]
    n_nodes = 1 + b + b * b
    assert boxes.shape == (n_nodes, 15)
    assert np.all(tri_node[0] == 0) and np.all(tri_node >= 0)
    for lv in range(1, L):
        assert np.array_equal(parent[tri_node[lv]], tri_node[lv - 1])
    for node in range(n_nodes):
        tris = np.nonzero((tri_node == node).any(axis=0))[0]
        if len(tris) == 0:
            continue
        bx = boxes[node].astype(np.float64)
        idx = np.unique(F[tris])
        loc = (V[idx].astype(np.float64) - bx[:3]) @ bx[3:12].reshape(3, 3).T
        assert np.all(np.abs(loc) <= bx[12:] * (1 + 1e-6) + 1e-6), node
    assert np.all(np.diff(e) <= 0)
    # Eq. 7 with omega = layers to the leaves, from OBVs recomputed on the device
    key = torch.from_numpy(np.arange(n_nodes, dtype=np.int32)).cuda()
    re = api.outer_volume(Vt, Ft, torch.from_numpy(boxes).cuda(), R, seed=seed, box_key=key).cpu().numpy()
    level = np.concatenate([[lv] * b ** lv for lv in range(L)])
    used = np.array([(tri_node == n).any() for n in range(n_nodes)])
    assert np.allclose(re[used], obv[used], rtol=0, atol=1e-12)
    w = (L - level).astype(np.float64)
    assert abs(np.sum(w * obv) - e[-1]) <= 1e-9 * max(1.0, e[-1])


def test_jitter_table_gives_the_same_bits_as_computed_draws(api, monkeypatch):
    """The Lloyd evaluator reads the ray jitter from a per-key table when the
    keys are few; with the table turned off the ray-test kernel recomputes
    every SplitMix64 draw.  Both must give bit-identical hierarchies."""
    V, F = synth.noisy_cube_sphere(6, seed=21)
    Vt, Ft = _dev(V, F)
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("OBBV_JITTER_TABLE", flag)
        out[flag] = api.build_hierarchy(Vt, Ft, levels=3, branching=2, iters=2, sweeps=1, R=16, seed=4,
                                        pops_per_round=8)
    for k in ("boxes", "obv", "parent", "tri_node", "e"):
        assert np.array_equal(out["1"][k], out["0"][k]), k


def test_containment_masks_give_the_same_bits_as_candidate_boxes(api, monkeypatch):
    """The flood decides a pop that a box of its group already contains from a
    containment mask taken while the device works, re-testing only boxes that
    grew since; with the masks turned off every pop builds its candidate boxes
    and the decision loop finds the contained ones.  Both must give
    bit-identical hierarchies and counters."""
    V, F = synth.noisy_cube_sphere(8, seed=23)
    Vt, Ft = _dev(V, F)
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("OBBV_FLOOD_MASKS", flag)
        out[flag] = api.build_hierarchy(Vt, Ft, levels=3, branching=4, iters=3, sweeps=1, R=16, seed=6,
                                        pops_per_round=8)
    for k in ("boxes", "obv", "parent", "tri_node", "e"):
        assert np.array_equal(out["1"][k], out["0"][k]), k
    assert out["1"]["counters"] == out["0"]["counters"]
    assert out["1"]["counters"]["trivial"] > 0


def test_flood_on_several_streams_gives_the_same_bits(api, monkeypatch):
    """Floods of two or more independent groups (the children of different
    parents) run in parts of about equal size on host threads, each with its
    own evaluator and stream (OBBV_FLOOD_STREAMS parts, default 4); with 1, one
    thread floods every group in shared rounds.  The hierarchies are
    bit-identical and so are the counters, except rounds (the parts count their
    rounds separately)."""
    V, F = synth.noisy_cube_sphere(8, seed=29)
    Vt, Ft = _dev(V, F)
    out = {}
    for flag in ("1", "2", "4"):
        monkeypatch.setenv("OBBV_FLOOD_STREAMS", flag)
        out[flag] = api.build_hierarchy(Vt, Ft, levels=3, branching=4, iters=3, sweeps=1, R=16, seed=9,
                                        pops_per_round=8)
    # four streams with the frame lists built in two passes (each pass reads a
    # list total back through the host word of its own scratch set)
    monkeypatch.setenv("OBBV_FLOOD_STREAMS", "4")
    monkeypatch.setenv("OBBV_FRAME_LISTS", "2")
    out["4, two-pass lists"] = api.build_hierarchy(Vt, Ft, levels=3, branching=4, iters=3, sweeps=1, R=16, seed=9,
                                                   pops_per_round=8)
    c1 = dict(out["1"]["counters"])
    r1 = c1.pop("rounds")
    for flag in ("2", "4", "4, two-pass lists"):
        for k in ("boxes", "obv", "parent", "tri_node", "e"):
            assert np.array_equal(out[flag][k], out["1"][k]), (flag, k)
        c = dict(out[flag]["counters"])
        assert c.pop("rounds") >= r1
        assert c == c1


def test_smaller_items_for_calls_that_run_alone_give_the_same_bits(api, monkeypatch):
    """Calls of a flood on one stream that would have few cast units take
    smaller cast items (OBBV_ALONE_ITEM_TRIS entries below
    OBBV_ALONE_SPLIT_BELOW units).  With every flood on one stream and the
    threshold above any call's units, every call of the floods is split; the
    hierarchies and counters are bit-identical to unsplit calls.  12,288
    triangles: whole-mesh casts cut their span-culled runs into pieces, and
    grouped casts their frame lists."""
    V, F = synth.noisy_cube_sphere(32, seed=33)
    Vt, Ft = _dev(V, F)
    monkeypatch.setenv("OBBV_FLOOD_STREAMS", "1")
    monkeypatch.setenv("OBBV_ALONE_SPLIT_BELOW", str(1 << 30))
    out = {}
    for items in ("0", "768", "1536", "2304"):
        monkeypatch.setenv("OBBV_ALONE_ITEM_TRIS", items)
        out[items] = api.build_hierarchy(Vt, Ft, levels=3, branching=4, iters=3, sweeps=1, R=32, seed=12,
                                         pops_per_round=8)
    for items in ("768", "1536", "2304"):
        for k in ("boxes", "obv", "parent", "tri_node", "e"):
            assert np.array_equal(out[items][k], out["0"][k]), (items, k)
        assert out[items]["counters"] == out["0"]["counters"]


@pytest.mark.timeout(300)
def test_bench_hierarchy_full_size_properties_and_sampled_parity(api):
    """The timed workload at full size and in the same launch configuration
    (noisy torus of 65,536 triangles, 4 levels of branching 4, 20 Lloyd
    iterations per level, 2 sweeps, R = 128, 32 pops per round, floods on four
    streams): Definition 1 structure, every node's box encloses its triangles,
    e never increases, the returned OBVs are what the device gives for the
    returned boxes (keys = node ids) and their Eq. 7 sum is e; three sampled
    nodes (the root, one of level 1, one of level 3) match the oracle within
    1e-5 of their box volume."""
    import torch
    V, F = synth.noisy_torus()
    Vt, Ft = _dev(V, F)
    L, b, R, seed = 4, 4, 128, 23
    out = api.build_hierarchy(Vt, Ft, levels=L, branching=b, iters=20, sweeps=2, R=R, seed=seed,
                              pops_per_round=32)
    boxes, obv, parent, tri_node, e = out["boxes"], out["obv"], out["parent"], out["tri_node"], out["e"]
    n_nodes = sum(b ** lv for lv in range(L))
    assert boxes.shape == (n_nodes, 15)
    assert np.all(tri_node[0] == 0) and np.all(tri_node >= 0)
    for lv in range(1, L):
        assert np.array_equal(parent[tri_node[lv]], tri_node[lv - 1])
    used = np.array([(tri_node == n).any() for n in range(n_nodes)])
    for node in np.nonzero(used)[0]:
        tris = np.nonzero((tri_node == node).any(axis=0))[0]
        bx = boxes[node].astype(np.float64)
        idx = np.unique(F[tris])
        loc = (V[idx].astype(np.float64) - bx[:3]) @ bx[3:12].reshape(3, 3).T
        assert np.all(np.abs(loc) <= bx[12:] * (1 + 1e-6) + 1e-6), node
    assert np.all(np.diff(e) <= 0)
    key = torch.from_numpy(np.arange(n_nodes, dtype=np.int32)).cuda()
    re = api.outer_volume(Vt, Ft, torch.from_numpy(boxes).cuda(), R, seed=seed, box_key=key).cpu().numpy()
    assert np.allclose(re[used], obv[used], rtol=0, atol=1e-12)
    level = np.concatenate([[lv] * b ** lv for lv in range(L)])
    assert abs(np.sum((L - level) * obv) - e[-1]) <= 1e-9 * max(1.0, e[-1])
    worst = 0.0
    for node in (0, 1 + int(np.argmax(used[1:1 + b])), 1 + b + b * b + int(np.argmax(used[1 + b + b * b:]))):
        bx = boxes[node].astype(np.float32)
        ref = raygrid.raygrid_obv(V, F, bx[:3], bx[3:12].reshape(3, 3), bx[12:], R, seed, node)
        vb = 8.0 * np.prod(bx[12:].astype(np.float64))
        err = abs(obv[node] - ref["obv"]) / vb
        worst = max(worst, err)
        assert err <= 1e-5, (node, obv[node], ref["obv"])
    record_parity({"test": "bench_hierarchy_full_size", "nodes": int(used.sum()), "e": float(e[-1]),
                   "sampled_max_err_rel": worst})
