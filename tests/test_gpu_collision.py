"""Collision queries on the device (obbv_collision_queries) against the oracle,
count for count, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import collision

from conftest import record_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def _used(tri_node, levels, b):
    used, base = [], 0
    for l in range(levels):
        n = b ** l
        present = np.zeros(n, bool)
        ids = tri_node[l][tri_node[l] >= 0] - base
        present[ids[(ids >= 0) & (ids < n)]] = True
        used.append(present)
        base += n
    return used


@pytest.fixture(scope="module")
def hierarchies(api):
    import torch
    V, F = synth.noisy_torus(nu=64, nv=32)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    L, b = 3, 4
    hier = api.build_hierarchy(Vt, Ft, levels=L, branching=b, iters=2, sweeps=0, R=16, seed=3, pops_per_round=8)
    tree = api.build_obb_tree(Vt, Ft, L, b)
    return V, L, b, {"hierarchy": (hier["boxes"], _used(hier["tri_node"], L, b)),
                     "obb_tree": (tree["boxes"], _used(tree["tri_node"], L, b))}


@pytest.mark.parametrize("which", ["hierarchy", "obb_tree"])
def test_collision_counts_match_the_oracle(api, hierarchies, which):
    """2,000 spheres of mixed radii around the torus: tests and hits of every
    query equal the oracle's (float64 decisions on both sides)."""
    import torch
    V, L, b, h = hierarchies
    boxes, used = h[which]
    S = synth.query_spheres(V, 2000, seed=7)
    tests, hits = api.collision_queries(torch.from_numpy(boxes).cuda(), L, b, torch.from_numpy(S).cuda(),
                                        node_used=torch.from_numpy(np.concatenate(used).astype(np.uint8)).cuda())
    ot, oh = collision.queries(L, b, collision.boxes_by_level(boxes.astype(np.float64), L, b),
                               [u.tolist() for u in used], S.astype(np.float64))
    assert np.array_equal(tests.cpu().numpy(), np.array(ot, np.int32))
    assert np.array_equal(hits.cpu().numpy(), np.array(oh, np.int32))
    record_parity({"test": f"collision_queries_{which}", "spheres": len(S), "tests": int(sum(ot)),
                   "hits": int(sum(oh))})


def test_collision_all_nodes_used_and_edge_sizes(api, hierarchies):
    """Without a used mask every node is tested as used; an empty query list
    does nothing; a wrongly sized node array is rejected by the binding."""
    import torch
    V, L, b, h = hierarchies
    boxes, used = h["obb_tree"]
    S = synth.query_spheres(V, 300, seed=9)
    tests, hits = api.collision_queries(torch.from_numpy(boxes).cuda(), L, b, torch.from_numpy(S).cuda())
    ones = [[True] * (b ** l) for l in range(L)]
    ot, oh = collision.queries(L, b, collision.boxes_by_level(boxes.astype(np.float64), L, b), ones,
                               S.astype(np.float64))
    assert np.array_equal(tests.cpu().numpy(), np.array(ot, np.int32))
    assert np.array_equal(hits.cpu().numpy(), np.array(oh, np.int32))
    t0, h0 = api.collision_queries(torch.from_numpy(boxes).cuda(), L, b, torch.zeros((0, 4), device="cuda"))
    assert t0.numel() == 0 and h0.numel() == 0
    with pytest.raises(ValueError):
        api.collision_queries(torch.from_numpy(boxes[:-1].copy()).cuda(), L, b, torch.from_numpy(S).cuda())


def test_collision_on_random_nested_trees(api):
    """Random trees whose children lie inside their parents, some nodes unused,
    3 to 4 levels and branching 2 to 5: every query's tests and hits equal the
    oracle's."""
    import torch
    rng = np.random.default_rng(4)
    I3 = np.eye(3)
    for levels, b in ((3, 5), (4, 2), (4, 3)):
        rows = [np.concatenate([[0.0, 0.0, 0.0], I3.reshape(-1), [1.0, 1.0, 1.0]])]
        used = [True]
        base, n = 0, 1
        for l in range(1, levels):
            for j in range(n):
                pc, ph = rows[base + j][0:3], rows[base + j][12:15]
                for k in range(b):
                    lo = pc[0] - ph[0] + 2 * ph[0] * k / b
                    hx = ph[0] / b * rng.uniform(0.4, 1.0)
                    cx = lo + ph[0] / b
                    hy, hz = ph[1] * rng.uniform(0.3, 1.0), ph[2] * rng.uniform(0.3, 1.0)
                    cy = pc[1] + rng.uniform(-(ph[1] - hy), ph[1] - hy)
                    cz = pc[2] + rng.uniform(-(ph[2] - hz), ph[2] - hz)
                    rows.append(np.concatenate([[cx, cy, cz], I3.reshape(-1), [hx, hy, hz]]))
                    used.append(bool(used[base + j]) and rng.uniform() > 0.15)
            base += n
            n *= b
        flat = np.array(rows, np.float32)
        u = np.array(used, np.uint8)
        S = np.concatenate([rng.uniform(-1.3, 1.3, (500, 3)), rng.uniform(0.0, 0.5, (500, 1))], axis=1)
        S = S.astype(np.float32)
        tests, hits = api.collision_queries(torch.from_numpy(flat).cuda(), levels, b, torch.from_numpy(S).cuda(),
                                            node_used=torch.from_numpy(u).cuda())
        bl = collision.boxes_by_level(flat.astype(np.float64), levels, b)
        ul, base = [], 0
        for l in range(levels):
            ul.append([bool(x) for x in u[base:base + b ** l]])
            base += b ** l
        ot, oh = collision.queries(levels, b, bl, ul, S.astype(np.float64))
        assert np.array_equal(tests.cpu().numpy(), np.array(ot, np.int32)), (levels, b)
        assert np.array_equal(hits.cpu().numpy(), np.array(oh, np.int32)), (levels, b)
