"""Pins of the hierarchy oracle: top-down build, bottom-up merge and the Eq. 7
keep / undo rule of the sweeps (Sec. 4.2.2), weights of Sec. 5."""
import numpy as np

import synth
from oracle import exact, hierarchy, raygrid
from oracle import lloyd as ol


def _two_pairs():
    """Four equal aligned cuboids in two pairs far apart (dyadic coordinates)."""
    Vs, Fs, comp = [], [], []
    for k, c in enumerate([(-3, 0.75, 0), (-3, -0.75, 0), (3, 0.75, 0), (3, -0.75, 0)]):
        V, F = synth.cuboid((0.5, 0.25, 0.375), c)
        Vs.append(V)
        Fs.append(F + 8 * k)
        comp += [k] * len(F)
    return np.vstack(Vs), np.vstack(Fs).astype(np.int32), np.array(comp)


def _exact_eval(V, F):
    def ev(items):
        out = []
        for _, c, Q, h in items:
            u, _, vt = np.linalg.svd(np.asarray(Q, np.float64))
            out.append(exact.obv(V, F, c, u @ vt, h))
        return out
    return ev


def _raygrid_eval(V, F, R=8, seed=5):
    def ev(items):
        return [raygrid.raygrid_obv(V, F, c, Q, h, R, seed, int(k))["obv"] for k, c, Q, h in items]
    return ev


def test_two_pairs_of_cuboids_reach_the_closed_form_error():
    """Root = bounding box of all four cuboids, layer 1 = the two pair boxes,
    leaves = the cuboids (OBV 0), so e = 3 OBV(root) + 2 (2 OBV(pair)) + 0 by hand.
    The seed is one whose draws put the two layer-1 children in different
    pairs (checked) and the leaves in different cuboids (checked below)."""
    V, F, comp = _two_pairs()
    seed = 16
    first = hierarchy.random_seeds(np.arange(len(F)), 2, seed, 1, 0)
    assert comp[first[0]] // 2 != comp[first[1]] // 2
    H, e, td = hierarchy.build(V, F, 3, 2, _exact_eval(V, F), seed, iters=1, sweeps=1, K=8)
    v_cub = 1.0 * 0.5 * 0.75
    root = 7.0 * 2.0 * 0.75 - 4 * v_cub
    pair = 1.0 * 2.0 * 0.75 - 2 * v_cub
    e_star = 3 * root + 2 * (2 * pair) + 1 * 0.0
    assert abs(e[0] - e_star) <= 1e-9 and abs(e[-1] - e_star) <= 1e-9
    A = H.arrays()
    leaves = [sorted(set(comp[A["tri_node"][2] == n])) for n in range(3, 7)]
    assert sorted(leaves) == [[0], [1], [2], [3]]
    pairs = [sorted(set(comp[A["tri_node"][1] == n] // 2)) for n in (1, 2)]
    assert sorted(pairs) == [[0], [1]]
    # the merge regroups the leaves into the same pairs: e does not drop, the merge is undone
    assert H.trace == [("merge", 1, e[0], e[0], False)]


def test_a_merge_that_raises_e_is_undone():
    """A build whose bottom-up merge of layer 1 raises e: the sweep restores the
    top-down state bit for bit and, with no layer merged, re-solves nothing."""
    V, F = synth.noisy_cube_sphere(4, seed=100)
    H, e, td = hierarchy.build(V, F, 3, 3, _raygrid_eval(V, F), 3, iters=1, sweeps=1, K=8)
    (kind, l, e0, e1, kept), = H.trace
    assert kind == "merge" and l == 1 and not kept and e1 > e0 * (1 + 1e-3)
    assert e == [e0, e0]
    A = H.arrays()
    for k in td:
        assert np.array_equal(A[k], td[k]), k


def test_a_resolve_that_raises_e_is_undone():
    """A sweep whose merge lowers e (kept) and whose re-solve of the leaves then
    raises it: the result is the state right after the merge."""
    V, F = synth.noisy_cube_sphere(4, seed=101)
    ev = _raygrid_eval(V, F)
    H, e, td = hierarchy.build(V, F, 3, 3, ev, 3, iters=1, sweeps=1, K=8)
    assert [(t[0], t[1], t[4]) for t in H.trace] == [("merge", 1, True), ("solve", 2, False)]
    assert H.trace[0][3] < H.trace[0][2] and H.trace[1][3] > H.trace[1][2]
    G = hierarchy.Hierarchy(V, F, 3, 3, ev, 3, K=8, iters=1)
    G.top_down()
    G.merge(1)
    assert e[-1] == G.error()
    A, B = H.arrays(), G.arrays()
    for k in A:
        assert np.array_equal(A[k], B[k]), k


def test_hierarchy_structure_enclosure_and_weighted_error():
    """Definition 1 and Eq. 7 on a two-sweep build: every triangle has a node per
    layer, a node's triangles lie in its parent's, every box encloses its
    triangles, e never increases, and e is Sec. 5's weighted sum of outer
    volumes recomputed from the returned boxes."""
    V, F = synth.noisy_cube_sphere(4, seed=102)
    ev = _raygrid_eval(V, F)
    L, b = 3, 3
    H, e, _ = hierarchy.build(V, F, L, b, ev, 7, iters=1, sweeps=2, K=8)
    A = H.arrays()
    tn, parent, boxes = A["tri_node"], A["parent"], A["boxes"]
    assert np.all(tn[0] == 0) and np.all(tn >= 0)
    for lv in range(1, L):
        assert np.array_equal(parent[tn[lv]], tn[lv - 1])
    for node in range(len(boxes)):
        tris = np.nonzero((tn == node).any(axis=0))[0]
        if len(tris) == 0:
            continue
        bx = boxes[node].astype(np.float64)
        loc = (V[np.unique(F[tris])].astype(np.float64) - bx[:3]) @ bx[3:12].reshape(3, 3).T
        assert np.all(np.abs(loc) <= bx[12:]), node
    assert all(x >= y for x, y in zip(e, e[1:]))
    level = np.concatenate([[lv] * b ** lv for lv in range(L)])
    used = np.array([(tn == n).any() for n in range(len(boxes))])
    again = np.array(ev([(n, boxes[n][:3], boxes[n][3:12].reshape(3, 3), boxes[n][12:]) for n in range(len(boxes))]))
    w = np.array(ol.layer_weights(L))[level]
    assert abs(np.sum(w[used] * again[used]) - e[-1]) <= 1e-12 * e[-1]


def test_following_another_build_changes_nothing_beyond_the_tie_tolerance():
    """Named choices are taken only where they are as valid as the build's own:
    with both tolerances 0 another build's choices are ignored, and naming the
    build's own choices reproduces it with nothing taken."""
    V, F = synth.noisy_cube_sphere(4, seed=103)
    ev = _raygrid_eval(V, F)
    H0, e0, td0 = hierarchy.build(V, F, 3, 2, ev, 1, iters=1, sweeps=1, K=8)
    A0 = H0.arrays()
    _, _, other = hierarchy.build(V, F, 3, 2, ev, 2, iters=1, sweeps=0, K=8)
    fol = hierarchy.FollowArrays(other, 3, 2)
    H1, e1, _ = hierarchy.build(V, F, 3, 2, ev, 1, iters=1, sweeps=1, K=8, follow_top_down=fol,
                                follow_sweeps=fol, tie=0.0, eps=0.0)
    H2, e2, _ = hierarchy.build(V, F, 3, 2, ev, 1, iters=1, sweeps=1, K=8,
                                follow_top_down=hierarchy.FollowArrays(td0, 3, 2),
                                follow_sweeps=hierarchy.FollowArrays(A0, 3, 2))
    assert e1 == e0 and e2 == e0
    for H in (H1, H2):
        assert H.counters["ties"] == 0 and H.counters["update_ties"] == 0
    for k in A0:
        assert np.array_equal(H1.arrays()[k], A0[k]) and np.array_equal(H2.arrays()[k], A0[k]), k


def test_unit_adjacency_is_mesh_edges_between_units():
    """Two units are neighbours exactly when some mesh edge joins a triangle of
    each (brute force over all triangle pairs sharing two vertices)."""
    V, F = synth.icosphere(1)
    rng = np.random.default_rng(0)
    unit_of = rng.integers(0, 6, len(F))
    units = [np.nonzero(unit_of == u)[0] for u in range(6)]
    E = ol.unit_elements(V, F, ol.adjacency(F), units, np.zeros((6, 3), np.float32))
    want = [set() for _ in range(6)]
    for s in range(len(F)):
        for t in range(len(F)):
            if len(set(F[s]) & set(F[t])) == 2 and unit_of[s] != unit_of[t]:
                want[unit_of[s]].add(unit_of[t])
    assert [set(a) for a in E.adj] == want
