"""Pins of the Lloyd oracle (Sec. 4.2.1) and the layer weights (Sec. 5)."""
import numpy as np

import synth
from oracle import exact, lloyd, raygrid


def _raygrid_eval(V, F, R=6, seed=3):
    def ev(items):
        return [raygrid.raygrid_obv(V, F, c, Q, h, R, seed, int(slot))["obv"] for slot, c, Q, h in items]
    return ev


def _exact_eval(V, F):
    def ev(items):
        out = []
        for _, c, Q, h in items:
            Q64 = Q.astype(np.float64)
            u, _, vt = np.linalg.svd(Q64)
            out.append(exact.obv(V, F, c, u @ vt, h))
        return out
    return ev


def test_bulk_flood_with_one_pop_per_round_is_the_serial_flood():
    V, F = synth.icosphere(1)
    adj = lloyd.adjacency(F)
    group = list(range(len(F)))
    centers = np.array([[0.9, 0.1, 0.0], [-0.5, 0.6, 0.3], [0.0, -0.7, -0.5]], np.float32)
    axes = np.stack([np.eye(3, dtype=np.float32)] * 3)
    ev = _raygrid_eval(V, F)
    a1, b1, o1, _ = lloyd.flood_partition(V, F, adj, group, centers, axes, [0, 1, 2], ev, K=1)
    a2, b2, o2 = lloyd.serial_flood(V, F, adj, group, centers, axes, [0, 1, 2], ev)
    assert a1 == a2
    for x, y in zip(b1, b2):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
    assert np.array_equal(o1, o2)


def test_disjoint_cuboids_one_seed_each_reach_zero_error():
    """k disjoint rotated cuboids (distinct sides), one box per component with
    the component's axes and centre: one Lloyd iteration gives e = 0."""
    V, F, comp, params = synth.disjoint_cuboids(3, seed=7)
    adj = lloyd.adjacency(F)
    centers = np.array([p[0] for p in params], np.float32)
    axes = np.array([p[1] for p in params], np.float32)
    ev = _exact_eval(V, F)
    clusters, boxes, obv, e, _ = lloyd.lloyd_iteration(V, F, adj, range(len(F)), centers, axes, [0, 1, 2],
                                                       ev, K=4)
    for k in range(3):
        assert sorted(clusters[k]) == sorted(np.nonzero(comp == k)[0].tolist())
    vb = sum(8 * np.prod(p[2]) for p in params)
    assert e <= 1e-5 * vb


def test_fig4_min_outer_volume_increase_beats_nearest_centre():
    """Fig. 4: the triangle goes to the box whose outer volume grows least, even
    when another box's centre is nearer."""
    V, F = synth.cuboid((2.0, 0.25, 0.25))
    adj = lloyd.adjacency(F)
    # box 0 rotated 45 degrees about z around (-0.5, 0, 0); box 1 aligned around (1.2, 0, 0)
    r = np.sqrt(0.5)
    Q0 = np.array([[r, r, 0], [-r, r, 0], [0, 0, 1]], np.float32)
    Q1 = np.eye(3, dtype=np.float32)
    ev = _exact_eval(V, F)
    # a small extra triangle near x = 0.2 is emulated by a vertex probe of one mesh triangle:
    # use the flood's own decision on the full strip with fixed seeds instead
    centers = np.array([[-0.5, 0.0, 0.0], [1.2, 0.0, 0.0]], np.float32)
    axes = np.stack([Q0, Q1])
    m = V[F].astype(np.float64).mean(axis=1)
    d0 = np.linalg.norm(m - centers[0], axis=1)
    d1 = np.linalg.norm(m - centers[1], axis=1)
    assign, boxes, obv, _ = lloyd.flood_partition(V, F, adj, range(len(F)), centers, axes, [0, 1], ev, K=1)
    nearer0_to1 = [t for t in assign if d0[t] < d1[t] and assign[t] == 1]
    assert nearer0_to1, "some triangle nearer to centre 0 must be given to box 1"
    # every decision minimises the outer-volume increase (dOBV >= 0 by monotonicity)
    assert all(v >= -1e-12 for v in obv)


def test_parameter_update_never_increases_and_fixes_a_rotated_box():
    V, F = synth.cuboid((0.8, 0.4, 0.2))
    ev = _exact_eval(V, F)
    tris = list(range(len(F)))
    Q = (lloyd.rot_local(2, 0.06) @ np.eye(3)).astype(np.float32)
    base = lloyd.tight_box(V, F, tris, Q)
    base_v = ev([(0, *base)])[0]
    box, v, accepted = lloyd.update_box(V, F, tris, Q, 0, ev)
    assert v <= base_v
    assert accepted and v < 0.5 * base_v


def test_outer_volume_monotone_under_growth():
    """OBV(O') >= OBV(O) for O inside O' (exact evaluator), hence dOBV >= 0."""
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(5, seed=4)
    g = np.random.default_rng(0)
    for b in range(5):
        u, _, vt = np.linalg.svd(a[b].astype(np.float64))
        Q = u @ vt
        h2 = h[b] + g.uniform(0, 0.3, 3)
        assert exact.obv(V, F, c[b], Q, h2) >= exact.obv(V, F, c[b], Q, h[b]) - 1e-12


def test_layer_weights_example():
    """Sec. 5: leaf weight 1.0, the layer above 2.0, and so on."""
    assert lloyd.layer_weights(2) == [2.0, 1.0]
    assert lloyd.layer_weights(4) == [4.0, 3.0, 2.0, 1.0]
    assert lloyd.hierarchy_error([[1.0], [0.5, 0.25]], [2.0, 1.0]) == 2.75


def test_update_takes_a_twin_within_noise_but_not_another_rotation():
    """The parameter update is an argmin over noisy estimates: a twin update
    whose evaluator differs by 5e-7 of the box volume per call is accepted as
    valid (the gradient-noise bound covers it), while the same step taken about
    a direction at right angles to the descent direction is rejected."""
    V, F = synth.noisy_cube_sphere(4, seed=3)
    tris = list(range(0, len(F), 3))
    ev = _raygrid_eval(V, F, R=8)
    rng = np.random.default_rng(1)

    def noisy(items):
        return [v + 5e-7 * lloyd.box_volume(h) * rng.standard_normal() for v, (_, _, _, h) in zip(ev(items), items)]

    Q = (lloyd.rot_local(0, 0.3) @ lloyd.rot_local(2, 0.2)).astype(np.float32)
    mine = lloyd.update_box(V, F, tris, Q, 4, ev)
    twin = lloyd.update_box(V, F, tris, Q, 4, noisy)
    assert np.abs(twin[0][1] - mine[0][1]).max() > 1e-6       # the noise turned the step
    cnt = {}
    got = lloyd.update_box(V, F, tris, Q, 4, ev, follow_box=twin[0], counters=cnt)
    assert cnt["update_ties"] == 1
    assert np.array_equal(got[0][1], twin[0][1]) and np.array_equal(got[0][2], twin[0][2])
    assert abs(got[1] - mine[1]) <= 2e-5 * lloyd.box_volume(mine[0][2])
    # a step of the chosen length about an axis orthogonal to the descent direction
    r = lloyd.rotation_vector(mine[0][1].astype(np.float64) @ Q.astype(np.float64).T)
    assert np.linalg.norm(r) > 0
    perp = np.cross(r, [0.3, -0.5, 0.8])
    perp *= np.linalg.norm(r) / np.linalg.norm(perp)
    wrong = lloyd.tight_box(V, F, tris, lloyd.rodrigues(perp) @ Q.astype(np.float64))
    cnt = {}
    got = lloyd.update_box(V, F, tris, Q, 4, ev, follow_box=wrong, counters=cnt)
    assert cnt.get("update_ties", 0) == 0
    assert np.array_equal(got[0][1], mine[0][1]) and got[1] == mine[1]


def _stalled_cuboids():
    """Three disjoint cuboids; two boxes start in cuboid 0 and one in cuboid 1,
    so no flood reaches cuboid 2 and the partition mixes cuboids 1 and 2."""
    V, F, comp, params = synth.disjoint_cuboids(3, seed=7, spacing=3.0)
    cen = V[F].astype(np.float64).mean(1)
    t0, t1 = np.nonzero(comp == 0)[0], np.nonzero(comp == 1)[0]
    centers = np.array([cen[t0[0]], cen[t0[-1]], cen[t1[0]]], np.float32)
    axes = np.array([params[0][1], params[0][1], params[1][1]], np.float32)
    return V, F, comp, centers, axes


def test_adjustment_reseeds_a_redundant_box():
    """Sec. 4.2.1, third step: plain iterations keep two boxes in one cuboid and
    one box over the other two; each adjustment moves the least important box
    (fewest triangles) into the worst-fitting box and is kept because the error
    drops; after two, every box holds exactly one cuboid; a third is undone and
    leaves the state as it was."""
    V, F, comp, centers, axes = _stalled_cuboids()
    adj = lloyd.adjacency(F)
    ev = _exact_eval(V, F)
    group, slots = range(len(F)), [0, 1, 2]
    cl, bx, obv, e, _ = lloyd.lloyd_iteration(V, F, adj, group, centers, axes, slots, ev, K=4)
    c2, b2, o2, e2, _ = lloyd.lloyd_iteration(V, F, adj, group, [b[0] for b in bx], [b[1] for b in bx], slots, ev,
                                              K=4)
    assert sorted(sorted(set(comp[c])) for c in c2) == [[0], [0], [1, 2]]
    assert lloyd.least_important(cl, obv) in (0, 1)
    state = (cl, bx, obv, e)
    errors = [e]
    for k in range(2):
        acc, *state = lloyd.adjust(V, F, adj, group, *state[:3], slots, ev, K=4)
        assert acc and state[3] < errors[-1]
        errors.append(state[3])
    assert sorted(sorted(set(comp[c])) for c in state[0]) == [[0], [1], [2]]
    acc, c3, b3, o3, e3 = lloyd.adjust(V, F, adj, group, *state[:3], slots, ev, K=4)
    assert not acc and c3 is state[0] and b3 is state[1] and o3 is state[2] and e3 == state[3]


def test_adjustment_is_kept_only_when_the_error_drops():
    """Iterations and adjustments alternating on a noisy sphere: every kept
    adjustment lowers the group's error, every undone one returns the state
    unchanged, so the error after each adjustment never exceeds the error before."""
    V, F = synth.noisy_cube_sphere(4, seed=12)
    adj = lloyd.adjacency(F)
    ev = _raygrid_eval(V, F, R=6)
    g = np.random.default_rng(2)
    cen = V[F].astype(np.float64).mean(1)
    centers = cen[g.choice(len(F), 4, replace=False)].astype(np.float32)
    axes = np.stack([np.eye(3, dtype=np.float32)] * 4)
    group, slots = range(len(F)), [3, 4, 5, 6]
    cl, bx, obv, e, _ = lloyd.lloyd_iteration(V, F, adj, group, centers, axes, slots, ev, K=8)
    outcomes = []
    for _ in range(3):
        acc, cl2, bx2, obv2, e2 = lloyd.adjust(V, F, adj, group, cl, bx, obv, slots, ev, K=8)
        assert e2 <= e
        if acc:
            assert e2 < e
        else:
            assert cl2 is cl and e2 == e
        outcomes.append(acc)
        cl, bx, obv, e, _ = lloyd.lloyd_iteration(V, F, adj, group, [b[0] for b in bx2], [b[1] for b in bx2], slots,
                                                  ev, K=8)
    assert len(outcomes) == 3
