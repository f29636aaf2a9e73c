"""Pins of the collision-query oracle (synthetic stand-in for the paper's
collision experiment, Sec. 5) against geometry fixed independently of it."""
import numpy as np
import pytest
from scipy.optimize import minimize

import synth
from oracle import collision


I3 = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]


def test_touching_faces_edges_and_corners():
    """Unit half-extent box at the origin: a sphere reaching exactly to a face,
    an edge or a corner overlaps (closed sets); one 1e-9 short does not."""
    h = [1.0, 1.0, 1.0]
    c = [0.0, 0.0, 0.0]
    assert collision.sphere_overlaps_box([3.0, 0.0, 0.0], 2.0, c, I3, h)
    assert not collision.sphere_overlaps_box([3.0, 0.0, 0.0], 2.0 - 1e-9, c, I3, h)
    assert collision.sphere_overlaps_box([4.0, 5.0, 0.5], 5.0, c, I3, h)           # edge: 3-4-5
    assert not collision.sphere_overlaps_box([4.0, 5.0, 0.5], 5.0 - 1e-9, c, I3, h)
    assert collision.sphere_overlaps_box([3.0, 3.0, 2.0], 3.0, c, I3, h)           # corner: 2,2,1 -> 3
    assert not collision.sphere_overlaps_box([3.0, 3.0, 2.0], 3.0 - 1e-9, c, I3, h)
    assert collision.sphere_overlaps_box([0.2, -0.3, 0.1], 0.0, c, I3, h)          # centre inside, r = 0


def _distance_by_minimisation(x, c, Q, h):
    """Distance from x to the box found numerically: minimise |c + Q^T p - x|
    over the box p in [-h, h] (bounded quasi-Newton from the box centre)."""
    Qa = np.asarray(Q, np.float64)
    f = lambda p: float(np.sum((np.asarray(c) + Qa.T @ p - np.asarray(x)) ** 2))
    g = lambda p: 2.0 * (Qa @ (np.asarray(c) + Qa.T @ p - np.asarray(x)))
    res = minimize(f, np.zeros(3), jac=g, method="L-BFGS-B", bounds=[(-hk, hk) for hk in h],
                   options={"ftol": 1e-15, "gtol": 1e-12})
    return float(np.sqrt(res.fun))


def test_overlap_agrees_with_numerical_distance_on_rotated_boxes():
    """Random rotated boxes and spheres, away from tangency (|distance - r| >
    1e-4): the overlap decision agrees with the distance found by bounded
    minimisation."""
    rng = np.random.default_rng(3)
    c, a, h = synth.random_boxes(40, seed=19, center_range=0.5, half_range=(0.1, 0.7))
    checked = 0
    for i in range(40):
        for _ in range(10):
            x = rng.uniform(-2.0, 2.0, 3)
            dist = _distance_by_minimisation(x, c[i].astype(np.float64), a[i].astype(np.float64),
                                             h[i].astype(np.float64))
            r = float(rng.uniform(0.0, 1.5))
            if abs(dist - r) < 1e-4:
                continue
            assert collision.sphere_overlaps_box(x, r, c[i], a[i].tolist(), h[i]) == (dist <= r), (i, dist, r)
            checked += 1
    assert checked > 350


def _nested_tree(levels, b, seed):
    """Axis-aligned boxes, each child inside its parent (a random sub-box of
    one cell of the parent split along x), some nodes unused."""
    rng = np.random.default_rng(seed)
    boxes = [[([0.0, 0.0, 0.0], I3, [1.0, 1.0, 1.0])]]
    used = [[True]]
    for l in range(1, levels):
        lv, uv = [], []
        for j, (pc, _, ph) in enumerate(boxes[l - 1]):
            for k in range(b):
                lo = pc[0] - ph[0] + 2 * ph[0] * k / b
                hi = lo + 2 * ph[0] / b
                cx = rng.uniform(lo + 0.25 * (hi - lo), hi - 0.25 * (hi - lo))
                hx = min(cx - lo, hi - cx) * rng.uniform(0.5, 1.0)
                hy, hz = ph[1] * rng.uniform(0.3, 1.0), ph[2] * rng.uniform(0.3, 1.0)
                cy = pc[1] + rng.uniform(-(ph[1] - hy), ph[1] - hy)
                cz = pc[2] + rng.uniform(-(ph[2] - hz), ph[2] - hz)
                lv.append(([cx, cy, cz], I3, [hx, hy, hz]))
                uv.append(bool(used[l - 1][j]) and rng.uniform() > 0.1)
        boxes.append(lv)
        used.append(uv)
    return boxes, used


def test_traversal_counts_match_a_scan_of_a_nested_tree():
    """With every child inside its parent, a node is tested iff its parent is
    used and overlapped (a node overlapped implies its ancestors are), and the
    hits are the used leaves whose box the sphere overlaps: both counted by a
    plain scan of all nodes, without descending."""
    L, b = 4, 3
    boxes, used = _nested_tree(L, b, seed=8)
    rng = np.random.default_rng(11)
    for _ in range(200):
        x = rng.uniform(-1.3, 1.3, 3)
        r = float(rng.uniform(0.0, 0.6))
        tests, hits = collision.query(L, b, boxes, used, x, r)
        ov = [[used[l][j] and collision.sphere_overlaps_box(x, r, *boxes[l][j]) for j in range(b ** l)]
              for l in range(L)]
        want_tests = 1 + sum(1 for l in range(1, L) for j in range(b ** l)
                             if used[l][j] and ov[l - 1][j // b])
        want_hits = sum(ov[L - 1])
        assert (tests, hits) == (want_tests, want_hits)


def test_everything_and_nothing():
    """A sphere holding the whole tree tests every used node and hits every used
    leaf; a sphere far away tests the root only."""
    L, b = 3, 4
    boxes, used = _nested_tree(L, b, seed=2)
    n_used = sum(sum(u) for u in used)
    t, h = collision.query(L, b, boxes, used, [0.0, 0.0, 0.0], 10.0)
    assert t == n_used and h == sum(used[L - 1])
    assert collision.query(L, b, boxes, used, [50.0, 0.0, 0.0], 1.0) == (1, 0)


def test_boxes_by_level_layout():
    """Level-order rows map to boxes[l][j] with centre, axis rows and half extents."""
    flat = np.arange(5 * 15, dtype=np.float64).reshape(5, 15)
    bl = collision.boxes_by_level(flat, 2, 4)
    assert len(bl) == 2 and len(bl[0]) == 1 and len(bl[1]) == 4
    c, Q, h = bl[1][2]
    assert c == list(flat[3, 0:3]) and Q[1] == list(flat[3, 6:9]) and h == list(flat[3, 12:15])
