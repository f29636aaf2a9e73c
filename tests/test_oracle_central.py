"""Pins of the central-projection oracle (Sec. 4.1, Eq. 9-10) against facts
fixed independently of it: closed-form solid angles, the paper's worked
example of Eq. 9, exact cases, watertightness on exact edge and vertex hits,
and convergence to the exact outer volume (itself pinned by closed forms)."""
import math

import numpy as np
import pytest

import synth
from oracle import central, exact


def test_pixel_solid_angles_cover_the_sphere():
    """The 6 m^2 pixel cones cover the sphere once (4 pi) and each face 4 pi / 6;
    the centre pixel of m = 1 is a whole face."""
    for m in (1, 3, 8):
        d, W = central.face_pixels(m)
        assert len(d) == 6 * m * m and np.all(W > 0)
        assert abs(W.sum() - 4 * math.pi) < 1e-12
        assert abs(W[: m * m].sum() - 4 * math.pi / 6) < 1e-12


def test_eq9_worked_example():
    """Eq. 9's example (centre inside; crossings p0 leaving, p1 entering, p2
    leaving, all before p_e): l_out = p_e o - (p_2 o - p_1 o + p_0 o).  A
    crossing beyond the box counts as reaching p_e."""
    r0, r1, r2, re = 0.3, 0.7, 1.1, 1.6
    l_in = central.cone_terms([r0, r1, r2], [1, -1, 1], re, power=1)
    assert abs((re - l_in) - (re - (r2 - r1 + r0))) < 1e-15
    # centre outside, entering at 0.4, leaving beyond the box at 2.0: inside from 0.4 to p_e
    assert abs(central.cone_terms([0.4, 2.0], [-1, 1], re, power=1) - (re - 0.4)) < 1e-15


def test_box_inside_the_solid_is_zero_and_far_box_is_its_own_quadrature():
    """A box inside the solid gives exactly 0 (every ray's crossings lie beyond
    it and sum to one exit); a box away from the solid gives the quadrature of
    its own volume, which tends to 8 h0 h1 h2."""
    V, F = synth.icosphere(3)
    I3 = np.eye(3)
    assert central.obv(V, F, [0.05, -0.02, 0.03], I3, [0.2, 0.15, 0.25], 6) == 0.0
    h = np.array([0.3, 0.2, 0.4])
    q = []
    for m in (4, 16):
        d, W = central.face_pixels(m)
        re = np.array([min(h[k] / abs(x[k]) for k in range(3) if x[k] != 0.0) * np.linalg.norm(x) for x in d])
        q.append(float(np.sum(re ** 3 * W) / 3.0))
        assert central.obv(V, F, [5.0, 0.0, 0.0], I3, h, m) == pytest.approx(q[-1], rel=1e-14)
    vb = 8 * h.prod()
    assert abs(q[1] - vb) < abs(q[0] - vb) < 0.05 * vb


def test_exact_edge_and_vertex_hits_count_once():
    """Octahedron |x| + |y| + |z| <= 1 around the centre: rays through its
    vertices (4 triangles meet) and edge midpoints (2 meet) and a generic ray
    each cross it exactly once, leaving, at the right depth; from outside, a
    ray through an edge enters and leaves once each."""
    V, F = synth.octahedron(1.0)
    T = np.asarray(V, np.float64)[np.asarray(F, np.int64)]
    for d, t_want in (([1.0, 0.0, 0.0], 1.0), ([0.0, -1.0, 0.0], 1.0), ([0.0, 0.0, 1.0], 1.0),
                      ([1.0, 1.0, 0.0], 0.5), ([0.0, -1.0, 1.0], 0.5), ([1.0, 1.0, 1.0], 1.0 / 3.0),
                      ([0.3, 0.2, 0.5], 1.0)):
        t, s = central.ray_crossings(T, np.array(d))
        assert len(t) == 1 and s[0] == 1.0, (d, t, s)
        assert abs(t[0] - t_want) < 1e-15
    # shift the solid so the ray from the origin along +x passes through the
    # edge from (1, 0, 0) to (0, 1, 0) of the moved octahedron's near side
    T2 = T + np.array([2.0, -0.5, 0.0])
    t, s = central.ray_crossings(T2, np.array([1.0, 0.0, 0.0]))
    assert sorted(s.tolist()) == [-1.0, 1.0]
    assert abs(t.min() - 1.5) < 1e-15 and abs(t.max() - 2.5) < 1e-15


def test_estimator_converges_to_the_exact_outer_volume():
    """Random boxes over the icosphere: the mean error against the exact OBV
    (relative to V_box) shrinks from m = 4 to m = 16 and is below 2e-3 at 16."""
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(6, seed=3, center_range=0.6, half_range=(0.2, 0.6))
    err = {}
    for m in (4, 16):
        e = []
        for i in range(6):
            ex = exact.obv(V, F, c[i], a[i], h[i].astype(np.float64))
            e.append(abs(central.obv(V, F, c[i], a[i], h[i], m) - ex) / exact.box_volume(h[i]))
        err[m] = float(np.mean(e))
    assert err[16] < err[4] and err[16] < 2e-3
