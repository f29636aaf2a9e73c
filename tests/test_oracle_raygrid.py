"""Pins of the discrete ray-grid oracle D_R (Sec. 4.1, Eq. 9 generalised)."""
import numpy as np
import pytest

import synth
from oracle import exact, raygrid


def _ortho(a):
    u, _, vt = np.linalg.svd(np.asarray(a, dtype=np.float64))
    return u @ vt


def test_eq9_worked_example():
    """Sec. 4.1: centre inside the solid, the ray crosses p0 (leaving), p1
    (entering), p2 (leaving) before hitting the box at p_e:
    l_out = |p_e o| - (|p2 o| - |p1 o| + |p0 o|)."""
    t0, t1, t2, te = 0.3, 0.55, 0.8, 1.0
    got = raygrid.eq9_outside_length([t0, t1, t2], [+1, -1, +1], te)
    assert got == pytest.approx(te - (t2 - t1 + t0), abs=1e-15)
    # the generalised form also covers the box face being inside the solid
    # (a crossing beyond p_e): then the segment past t2 is inside again
    got2 = raygrid.eq9_outside_length([t0, t1, 1.4], [+1, -1, +1], te)
    assert got2 == pytest.approx((t1 - t0), abs=1e-15)


def test_parity_length_brute_force():
    """Parity length of a line against a fine sampling of the parity rule."""
    g = np.random.default_rng(3)
    for _ in range(50):
        d = np.sort(g.uniform(-2, 2, size=g.integers(0, 7)))
        h = g.uniform(0.1, 1.5)
        L = raygrid.parity_inside_length(d, h)
        t = np.linspace(-h, h, 200001)[:-1] + h / 200000
        inside = (np.searchsorted(d, t) % 2) == 1
        assert abs(L - inside.mean() * 2 * h) <= 2e-4 * h


def test_inside_and_disjoint_are_exact_for_any_seed():
    V, F = synth.icosphere(3)
    _, a, _ = synth.random_boxes(1, seed=8)
    for seed in (1, 2, 3):
        r_in = raygrid.raygrid_obv(V, F, [0.05, 0.0, -0.05], a[0], [0.3, 0.25, 0.2], 8, seed)
        assert r_in["obv"] == 0.0
        r_out = raygrid.raygrid_obv(V, F, [3.0, 0.2, 0.0], a[0], [0.3, 0.25, 0.2], 8, seed)
        assert r_out["obv"] == r_out["v_box"]


def test_aligned_cuboid_on_grid_lines_is_exact():
    """Cuboid faces on grid lines of the ray grid: every ray is fully in or out
    in (u, v), so D_R equals the exact value for any jitter."""
    V, F = synth.cuboid((0.5, 0.25, 0.75), center=(0.25, 0.0, 0.0))
    # box [-1, 1]^3 with R = 8: grid lines at multiples of 0.25
    for seed in (5, 6):
        r = raygrid.raygrid_obv(V.astype(np.float64), F, [0, 0, 0], np.eye(3), [1, 1, 1], 8, seed)
        assert abs(r["v_in"] - 0.5 * 2 * 0.25 * 2 * 0.75 * 2) <= 1e-14


def test_parity_equals_signed_per_ray():
    V, F = synth.noisy_torus(nu=48, nv=24)
    c, a, h = synth.random_boxes(3, seed=12, center_range=1.0, half_range=(0.2, 0.7))
    for b in range(3):
        r = raygrid.raygrid_obv(V, F, c[b], a[b], h[b], 16, 1, b, keep_rays=True)
        for w, ray in r["rays"].items():
            flag = ray["near_edge"] | ray["near_slab"]
            diff = np.abs(ray["L"] - ray["L_signed"])[~flag]
            assert diff.max(initial=0.0) <= 1e-12 * h[b].max()


def test_unbiased_over_seeds():
    """Stratified jitter: the mean of D_R over S seeds equals the exact OBV
    within 4 standard errors."""
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(2, seed=23, center_range=0.9, half_range=(0.3, 0.8))
    S = 48
    for b in range(2):
        Q = _ortho(a[b])
        ex = exact.obv(V, F, c[b], Q, h[b])
        vals = np.array([raygrid.raygrid_obv(V, F, c[b], Q, h[b], 6, 1000 + s, b)["obv"]
                         for s in range(S)])
        se = vals.std(ddof=1) / np.sqrt(S)
        assert abs(vals.mean() - ex) <= 4 * se + 1e-12


def test_error_shrinks_with_resolution():
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(1, seed=29, center_range=0.7, half_range=(0.4, 0.8))
    Q = _ortho(a[0])
    ex = exact.obv(V, F, c[0], Q, h[0])
    errs = []
    for R in (4, 16, 64):
        e = [raygrid.raygrid_obv(V, F, c[0], Q, h[0], R, 7 + s, 0)["obv"] - ex for s in range(6)]
        errs.append(np.sqrt(np.mean(np.square(e))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < errs[0] / 20


def test_axes_estimates_agree_with_exact_on_config1_boxes():
    V, F = synth.icosphere(3)
    c, a, h = synth.random_boxes(4, seed=12)
    for b in range(4):
        r = raygrid.raygrid_obv(V, F, c[b], a[b], h[b], 32, 13, b)
        ex = exact.inside_volume(V, F, c[b], a[b], h[b], axis=0)
        # statistical agreement of the 3-axis mean at R = 32
        assert abs(r["v_in"] - ex) <= 2e-2 * r["v_box"]


def test_occupancy_cuboid_face_splits_sub_slabs_exactly():
    """An axis-aligned cuboid whose top face lies on the boundary between the
    4th and 5th sub-slab of the box (and whose sides contain the box's column):
    sub-slabs 0-3 are inside (1), 4-7 outside (0), on every ray (up to the
    rounding of the sub-slab bounds)."""
    V, F = synth.cuboid((2.0, 2.0, 1.0), center=(0.0, 0.0, -1.0))   # solid z in [-2, 0]
    occ = raygrid.occupancy(V.astype(np.float64), F, [0.1, -0.2, 0.0], np.eye(3), [0.5, 0.4, 0.8], 3, 7)
    assert np.abs(occ[:, :, :4] - 1.0).max() <= 1e-12
    assert np.abs(occ[:, :, 4:]).max() <= 1e-12


def test_occupancy_mean_is_the_inside_fraction_of_its_rays():
    """Summed over the 8 sub-slabs, the occupancy of a ray is its inside length
    over the slab: the mean over (i, j, k) is V_in along axis 2 / V_box for the
    same 8 x 8 jittered rays."""
    V, F = synth.noisy_torus(nu=48, nv=24)
    c, a, h = synth.random_boxes(3, seed=4, center_range=0.8, half_range=(0.3, 0.7))
    for b in range(3):
        occ = raygrid.occupancy(V, F, c[b], a[b], h[b], 11, b)
        r = raygrid.raygrid_obv(V, F, c[b], a[b], h[b], 8, 11, b, axis_mask=4)
        assert abs(occ.mean() - r["v_in"] / r["v_box"]) <= 1e-12
