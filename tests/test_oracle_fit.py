"""Pins of the covariance-OBB fit oracle."""
from fractions import Fraction

import numpy as np

import synth
from oracle import fit


def _monomial_second_moment(p, q, r):
    """E[x x^T] of the uniform density on triangle (p, q, r) from the exact
    monomial integrals over the unit simplex: x = p + s (q - p) + t (r - p),
    ∫1 = 1/2, ∫s = ∫t = 1/6, ∫s^2 = ∫t^2 = 1/12, ∫st = 1/24 (Fractions)."""
    p, q, r = ([Fraction(x) for x in v] for v in (p, q, r))
    a = [q[i] - p[i] for i in range(3)]
    b = [r[i] - p[i] for i in range(3)]
    M = [[Fraction(0)] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            val = (p[i] * p[j] * Fraction(1, 2)
                   + (p[i] * a[j] + a[i] * p[j]) * Fraction(1, 6)
                   + (p[i] * b[j] + b[i] * p[j]) * Fraction(1, 6)
                   + a[i] * a[j] * Fraction(1, 12) + b[i] * b[j] * Fraction(1, 12)
                   + (a[i] * b[j] + b[i] * a[j]) * Fraction(1, 24))
            M[i][j] = val * 2          # divide by the simplex area 1/2
    return np.array([[float(x) for x in row] for row in M])


def test_single_triangle_moments_closed_form():
    g = np.random.default_rng(0)
    for _ in range(5):
        P = g.uniform(-1, 1, (3, 3))
        mu, C, S = fit.cluster_covariance(P, np.array([[0, 1, 2]]))
        E = _monomial_second_moment(*P)
        assert np.allclose(C + np.outer(mu, mu), E, atol=1e-13)
        assert np.allclose(mu, P.mean(0), atol=1e-15)
        assert abs(S - 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))) < 1e-15


def test_rotated_cuboid_axes_and_extents():
    g = np.random.default_rng(4)
    for k in range(4):
        _, a, _ = synth.random_boxes(1, seed=200 + k)
        u, _, vt = np.linalg.svd(a[0].astype(np.float64))
        Q = u @ vt
        half = np.array([0.9, 0.5, 0.2])      # distinct sides -> distinct eigenvalues
        ctr = g.uniform(-1, 1, 3)
        _, F = synth.cuboid(half, ctr, Q)
        corners = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], float)
        V = (corners * half) @ Q + ctr
        c, Qf, h, lam = fit.fit_cluster(V, F)
        for i in range(3):
            assert abs(abs(Qf[i] @ Q[i]) - 1.0) < 1e-12
        assert np.allclose(h, half, atol=1e-12)
        assert np.allclose(c, ctr, atol=1e-12)
        assert lam[0] > lam[1] > lam[2] > 0
        assert abs(np.linalg.det(Qf) - 1.0) < 1e-12


def test_jacobi_matches_lapack():
    V, F = synth.noisy_torus(nu=32, nv=16)
    for sel in (slice(0, 200), slice(100, 700), slice(None)):
        _, C, _ = fit.cluster_covariance(V, F[sel])
        Qa, la = fit.axes_from_covariance(C)
        Qb, lb = fit.axes_from_covariance(C, use_jacobi=True)
        assert np.allclose(la, lb, rtol=1e-12, atol=1e-15)
        assert np.allclose(Qa, Qb, atol=1e-9)


def test_rigid_motion_equivariance():
    V, F = synth.noisy_cube_sphere(4)
    V = V.astype(np.float64)
    V = V * np.array([1.5, 1.0, 0.6])      # distinct principal axes
    sel = F[:150]
    c0, Q0, h0, _ = fit.fit_cluster(V, sel)
    _, a, _ = synth.random_boxes(1, seed=3)
    u, _, vt = np.linalg.svd(a[0].astype(np.float64))
    Rm = u @ vt
    t = np.array([0.5, -2.0, 1.0])
    c1, Q1, h1, _ = fit.fit_cluster(V @ Rm + t, sel)
    assert np.allclose(h1, h0, atol=1e-10)
    assert np.allclose(c1, c0 @ Rm + t, atol=1e-10)
    for i in range(3):
        assert abs(abs(Q1[i] @ (Q0[i] @ Rm)) - 1.0) < 1e-9


def test_fit_encloses_cluster_vertices():
    V, F = synth.noisy_torus(nu=32, nv=16)
    cl = (np.arange(len(F)) * 7 // len(F)).astype(np.int32)
    boxes = fit.fit_clusters(V, F, cl, 7)
    for k, (c, Q, h, _) in enumerate(boxes):
        idx = np.unique(F[cl == k])
        loc = (V[idx].astype(np.float64) - c) @ Q.T
        assert np.all(np.abs(loc) <= h + 1e-12)
