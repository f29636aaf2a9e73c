"""Mesh and box helpers of the oracle (float64 or exact rationals).

Conventions (Sec. 3 of the paper: X is a closed solid triangle mesh, O an
oriented box):

* a box is (c, Q, h); row k of Q is unit local axis k; local coordinates of a
  point x are x' = Q (x - c); the box is {|x'_k| <= h_k};
* a cast along local axis w uses the other two axes in cyclic order as the
  face coordinates (u, v): w=0 -> (1, 2), w=1 -> (2, 0), w=2 -> (0, 1);
* triangles are counter-clockwise seen from outside (outward normal
  (b - a) x (c - a)).
"""
from fractions import Fraction

import numpy as np


def face_axes(w):
    return (w + 1) % 3, (w + 2) % 3


def directed_edge_report(F):
    """Closed + consistently oriented check: every directed edge (a, b) occurs
    exactly once and its reverse (b, a) occurs exactly once.

    Returns (closed_and_oriented, n_bad_edges).
    """
    F = np.asarray(F, dtype=np.int64)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
    counts = {}
    for a, b in e.tolist():
        counts[(a, b)] = counts.get((a, b), 0) + 1
    bad = 0
    for (a, b), k in counts.items():
        if k != 1 or counts.get((b, a), 0) != 1:
            bad += 1
    return bad == 0, bad


def signed_volume(V, F):
    """Enclosed volume by the divergence theorem: sum over triangles of det[a, b, c] / 6."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def to_local(V, center, axes):
    """x' = Q (x - c) for all vertices, float64 (inputs promoted exactly)."""
    V = np.asarray(V, dtype=np.float64)
    c = np.asarray(center, dtype=np.float64).reshape(3)
    Q = np.asarray(axes, dtype=np.float64).reshape(3, 3)
    return (V - c) @ Q.T


def to_local_exact(V, center, axes):
    """Same transform in exact rational arithmetic (lists of Fractions)."""
    out = []
    for x in V:
        d = [Fraction(x[k]) - Fraction(center[k]) for k in range(3)]
        out.append([sum(Fraction(axes[r][k]) * d[k] for k in range(3)) for r in range(3)])
    return out


def rational_rotation(a, b, c, d):
    """Exactly orthogonal rational rotation from an integer quaternion (a, b, c, d)
    (w = a): R(q) / |q|^2 with Fraction entries; returns axes = R^T (rows = local axes)."""
    a, b, c, d = (Fraction(t) for t in (a, b, c, d))
    n = a * a + b * b + c * c + d * d
    R = [[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
         [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
         [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]]
    return [[R[k][r] / n for k in range(3)] for r in range(3)]
