"""Exact outer volume of one box (Sec. 3, Eq. 4), by the divergence theorem.

OBV(X, O) is the volume of the part of box O outside the solid X, i.e.
V_box - vol(X ∩ O).  Pinned in the tests by closed forms, exact rationals,
Monte-Carlo winding numbers and a partition invariant.

Derivation used here.  Cast lines parallel to local axis w through every face
point (u, v).  A closed, outward oriented surface crosses such a line with sign
s_T = sign(n_T . e_w) (+1 leaving the solid when moving along +w).  The solid's
indicator at depth t on the line is the sum of s_k over the crossings above t,
so the inside length of the slab [-h_w, h_w] is
    sum_k s_k (clamp(w_k, -h_w, h_w) + h_w),
and integrating over the face rectangle gives
    vol(X ∩ O) = sum_T s_T  ∬_{P_T ∩ rect} (clamp(w_T(u, v), -h_w, h_w) + h_w) du dv,
with P_T the projection of triangle T on (u, v) and w_T its (affine) depth.
Per triangle: clip P_T to the rectangle, split it by w_T = +h_w and w_T = -h_w;
the part above contributes 2 h_w * area, the middle part area * (w_T(centroid) + h_w),
the part below nothing.

The same routine runs on Python floats (float64) or on ``fractions.Fraction``
(exact when vertices, centre, half extents and axes are rational).
"""
from fractions import Fraction

import numpy as np

from .geometry import face_axes, to_local, to_local_exact


def clip_polygon(poly, g):
    """Sutherland-Hodgman: the part of ``poly`` where the affine function g >= 0.

    ``poly`` is a list of (u, v, w) points of a planar convex polygon; the new
    vertices are linear interpolations of all three coordinates, so the depth w
    stays exact along the clipped edges.  Keeps the input orientation.
    """
    out = []
    n = len(poly)
    for k in range(n):
        p, q = poly[k], poly[(k + 1) % n]
        gp, gq = g(p), g(q)
        if gp >= 0:
            out.append(p)
        if (gp > 0 and gq < 0) or (gp < 0 and gq > 0):
            t = gp / (gp - gq)
            out.append(tuple(p[i] + t * (q[i] - p[i]) for i in range(3)))
    return out


def _sign(x):
    return int(x > 0) - int(x < 0)


def _area2(p, q, r):
    """Twice the signed area of the projection of (p, q, r) on (u, v)."""
    return (q[0] - p[0]) * (r[1] - p[1]) - (q[1] - p[1]) * (r[0] - p[0])


def fan_integrals(poly):
    """(area, ∬ w du dv) of a convex planar polygon, by a triangle fan from vertex 0.

    On each fan triangle w is affine, so its integral is area * mean of the
    three vertex depths.
    """
    area = 0
    wint = 0
    for k in range(1, len(poly) - 1):
        a = abs(_area2(poly[0], poly[k], poly[k + 1])) / 2
        area += a
        wint += a * (poly[0][2] + poly[k][2] + poly[k + 1][2]) / 3
    return area, wint


def triangle_inside_contribution(pa, pb, pc, hu, hv, hw):
    """s_T ∬_{P_T ∩ rect} (clamp(w_T, -hw, hw) + hw) du dv for one triangle.

    pa, pb, pc are (u, v, w) triples in the cast frame.  The triangle is clipped
    to the prism over the face rectangle, then split by the planes w = +hw and
    w = -hw: the piece above contributes 2 hw * area, the middle piece
    ∬ (w + hw), the piece below nothing.
    """
    s = _sign(_area2(pa, pb, pc))
    if s == 0:
        return 0
    poly = [tuple(pa), tuple(pb), tuple(pc)]
    for g in (lambda p: p[0] + hu, lambda p: hu - p[0],
              lambda p: p[1] + hv, lambda p: hv - p[1]):
        poly = clip_polygon(poly, g)
        if len(poly) < 3:
            return 0
    if all(p[2] == hw for p in poly):
        # lying in the plane w = +h_w: both closed half-spaces below would keep
        # it, but it is one piece, inside over the whole slab
        a, _ = fan_integrals(poly)
        return s * 2 * hw * a
    top = clip_polygon(poly, lambda p: p[2] - hw)
    mid = clip_polygon(clip_polygon(poly, lambda p: hw - p[2]), lambda p: p[2] + hw)
    total = 0
    if len(top) >= 3:
        a, _ = fan_integrals(top)
        total += 2 * hw * a
    if len(mid) >= 3:
        a, wi = fan_integrals(mid)
        total += wi + hw * a
    return s * total


def inside_volume_axis(P, F, half, w):
    """vol(X ∩ O) by casting along local axis w; P = local vertex coordinates."""
    ua, va = face_axes(w)
    hu, hv, hw = half[ua], half[va], half[w]
    total = 0
    for t in range(len(F)):
        a, b, c = (P[F[t][k]] for k in range(3))
        total += triangle_inside_contribution((a[ua], a[va], a[w]), (b[ua], b[va], b[w]),
                                              (c[ua], c[va], c[w]), hu, hv, hw)
    return total


def _relevant_triangles(P, F, half, w):
    """Triangles whose projection meets the face rectangle and that reach above -h_w
    (all others contribute exactly zero)."""
    ua, va = face_axes(w)
    tri = P[F]  # [T,3,3]
    lo = tri.min(axis=1)
    hi = tri.max(axis=1)
    keep = ((hi[:, ua] >= -half[ua]) & (lo[:, ua] <= half[ua])
            & (hi[:, va] >= -half[va]) & (lo[:, va] <= half[va])
            & (hi[:, w] > -half[w]))
    return np.nonzero(keep)[0]


def inside_volume(V, F, center, axes, half, axis=None):
    """float64 vol(X ∩ O); per cast axis (list of 3) or for one axis."""
    P = to_local(V, center, axes)
    h = [float(x) for x in np.asarray(half, dtype=np.float64).reshape(3)]
    F = np.asarray(F, dtype=np.int64)
    axes_list = [axis] if axis is not None else [0, 1, 2]
    out = []
    for w in axes_list:
        idx = _relevant_triangles(P, F, h, w)
        Pl = P.tolist()
        out.append(float(inside_volume_axis(Pl, F[idx].tolist(), h, w)))
    return out[0] if axis is not None else out


def box_volume(half):
    h = np.asarray(half, dtype=np.float64).reshape(3)
    return float(8.0 * h[0] * h[1] * h[2])


def obv(V, F, center, axes, half, axis=0):
    """OBV = V_box - vol(X ∩ O) (float64)."""
    return box_volume(half) - inside_volume(V, F, center, axes, half, axis=axis)


def inside_volume_exact(V, F, center, axes, half, axis=0):
    """Exact rational vol(X ∩ O) (inputs converted to Fractions exactly)."""
    P = to_local_exact([[Fraction(x) for x in row] for row in np.asarray(V).tolist()]
                       if not isinstance(V, list) else V,
                       [Fraction(x) for x in center],
                       [[Fraction(x) for x in row] for row in axes])
    h = [Fraction(x) for x in half]
    return inside_volume_axis(P, [list(map(int, t)) for t in np.asarray(F).tolist()], h, axis)
