"""The paper's central-projection estimator of the outer volume (Sec. 4.1,
Eq. 9-10) in float64 -- test infrastructure only, never imported by the library.

Rays leave the box centre o through the pixel centres of a cube map of 6 x m x m
pixels in the box frame (face +x: direction (1, a, b) with a, b the pixel
centre in [-1, 1]; the other faces alike).  A pixel is a cone of directions of
solid angle W (exact: the solid angle of the pixel's square on the unit cube).
Along the ray o + t d (d not normalised) the box is left at t_e = min_k h_k /
|d_k|, and the mesh is crossed at t_k > 0 with s_k = +1 where the ray leaves
the solid (outward normal . d > 0) and -1 where it enters.  Reading of Eq. 9
(the printed form drops the crossings beyond the box): the solid's indicator
at t is the sum of s_k over the crossings beyond t, so the inside part of the
cone is sum_k s_k min(r_k, r_e)^3 W / 3 with r = t |d| (cone volumes: the cubic
weights of the paper's GPU variant; with power 1 the same sum is Eq. 9's
inside length).  Outer volume: OBV = sum over pixels of (r_e^3 - sum_k s_k
min(r_k, r_e)^3) W / 3, so a box inside the solid gives exactly 0 and a box
away from it the quadrature of its own volume.

Crossings are found with a watertight ray-triangle test (Woop, Benthin and
Wald, JCGT 2013: axes permuted so the ray's largest component is z, vertices
sheared so the ray runs along z, three 2-D edge functions) with one owner for
points on a shared edge: after orienting the edge functions so the inside is
positive, an edge function equal to 0 passes only for a top-left edge.  Every
step is a float64 operation in one fixed order (the device evaluator makes the
same decisions).
"""
import math

import numpy as np


def to_local_ordered(V, center, axes):
    """x' = Q (x - c) in float64, each coordinate as (Q_r0 d0 + Q_r1 d1) + Q_r2 d2
    (one fixed order of operations, so both sides of a parity test place the
    vertices identically)."""
    V = np.asarray(V, np.float64)
    c = np.asarray(center, np.float64).reshape(3)
    Q = np.asarray(axes, np.float64).reshape(3, 3)
    d0, d1, d2 = V[:, 0] - c[0], V[:, 1] - c[1], V[:, 2] - c[2]
    return np.stack([(Q[r, 0] * d0 + Q[r, 1] * d1) + Q[r, 2] * d2 for r in range(3)], axis=1)


def face_pixels(m):
    """[6 m^2] directions d (float64, not normalised) and solid angles W."""
    c = -1.0 + (2.0 * np.arange(m) + 1.0) / m          # pixel centres
    e = -1.0 + 2.0 * np.arange(m + 1) / m               # pixel edges

    def F(a, b):
        return np.arctan(a * b / np.sqrt(1.0 + a * a + b * b))

    A0, B0 = np.meshgrid(e[:-1], e[:-1], indexing="ij")
    A1, B1 = np.meshgrid(e[1:], e[1:], indexing="ij")
    W = (F(A1, B1) - F(A0, B1) - F(A1, B0) + F(A0, B0)).reshape(-1)
    Ac, Bc = np.meshgrid(c, c, indexing="ij")
    a, b = Ac.reshape(-1), Bc.reshape(-1)
    one = np.ones_like(a)
    dirs, ws = [], []
    for axis in range(3):
        for sgn in (1.0, -1.0):
            d = np.zeros((m * m, 3))
            d[:, axis] = sgn * one
            d[:, (axis + 1) % 3] = a
            d[:, (axis + 2) % 3] = b
            dirs.append(d)
            ws.append(W)
    return np.concatenate(dirs), np.concatenate(ws)


def _topleft(px, py, qx, qy):
    """Edge p -> q of a counter-clockwise oriented 2-D triangle owns its points
    when it is a top edge (horizontal, running left) or a left edge (running
    down)."""
    dx = qx - px
    dy = qy - py
    return (dy < 0.0) | ((dy == 0.0) & (dx < 0.0))


def ray_crossings(T, d):
    """Crossings of the ray t d (t > 0) with triangles T [n, 3, 3] (box frame,
    ray origin at 0): (t, s) arrays of the triangles it crosses."""
    ad = np.abs(d)
    kz = int(np.argmax(ad))
    kx, ky = (kz + 1) % 3, (kz + 2) % 3
    if d[kz] < 0.0:
        kx, ky = ky, kx
    Sx = d[kx] / d[kz]
    Sy = d[ky] / d[kz]
    Sz = 1.0 / d[kz]
    Ax = T[:, 0, kx] - Sx * T[:, 0, kz]
    Ay = T[:, 0, ky] - Sy * T[:, 0, kz]
    Bx = T[:, 1, kx] - Sx * T[:, 1, kz]
    By = T[:, 1, ky] - Sy * T[:, 1, kz]
    Cx = T[:, 2, kx] - Sx * T[:, 2, kz]
    Cy = T[:, 2, ky] - Sy * T[:, 2, kz]
    U = Cx * By - Cy * Bx      # edge B -> C
    V = Ax * Cy - Ay * Cx      # edge C -> A
    Wf = Bx * Ay - By * Ax     # edge A -> B
    det = (U + V) + Wf
    o = np.where(det < 0.0, -1.0, 1.0)
    # oriented so that the inside is positive; a zero passes on a top-left edge
    # (the edges' directions flip with the orientation)
    Uo, Vo, Wo = o * U, o * V, o * Wf
    flip = det < 0.0
    tlU = np.where(flip, _topleft(Cx, Cy, Bx, By), _topleft(Bx, By, Cx, Cy))
    tlV = np.where(flip, _topleft(Ax, Ay, Cx, Cy), _topleft(Cx, Cy, Ax, Ay))
    tlW = np.where(flip, _topleft(Bx, By, Ax, Ay), _topleft(Ax, Ay, Bx, By))
    inside = (((Uo > 0.0) | ((Uo == 0.0) & tlU)) & ((Vo > 0.0) | ((Vo == 0.0) & tlV))
              & ((Wo > 0.0) | ((Wo == 0.0) & tlW)) & (det != 0.0))
    Az = Sz * T[:, 0, kz]
    Bz = Sz * T[:, 1, kz]
    Cz = Sz * T[:, 2, kz]
    tnum = (U * Az + V * Bz) + Wf * Cz
    with np.errstate(divide="ignore", invalid="ignore"):
        t = tnum / det
    hit = inside & (t > 0.0)
    e1 = T[:, 1] - T[:, 0]
    e2 = T[:, 2] - T[:, 0]
    n = np.cross(e1, e2)
    nd = (n[:, 0] * d[0] + n[:, 1] * d[1]) + n[:, 2] * d[2]
    s = np.where(nd > 0.0, 1.0, -1.0)
    keep = hit & (nd != 0.0)
    return t[keep], s[keep]


def cube(x):
    """x^3 as (x x) x, the one rounding sequence used for every cone depth."""
    return (x * x) * x


def cone_terms(r, s, r_e, power=3):
    """sum_k s_k min(r_k, r_e)^power (power 3: cone volumes times 3 / W;
    power 1: Eq. 9's inside length), summed in crossing order."""
    m = np.minimum(np.asarray(r, np.float64), r_e)
    terms = np.asarray(s, np.float64) * (cube(m) if power == 3 else m)
    total = 0.0
    for x in terms.tolist():
        total = total + x
    return total


def obv(V, F, center, axes, half, m):
    """Central-projection outer volume of one box (float64)."""
    P = to_local_ordered(V, center, axes)
    T = P[np.asarray(F, np.int64)]
    h = np.asarray(half, np.float64).reshape(3)
    dirs, W = face_pixels(m)
    total = 0.0
    for d, w in zip(dirs, W):
        with np.errstate(divide="ignore"):
            te = min(h[k] / abs(d[k]) for k in range(3) if d[k] != 0.0)
        dn = math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        re = te * dn
        t, s = ray_crossings(T, d)
        total += (cube(re) - cone_terms(t * dn, s, re)) * w / 3.0
    return total
