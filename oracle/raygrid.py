"""Discrete outer volume D_R on a jittered parallel-ray grid (float64 oracle).

This is the estimator the HIP path computes (Sec. 4.1 casts rays and sums the
inside/outside length along each ray, Eq. 9; here the rays are parallel to a
box axis instead of leaving the box centre):

for each cast axis w of the box (all three by default) and each cell (i, j) of
an R x R grid on the face rectangle [-h_u, h_u] x [-h_v, h_v]:
  1. jitter (xi, eta) from SplitMix64 (see ``rng``);
  2. the ray is the line through (u, v) = (-h_u + (i + xi) du, -h_v + (j + eta) dv)
     parallel to e_w, with du = 2 h_u / R, dv = 2 h_v / R;
  3. collect every triangle whose projection contains (u, v) and its depth;
     a point at depth t is inside the solid iff the number of crossings below t
     is odd (parity); L = length of the inside part of [-h_w, h_w];
  4. V_in,w = sum L du dv; V_in = mean over the cast axes; D_R = V_box - V_in.

Per ray the oracle also reports the crossing counts, the orientation-signed
inside length sum_k s_k (clamp(w_k) + h_w) (equal to the parity length on a
closed, consistently oriented, non-self-intersecting mesh) and two flags: the
ray passes within ``tol`` of a projected triangle edge, or a crossing lies
within ``tol`` of a slab face.  Either classification is correct on flagged rays.
"""
import numpy as np

from . import rng
from .geometry import face_axes, to_local


def ray_positions(half, w, R, seed, box_key):
    """Ray coordinates (u[i, j], v[i, j]) on the face of cast axis w (float64)."""
    ua, va = face_axes(w)
    hu, hv = float(half[ua]), float(half[va])
    du, dv = 2.0 * hu / R, 2.0 * hv / R
    i, j = np.meshgrid(np.arange(R, dtype=np.uint64), np.arange(R, dtype=np.uint64), indexing="ij")
    xi, eta = rng.jitter(seed, box_key, w, i, j)
    u = -hu + (i.astype(np.float64) + xi) * du
    v = -hv + (j.astype(np.float64) + eta) * dv
    return u, v


def parity_inside_length(depths, h):
    """Inside length of [-h, h] on one line from its crossing depths (parity rule)."""
    d = np.sort(np.asarray(depths, dtype=np.float64))
    n_below = int(np.sum(d < -h))
    inside = (n_below % 2) == 1
    pos = -h
    L = 0.0
    for t in d[(d >= -h) & (d <= h)]:
        if inside:
            L += t - pos
        pos = t
        inside = not inside
    if inside:
        L += h - pos
    return L


def parity_inside_length_interval(depths, a, b):
    """Inside length of [a, b] on one line from its crossing depths (parity rule)."""
    d = np.sort(np.asarray(depths, dtype=np.float64))
    inside = (int(np.sum(d < a)) % 2) == 1
    pos, L = a, 0.0
    for t in d[(d >= a) & (d <= b)]:
        if inside:
            L += t - pos
        pos = t
        inside = not inside
    if inside:
        L += b - pos
    return L


def occupancy(V, F, center, axes, half, seed, box_key=0):
    """8 x 8 x 8 inside fractions of a box: 8 x 8 jittered rays along local axis 2,
    inside length within each of the 8 equal sub-slabs of [-h2, h2] / sub-slab length."""
    P = to_local(V, center, axes)
    h = np.asarray(half, dtype=np.float64).reshape(3)
    res = cast_axis(P, np.asarray(F, np.int64), h, 2, 8, seed, box_key, keep_depths=True)
    occ = np.zeros((8, 8, 8))
    step = 2.0 * h[2] / 8
    for i in range(8):
        for j in range(8):
            d = res["depths"][i * 8 + j]
            for k in range(8):
                a = -h[2] + k * step
                occ[i, j, k] = parity_inside_length_interval(d, a, a + step) / step
    return occ


def signed_inside_length(depths, signs, h):
    """sum_k s_k (clamp(w_k, -h, h) + h) with s_k = +1 when the line leaves the solid."""
    d = np.clip(np.asarray(depths, dtype=np.float64), -h, h)
    return float(np.sum(np.asarray(signs, dtype=np.float64) * (d + h)))


def eq9_outside_length(t_hits, signs, t_e):
    """Outside length of the segment [0, t_e] of a ray leaving the box centre.

    Generalisation of Eq. 9: inside length = sum_k s_k min(t_k, t_e) over the
    crossings at t_k > 0 (s_k = +1 leaving the solid), outside = t_e - inside.
    With every crossing before t_e this is the paper's
    l_out = |p_e o| - sum_i sign(n(p_i) . w) |p_i o|.
    """
    t = np.asarray(t_hits, dtype=np.float64)
    s = np.asarray(signs, dtype=np.float64)
    keep = t > 0
    return float(t_e - np.sum(s[keep] * np.minimum(t[keep], t_e)))


def integrate_rays(ray, depth, sign, n_rays, h, tol):
    """Per-ray quantities of crossings sorted by (ray, depth), all rays at once.

    The parity length of a ray adds, in depth order, the length of every inside
    segment of [-h, h] between consecutive in-slab crossings (the ray starts
    inside when an odd number of crossings lies below -h), then the last
    segment up to +h: the sums of ``parity_inside_length`` term by term and in
    its order.  The signed length is ``signed_inside_length``.
    """
    below = depth < -h
    above = depth > h
    inn = ~below & ~above
    n_below = np.bincount(ray[below], minlength=n_rays).astype(np.int64)
    n_in = np.bincount(ray[inn], minlength=n_rays).astype(np.int64)
    n_above = np.bincount(ray[above], minlength=n_rays).astype(np.int64)
    near_slab = np.bincount(ray[np.abs(np.abs(depth) - h) < tol], minlength=n_rays) > 0
    L_sgn = np.bincount(ray, weights=sign * (np.clip(depth, -h, h) + h), minlength=n_rays).astype(np.float64)
    # in-slab crossings: rank within the ray and the previous position
    r_in, d_in = ray[inn], depth[inn]
    first = np.ones(len(r_in), dtype=bool)
    first[1:] = r_in[1:] != r_in[:-1]
    start = np.maximum.accumulate(np.where(first, np.arange(len(r_in)), 0)) if len(r_in) else np.zeros(0, int)
    rank = np.arange(len(r_in)) - start
    prev = np.where(first, -h, np.concatenate([[-h], d_in[:-1]]))
    was_inside = (n_below[r_in] + rank) % 2 == 1
    L_par = np.bincount(r_in[was_inside], weights=(d_in - prev)[was_inside],
                        minlength=n_rays).astype(np.float64)
    # the last segment: inside after all in-slab crossings
    last = np.full(n_rays, -h)
    last[r_in] = d_in            # crossings are in depth order: the last write wins
    tail = (n_below + n_in) % 2 == 1
    L_par[tail] += h - last[tail]
    return L_par, L_sgn, n_below, n_in, n_above, near_slab


def cast_axis(P, F, half, w, R, seed, box_key, tol=1e-6, keep_depths=False):
    """All rays of one cast axis.  Returns a dict of per-ray [R, R] arrays."""
    ua, va = face_axes(w)
    hu, hv, hw = float(half[ua]), float(half[va]), float(half[w])
    du, dv = 2.0 * hu / R, 2.0 * hv / R
    u, v = ray_positions(half, w, R, seed, box_key)

    tri = P[F]                               # [T, 3 vertices, 3 coords]
    U, Vv, W = tri[:, :, ua], tri[:, :, va], tri[:, :, w]
    A2 = (U[:, 1] - U[:, 0]) * (Vv[:, 2] - Vv[:, 0]) - (Vv[:, 1] - Vv[:, 0]) * (U[:, 2] - U[:, 0])
    # candidate cells: the projected bounding box (grown by tol) of each triangle
    i0 = np.floor((U.min(1) - tol + hu) / du).astype(np.int64)
    i1 = np.floor((U.max(1) + tol + hu) / du).astype(np.int64)
    j0 = np.floor((Vv.min(1) - tol + hv) / dv).astype(np.int64)
    j1 = np.floor((Vv.max(1) + tol + hv) / dv).astype(np.int64)
    i0, j0 = np.maximum(i0, 0), np.maximum(j0, 0)
    i1, j1 = np.minimum(i1, R - 1), np.minimum(j1, R - 1)
    ok = (A2 != 0) & (i1 >= i0) & (j1 >= j0)
    tid = np.nonzero(ok)[0]
    ni = (i1 - i0 + 1)[tid]
    nj = (j1 - j0 + 1)[tid]
    cnt = ni * nj
    hits_ray, hits_w, hits_s = [], [], []
    near_edge = np.zeros((R, R), dtype=bool)
    chunk = 2_000_000
    start = 0
    while start < len(tid):
        # expand (triangle, cell) pairs chunk by chunk to bound memory
        csum = np.cumsum(cnt[start:])
        stop = start + int(np.searchsorted(csum, chunk, side="right")) + 1
        stop = min(stop, len(tid))
        t_ids = tid[start:stop]
        c = cnt[start:stop]
        rep_t = np.repeat(t_ids, c)
        local = np.arange(int(c.sum())) - np.repeat(np.cumsum(c) - c, c)
        nj_r = np.repeat(nj[start:stop], c)
        ci = np.repeat(i0[t_ids], c) + local // nj_r
        cj = np.repeat(j0[t_ids], c) + local % nj_r
        pu, pv = u[ci, cj], v[ci, cj]
        s = np.sign(A2[rep_t])
        ua_, va_ = U[rep_t], Vv[rep_t]
        e = []
        dist = []
        for k in range(3):
            a, b = k, (k + 1) % 3
            ex = ua_[:, b] - ua_[:, a]
            ey = va_[:, b] - va_[:, a]
            ek = (ex * (pv - va_[:, a]) - ey * (pu - ua_[:, a])) * s   # >= 0 inside
            e.append(ek)
            dist.append(ek / np.hypot(ex, ey))
        e = np.stack(e, 1)
        dist = np.stack(dist, 1)
        inside = np.all(e >= 0, axis=1)
        near = (dist.min(1) > -tol) & (np.abs(dist).min(1) < tol)
        near_edge[ci[near], cj[near]] = True
        # barycentric depth: weight of vertex k is the edge function opposite to it
        area2 = np.abs(A2[rep_t])
        wts = np.stack([e[:, 1], e[:, 2], e[:, 0]], 1) / area2[:, None]
        depth = np.sum(wts * W[rep_t], axis=1)
        hits_ray.append((ci * R + cj)[inside])
        hits_w.append(depth[inside])
        hits_s.append(s[inside])
        start = stop
    if hits_ray:
        hr = np.concatenate(hits_ray)
        hwv = np.concatenate(hits_w)
        hs = np.concatenate(hits_s)
    else:
        hr = np.zeros(0, np.int64)
        hwv = np.zeros(0)
        hs = np.zeros(0)
    order = np.lexsort((hwv, hr))
    hr, hwv, hs = hr[order], hwv[order], hs[order]
    L_par, L_sgn, n_below, n_in, n_above, near_slab = integrate_rays(hr, hwv, hs, R * R, hw, tol)
    bounds = np.searchsorted(hr, np.arange(R * R + 1))
    depths = [hwv[bounds[r]:bounds[r + 1]] for r in range(R * R)] if keep_depths else None
    V_in = float(L_par.sum() * du * dv)
    return {
        "V_in": V_in,
        "L": L_par.reshape(R, R), "L_signed": L_sgn.reshape(R, R),
        "n_below": n_below.reshape(R, R), "n_in": n_in.reshape(R, R),
        "n_above": n_above.reshape(R, R),
        "near_edge": near_edge, "near_slab": near_slab.reshape(R, R),
        "u": u, "v": v, "depths": depths,
    }


def raygrid_obv(V, F, center, axes, half, R, seed, box_key=0, axis_mask=7, tol=1e-6,
                keep_rays=False):
    """D_R for one box.  Returns dict(obv, v_box, v_in, v_in_axis, rays)."""
    P = to_local(V, center, axes)
    F = np.asarray(F, dtype=np.int64)
    h = np.asarray(half, dtype=np.float64).reshape(3)
    v_box = float(8.0 * h[0] * h[1] * h[2])
    per_axis = {}
    rays = {}
    # local bounds of every triangle: a triangle whose projection misses the face
    # rectangle of an axis (by more than the candidate-cell margin) meets none of
    # its rays, so it is left out of that axis before the per-cell work
    p0, p1, p2 = P[F[:, 0]], P[F[:, 1]], P[F[:, 2]]
    lo = np.minimum(np.minimum(p0, p1), p2)
    hi = np.maximum(np.maximum(p0, p1), p2)
    for w in range(3):
        if not (axis_mask >> w) & 1:
            continue
        if v_box == 0.0:
            per_axis[w] = 0.0
            continue
        ua, va = face_axes(w)
        near = ((hi[:, ua] >= -h[ua] - 2 * tol) & (lo[:, ua] <= h[ua] + 2 * tol)
                & (hi[:, va] >= -h[va] - 2 * tol) & (lo[:, va] <= h[va] + 2 * tol))
        res = cast_axis(P, F[near], h, w, R, seed, box_key, tol)
        per_axis[w] = res["V_in"]
        if keep_rays:
            rays[w] = res
    v_in = float(np.mean(list(per_axis.values()))) if per_axis else 0.0
    return {"obv": v_box - v_in, "v_box": v_box, "v_in": v_in, "v_in_axis": per_axis,
            "rays": rays}


def raygrid_obv_many(V, F, centers, axes, halves, R, seed, box_keys=None, axis_mask=7):
    """D_R for a batch of boxes (float64 array)."""
    n = len(centers)
    keys = np.arange(n) if box_keys is None else box_keys
    return np.array([raygrid_obv(V, F, centers[b], axes[b], halves[b], R, seed,
                                 int(keys[b]), axis_mask)["obv"] for b in range(n)])
