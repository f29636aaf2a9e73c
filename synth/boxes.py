"""Seeded oriented boxes.

A box is (center[3], axes[3][3], half[3]); row k of ``axes`` is the unit local
axis k in world coordinates (right handed).  Packed as 15 float32 values in the
order center, axes (row major), half -- the layout of ``obbv_box``.
"""
import numpy as np


def quat_to_axes(q):
    """Rotation of a unit quaternion (x, y, z, w); returns axes with rows = R[:, k]."""
    x, y, z, w = (float(t) for t in q)
    R = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])
    return R.T.copy()


def _uniform_quaternions(rng, n):
    """Uniform random unit quaternions (Shoemake, Graphics Gems III, 1992)."""
    u1, u2, u3 = rng.uniform(size=(3, n))
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                     b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=-1)


def random_boxes(n, seed, center_range=1.2, half_range=(0.1, 0.8)):
    """n boxes: centers U[-c, c]^3, half extents U[lo, hi]^3, uniform rotations.

    Returns float32 arrays center [n,3], axes [n,3,3], half [n,3].
    """
    rng = np.random.default_rng(seed)
    center = rng.uniform(-center_range, center_range, size=(n, 3))
    half = rng.uniform(half_range[0], half_range[1], size=(n, 3))
    qs = _uniform_quaternions(rng, n)
    axes = np.stack([quat_to_axes(q) for q in qs]) if n else np.zeros((0, 3, 3))
    return (center.astype(np.float32), axes.astype(np.float32), half.astype(np.float32))


def axis_aligned_box(center, half):
    c = np.asarray(center, dtype=np.float32).reshape(1, 3)
    h = np.asarray(half, dtype=np.float32).reshape(1, 3)
    return c, np.eye(3, dtype=np.float32)[None], h


def boxes_to_array(center, axes, half):
    """Pack into the [n, 15] float32 layout (center, axes row major, half)."""
    center = np.asarray(center, dtype=np.float32).reshape(-1, 3)
    n = center.shape[0]
    axes = np.asarray(axes, dtype=np.float32).reshape(n, 9)
    half = np.asarray(half, dtype=np.float32).reshape(n, 3)
    return np.ascontiguousarray(np.concatenate([center, axes, half], axis=1))


def mixed_boxes(V, n, seed, surface_frac=0.5):
    """n boxes around a mesh with vertices V: a `surface_frac` share centred near
    random vertices (half extents U[0.02, 0.3] x diagonal, like boxes grown around
    surface patches), the rest with centres uniform in the bounding box grown by
    10% (half extents U[0.03, 0.5] x diagonal); uniform random rotations.
    Returns float32 [n, 15] rows (center, axes, half)."""
    rng = np.random.default_rng(seed)
    V = np.asarray(V, dtype=np.float64)
    lo, hi = V.min(0), V.max(0)
    diag = float(np.linalg.norm(hi - lo))
    ns = int(round(n * surface_frac))
    c_s = V[rng.integers(0, len(V), ns)] + rng.normal(0, 0.02 * diag, (ns, 3))
    h_s = rng.uniform(0.02, 0.3, (ns, 3)) * diag
    span = hi - lo
    c_r = rng.uniform(lo - 0.1 * span, hi + 0.1 * span, (n - ns, 3))
    h_r = rng.uniform(0.03, 0.5, (n - ns, 3)) * diag
    qs = _uniform_quaternions(rng, n)
    axes = np.stack([quat_to_axes(q) for q in qs]) if n else np.zeros((0, 3, 3))
    return boxes_to_array(np.vstack([c_s, c_r]), axes, np.vstack([h_s, h_r]))


def _f32_up(x):
    y = np.asarray(x, np.float64).astype(np.float32)
    return np.where(y.astype(np.float64) < x, np.nextafter(y, np.float32(np.inf)), y).astype(np.float32)


def flood_candidates(V, F, n_groups, seed, k=8, patch=48, reach=6):
    """Candidate boxes as a flood meets them: n_groups base boxes, each with k
    grown copies.  A base box has a uniform random rotation, its centre at the
    centroid of a random triangle, and half extents enclosing (symmetrically
    about that centre) the `patch` triangles whose centroids are nearest to it;
    candidate j encloses the base's triangles plus one more triangle, drawn from
    the next reach x k nearest, that lies partly outside the base box.  Returns
    float32 (base [G, 15], candidates [G, k, 15]); groups without k such
    triangles are skipped."""
    rng = np.random.default_rng(seed)
    V = np.asarray(V, np.float64)
    T = V[np.asarray(F)]
    cen = T.mean(axis=1)
    qs = _uniform_quaternions(rng, n_groups)
    base, cand = [], []
    for g in range(n_groups):
        Q = quat_to_axes(qs[g])
        s = int(rng.integers(0, len(cen)))
        c = cen[s].astype(np.float32).astype(np.float64)
        near = np.argsort(np.linalg.norm(cen - c, axis=1))[:patch + reach * k]
        loc = np.abs((T[near] - c) @ Q.T).max(axis=1)          # [n, 3] extents per triangle
        h = _f32_up(loc[:patch].max(axis=0))
        grows = [int(i) for i in range(patch, len(near)) if np.any(_f32_up(np.maximum(loc[i], h)) != h)]
        if len(grows) < k:
            continue
        pick = rng.choice(grows, size=k, replace=False)
        base.append(np.concatenate([c.astype(np.float32), Q.reshape(-1).astype(np.float32), h]))
        cand.append([np.concatenate([c.astype(np.float32), Q.reshape(-1).astype(np.float32),
                                     _f32_up(np.maximum(loc[i], h))]) for i in pick])
    return np.array(base, np.float32).reshape(-1, 15), np.array(cand, np.float32).reshape(-1, k, 15)


def query_spheres(V, n, seed, r_lo=0.01, r_hi=0.2):
    """[n, 4] float32 spheres (centre, radius) for collision queries: centres
    uniform in the mesh's bounding box grown by 20 % on every side, radii
    log-uniform in [r_lo, r_hi] times the box diagonal."""
    V = np.asarray(V, np.float64)
    lo, hi = V.min(axis=0), V.max(axis=0)
    pad = 0.2 * (hi - lo)
    rng = np.random.default_rng(seed)
    c = rng.uniform(lo - pad, hi + pad, size=(n, 3))
    diag = float(np.linalg.norm(hi - lo))
    r = np.exp(rng.uniform(np.log(r_lo), np.log(r_hi), size=n)) * diag
    return np.concatenate([c, r[:, None]], axis=1).astype(np.float32)
