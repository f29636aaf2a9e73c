"""Seeded closed triangle meshes (float32 vertices, int32 triangles, outward CCW).

Every generator returns ``(V, F)`` with ``V`` float32 ``[n_vertices, 3]`` and
``F`` int32 ``[n_triangles, 3]``; triangles are ordered counter-clockwise when
seen from outside, so the outward normal is ``(b - a) x (c - a)``.
Shapes and sizes follow the synthetic workloads that stand in for the paper's
solid models (icosphere, noisy torus, noisy cube-sphere, helix tube).
"""
import math

import numpy as np


def _orient_outward(V, F):
    """Flip every triangle whose normal points towards the centroid of the mesh.

    Only used for star-shaped generators (convex or radial meshes), where
    "outward" is well defined with respect to the centre.
    """
    V64 = V.astype(np.float64)
    ctr = V64.mean(axis=0)
    a, b, c = V64[F[:, 0]], V64[F[:, 1]], V64[F[:, 2]]
    n = np.cross(b - a, c - a)
    m = (a + b + c) / 3.0 - ctr
    flip = np.einsum("ij,ij->i", n, m) < 0
    F = F.copy()
    F[flip] = F[flip][:, [0, 2, 1]]
    return F


def icosahedron(radius=1.0):
    """Regular icosahedron with vertices on a sphere of the given radius."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts += [(0.0, s1, s2 * p), (s1, s2 * p, 0.0), (s2 * p, 0.0, s1)]
    V = np.array(pts, dtype=np.float64)
    # faces: triples of mutually adjacent vertices (edge length 2)
    n = len(V)
    d = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    F = np.array(faces, dtype=np.int32)
    V = V / np.linalg.norm(V, axis=1, keepdims=True) * radius
    F = _orient_outward(V, F)
    return V.astype(np.float32), F


def icosphere(subdiv=3, radius=1.0):
    """Icosahedron refined ``subdiv`` times by edge midpoints, projected to the sphere.

    subdiv=3 gives 642 vertices and 1,280 triangles.
    """
    V, F = icosahedron(1.0)
    V = V.astype(np.float64)
    for _ in range(subdiv):
        cache = {}
        verts = list(V)

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = (verts[a] + verts[b]) / 2.0
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        V = np.array(verts)
        F = np.array(nf, dtype=np.int32)
    V = V * radius
    return V.astype(np.float32), F.astype(np.int32)


def cuboid(half=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0), axes=None):
    """Closed cuboid: 8 vertices, 12 triangles.

    ``axes`` (3x3, rows = the cuboid's local axes in world coordinates) rotates
    it; by default it is axis aligned.
    """
    h = np.asarray(half, dtype=np.float64)
    corners = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)],
                       dtype=np.float64)
    local = corners * h
    Q = np.eye(3) if axes is None else np.asarray(axes, dtype=np.float64)
    V = local @ Q + np.asarray(center, dtype=np.float64)
    # index = 4*ix + 2*iy + iz with ix,iy,iz in {0,1}
    quads = [(0, 1, 3, 2), (4, 6, 7, 5),   # x = -1, x = +1
             (0, 4, 5, 1), (2, 3, 7, 6),   # y = -1, y = +1
             (0, 2, 6, 4), (1, 5, 7, 3)]   # z = -1, z = +1
    F = []
    for a, b, c, d in quads:
        F += [(a, b, c), (a, c, d)]
    F = np.array(F, dtype=np.int32)
    # orient using the cuboid centre (convex)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    m = (a + b + c) / 3.0 - np.asarray(center, dtype=np.float64)
    flip = np.einsum("ij,ij->i", n, m) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V.astype(np.float32), F


def octahedron(radius=1.0):
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64) * radius
    F = []
    for x in (0, 1):
        for y in (2, 3):
            for z in (4, 5):
                F.append((x, y, z))
    F = _orient_outward(V, np.array(F, dtype=np.int32))
    return V.astype(np.float32), F


def tetrahedron(scale=1.0):
    V = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) * scale
    F = _orient_outward(V, np.array([(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)], dtype=np.int32))
    return V.astype(np.float32), F


def _grid_quads(nu, nv, idx):
    """Triangles of a periodic nu x nv quad grid with vertex index function idx(i, j)."""
    i = np.arange(nu)[:, None]
    j = np.arange(nv)[None, :]
    a = idx(i, j)
    b = idx((i + 1) % nu, j)
    c = idx((i + 1) % nu, (j + 1) % nv)
    d = idx(i, (j + 1) % nv)
    t1 = np.stack([a, b, c], axis=-1).reshape(-1, 3)
    t2 = np.stack([a, c, d], axis=-1).reshape(-1, 3)
    out = np.empty((2 * nu * nv, 3), dtype=np.int64)
    out[0::2] = t1
    out[1::2] = t2
    return out.astype(np.int32)


def noisy_torus(R=1.0, r=0.35, nu=256, nv=128, amp=0.02, modes=8, seed=21):
    """Torus with a smooth seeded radial displacement.

    Tube radius r' = r + amp * f(u, v), with
    f = sum_{j,k=1..modes} a_jk cos(j u + alpha_jk) cos(k v + beta_jk),
    a_jk ~ N(0,1)/(j k), normalised so max |f| = 1 over the vertices.  Integer
    frequencies keep the displaced surface closed.  256 x 128 gives 65,536 triangles.
    """
    rng = np.random.default_rng(seed)
    jj = np.arange(1, modes + 1)[:, None]
    kk = np.arange(1, modes + 1)[None, :]
    a = rng.standard_normal((modes, modes)) / (jj * kk)
    al = rng.uniform(0, 2 * np.pi, (modes, modes))
    be = rng.uniform(0, 2 * np.pi, (modes, modes))
    u = 2 * np.pi * np.arange(nu) / nu
    v = 2 * np.pi * np.arange(nv) / nv
    U, Vv = np.meshgrid(u, v, indexing="ij")
    f = np.zeros_like(U)
    for j in range(modes):
        cu = np.cos((j + 1) * U[..., None] + al[j][None, None, :])  # [nu,nv,modes(k)]
        cv = np.cos((np.arange(1, modes + 1))[None, None, :] * Vv[..., None] + be[j][None, None, :])
        f += np.sum(a[j][None, None, :] * cu * cv, axis=-1)
    f /= np.abs(f).max()
    rr = r + amp * f
    X = (R + rr * np.cos(Vv)) * np.cos(U)
    Y = (R + rr * np.cos(Vv)) * np.sin(U)
    Z = rr * np.sin(Vv)
    V = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    F = _grid_quads(nu, nv, lambda i, j: i * nv + j)
    F = _orient_by_volume(V, F)
    return V.astype(np.float32), F


def _orient_by_volume(V, F):
    """Flip all triangles if the signed volume is negative (consistent grids only)."""
    V64 = np.asarray(V, dtype=np.float64)
    a, b, c = V64[F[:, 0]], V64[F[:, 1]], V64[F[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    if vol < 0:
        F = F[:, [0, 2, 1]].copy()
    return F


def _legendre_normalised(x, lmax):
    """Orthonormal associated Legendre functions with the Condon-Shortley phase:
    P[l][m] = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(x), by the standard
    three-term recurrences in l (stable for all degrees used here)."""
    s = np.sqrt(np.maximum(1.0 - x * x, 0.0))
    P = [[None] * (lmax + 1) for _ in range(lmax + 1)]
    P[0][0] = np.full_like(x, np.sqrt(1.0 / (4.0 * np.pi)))
    for m in range(1, lmax + 1):
        P[m][m] = -np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * P[m - 1][m - 1]
    for m in range(0, lmax):
        P[m + 1][m] = np.sqrt(2.0 * m + 3.0) * x * P[m][m]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            P[l][m] = a * (x * P[l - 1][m] - b * P[l - 2][m])
    return P


def _real_sph_harm_field(dirs, lmax, rng, decay_plus=1.0):
    """Seeded real spherical-harmonic field g(d) = sum_{l=1..lmax} sum_m c_lm Y_lm(d),
    with Y_l0 = Y_l^0, Y_lm = sqrt(2) Re Y_l^m and Y_l,-m = sqrt(2) Im Y_l^m (m > 0),
    Y_l^m the complex orthonormal harmonics with the Condon-Shortley phase."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    phi = np.arctan2(y, x)                         # azimuth
    P = _legendre_normalised(np.clip(z, -1.0, 1.0), lmax)
    g = np.zeros(len(dirs))
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            c = rng.standard_normal() / (l + decay_plus)
            if m < 0:
                yr = np.sqrt(2.0) * P[l][-m] * np.sin(-m * phi)
            elif m == 0:
                yr = P[l][0]
            else:
                yr = np.sqrt(2.0) * P[l][m] * np.cos(m * phi)
            g += c * yr
    return g


def noisy_cube_sphere(n, amp=0.05, lmax=8, seed=31):
    """Star-shaped noisy sphere from a cube grid with n quads per face edge.

    Triangles = 12 n^2.  Radius rho(d) = 1 + amp * g(d) with g a seeded real
    spherical-harmonic field up to degree lmax (c_lm ~ N(0,1)/(l+1)),
    normalised to max |g| = 1.
    """
    n = int(n)
    # integer lattice on the cube [-n, n]^3 (step 2), one (n+1)^2 grid per face
    lin = -n + 2 * np.arange(n + 1)
    grids, quads = [], []
    for axis in range(3):
        for sgn in (-1, 1):
            a1, a2 = (axis + 1) % 3, (axis + 2) % 3
            p = np.zeros((n + 1, n + 1, 3), dtype=np.int64)
            p[..., axis] = sgn * n
            p[..., a1] = lin[:, None]
            p[..., a2] = lin[None, :]
            grids.append(p.reshape(-1, 3))
    keys = np.concatenate(grids)
    pts, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(6, n + 1, n + 1)
    F = []
    for f, (axis, sgn) in enumerate([(ax, sg) for ax in range(3) for sg in (-1, 1)]):
        g = inv[f]
        a, b, c, d = g[:-1, :-1], g[1:, :-1], g[1:, 1:], g[:-1, 1:]
        # (a1, a2, axis) is right handed, so (a, b, c) is CCW seen from +axis
        if sgn > 0:
            t1, t2 = np.stack([a, b, c], -1), np.stack([a, c, d], -1)
        else:
            t1, t2 = np.stack([a, c, b], -1), np.stack([a, d, c], -1)
        F.append(np.stack([t1, t2], 2).reshape(-1, 3))
    F = np.concatenate(F)
    P = pts.astype(np.float64)
    dirs = P / np.linalg.norm(P, axis=1, keepdims=True)
    rng = np.random.default_rng(seed)
    g = _real_sph_harm_field(dirs, lmax, rng)
    g /= np.abs(g).max()
    V = dirs * (1.0 + amp * g)[:, None]
    return V.astype(np.float32), np.array(F, dtype=np.int32)


def lognormal_triangle_counts(count, seed, median=20000, sigma=np.log(10.0) / 2, lo=2000, hi=200000):
    """Triangle-count targets T ~ lognormal(median, sigma), redrawn until in [lo, hi]."""
    rng = np.random.default_rng(seed)
    T = np.empty(count)
    todo = np.arange(count)
    while len(todo):
        T[todo] = median * np.exp(sigma * rng.standard_normal(len(todo)))
        todo = todo[(T[todo] < lo) | (T[todo] > hi)]
    return T


def noisy_sphere_batch(count=256, seed=3, amp=0.05, lmax=8):
    """A batch of noisy cube-spheres with lognormal triangle counts: mesh m has
    n = round(sqrt(T_m / 12)) quads per face edge (12 n^2 triangles) and its own
    spherical-harmonic field (seed 1000 * seed + m).  Returns a list of (V, F)."""
    T = lognormal_triangle_counts(count, seed)
    out = []
    for m in range(count):
        n = max(1, int(round(np.sqrt(T[m] / 12.0))))
        out.append(noisy_cube_sphere(n, amp=amp, lmax=lmax, seed=1000 * seed + m))
    return out


def helix_tube(turns=4, radius=1.0, pitch=0.6, tube_r=0.15, noise=0.01,
               rings=7814, around=128, seed=41):
    """Capped tube swept along a helix, with seeded smooth surface noise.

    Centreline (radius cos 2 pi s, radius sin 2 pi s, pitch s), s in [0, turns],
    Frenet frame.  Tube radius tube_r + noise * n(s, phi), n a smooth field
    periodic in phi (frequencies 1..8) with up to 32 cycles along s, max |n| = 1.
    rings x around quads plus two cap fans: 7,814 x 128 gives 2,000,128 + 256 triangles.
    """
    rng = np.random.default_rng(seed)
    s = np.linspace(0.0, turns, rings)
    t = 2 * np.pi * s
    C = np.stack([radius * np.cos(t), radius * np.sin(t), pitch * s], axis=-1)
    # Frenet frame of a helix (closed form)
    k = 2 * np.pi
    T = np.stack([-radius * k * np.sin(t), radius * k * np.cos(t), np.full_like(t, pitch)], -1)
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    N = np.stack([-np.cos(t), -np.sin(t), np.zeros_like(t)], -1)
    B = np.cross(T, N)
    phi = 2 * np.pi * np.arange(around) / around
    nf = np.zeros((rings, around))
    for fphi in range(1, 9):
        cyc = rng.integers(1, 33)
        amp_ = rng.standard_normal() / fphi
        ph1, ph2 = rng.uniform(0, 2 * np.pi, 2)
        nf += amp_ * np.cos(fphi * phi[None, :] + ph1) * np.cos(2 * np.pi * cyc * s[:, None] / turns + ph2)
    nf /= np.abs(nf).max()
    rr = tube_r + noise * nf
    P = (C[:, None, :]
         + rr[..., None] * (np.cos(phi)[None, :, None] * N[:, None, :]
                            + np.sin(phi)[None, :, None] * B[:, None, :]))
    V = P.reshape(-1, 3)
    i = np.arange(rings - 1)[:, None]
    j = np.arange(around)[None, :]
    a = i * around + j
    b = (i + 1) * around + j
    c = (i + 1) * around + (j + 1) % around
    d = i * around + (j + 1) % around
    F1 = np.stack([a, b, c], -1).reshape(-1, 3)
    F2 = np.stack([a, c, d], -1).reshape(-1, 3)
    Fq = np.empty((2 * F1.shape[0], 3), dtype=np.int64)
    Fq[0::2] = F1
    Fq[1::2] = F2
    c0 = len(V)
    c1 = c0 + 1
    V = np.vstack([V, C[0][None, :], C[-1][None, :]])
    jj = np.arange(around)
    cap0 = np.stack([np.full(around, c0), jj, (jj + 1) % around], -1)
    last = (rings - 1) * around
    cap1 = np.stack([np.full(around, c1), last + (jj + 1) % around, last + jj], -1)
    F = np.vstack([Fq, cap0, cap1]).astype(np.int32)
    F = _orient_by_volume(V, F)
    return V.astype(np.float32), F


def disjoint_cuboids(k=3, seed=7, spacing=3.0):
    """k rotated cuboids with distinct side lengths, far apart from each other.

    Returns (V, F, comp) with comp[t] = index of the cuboid triangle t belongs to,
    plus the list of (center, axes, half) of each cuboid.
    """
    rng = np.random.default_rng(seed)
    Vs, Fs, comp, params = [], [], [], []
    off = 0
    for i in range(k):
        half = np.sort(rng.uniform(0.2, 0.9, 3))[::-1] * np.array([1.0, 0.8, 0.6])
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        from .boxes import quat_to_axes
        axes = quat_to_axes(q)
        center = np.array([spacing * i, 0.0, 0.0])
        V, F = cuboid(half, center, axes)
        Vs.append(V)
        Fs.append(F + off)
        comp += [i] * len(F)
        params.append((center, axes, half))
        off += len(V)
    return (np.vstack(Vs).astype(np.float32), np.vstack(Fs).astype(np.int32),
            np.array(comp, dtype=np.int32), params)


def split_top_slab(rv, u_half=0.5, v_lo=-0.4, v_hi=0.45, z_lo=-0.25, z_hi=0.3):
    """Closed axis-aligned slab [-u_half, u_half] x [v_lo, v_hi] x [z_lo, z_hi]
    whose top face (z = z_hi) is cut in two along the line y = rv, so that an
    interior edge from (-u_half, rv, z_hi) to (u_half, rv, z_hi) is shared by two
    top triangles facing +z; the side faces x = +-u_half carry the extra vertex
    as a pentagon fan.  Vertices float32, triangles outward (counter-clockwise
    seen from outside)."""
    x0, x1 = -u_half, u_half
    P = [(x0, v_lo, z_lo), (x1, v_lo, z_lo), (x1, v_hi, z_lo), (x0, v_hi, z_lo),      # 0-3 bottom
         (x0, v_lo, z_hi), (x1, v_lo, z_hi), (x1, rv, z_hi), (x0, rv, z_hi),          # 4-7 top, lower half
         (x1, v_hi, z_hi), (x0, v_hi, z_hi)]                                          # 8-9 top, upper half
    tris = [
        ((0, 2, 1), (0, 0, -1)), ((0, 3, 2), (0, 0, -1)),          # bottom
        ((4, 5, 6), (0, 0, 1)), ((4, 6, 7), (0, 0, 1)),            # top, y in [v_lo, rv]: edge 6-7 on y = rv
        ((7, 6, 8), (0, 0, 1)), ((7, 8, 9), (0, 0, 1)),            # top, y in [rv, v_hi]: edge 7-6 on y = rv
        ((0, 1, 5), (0, -1, 0)), ((0, 5, 4), (0, -1, 0)),          # y = v_lo
        ((3, 9, 8), (0, 1, 0)), ((3, 8, 2), (0, 1, 0)),            # y = v_hi
        ((1, 2, 8), (1, 0, 0)), ((1, 8, 6), (1, 0, 0)), ((1, 6, 5), (1, 0, 0)),    # x = +u_half
        ((0, 4, 7), (-1, 0, 0)), ((0, 7, 9), (-1, 0, 0)), ((0, 9, 3), (-1, 0, 0)),  # x = -u_half
    ]
    V = np.array(P, dtype=np.float32)
    F = []
    for (a, b, c), n in tris:
        pa, pb, pc = V[a].astype(np.float64), V[b].astype(np.float64), V[c].astype(np.float64)
        if np.dot(np.cross(pb - pa, pc - pa), n) < 0:
            b, c = c, b
        F.append((a, b, c))
    return V, np.array(F, dtype=np.int32)
