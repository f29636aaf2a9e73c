"""Area-weighted covariance OBB of a triangle cluster (float64 oracle).

The paper fixes a box by its centre and its three axes; the extents then follow
from enclosing the cluster (Sec. 4.2.1).  The axes used to seed a cluster's box
are the principal directions of the cluster's surface (the covariance fit the
paper cites among top-down builders, Sec. 2; continuous-surface form of
Gottschalk et al.'s OBB-tree):

* triangle T with vertices p, q, r: area A_T, centroid m_T;
  second moment of the uniform density on T:
      E_T[x x^T] = (9 m m^T + p p^T + q q^T + r r^T) / 12;
* mu = sum A_T m_T / sum A_T;
  C  = sum A_T E_T[(x - mu)(x - mu)^T] / sum A_T  (evaluated with vertices - mu);
* axes: eigenvectors of C by decreasing eigenvalue; e2 = e0 x e1; the largest
  |component| of e0 and of e1 is made positive;
* extents: min / max of Q (v - 0) over the cluster's vertices; c = Q^T mid,
  h = (max - min) / 2.
"""
import numpy as np


def cluster_covariance(V, F):
    """(mu, C, total_area) of the triangle set F (float64)."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64).reshape(-1, 3)
    p, q, r = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(q - p, r - p), axis=1)
    S = area.sum()
    m = (p + q + r) / 3.0
    mu = (area[:, None] * m).sum(0) / S
    pc, qc, rc, mc = p - mu, q - mu, r - mu, m - mu
    E = (9.0 * np.einsum("ti,tj->tij", mc, mc) + np.einsum("ti,tj->tij", pc, pc)
         + np.einsum("ti,tj->tij", qc, qc) + np.einsum("ti,tj->tij", rc, rc)) / 12.0
    C = (area[:, None, None] * E).sum(0) / S
    return mu, C, S


def jacobi_eigh(C, sweeps=50):
    """Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (float64).

    Returns (eigenvalues, eigenvectors as columns), unsorted.
    """
    A = np.array(C, dtype=np.float64)
    Vm = np.eye(3)
    for _ in range(sweeps):
        off = A[0, 1] ** 2 + A[0, 2] ** 2 + A[1, 2] ** 2
        if off < 1e-300:
            break
        for p in range(2):
            for q in range(p + 1, 3):
                if A[p, q] == 0.0:
                    continue
                theta = (A[q, q] - A[p, p]) / (2.0 * A[p, q])
                if theta == 0:
                    t = 1.0
                elif abs(theta) > 1e150:          # theta^2 would overflow
                    t = 1.0 / (2.0 * theta)
                else:
                    t = np.sign(theta) / (abs(theta) + np.sqrt(theta * theta + 1.0))
                c = 1.0 / np.sqrt(t * t + 1.0)
                s = t * c
                J = np.eye(3)
                J[p, p] = c
                J[q, q] = c
                J[p, q] = s
                J[q, p] = -s
                A = J.T @ A @ J
                Vm = Vm @ J
    return np.diag(A).copy(), Vm


def axes_from_covariance(C, use_jacobi=False):
    """Rows = local axes (decreasing eigenvalue, right handed, sign rule); eigenvalues."""
    if use_jacobi:
        lam, vec = jacobi_eigh(C)
    else:
        lam, vec = np.linalg.eigh(C)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    e0, e1 = vec[:, order[0]].copy(), vec[:, order[1]].copy()
    for e in (e0, e1):
        k = int(np.argmax(np.abs(e)))
        if e[k] < 0:
            e *= -1.0
    e2 = np.cross(e0, e1)
    return np.stack([e0, e1, e2]), lam


def tight_box(V, F, axes):
    """Centre and half extents of the tightest box with the given axes around F's vertices."""
    V = np.asarray(V, dtype=np.float64)
    idx = np.unique(np.asarray(F, dtype=np.int64).reshape(-1))
    Q = np.asarray(axes, dtype=np.float64)
    proj = V[idx] @ Q.T
    lo, hi = proj.min(0), proj.max(0)
    mid = 0.5 * (lo + hi)
    return Q.T @ mid, 0.5 * (hi - lo)


def fit_cluster(V, F, use_jacobi=False):
    """(center, axes, half, eigenvalues) of the covariance OBB of triangles F."""
    _, C, _ = cluster_covariance(V, F)
    Q, lam = axes_from_covariance(C, use_jacobi)
    c, h = tight_box(V, F, Q)
    return c, Q, h, lam


def fit_clusters(V, F, tri_cluster, n_clusters, use_jacobi=False):
    """Fit every cluster id in [0, n_clusters); triangles with id -1 are ignored.

    Empty clusters get a zero box (center 0, identity axes, half 0) and zero eigenvalues.
    """
    F = np.asarray(F)
    tri_cluster = np.asarray(tri_cluster)
    out = []
    for k in range(n_clusters):
        sel = F[tri_cluster == k]
        if len(sel) == 0:
            out.append((np.zeros(3), np.eye(3), np.zeros(3), np.zeros(3)))
        else:
            out.append(fit_cluster(V, sel, use_jacobi))
    return out
