"""Independent checks used to pin the oracle (none of them share its arithmetic)."""
import numpy as np


def winding_number(V, F, pts, chunk=200_000):
    """Generalised winding number of closed mesh (V, F) at points ``pts``.

    Sum of the signed solid angles of the triangles seen from each point,
    divided by 4 pi; solid angle of a triangle by Van Oosterom and Strackee
    (IEEE Trans. Biomed. Eng., 1983).  Independent of any ray parity rule.
    """
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    out = np.empty(len(pts))
    for s in range(0, len(pts), chunk):
        p = pts[s:s + chunk]
        acc = np.zeros(len(p))
        for a_i, b_i, c_i in F:
            a = V[a_i] - p
            b = V[b_i] - p
            c = V[c_i] - p
            la, lb, lc = (np.linalg.norm(x, axis=1) for x in (a, b, c))
            det = np.einsum("ij,ij->i", a, np.cross(b, c))
            den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc
                   + np.einsum("ij,ij->i", b, c) * la + np.einsum("ij,ij->i", c, a) * lb)
            acc += 2.0 * np.arctan2(det, den)
        out[s:s + chunk] = acc / (4.0 * np.pi)
    return out


def points_in_box(rng, n, center, axes, half):
    """Uniform points in an oriented box (rows of axes = local axes)."""
    loc = rng.uniform(-1.0, 1.0, size=(n, 3)) * np.asarray(half, dtype=np.float64)
    return loc @ np.asarray(axes, dtype=np.float64) + np.asarray(center, dtype=np.float64)


def interval_overlap(a0, a1, b0, b1):
    return max(0.0, min(a1, b1) - max(a0, b0))
