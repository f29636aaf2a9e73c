"""Top-down OBB tree of covariance boxes (float64 oracle) -- the baseline the
paper compares its hierarchy against (Sec. 5, Fig. 6: OBB-tree style top-down
construction).  Test infrastructure only: never imported by the library.

Rule (the classic top-down builder): the root box is the area-weighted
covariance box of all triangles; every node's triangles are ordered by the
projection of their centroids on the longest axis of the node's box (ties by
triangle index) and cut into `branching` parts of equal count (rank * b //
count); each part's box is again its covariance box.  Node numbering is
level-major; node j of level l has children b j .. b j + b - 1.
"""
import numpy as np

from . import fit as ofit


def centroids(V, F):
    T = np.asarray(V, np.float64)[np.asarray(F, np.int64)]
    return ((T[:, 0] + T[:, 1]) + T[:, 2]) / 3.0


def build_obb_tree(V, F, levels, branching):
    """Returns (boxes per level: list of [(c, Q, h)], tri_node per level: list of int arrays)."""
    V = np.asarray(V)
    F = np.asarray(F)
    nt = len(F)
    cen = centroids(V, F)
    cluster = np.zeros(nt, np.int64)
    boxes, tri_node = [], []
    n = 1
    for lv in range(levels):
        fits = ofit.fit_clusters(V, F, cluster.astype(np.int32), n)
        boxes.append(fits)
        tri_node.append(cluster.copy())
        if lv + 1 == levels:
            break
        nxt = np.empty(nt, np.int64)
        for j in range(n):
            members = np.nonzero(cluster == j)[0]
            if len(members) == 0:
                continue
            Q, h = fits[j][1], fits[j][2]
            # longest axis: the first of equal longest extents
            k = 0 if h[0] >= h[1] and h[0] >= h[2] else (1 if h[1] >= h[2] else 2)
            p = cen[members] @ np.asarray(Q, np.float64)[k]
            order = members[np.lexsort((members, p))]
            rank = np.arange(len(order))
            part = np.minimum(rank * branching // len(order), branching - 1)
            nxt[order] = j * branching + part
        cluster = nxt
        n *= branching
    return boxes, tri_node
