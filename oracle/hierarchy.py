"""Hierarchy of boxes built top-down, then improved by multigrid-like sweeps
(Sec. 4.2.2), scored by the weighted error of Eq. 7 -- float64 oracle.

Test infrastructure: this module is the plain reference the HIP path is checked
against; nothing in the library imports it.

Readings of the paper (each layer is a same-layer Lloyd clustering, Sec. 4.2.1,
see ``lloyd``):

* layer 0 is one box over the whole mesh: the covariance box of all triangles
  (its axes seed the box), then ``iters`` parameter updates;
* top-down: the triangles of every node of layer l-1 are clustered into
  ``branching`` children.  A child starts from a triangle of its parent drawn
  with SplitMix64 (seed ^ 0x243F6A8885A308D3, counter (l << 48) | (parent << 20)
  | draw, modulo the parent's triangle count, repeats rejected): its centre is
  that triangle's centroid, its axes are its parent's.  A parent with fewer
  triangles than ``branching`` gets as many children as it has triangles; the
  others stay empty;
* bottom-up merge of layer l: the boxes of layer l+1 become the elements of a
  flood (an element's vertices are its triangles' vertices, its centroid is the
  box centre, two elements are adjacent when a mesh edge joins them) that
  regroups them under the non-empty boxes of layer l, within the groups of
  their grandparents; the layer-l boxes then get their parameter update;
* Eq. 7 with omega = number of layers down to the leaves (leaf 1, Sec. 5) scores
  every change: a sweep merges layers L-2, ..., 1 while e drops (the first merge
  that does not lower e is undone and ends the up pass), then re-solves the
  layers below the highest merged one, top-down, keeping each re-solve only if
  e drops.

Node numbering: layer-major; the jitter key of a node is its number (root 0).
"""
import copy

import numpy as np

from . import fit as ofit
from . import lloyd as ol
from . import rng

SEED_SALT = 0x243F6A8885A308D3


def random_seeds(G, count, seed, level, parent):
    """``count`` distinct triangles of the list G (SplitMix64 draws, repeats rejected)."""
    out = []
    draw = 0
    while len(out) < count:
        n = (level << 48) | (parent << 20) | draw
        draw += 1
        t = int(G[rng.splitmix64(seed ^ SEED_SALT, n) % len(G)])
        if t not in out:
            out.append(t)
    return out


class Level:
    def __init__(self, n, nt):
        self.box = [None] * n            # (c, Q, h) float32
        self.obv = [0.0] * n
        self.parent = [-1] * n           # index into the layer above
        self.slot = [0] * n              # jitter key
        self.tri_node = np.full(nt, -1, np.int64)


class Hierarchy:
    """State of the build, with the plain steps of Sec. 4.2.2 as methods.

    ``evaluate`` maps a list of (key, c, Q, h) to OBV values.  ``follow``
    (optional) names the choices of another implementation, taken only where
    they are as valid as this build's own (near-ties of the flood,
    ``lloyd.flood``; updates within the estimate's noise, ``lloyd.update_box``):
    follow.element(level, kind, index) and follow.box(level, j)."""

    def __init__(self, V, F, levels, branching, evaluate, seed, K=32, delta=0.02, iters=1, follow=None,
                 tie=2e-5, eps=1e-5):
        self.V = np.asarray(V)
        self.F = np.asarray(F, np.int64)
        self.nt = len(self.F)
        self.L, self.b = levels, branching
        self.evaluate, self.seed, self.K, self.delta, self.iters = evaluate, seed, K, delta, iters
        self.follow, self.tie, self.eps = follow, tie, eps
        self.adj = ol.adjacency(self.F)
        self.tri_E = ol.triangle_elements(self.V, self.F, self.adj)
        self.cen = ol._centroids(self.V, self.F)
        self.counters = {"ties": 0, "update_ties": 0, "evals": 0}
        self.trace = []
        self.lv = []

    # -- Eq. 7 ---------------------------------------------------------------
    def error(self):
        return float(sum((self.L - l) * float(np.sum(self.lv[l].obv)) for l in range(self.L)))

    # -- one Lloyd iteration over groups of (elements, boxes) -----------------
    def _iterate(self, E, groups, boxes, obv, slot, level, kind, ids=None):
        """Partition (flood per group with several boxes; a group with one box
        takes all its elements), then the parameter update of every box that
        received triangles.  Returns the box of every element (-1: none)."""
        eb = np.full(E.n, -1, np.int64)
        fol = self.follow
        for elems, bxs in groups:
            if not elems or not bxs:
                continue
            if len(bxs) == 1:
                eb[elems] = bxs[0]
                continue
            local = {j: i for i, j in enumerate(bxs)}
            follow = None
            if fol is not None:
                def follow(e, bxs=bxs, local=local):
                    j = fol.element(level, kind, e if ids is None else ids[e])
                    return local.get(j) if j is not None else None
            assign, grown, gobv, cnt = ol.flood(E, elems, [boxes[j][0] for j in bxs], [boxes[j][1] for j in bxs],
                                                [slot[j] for j in bxs], self._ev, self.K, follow, self.tie)
            self.counters["ties"] += cnt["ties"]
            for e, i in assign.items():
                eb[e] = bxs[i]
            for i, j in enumerate(bxs):
                boxes[j] = grown[i]
                obv[j] = float(gobv[i])
        tris = [[] for _ in boxes]
        for e in range(E.n):
            if eb[e] >= 0:
                tris[eb[e]].extend(int(t) for t in E.tris[e])
        for j in range(len(boxes)):
            if not tris[j]:
                continue
            fb = fol.box(level, j) if fol is not None else None
            bx, v, _ = ol.update_box(self.V, self.F, sorted(tris[j]), boxes[j][1], slot[j], self._ev, self.delta,
                                     follow_box=fb, tie=self.tie, eps=self.eps, counters=self.counters)
            boxes[j] = bx
            obv[j] = v
        return eb, tris

    def _ev(self, items):
        self.counters["evals"] += len(items)
        return self.evaluate(items)

    # -- layer 0 ---------------------------------------------------------------
    def root(self):
        R0 = Level(1, self.nt)
        c, Q, h, _ = ofit.fit_cluster(self.V, self.F)
        R0.box[0] = ol.make_box(c, Q, h)
        R0.tri_node[:] = 0
        self.lv = [R0]
        groups = [(list(range(self.nt)), [0])]
        for _ in range(self.iters):
            self._iterate(self.tri_E, groups, R0.box, R0.obv, R0.slot, 0, "tri")

    # -- top-down: children of every node of layer l-1 ------------------------
    def split(self, l, node_base):
        P = self.lv[l - 1]
        n_par = len(P.box)
        C = Level(n_par * self.b, self.nt)
        for q in range(n_par):
            G = np.nonzero(P.tri_node == q)[0]
            nseed = min(self.b, len(G))
            seeds = random_seeds(G, nseed, self.seed, l, q) if nseed else []
            for k in range(self.b):
                j = q * self.b + k
                C.parent[j] = q
                C.slot[j] = node_base + j
                Qp = P.box[q][1]
                if k < nseed:
                    C.box[j] = (self.cen[seeds[k]].astype(np.float32), Qp.copy(), np.zeros(3, np.float32))
                else:   # more children than triangles: an empty node
                    C.box[j] = (P.box[q][0].copy(), Qp.copy(), np.full(3, -1.0, np.float32))
        self.lv.append(C)
        self.solve(l)
        for j, bx in enumerate(C.box):
            if bx[2][0] < 0:
                C.box[j] = (bx[0], bx[1], np.zeros(3, np.float32))

    # -- the same-layer solve of layer l under its current parents ------------
    def solve(self, l):
        C, P = self.lv[l], self.lv[l - 1]
        groups = []
        for q in range(len(P.box)):
            elems = [int(t) for t in np.nonzero(P.tri_node == q)[0]]
            bxs = [j for j in range(len(C.box)) if C.parent[j] == q and C.box[j][2][0] >= 0]
            groups.append((elems, bxs[:len(elems)]))
        boxes, obv = list(C.box), list(C.obv)
        for _ in range(self.iters):
            eb, tris = self._iterate(self.tri_E, groups, boxes, obv, C.slot, l, "tri")
        for j in range(len(boxes)):
            if tris[j]:
                C.box[j], C.obv[j] = boxes[j], obv[j]
            else:
                C.box[j], C.obv[j] = (boxes[j][0], boxes[j][1], np.zeros(3, np.float32)), 0.0
        C.tri_node = eb.copy()

    # -- bottom-up merge of layer l -------------------------------------------
    def merge(self, l):
        A, U, G = self.lv[l], self.lv[l + 1], self.lv[l - 1]
        units = [u for u in range(len(U.box)) if np.any(U.tri_node == u)]
        unit_tris = [np.nonzero(U.tri_node == u)[0] for u in units]
        E = ol.unit_elements(self.V, self.F, self.adj, unit_tris, [U.box[u][0] for u in units])
        groups = []
        for g in range(len(G.box)):
            elems = [e for e, u in enumerate(units) if A.parent[U.parent[u]] == g]
            bxs = [j for j in range(len(A.box)) if A.parent[j] == g and (A.box[j][2][0] > 0 or A.box[j][2][1] > 0)]
            groups.append((elems, bxs[:len(elems)]))
        boxes, obv = list(A.box), list(A.obv)
        eb, tris = self._iterate(E, groups, boxes, obv, A.slot, l, "unit", ids=units)
        for e, u in enumerate(units):
            if eb[e] >= 0:
                U.parent[u] = int(eb[e])
        for j in range(len(boxes)):
            if tris[j]:
                A.box[j], A.obv[j] = boxes[j], obv[j]
            else:
                A.box[j], A.obv[j] = (boxes[j][0], boxes[j][1], np.zeros(3, np.float32)), 0.0
        A.tri_node = np.array([U.parent[u] if u >= 0 else -1 for u in U.tri_node], np.int64)

    # -- the whole build ---------------------------------------------------------
    def top_down(self):
        self.root()
        base = 1
        for l in range(1, self.L):
            self.split(l, base)
            base += len(self.lv[l].box)
        return self.error()

    def sweep(self, e):
        """One up pass and one down pass; returns the new e."""
        top = self.L
        for l in range(self.L - 2, 0, -1):
            saved = copy.deepcopy(self.lv)
            self.merge(l)
            e2 = self.error()
            self.trace.append(("merge", l, e, e2, e2 < e))
            if e2 < e:
                e, top = e2, l
            else:
                self.lv = saved
                break
        for l in range(max(1, top + 1), self.L):
            saved = copy.deepcopy(self.lv)
            self.solve(l)
            e2 = self.error()
            self.trace.append(("solve", l, e, e2, e2 < e))
            if e2 < e:
                e = e2
            else:
                self.lv = saved
        return e

    def arrays(self):
        """Layer-major arrays: boxes [n, 15] float32, obv, parent, tri_node [L, nt]."""
        n = sum(len(x.box) for x in self.lv)
        boxes = np.zeros((n, 15), np.float32)
        obv = np.zeros(n)
        parent = np.full(n, -1, np.int64)
        tri_node = np.full((self.L, self.nt), -1, np.int64)
        g0 = 0
        for l, Lv in enumerate(self.lv):
            pbase = g0 - len(self.lv[l - 1].box) if l > 0 else 0
            for j, (c, Q, h) in enumerate(Lv.box):
                boxes[g0 + j] = np.concatenate([c, np.asarray(Q).reshape(-1), h])
                obv[g0 + j] = Lv.obv[j]
                parent[g0 + j] = pbase + Lv.parent[j] if Lv.parent[j] >= 0 else -1
            tri_node[l] = np.where(Lv.tri_node >= 0, Lv.tri_node + g0, -1)
            g0 += len(Lv.box)
        return {"boxes": boxes, "obv": obv, "parent": parent, "tri_node": tri_node}


class FollowArrays:
    """Near-tie choices read from layer-major output arrays of a build (see
    ``Hierarchy``): the node of a triangle, the parent of a unit, a node's box."""

    def __init__(self, out, levels, branching):
        self.out = out
        self.base = [0]
        w = 1
        for _ in range(levels):
            self.base.append(self.base[-1] + w)
            w *= branching

    def element(self, level, kind, i):
        """Layer-``level`` node taking triangle i (kind "tri") or the layer-(level+1)
        node i (kind "unit", a merge), as a layer-local index."""
        b0 = self.base[level]
        if kind == "tri":
            g = int(self.out["tri_node"][level][i])
        else:
            g = int(self.out["parent"][self.base[level + 1] + i])
        return g - b0 if g >= 0 else None

    def box(self, level, j):
        row = self.out["boxes"][self.base[level] + j]
        return row[:3], row[3:12].reshape(3, 3), row[12:]


def build(V, F, levels, branching, evaluate, seed, iters=1, sweeps=1, K=32, delta=0.02, follow_top_down=None,
          follow_sweeps=None, tie=2e-5, eps=1e-5):
    """Top-down build and ``sweeps`` sweeps.  Returns (hierarchy, e history,
    layer-major arrays after the top-down build)."""
    H = Hierarchy(V, F, levels, branching, evaluate, seed, K, delta, iters, follow_top_down, tie, eps)
    e = [H.top_down()]
    top_down = H.arrays()
    H.follow = follow_sweeps
    for _ in range(sweeps):
        e.append(H.sweep(e[-1]))
    return H, e, top_down
