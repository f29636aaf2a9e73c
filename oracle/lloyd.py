"""Same-layer Lloyd clustering of triangles into boxes (Sec. 4.2.1) and the
layer weights of the hierarchy error (Sec. 3, Eq. 7; Sec. 5) -- float64 oracle.

A box O_i of a layer has a centre c_i and axes Q_i (its 6 free parameters); its
half extents S_i follow from enclosing its triangle set F_i.  During the
partition the centre stays fixed, so the box is symmetric about c_i:
h_i = max over the vertices v of F_i of |Q_i (v - c_i)|.

Partition (flooding, Sec. 4.2.1 step 1), in the paper's order:
  * every triangle t of the group gets the key |m_t - c_nearest| (centroid to the
    nearest box centre); each box starts from the triangle nearest its centre;
  * repeatedly take t_min, the frontier triangle with the smallest key; for every
    box O_i compute dOBV_i = |OBV(O_i(S_i')) - OBV(O_i(S_i))| (Eq. 12) where S_i'
    encloses F_i and t_min; give t_min to the box with the smallest dOBV (Eq. 13;
    ties: nearer centre, then lower index); put its unassigned neighbours in the
    queue.  A box that already contains t_min has dOBV = 0, so when one exists
    t_min goes to the nearest such box without evaluating the others.
  * bulk-synchronous rounds take the K smallest frontier triangles at once and
    evaluate them all against the boxes of the round start (K = 1 is the serial
    flood); triangles no flood reaches (other components) are assigned one by
    one by the same rule at the end.
Parameter update (step 2): tight box for the current axes, then a finite
difference gradient of OBV over the three rotation angles (+-delta about each
local axis) and a steepest-descent line search; the best candidate is kept if
it lowers OBV.
Adjustment (step 3, for a stalled iteration): the least important box (fewest
triangles) is re-seeded inside the worst-fitting box; kept only if the group's
error drops (``adjust``).

Boxes are stored as float32 (centre and axes rounded to nearest, half extents
rounded up so the box still encloses), as the HIP path stores them; OBV values
come from an evaluator callable (the ray-grid oracle in the tests).
"""
import heapq

import numpy as np


# ---------------------------------------------------------------------------
# float32 box storage
# ---------------------------------------------------------------------------
def f32_up(x):
    """Round float64 values up to float32."""
    x = np.asarray(x, dtype=np.float64)
    y = x.astype(np.float32)
    lo = y.astype(np.float64) < x
    y = np.where(lo, np.nextafter(y, np.float32(np.inf)), y)
    return y.astype(np.float32)


def make_box(c, Q, h):
    return (np.asarray(c, np.float64).astype(np.float32), np.asarray(Q, np.float64).astype(np.float32),
            f32_up(h))


def project(P, Q):
    """Local coordinates Q p of points P [n,3] (float64), summed in axis order."""
    P = np.asarray(P, np.float64)
    Q = np.asarray(Q, np.float64)
    return np.stack([(P[:, 0] * Q[r, 0] + P[:, 1] * Q[r, 1]) + P[:, 2] * Q[r, 2] for r in range(3)], axis=1)


def tri_extent(V, F, t, c, Q):
    """max over the vertices of triangle t of |Q (v - c)| per local axis (float64)."""
    P = project(V[F[t]].astype(np.float64) - np.asarray(c, np.float64), Q)
    return np.abs(P).max(axis=0)


def tight_box(V, F, tris, Q):
    """Tightest box with axes Q (float32) around the vertices of triangles `tris`."""
    Q32 = np.asarray(Q, np.float32)
    Q64 = Q32.astype(np.float64)
    idx = np.unique(F[np.asarray(tris)].reshape(-1))
    proj = project(V[idx].astype(np.float64), Q64)
    lo, hi = proj.min(0), proj.max(0)
    mid = 0.5 * (lo + hi)
    c = np.array([(Q64[0, k] * mid[0] + Q64[1, k] * mid[1]) + Q64[2, k] * mid[2] for k in range(3)])
    c32 = c.astype(np.float32)
    # extents about the stored (rounded) centre so the float32 box encloses
    P = project(V[idx].astype(np.float64) - c32.astype(np.float64), Q64)
    return c32, Q32, f32_up(np.abs(P).max(axis=0))


def adjacency(F):
    """Edge-adjacent triangles (sharing an undirected edge)."""
    edges = {}
    for t, (a, b, c) in enumerate(np.asarray(F).tolist()):
        for u, v in ((a, b), (b, c), (c, a)):
            edges.setdefault((min(u, v), max(u, v)), []).append(t)
    nb = [[] for _ in range(len(F))]
    for ts in edges.values():
        for x in ts:
            for y in ts:
                if x != y:
                    nb[x].append(y)
    return [sorted(set(n)) for n in nb]


# ---------------------------------------------------------------------------
# partition
# ---------------------------------------------------------------------------
def _centroids(V, F):
    T = V[F].astype(np.float64)
    return ((T[:, 0] + T[:, 1]) + T[:, 2]) / 3.0


class Elements:
    """What a flood distributes among boxes: single triangles (the same-layer
    clustering, Sec. 4.2.1) or units of several triangles (the bottom-up merge
    of Sec. 4.2.2 regroups the child boxes of a layer).  Per element: the
    float64 coordinates of its triangles' vertices, a centroid and its
    edge-adjacent elements; ``tris`` lists its triangles."""

    def __init__(self, verts, cen, adj, tris):
        self.verts = verts
        self.cen = np.asarray(cen, np.float64)
        self.adj = adj
        self.tris = tris
        self.n = len(verts)

    def extent(self, e, c, Q):
        """max over the element's vertices of |Q (v - c)| per local axis (float64)."""
        P = project(self.verts[e] - np.asarray(c, np.float64), Q)
        return np.abs(P).max(axis=0)


def triangle_elements(V, F, adj=None):
    V64 = np.asarray(V).astype(np.float64)
    F = np.asarray(F)
    return Elements([V64[f] for f in F], _centroids(np.asarray(V), F), adjacency(F) if adj is None else adj,
                    [np.array([t]) for t in range(len(F))])


def unit_elements(V, F, tri_adj, unit_tris, unit_centres):
    """Units of triangles as elements: the centroid of a unit is its box centre;
    two units are adjacent when a mesh edge joins a triangle of each."""
    V64 = np.asarray(V).astype(np.float64)
    F = np.asarray(F)
    unit_of = {}
    for e, ts in enumerate(unit_tris):
        for t in ts:
            unit_of[int(t)] = e
    adj = []
    for e, ts in enumerate(unit_tris):
        nb = set()
        for t in ts:
            for t2 in tri_adj[int(t)]:
                u = unit_of.get(t2, -1)
                if u >= 0 and u != e:
                    nb.add(u)
        adj.append(sorted(nb))
    verts = [V64[F[np.asarray(ts)].reshape(-1)] for ts in unit_tris]
    cen = np.asarray(unit_centres, np.float32).astype(np.float64)
    return Elements(verts, cen, adj, [np.asarray(ts) for ts in unit_tris])


def box_volume(h):
    h = np.asarray(h, np.float64)
    return float(8.0 * h[0] * h[1] * h[2])


def flood(E, group, centers, axes, slots, evaluate, K=32, follow=None, tie=2e-5):
    """Bulk-synchronous flood of the elements `group` into len(centers) boxes.

    evaluate(list of (slot, c, Q, h)) -> float64 array of OBV.

    ``follow`` (optional, element -> box index) names the choice another
    implementation took.  Where the two best moves of an element differ in dOBV
    by less than ``tie`` times the larger grown box volume (the estimator's
    noise), either choice is correct; the flood then takes the named one and
    counts it in ``counters["ties"]``.  Every value it uses is still its own.

    Returns (assign: dict element -> box index, boxes: list of (c, Q, h), obv
    array, counters dict).
    """
    b = len(centers)
    group = [int(e) for e in group]
    in_group = set(group)
    C = np.asarray(centers, np.float32).astype(np.float64)
    dist = {e: np.linalg.norm(E.cen[e] - C, axis=1) for e in group}
    key = {e: float(dist[e].min()) for e in group}
    assign = {}
    boxes = []
    chosen = set()
    for i in range(b):
        cand = [e for e in group if e not in chosen]
        s = min(cand, key=lambda e: (float(dist[e][i]), e))
        chosen.add(s)
        assign[s] = i
        c32, Q32 = np.float32(centers[i]), np.asarray(axes[i], np.float32)
        boxes.append(make_box(c32, Q32, E.extent(s, c32.astype(np.float64), Q32.astype(np.float64))))
    obv = np.array(evaluate([(slots[i], *boxes[i]) for i in range(b)]), dtype=np.float64)
    counters = {"rounds": 0, "evals": b, "trivial": 0, "moves": 0, "ties": 0}
    heap = []
    queued = set(assign)
    for s in list(assign):
        for n in E.adj[s]:
            if n in in_group and n not in queued:
                queued.add(n)
                heapq.heappush(heap, (key[n], n))

    def decide(pops):
        """Evaluate the (e, box) candidates of this round against the current boxes.

        A box that already contains e has dOBV = 0, the smallest possible value,
        so when one exists e goes to the nearest such box and the other boxes
        of e need no evaluation.
        """
        grown = {}
        req = []
        for e in pops:
            trivial_any = False
            for i in range(b):
                c, Q, h = boxes[i]
                ext = E.extent(e, c.astype(np.float64), Q.astype(np.float64))
                h2 = f32_up(np.maximum(h.astype(np.float64), ext))
                grown[(e, i)] = h2
                if np.array_equal(h2, h):
                    counters["trivial"] += 1
                    trivial_any = True
            if not trivial_any:
                req += [(e, i) for i in range(b)]
        vals = evaluate([(slots[i], boxes[i][0], boxes[i][1], grown[(e, i)]) for e, i in req]) if req else []
        counters["evals"] += len(req)
        dval = {k: v for k, v in zip(req, vals)}
        choice = {}
        for e in pops:
            best = None
            for i in range(b):
                if (e, i) in dval:
                    d = abs(dval[(e, i)] - obv[i])
                elif np.array_equal(grown[(e, i)], boxes[i][2]):
                    d = 0.0
                else:
                    continue          # not evaluated: another box contains e
                k = (d, float(dist[e][i]), i)
                if best is None or k < best:
                    best = k
            pick = best[2]
            f = None if follow is None else follow(e)
            if f is not None and f != pick and 0 <= f < b and (e, f) in dval:
                df = abs(dval[(e, f)] - obv[f])
                vb = max(box_volume(grown[(e, f)]), box_volume(grown[(e, pick)]))
                if df != best[0] and abs(df - best[0]) <= tie * vb:
                    pick = f
                    counters["ties"] += 1
            choice[e] = pick
        return choice, grown, dval

    def apply(choice, grown, dval):
        per_box = {}
        for e, i in choice.items():
            assign[e] = i
            per_box.setdefault(i, []).append(e)
            counters["moves"] += 1
        extra = []
        for i, es in per_box.items():
            c, Q, h = boxes[i]
            hs = [grown[(e, i)] for e in es]
            hn = hs[0]
            for x in hs[1:]:
                hn = np.maximum(hn, x)
            if np.array_equal(hn, h):
                continue
            boxes[i] = (c, Q, hn)
            same = [e for e in es if np.array_equal(grown[(e, i)], hn) and (e, i) in dval]
            if same:
                obv[i] = dval[(same[0], i)]
            else:
                extra.append(i)
        if extra:
            vals = evaluate([(slots[i], *boxes[i]) for i in extra])
            counters["evals"] += len(extra)
            for i, v in zip(extra, vals):
                obv[i] = v

    while heap:
        pops = []
        while heap and len(pops) < K:
            _, e = heapq.heappop(heap)
            if e not in assign:
                pops.append(e)
        if not pops:
            break
        counters["rounds"] += 1
        choice, grown, dval = decide(pops)
        apply(choice, grown, dval)
        for e in pops:
            for n in E.adj[e]:
                if n in in_group and n not in assign and n not in queued:
                    queued.add(n)
                    heapq.heappush(heap, (key[n], n))
    # elements the flood cannot reach
    for e in sorted(group):
        if e not in assign:
            choice, grown, dval = decide([e])
            apply(choice, grown, dval)
    return assign, boxes, obv, counters


def flood_partition(V, F, adj, group, centers, axes, slots, evaluate, K=32, follow=None, tie=2e-5):
    """The flood over single triangles (see ``flood``)."""
    return flood(triangle_elements(V, F, adj), group, centers, axes, slots, evaluate, K, follow, tie)


def serial_flood(V, F, adj, group, centers, axes, slots, evaluate):
    """The paper's serial flood: one t_min at a time (reference for K = 1)."""
    V = np.asarray(V)
    F = np.asarray(F)
    b = len(centers)
    in_group = set(int(t) for t in group)
    m = _centroids(V, F)
    C = np.asarray(centers, np.float32).astype(np.float64)
    boxes, assign, chosen = [], {}, set()
    for i in range(b):
        s = min((t for t in in_group if t not in chosen),
                key=lambda t: (float(np.linalg.norm(m[t] - C[i])), t))
        chosen.add(s)
        assign[s] = i
        boxes.append(make_box(centers[i], axes[i],
                              tri_extent(V, F, s, np.float32(centers[i]), np.float32(axes[i]))))
    obv = [float(v) for v in evaluate([(slots[i], *boxes[i]) for i in range(b)])]
    heap = []
    seen = set(assign)

    def push_neighbours(t):
        for n in adj[t]:
            if n in in_group and n not in seen:
                seen.add(n)
                heapq.heappush(heap, (float(np.linalg.norm(m[n] - C, axis=1).min()), n))

    for s in list(assign):
        push_neighbours(s)

    def take(t):
        best, best_h, best_v = None, None, None
        grown = []
        for i in range(b):
            c, Q, h = boxes[i]
            grown.append(f32_up(np.maximum(h.astype(np.float64), tri_extent(V, F, t, c, Q))))
        inside = [i for i in range(b) if np.array_equal(grown[i], boxes[i][2])]
        for i in (inside if inside else range(b)):
            c, Q, h = boxes[i]
            h2 = grown[i]
            if inside:
                d, v = 0.0, obv[i]
            else:
                v = float(evaluate([(slots[i], c, Q, h2)])[0])
                d = abs(v - obv[i])
            k = (d, float(np.linalg.norm(m[t] - C[i])), i)
            if best is None or k < best:
                best, best_h, best_v = k, h2, v
        i = best[2]
        assign[t] = i
        boxes[i] = (boxes[i][0], boxes[i][1], best_h)
        obv[i] = best_v

    while heap:
        _, t = heapq.heappop(heap)
        if t in assign:
            continue
        take(t)
        push_neighbours(t)
    for t in sorted(in_group):
        if t not in assign:
            take(t)
    return assign, boxes, np.array(obv)


# ---------------------------------------------------------------------------
# parameter update
# ---------------------------------------------------------------------------
def rot_local(k, theta):
    """Rotation by theta about local axis k, acting on the local axis frame."""
    cth, sth = np.cos(theta), np.sin(theta)
    R = np.eye(3)
    a, b = (k + 1) % 3, (k + 2) % 3
    R[a, a], R[a, b], R[b, a], R[b, b] = cth, -sth, sth, cth
    return R


def rodrigues(r):
    th = float(np.linalg.norm(r))
    if th == 0.0:
        return np.eye(3)
    k = np.asarray(r, np.float64) / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * (Kx @ Kx)


def rotation_vector(Rm):
    """Axis times angle of a rotation matrix (log map; angles well below pi)."""
    c = np.clip((np.trace(Rm) - 1.0) / 2.0, -1.0, 1.0)
    th = float(np.arccos(c))
    if th == 0.0:
        return np.zeros(3)
    w = np.array([Rm[2, 1] - Rm[1, 2], Rm[0, 2] - Rm[2, 0], Rm[1, 0] - Rm[0, 1]])
    return th * w / (2.0 * np.sin(th))


def update_box(V, F, tris, Q, slot, evaluate, delta=0.02, steps=(8.0, 4.0, 2.0, 1.0, 0.5),
               follow_box=None, tie=2e-5, eps=1e-5, counters=None):
    """Step 2 of the Lloyd iteration for one box: tight box, FD gradient over the
    three rotation angles, line search along -gradient; returns (box, obv, accepted).

    ``follow_box`` (optional (c, Q, h)) is the box another implementation kept
    whose outer-volume estimates agree with these to ``eps`` of the box volume.
    Its finite-difference gradient then differs by at most sqrt(3) eps V / delta
    per component, so its descent direction by at most
    kappa = 2 sqrt(3) eps V / (delta |g|) (plus float32 rounding of the axes):
    the update is ill-conditioned where |g| is small.  The named box is taken
    when it is valid under that bound:
    it is this oracle's tight box for its own axes; its axes are the current
    ones or a rotation of them by one of the line-search steps about a direction
    within kappa of -g / |g|; and its outer volume (evaluated here) agrees with
    this update's value at the same step to tie V plus the first-order change
    2 s delta |g| |d' - d|, with the choice among candidates a near-tie (within
    tie V, plus the same direction allowance) when it differs from this one.
    Taken boxes are counted in ``counters["update_ties"]``.
    """
    Q = np.asarray(Q, np.float32).astype(np.float64)
    base = tight_box(V, F, tris, Q)
    cands = [base]
    for k in range(3):
        for sgn in (+1.0, -1.0):
            cands.append(tight_box(V, F, tris, rot_local(k, sgn * delta) @ Q))
    vals = np.asarray(evaluate([(slot, *bx) for bx in cands]), dtype=np.float64)
    g = np.array([(vals[1 + 2 * k] - vals[2 + 2 * k]) / (2 * delta) for k in range(3)])
    gn = float(np.linalg.norm(g))
    options = [(base, float(vals[0]), False)]
    pick = 0
    d = np.zeros(3)
    lv = np.zeros(0)
    if gn != 0.0:
        d = -g / gn
        line = [tight_box(V, F, tris, rodrigues(s * delta * d) @ Q) for s in steps]
        lv = np.asarray(evaluate([(slot, *bx) for bx in line]), dtype=np.float64)
        options += [(line[j], float(lv[j]), True) for j in range(len(steps))]
        j = int(np.argmin(lv))
        if lv[j] < vals[0]:
            pick = 1 + j
    if follow_box is None:
        return options[pick]
    fc, fQ, fh = (np.asarray(x, np.float64) for x in follow_box)
    fQ = fQ.reshape(3, 3)
    row = np.concatenate([fc, fQ.reshape(-1), fh])

    def gap(bx):
        return float(np.max(np.abs(np.concatenate([bx[0], bx[1].reshape(-1), bx[2]]).astype(np.float64) - row)))

    if gap(options[pick][0]) <= 1e-6:
        return options[pick]
    mine = tight_box(V, F, tris, fQ)
    if gap(mine) > 1e-6:
        return options[pick]                 # not the tight box of its own axes
    vbox = max(box_volume(mine[2]), box_volume(options[pick][0][2]))
    v_f = float(np.asarray(evaluate([(slot, *mine)]), dtype=np.float64)[0])
    r = rotation_vector(fQ @ Q.T)
    th = float(np.linalg.norm(r))
    kappa = (2.0 * np.sqrt(3.0) * eps * vbox / (delta * gn) if gn > 0 else np.inf)
    if th < 1e-6:                            # the named box kept the current axes
        allow = tie * vbox + (2.0 * max(steps) * delta * gn * min(kappa, 2.0) if pick else 0.0)
        ok = abs(v_f - vals[0]) <= tie * vbox and (pick == 0 or vals[0] - options[pick][1] <= allow)
    else:
        jf = int(np.argmin([abs(th - s * delta) for s in steps]))
        s_f = steps[jf]
        dd = float(np.linalg.norm(r / th - d)) if gn > 0 else np.inf
        round_off = 1e-6 / (s_f * delta)
        ok = gn > 0 and abs(th - s_f * delta) <= 1e-3 * s_f * delta and dd <= kappa + round_off
        if ok:
            drift = 2.0 * s_f * delta * gn * dd
            ok = abs(v_f - lv[jf]) <= tie * vbox + drift and v_f <= vals[0] + tie * vbox
            if ok and 1 + jf != pick:
                ok = abs(lv[jf] - options[pick][1]) <= tie * vbox + drift
    if not ok:
        return options[pick]
    if counters is not None:
        counters["update_ties"] = counters.get("update_ties", 0) + 1
    return (mine, v_f, th >= 1e-6)


# ---------------------------------------------------------------------------
# one Lloyd iteration of a group, and the hierarchy weights
# ---------------------------------------------------------------------------
def lloyd_iteration(V, F, adj, group, centers, axes, slots, evaluate, K=32, follow=None, follow_boxes=None,
                    tie=2e-5, counters=None):
    """Partition then update every box; returns (clusters, boxes, obv, layer error, flood counters).
    ``follow`` / ``follow_boxes`` (optional) name another implementation's
    choices, taken only where they are as valid as this one's (see ``flood`` and
    ``update_box``)."""
    assign, boxes, obv, cnt = flood_partition(V, F, adj, group, centers, axes, slots, evaluate, K, follow, tie)
    b = len(centers)
    clusters = [sorted(t for t, i in assign.items() if i == k) for k in range(b)]
    out_boxes, out_obv = [], []
    for k in range(b):
        if not clusters[k]:
            out_boxes.append(boxes[k])
            out_obv.append(float(obv[k]))
            continue
        fb = follow_boxes(k) if follow_boxes is not None else None
        bx, v, _ = update_box(V, F, clusters[k], boxes[k][1], slots[k], evaluate, follow_box=fb, tie=tie,
                              counters=counters)
        out_boxes.append(bx)
        out_obv.append(v)
    return clusters, out_boxes, np.array(out_obv), float(np.sum(out_obv)), cnt


# ---------------------------------------------------------------------------
# adjustment (Sec. 4.2.1, third step)
# ---------------------------------------------------------------------------
def least_important(clusters, obv):
    """The box of least importance: the fewest triangles; ties go to the larger
    outer volume, then to the higher index."""
    return min(range(len(clusters)), key=lambda i: (len(clusters[i]), -float(obv[i]), -i))


def adjust(V, F, adj, group, clusters, boxes, obv, slots, evaluate, K=32, follow=None, follow_boxes=None,
           tie=2e-5, counters=None):
    """One adjustment of a group's boxes, for when the Lloyd iteration stalls.

    The least important box is re-seeded where the group fits worst: its centre
    moves to the centroid of the triangle farthest from the centre of the box
    with the largest outer volume (ties: lower index; farthest: ties to the lower
    triangle index), and it takes that box's axes.  One Lloyd iteration then
    runs from the adjusted centres and axes; its result is kept if the group's
    error (sum of OBV) is lower than before, else the group is left as it was.

    Returns (accepted, clusters, boxes, obv, error)."""
    b = len(boxes)
    e0 = float(np.sum(obv))
    if b < 2:
        return False, clusters, boxes, obv, e0
    j = least_important(clusters, obv)
    w = min((i for i in range(b) if i != j), key=lambda i: (-float(obv[i]), i))
    if not clusters[w]:
        return False, clusters, boxes, obv, e0
    cen = _centroids(np.asarray(V), np.asarray(F))
    cw = np.asarray(boxes[w][0], np.float32).astype(np.float64)
    tw = np.asarray(sorted(clusters[w]))
    d = np.linalg.norm(cen[tw] - cw, axis=1)
    t = int(tw[np.flatnonzero(d == d.max())[0]])
    centers = [np.asarray(bx[0], np.float32) for bx in boxes]
    axes = [np.asarray(bx[1], np.float32) for bx in boxes]
    centers[j] = cen[t].astype(np.float32)
    axes[j] = np.asarray(boxes[w][1], np.float32).copy()
    c2, b2, o2, e2, _ = lloyd_iteration(V, F, adj, group, centers, axes, slots, evaluate, K, follow, follow_boxes,
                                        tie, counters)
    if e2 < e0:
        return True, c2, b2, o2, e2
    return False, clusters, boxes, obv, e0


def layer_weights(n_levels):
    """Sec. 5: omega = number of layers from the layer to the leaves, leaf = 1."""
    return [float(n_levels - l) for l in range(n_levels)]


def hierarchy_error(level_obv, weights):
    """Eq. 7 with each layer's OMV replaced by its sum of OBV (Eq. 6)."""
    return float(sum(w * float(np.sum(o)) for w, o in zip(weights, level_obv)))
