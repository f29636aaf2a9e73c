"""Synthetic collision queries against a box hierarchy (float64 oracle) -- the
stand-in for the paper's collision experiment (Sec. 5: colliders against the
model's hierarchy, counting bounding-volume tests; the physics engine and the
models are absent).  Test infrastructure only: never imported by the library.

A query is a sphere (centre x, radius r).  The hierarchy is descended from the
root: a node is tested against the sphere; when the sphere overlaps its box and
the node has children, the children are tested in order; an overlapped leaf is
a hit.  Nodes marked unused (no triangles) are never tested.  The result of a
query is (tests, hits).

Sphere-box overlap: in the box frame (row k of Q is local axis k) the centre is
d_k = Q_k . (x - c); the squared distance from the centre to the box is
sum_k max(|d_k| - h_k, 0)^2, and the sphere overlaps the box iff it is <= r^2.
Written out in Python float64 with one fixed order of operations:
d_k = (Q_k0 (x0 - c0) + Q_k1 (x1 - c1)) + Q_k2 (x2 - c2), and the sum over k
left to right.

Layout (the hierarchy builders' output): nodes in level order, level l holding
b^l nodes; node j of level l (j counted within the level) has children
b j .. b j + b - 1 of level l + 1.
"""


def sphere_overlaps_box(x, r, c, Q, h):
    """True when the sphere (x, r) and the box (c, Q, h) intersect (float64)."""
    d = [float(x[k]) - float(c[k]) for k in range(3)]
    dist2 = 0.0
    for k in range(3):
        t = (float(Q[k][0]) * d[0] + float(Q[k][1]) * d[1]) + float(Q[k][2]) * d[2]
        e = abs(t) - float(h[k])
        if e > 0.0:
            dist2 = dist2 + e * e
    return dist2 <= float(r) * float(r)


def query(levels, branching, boxes, used, x, r):
    """(tests, hits) of one sphere.  boxes[l][j] = (c, Q, h), used[l][j] bool."""
    tests = 0
    hits = 0

    def visit(l, j):
        nonlocal tests, hits
        if not used[l][j]:
            return
        tests += 1
        c, Q, h = boxes[l][j]
        if not sphere_overlaps_box(x, r, c, Q, h):
            return
        if l + 1 == levels:
            hits += 1
            return
        for k in range(branching):
            visit(l + 1, branching * j + k)

    visit(0, 0)
    return tests, hits


def queries(levels, branching, boxes, used, spheres):
    """(tests, hits) arrays of every sphere (rows: x, y, z, r)."""
    out_t, out_h = [], []
    for s in spheres:
        t, h = query(levels, branching, boxes, used, s[:3], s[3])
        out_t.append(t)
        out_h.append(h)
    return out_t, out_h


def boxes_by_level(flat, levels, branching):
    """Split a level-order [n_nodes][15] array (centre, axes rows, half extents)
    into boxes[l][j] = (c, Q, h)."""
    out, base = [], 0
    for l in range(levels):
        n = branching ** l
        lv = []
        for j in range(n):
            row = flat[base + j]
            lv.append((list(row[0:3]), [list(row[3:6]), list(row[6:9]), list(row[9:12])], list(row[12:15])))
        out.append(lv)
        base += n
    return out
