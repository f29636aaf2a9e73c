"""Pins of the OBB-tree oracle (the top-down comparison baseline)."""
import numpy as np

import synth
from oracle import tree as otree


def _two_cuboids():
    VA, FA = synth.cuboid((0.5, 0.3, 0.2), (0.0, 0.0, 0.0))
    VB, FB = synth.cuboid((0.4, 0.35, 0.25), (5.0, 0.2, -0.1))
    V = np.vstack([VA, VB])
    F = np.vstack([FA, FB + len(VA)]).astype(np.int32)
    return V, F


def test_median_split_separates_two_far_cuboids_into_their_exact_boxes():
    """Two cuboids of 12 triangles each, 5 apart along x: the root's longest
    axis is x, the median cut puts each cuboid in one child, and each child's
    covariance box is its cuboid exactly (centre and half extents in closed form)."""
    V, F = _two_cuboids()
    boxes, tri_node = otree.build_obb_tree(V, F, 2, 2)
    Q0 = np.asarray(boxes[0][0][1])
    assert abs(Q0[0, 0]) > 0.99          # the cuboids lie 5 apart along x
    assert sorted(set(tri_node[1][:12])) == [tri_node[1][0]] and sorted(set(tri_node[1][12:])) == [tri_node[1][12]]
    assert tri_node[1][0] != tri_node[1][12]
    for comp, (half, centre) in ((tri_node[1][0], ((0.5, 0.3, 0.2), (0.0, 0.0, 0.0))),
                                 (tri_node[1][12], ((0.4, 0.35, 0.25), (5.0, 0.2, -0.1)))):
        c, Q, h = boxes[1][comp][:3]
        assert np.allclose(c, centre, atol=1e-6)
        assert np.allclose(np.sort(h), np.sort(half), atol=1e-6)
        assert abs(np.prod(h) - np.prod(half)) <= 1e-6 * np.prod(half)


def test_levels_partition_into_equal_counts_and_nest():
    V, F = synth.icosphere(2)
    b, L = 4, 3
    _, tri_node = otree.build_obb_tree(V, F, L, b)
    nt = len(F)
    for lv in range(L):
        n = b ** lv
        counts = np.bincount(tri_node[lv], minlength=n)
        assert counts.sum() == nt and len(counts) == n
        if lv:
            parent = tri_node[lv] // b
            assert np.array_equal(parent, tri_node[lv - 1])
            for p in range(b ** (lv - 1)):
                kids = counts[p * b:(p + 1) * b]
                assert kids.max() - kids.min() <= 1


def test_children_of_a_node_are_ordered_along_its_longest_axis():
    V, F = synth.noisy_torus(nu=32, nv=16)
    boxes, tri_node = otree.build_obb_tree(V, F, 2, 4)
    Q, h = np.asarray(boxes[0][0][1]), np.asarray(boxes[0][0][2])
    k = int(np.argmax(h))
    p = otree.centroids(V, F) @ Q[k]
    for part in range(3):
        assert p[tri_node[1] == part].max() <= p[tri_node[1] == part + 1].min()
