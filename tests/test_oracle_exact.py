"""Pins of the exact outer-volume oracle (Sec. 3, Eq. 4 / divergence theorem)."""
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import exact, geometry, rng as orng
from tests.pins import interval_overlap, points_in_box, winding_number

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_stream():
    vals = [int(x) for x in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if x.strip() and not x.startswith("#")]
    assert [orng.splitmix64(1234567, n) for n in range(5)] == vals
    assert [int(x) for x in orng.splitmix64_np(1234567, np.arange(5, dtype=np.uint64))] == vals


@pytest.mark.parametrize("mesh", ["icosphere", "torus", "cubesphere", "tetra"])
def test_enclosing_box_gives_mesh_volume(mesh):
    """Box containing the whole mesh: vol(X ∩ O) = vol(X) = sum det / 6."""
    if mesh == "icosphere":
        V, F = synth.icosphere(2)
    elif mesh == "torus":
        V, F = synth.noisy_torus(nu=32, nv=16)
    elif mesh == "cubesphere":
        V, F = synth.noisy_cube_sphere(4)
    else:
        V, F = synth.tetrahedron(0.7)
    vm = geometry.signed_volume(V, F)
    _, a, _ = synth.random_boxes(1, seed=5)
    u, _, vt = np.linalg.svd(a[0].astype(np.float64))
    Q = u @ vt                      # orthonormal to float64 precision (float32 axes are not)
    # a randomly rotated box large enough to contain everything
    vin = exact.inside_volume(V, F, [0.01, -0.02, 0.03], Q, [2.0, 2.1, 2.2])
    for w in range(3):
        assert abs(vin[w] - vm) <= 1e-12 * abs(vm)


def test_box_inside_solid_and_disjoint():
    V, F = synth.icosphere(3)
    _, a, _ = synth.random_boxes(1, seed=8)
    h = [0.3, 0.25, 0.2]            # corner radius < 0.45 < inradius of the icosphere
    assert abs(exact.obv(V, F, [0.05, 0.0, -0.05], a[0], h)) <= 1e-13
    far = [5.0, 0.0, 0.0]
    for w in range(3):
        # crossings above the slab cancel in pairs (exactly in rationals, to rounding here)
        assert abs(exact.obv(V, F, far, a[0], h, axis=w) - exact.box_volume(h)) <= 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_rotated_cuboid_vs_aligned_box(seed):
    """Cuboid mesh and a box sharing its axes: the inside volume is the product
    of the three interval overlaps in the common local frame."""
    r = np.random.default_rng(seed)
    _, a, _ = synth.random_boxes(1, seed=100 + seed)
    u, _, vt = np.linalg.svd(a[0].astype(np.float64))
    Q = u @ vt
    ch = r.uniform(0.3, 1.0, 3)
    cc = r.uniform(-0.3, 0.3, 3)
    bh = r.uniform(0.2, 0.9, 3)
    bc_local = r.uniform(-0.8, 0.8, 3)
    _, F = synth.cuboid(ch, cc @ Q, Q)          # cuboid centre cc in local coordinates
    corners = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], float)
    V = (corners * ch + cc) @ Q                 # same vertex order, exact float64 corners
    bc = bc_local @ Q
    vin = exact.inside_volume(V, F, bc, Q, bh)
    ref = np.prod([interval_overlap(cc[k] - ch[k], cc[k] + ch[k],
                                    bc_local[k] - bh[k], bc_local[k] + bh[k]) for k in range(3)])
    for w in range(3):
        assert abs(vin[w] - ref) <= 1e-12


def test_partition_invariant_tiles_sum_to_mesh_volume():
    """Boxes tiling a region that contains the mesh (common random frame):
    their inside volumes add up to vol(X)."""
    V, F = synth.noisy_torus(nu=24, nv=12)
    vm = geometry.signed_volume(V, F)
    _, a, _ = synth.random_boxes(1, seed=33)
    u, _, vt = np.linalg.svd(a[0].astype(np.float64))
    Q = u @ vt
    loc = V.astype(np.float64) @ Q.T
    lo, hi = loc.min(0) - 0.05, loc.max(0) + 0.05
    n = (3, 2, 2)
    edges = [np.linspace(lo[k], hi[k], n[k] + 1) for k in range(3)]
    total = 0.0
    for i in range(n[0]):
        for j in range(n[1]):
            for k in range(n[2]):
                cl = np.array([(edges[0][i] + edges[0][i + 1]) / 2,
                               (edges[1][j] + edges[1][j + 1]) / 2,
                               (edges[2][k] + edges[2][k + 1]) / 2])
                hl = np.array([(edges[0][i + 1] - edges[0][i]) / 2,
                               (edges[1][j + 1] - edges[1][j]) / 2,
                               (edges[2][k + 1] - edges[2][k]) / 2])
                total += exact.inside_volume(V, F, cl @ Q, Q, hl, axis=(i + j + k) % 3)
    assert abs(total - vm) <= 1e-11 * vm


def test_fraction_exact_matches_float():
    """Rational octahedron-like solid, rational rotation from an integer quaternion:
    the float64 result agrees with the exact rational one."""
    V = [[Fraction(3, 2), 0, 0], [Fraction(-5, 4), 0, 0], [0, Fraction(7, 5), 0],
         [0, Fraction(-6, 5), 0], [0, 0, Fraction(4, 3)], [0, 0, Fraction(-1, 1)]]
    V = [[Fraction(x) for x in row] for row in V]
    _, F = synth.octahedron()
    Qx = geometry.rational_rotation(3, 1, -2, 1)
    c = [Fraction(1, 7), Fraction(-1, 9), Fraction(1, 11)]
    h = [Fraction(3, 5), Fraction(4, 5), Fraction(1, 2)]
    Vf = np.array([[float(x) for x in r] for r in V])
    Qf = np.array([[float(x) for x in r] for r in Qx])
    for w in range(3):
        ex = exact.inside_volume_exact(V, F, c, Qx, h, axis=w)
        assert isinstance(ex, Fraction)
        fl = exact.inside_volume(Vf, F, [float(x) for x in c], Qf, [float(x) for x in h], axis=w)
        assert abs(fl - float(ex)) <= 1e-13 * max(1.0, abs(float(ex)))
    # exactness across axes (the three casts give the same rational number)
    e = [exact.inside_volume_exact(V, F, c, Qx, h, axis=w) for w in range(3)]
    assert e[0] == e[1] == e[2]


@pytest.mark.parametrize("mesh,n", [("cube", 400_000), ("octa", 400_000),
                                    ("icosa", 300_000), ("ico1", 150_000)])
def test_monte_carlo_winding_number(mesh, n):
    """|exact - MC| <= 4 sigma with inside points classified by the generalised
    winding number (solid angles, no ray parity)."""
    if mesh == "cube":
        V, F = synth.cuboid((0.6, 0.5, 0.4))
    elif mesh == "octa":
        V, F = synth.octahedron(0.9)
    elif mesh == "icosa":
        V, F = synth.icosahedron(0.9)
    else:
        V, F = synth.icosphere(1, 0.9)
    c, a, h = synth.random_boxes(3, seed=77, center_range=0.4, half_range=(0.2, 0.7))
    g = np.random.default_rng(5)
    for b in range(3):
        pts = points_in_box(g, n, c[b], a[b], h[b])
        inside = winding_number(V, F, pts) > 0.5
        vb = exact.box_volume(h[b])
        p = inside.mean()
        mc = vb * p
        sig = vb * np.sqrt(max(p * (1 - p), 1e-12) / n)
        ex = exact.inside_volume(V, F, c[b], a[b], h[b], axis=b % 3)
        assert abs(ex - mc) <= 4 * sig + 1e-12


def test_rigid_motion_and_scaling():
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(2, seed=9)
    _, Rm, _ = synth.random_boxes(1, seed=10)
    u, _, vt = np.linalg.svd(Rm[0].astype(np.float64))
    Rm = u @ vt
    t = np.array([0.3, -1.1, 2.0])
    V64 = V.astype(np.float64)
    for b in range(2):
        base = exact.inside_volume(V64, F, c[b], a[b], h[b], axis=0)
        # rotate + translate mesh and box together: x -> x Rm + t
        Vm = V64 @ Rm + t
        cm = c[b].astype(np.float64) @ Rm + t
        am = a[b].astype(np.float64) @ Rm
        moved = exact.inside_volume(Vm, F, cm, am, h[b], axis=1)
        assert abs(moved - base) <= 1e-11
        s = 1.7
        scaled = exact.inside_volume(V64 * s, F, c[b].astype(np.float64) * s, a[b],
                                     h[b].astype(np.float64) * s, axis=2)
        assert abs(scaled - s ** 3 * base) <= 1e-11 * s ** 3


def test_eq5_sum_of_obv_bounds_union_outer_volume():
    """Sum_j OBV(X, O_j) >= OMV(X, union O_j) (Sec. 3, Eq. 5); MC for the union."""
    V, F = synth.icosphere(2)
    c, a, h = synth.random_boxes(3, seed=41, center_range=0.6, half_range=(0.3, 0.8))
    s = sum(exact.obv(V, F, c[b], a[b], h[b]) for b in range(3))
    g = np.random.default_rng(1)
    lo = (c - np.linalg.norm(h, axis=1)[:, None]).min(0)
    hi = (c + np.linalg.norm(h, axis=1)[:, None]).max(0)
    n = 200_000
    pts = g.uniform(lo, hi, size=(n, 3))
    in_union = np.zeros(n, bool)
    for b in range(3):
        loc = (pts - c[b]) @ a[b].astype(np.float64).T
        in_union |= np.all(np.abs(loc) <= h[b], axis=1)
    outside = winding_number(V, F, pts) < 0.5
    omv = np.prod(hi - lo) * np.mean(in_union & outside)
    assert s >= omv - 4 * np.prod(hi - lo) * np.sqrt(0.25 / n)


def test_faces_in_the_box_faces_count_once():
    """Mesh faces lying exactly in the planes of the box faces (aligned cuboids
    and their bounding or tight boxes): the inside volume is the closed form
    along every cast axis, in float64 and in exact rationals."""
    parts = [synth.cuboid((0.5, 0.25, 0.375), c) for c in [(-3, 0.75, 0), (-3, -0.75, 0), (3, 0.75, 0)]]
    V = np.vstack([p[0] for p in parts])
    F = np.vstack([p[1] + 8 * k for k, p in enumerate(parts)])
    v_one = 1.0 * 0.5 * 0.75
    cases = [([0.0, 0.0, 0.0], [3.5, 1.0, 0.375], 3 * v_one),       # bounding box of all three
             ([-3.0, 0.0, 0.0], [0.5, 1.0, 0.375], 2 * v_one),      # bounding box of the pair
             ([3.0, 0.75, 0.0], [0.5, 0.25, 0.375], v_one),         # tight box of one cuboid
             ([3.0, 0.75, 0.0], [0.25, 0.25, 0.375], v_one / 2)]    # half of it, sharing 5 faces
    for c, h, vin in cases:
        got = exact.inside_volume(V, F, c, np.eye(3), h)
        assert np.allclose(got, vin, rtol=0, atol=1e-15), (c, h, got)
        for w in range(3):
            assert exact.inside_volume_exact(V, F, c, np.eye(3).tolist(), h, axis=w) == Fraction(vin)
