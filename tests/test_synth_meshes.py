"""The synthetic workloads are closed, outward oriented solids of the stated sizes."""
import numpy as np
import pytest

import synth
from oracle import geometry


@pytest.mark.parametrize("name", ["icosphere3", "torus", "cubesphere", "helix_small", "cuboid",
                                  "octa", "tetra", "icosa"])
def test_closed_oriented_positive(name):
    V, F = {
        "icosphere3": lambda: synth.icosphere(3),
        "torus": lambda: synth.noisy_torus(),
        "cubesphere": lambda: synth.noisy_cube_sphere(12),
        "helix_small": lambda: synth.helix_tube(rings=200, around=16),
        "cuboid": lambda: synth.cuboid((0.3, 0.6, 0.9)),
        "octa": lambda: synth.octahedron(),
        "tetra": lambda: synth.tetrahedron(),
        "icosa": lambda: synth.icosahedron(),
    }[name]()
    ok, bad = geometry.directed_edge_report(F)
    assert ok, bad
    assert geometry.signed_volume(V, F) > 0
    assert V.dtype == np.float32 and F.dtype == np.int32


def test_workload_sizes():
    V, F = synth.icosphere(3)
    assert (len(V), len(F)) == (642, 1280)
    V, F = synth.noisy_torus()
    assert (len(V), len(F)) == (32768, 65536)
    V, F = synth.noisy_cube_sphere(41)
    assert len(F) == 12 * 41 * 41
    V, F = synth.helix_tube(rings=100, around=128)
    assert len(F) == 99 * 128 * 2 + 256


def test_spherical_harmonic_recurrence_matches_scipy():
    from scipy.special import sph_harm_y
    from synth.meshes import _legendre_normalised
    g = np.random.default_rng(0)
    d = g.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    P = _legendre_normalised(d[:, 2], 8)
    for l in range(9):
        for m in range(l + 1):
            Y = sph_harm_y(l, m, theta, phi)
            assert np.allclose(P[l][m] * np.cos(m * phi), Y.real, atol=1e-12), (l, m)
            assert np.allclose(P[l][m] * np.sin(m * phi), Y.imag, atol=1e-12), (l, m)


def test_lognormal_counts_range_and_median():
    T = synth.lognormal_triangle_counts(4096, seed=3)
    assert T.min() >= 2000 and T.max() <= 200000
    # truncation at +-2 sigma is nearly symmetric in log space: median stays ~20k
    assert 17000 < np.median(T) < 23000
