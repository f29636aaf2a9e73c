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
