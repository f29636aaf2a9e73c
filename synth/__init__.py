"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only builds meshes (vertex/triangle arrays) and box parameter arrays
from seeds.  It holds none of the outer-volume, fitting or clustering arithmetic:
both the CPU oracle and the HIP library receive these arrays as plain inputs.
"""
from .meshes import (icosahedron, icosphere, cuboid, octahedron, tetrahedron,
                     noisy_torus, noisy_cube_sphere, helix_tube, disjoint_cuboids,
                     lognormal_triangle_counts, noisy_sphere_batch, split_top_slab)
from .boxes import (random_boxes, quat_to_axes, axis_aligned_box, boxes_to_array, mixed_boxes, flood_candidates,
                    query_spheres)

__all__ = [
    "icosahedron", "icosphere", "cuboid", "octahedron", "tetrahedron",
    "noisy_torus", "noisy_cube_sphere", "helix_tube", "disjoint_cuboids",
    "lognormal_triangle_counts", "noisy_sphere_batch", "split_top_slab",
    "random_boxes", "quat_to_axes", "axis_aligned_box", "mixed_boxes",
    "boxes_to_array", "flood_candidates", "query_spheres",
]
