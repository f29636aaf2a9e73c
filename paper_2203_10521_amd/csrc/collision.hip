// Synthetic collision queries against a box hierarchy, the stand-in for the
// paper's collision experiment (Sec. 5: colliders against the model's
// hierarchy, counting bounding-volume tests).  One thread per sphere descends
// the level-order tree without a stack: after a node, the walk goes to its
// first child when the sphere overlaps it and it has children, else to the
// next sibling, climbing while the node is the last of its siblings.  The
// sphere-box test is float64 with one fixed rounding sequence.
#include <algorithm>

#include "common.h"

// Built with -ffp-contract=off (build.py): every operation rounds on its own,
// in the order the oracle follows.

namespace obbv {
namespace {

constexpr int kCollThreads = 256;

// Sphere (x, r) against box b: the squared distance from x to the box in its
// frame, sum_k max(|Q_k . (x - c)| - h_k, 0)^2, against r^2.
__device__ inline bool sphere_box(const double x[3], double r2, const obbv_box& b) {
  const double d0 = __dsub_rn(x[0], (double)b.center[0]);
  const double d1 = __dsub_rn(x[1], (double)b.center[1]);
  const double d2 = __dsub_rn(x[2], (double)b.center[2]);
  double dist2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = __dadd_rn(__dadd_rn(__dmul_rn((double)b.axes[3 * k], d0), __dmul_rn((double)b.axes[3 * k + 1], d1)),
                               __dmul_rn((double)b.axes[3 * k + 2], d2));
    const double e = __dsub_rn(fabs(t), (double)b.half[k]);
    if (e > 0.0) dist2 = __dadd_rn(dist2, __dmul_rn(e, e));
  }
  return dist2 <= r2;
}

__global__ void __launch_bounds__(kCollThreads)
k_collide(const obbv_box* __restrict__ nodes, const uint8_t* __restrict__ used, int levels, int branching,
          const float4* __restrict__ spheres, int n_spheres, int32_t* __restrict__ out_tests,
          int32_t* __restrict__ out_hits) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_spheres) return;
  const float4 s = spheres[q];
  const double x[3] = {(double)s.x, (double)s.y, (double)s.z};
  const double r2 = __dmul_rn((double)s.w, (double)s.w);
  int64_t first[17];  // first node of each level
  first[0] = 0;
  int64_t width = 1;
  for (int l = 0; l < levels; ++l) {
    first[l + 1] = first[l] + width;
    width *= branching;
  }
  int l = 0;
  int64_t j = 0;
  int32_t tests = 0, hits = 0;
  for (;;) {
    const int64_t node = first[l] + j;
    bool ov = false;
    if (!used || used[node]) {
      ++tests;
      ov = sphere_box(x, r2, nodes[node]);
    }
    if (ov && l + 1 < levels) {  // first child
      ++l;
      j *= branching;
      continue;
    }
    if (ov) ++hits;
    while (l > 0 && j % branching == branching - 1) {  // last sibling: up
      --l;
      j /= branching;
    }
    if (l == 0) break;
    ++j;
  }
  out_tests[q] = tests;
  out_hits[q] = hits;
}

}  // namespace

int collision_queries(const obbv_box* nodes, const uint8_t* node_used, int32_t levels, int32_t branching,
                      const float* spheres, int32_t n_spheres, int32_t* out_tests, int32_t* out_hits, hipStream_t s) {
  OBBV_ARG(levels >= 1 && levels <= 16, "levels must be in [1, 16]");
  OBBV_ARG(branching >= 1 && branching <= 64, "branching must be in [1, 64]");
  OBBV_ARG(n_spheres >= 0, "n_spheres < 0");
  if (n_spheres == 0) return OBBV_OK;
  int64_t n_nodes = 0, width = 1;
  for (int l = 0; l < levels; ++l) {
    n_nodes += width;
    width *= branching;
    OBBV_ARG(n_nodes <= ((int64_t)1 << 40), "the hierarchy has too many nodes");
  }
  OBBV_ARG(nodes && spheres && out_tests && out_hits, "NULL argument");
  OBBV_ARG(((uintptr_t)spheres & 15u) == 0, "spheres must be 16-byte aligned");
  hipLaunchKernelGGL(k_collide, dim3((unsigned)ceil_div(n_spheres, kCollThreads)), dim3(kCollThreads), 0, s, nodes,
                     node_used, levels, branching, (const float4*)spheres, n_spheres, out_tests, out_hits);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

}  // namespace obbv

static int obbv_collision_queries_body(const obbv_box* nodes, const uint8_t* node_used, int32_t levels,
                                      int32_t branching, const float* spheres, int32_t n_spheres, int32_t* out_tests,
                                      int32_t* out_hits, void* stream);
extern "C" int obbv_collision_queries(const obbv_box* nodes, const uint8_t* node_used, int32_t levels,
                                      int32_t branching, const float* spheres, int32_t n_spheres, int32_t* out_tests,
                                      int32_t* out_hits, void* stream) {
  return obbv::guarded([&] { return obbv_collision_queries_body(nodes, node_used, levels, branching, spheres, n_spheres, out_tests, out_hits, stream); });
}
static int obbv_collision_queries_body(const obbv_box* nodes, const uint8_t* node_used, int32_t levels,
                                      int32_t branching, const float* spheres, int32_t n_spheres, int32_t* out_tests,
                                      int32_t* out_hits, void* stream) {
  obbv::clear_error();
  return obbv::collision_queries(nodes, node_used, levels, branching, spheres, n_spheres, out_tests, out_hits,
                                 (hipStream_t)stream);
}
