// Outer volume OBV(X, O) of oriented boxes against a closed mesh
// (Sec. 3, Eq. 4), by jittered parallel rays on each box face and the signed
// crossing sum along each ray (Sec. 4.1, Eq. 9 generalised to a line).
//
// Pipeline per call (all on one stream, no host round trip):
//   k_mesh_centre        centre of every mesh's bounding box (unless the caller
//                        gives it): every cast keeps the half prism on the far
//                        side of its box from it
//   [k_frame_list]       boxes grouped by shared centre and axes: per (group,
//                        cast axis), the frame-local coordinates of the triangles
//                        in the group's kept half prism, in one pass into
//                        fixed segments (lists beyond 2 GB: k_frame_cull
//                        counts, k_frame_scan sizes, k_frame_cull fills)
//   k_span_bounds        single-mesh calls on meshes of more than one cast item
//                        (unless the caller has them): the bounding box of every
//                        span of 256 consecutive triangles and of every run of 18
//                        spans (one cast item); spans the kept half prism of a
//                        cast cannot reach are skipped below (meshes whose
//                        triangle order follows the surface -- grids, strips --
//                        give tight spans; any order gives the same results)
//   k_box_chunks         one block: the triangle list of every (box, axis) (its
//                        group's list or the whole mesh) cut into cast items of
//                        kCastTris entries (whole-mesh runs whose bounds miss the
//                        cast's kept half prism are left out), the ray grid of
//                        every cast, and the per-call counters set to zero
//   k_cast               persistent workgroups take (item, ray block) units from
//                        a device queue: the item's triangles are culled against
//                        the box's kept half prism and the block, the survivors
//                        compacted (wave ballots + a workgroup prefix) into LDS
//                        with their bounding cell range; the jittered rays of that
//                        range go to LDS; each lane builds one survivor's FP32
//                        edge and depth planes in registers and tests the rays of
//                        the cells its projected bounding box covers (waves
//                        take chunks of 64 survivors from an LDS cursor;
//                        records covering many cells are broadcast from their
//                        lane and tested by the whole wave, one cell per lane);
//                        the exact integer inside lengths are summed
//                        per lane, per workgroup, then into the (box, axis) int64
//                        sum
//   k_finalize           float64 OBV per box, publication of the call
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace obbv {
namespace {

constexpr int kCullThreads = 256;
constexpr int kCastThreads = 768;    // 12 waves: three per SIMD, one workgroup per CU
constexpr int kCastWaves = kCastThreads / 64;
constexpr int kCastTris = 4608;      // triangle-list entries per cast item (6 cull steps; 384 per wave)
constexpr int kRayBatch = 8;        // rays a thread generates at once in the ray phase
constexpr int kRasterCells = 512;    // records covering more cells take the wave-wide test
constexpr int kBlockRaysDefault = 16384;  // rays of one LDS ray block (float2 each): a whole
                                          // face up to R = 128
constexpr int kBlockRaysMax = 16384;
constexpr int kSpanTris = 256;                     // triangles per span (bounds table)
constexpr int kSpansPerItem = kCastTris / kSpanTris;  // 18
static_assert(kCastTris % kSpanTris == 0 && kSpansPerItem <= 64, "spans of an item fit one wave");

struct BoxRegs {
  float Q[9];
  float c[3];
  float h[3];
};

__device__ inline BoxRegs load_box(const obbv_box* __restrict__ boxes, int b) {
  BoxRegs r;
  const float* p = reinterpret_cast<const float*>(boxes + b);
#pragma unroll
  for (int k = 0; k < 3; ++k) r.c[k] = p[k];
#pragma unroll
  for (int k = 0; k < 9; ++k) r.Q[k] = p[3 + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) r.h[k] = p[12 + k];
  return r;
}

// element k (0, 1 or 2, a run-time value) of a 3-vector held in registers: the
// bits blended by masks, which keeps the compiler from turning the choice into
// an indexed load from a private-memory copy of the vector
__device__ inline float pick3(const float v[3], int k) {
  const uint32_t m0 = 0u - (uint32_t)(k == 0), m1 = 0u - (uint32_t)(k == 1), m2 = 0u - (uint32_t)(k == 2);
  return __uint_as_float((__float_as_uint(v[0]) & m0) | (__float_as_uint(v[1]) & m1) | (__float_as_uint(v[2]) & m2));
}

// 0 = computable box, 1 = zero extent (OBV 0, nothing to cast), 2 = invalid (NaN / negative)
__device__ inline int box_state(const BoxRegs& B) {
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) finite = finite && isfinite(B.Q[k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) finite = finite && isfinite(B.c[k]) && isfinite(B.h[k]);
  if (!finite) return 2;
  if (B.h[0] < 0.f || B.h[1] < 0.f || B.h[2] < 0.f) return 2;
  if (B.h[0] == 0.f || B.h[1] == 0.f || B.h[2] == 0.f) return 1;
  return 0;
}

// The ray grid of one (box, axis) cast, computed once per call by k_box_sides:
// half extents of the face (float64 of the float32 extents), cell sizes
// du = 2 hu / R and their reciprocals, the 1e-6 cell-range margins, the
// SplitMix64 state of the cast's first u draw, seed + (2 ((key << 32) | (w << 30))
// + 1) GAMMA (draw (i, j) adds 2 ((i << 15) + j) GAMMA, its v draw one more
// GAMMA), and the box state (0 = castable; other boxes get no records).
struct RayFrame {
  double hu, hv, du, dv, idu, idv;
  uint64_t s0;
  float eu, ev;
  int32_t state;
  uint32_t key;  // the box's jitter key
  int32_t pad[2];
};
static_assert(sizeof(RayFrame) == 80, "RayFrame layout");

// Cast frame of one (box, axis): face axes (ua, va), half extents, cell sizes.
struct CastFrame {
  int ua, va;
  float hu, hv, hw;
  double du, dv;
  double idu, idv;  // 1 / du, 1 / dv
  float eu, ev;  // bounding-box margins for binning
};

// The face rectangle of cast axis w (no cell sizes: enough for projects_into_face).
__device__ inline CastFrame cast_bounds(const BoxRegs& B, int w) {
  CastFrame f;
  f.ua = (w + 1) % 3;
  f.va = (w + 2) % 3;
  f.hu = pick3(B.h, f.ua);
  f.hv = pick3(B.h, f.va);
  f.hw = pick3(B.h, w);
  f.du = f.dv = f.idu = f.idv = 0.0;
  f.eu = 1e-6f * f.hu;
  f.ev = 1e-6f * f.hv;
  return f;
}

__device__ inline CastFrame cast_frame(const BoxRegs& B, int w, int R) {
  CastFrame f = cast_bounds(B, w);
  f.du = __ddiv_rn(__dmul_rn(2.0, (double)f.hu), (double)R);
  f.dv = __ddiv_rn(__dmul_rn(2.0, (double)f.hv), (double)R);
  f.idu = 1.0 / f.du;
  f.idv = 1.0 / f.dv;
  return f;
}

// cast_frame with the cell sizes of the cast's ray grid table (the same values)
__device__ inline CastFrame cast_frame_rf(const BoxRegs& B, int w, const RayFrame& rf) {
  CastFrame f = cast_bounds(B, w);
  f.du = rf.du;
  f.dv = rf.dv;
  f.idu = rf.idu;
  f.idv = rf.idv;
  return f;
}

// The ray grid of cast w of box b (see RayFrame).
__device__ inline RayFrame make_ray_frame(const BoxRegs& B, int w, uint32_t key, int R, uint64_t seed) {
  const int ua = (w + 1) % 3, va = (w + 2) % 3;
  const float huf = pick3(B.h, ua), hvf = pick3(B.h, va);
  RayFrame f;
  f.hu = huf;
  f.hv = hvf;
  f.du = __ddiv_rn(__dmul_rn(2.0, f.hu), (double)R);
  f.dv = __ddiv_rn(__dmul_rn(2.0, f.hv), (double)R);
  f.idu = 1.0 / f.du;
  f.idv = 1.0 / f.dv;
  f.eu = 1e-6f * huf;
  f.ev = 1e-6f * hvf;
  f.s0 = seed + (2ull * (((uint64_t)key << 32) | ((uint64_t)w << 30)) + 1ull) * kGamma;
  f.state = box_state(B);
  f.key = key;
  f.pad[0] = f.pad[1] = 0;
  return f;
}

// The triangle in the cast frame of axis w, optionally mirrored (z -> -z).
struct CastTri {
  float u[3], v[3], z[3];
  double A2;  // twice the signed projected area (float64 of the float coordinates)
};

__device__ inline CastTri cast_tri(const float P[3][3], int w, const CastFrame& f, bool mirror) {
  CastTri t;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    // coordinates picked by selects (the axes are not compile-time indices)
    t.u[k] = pick3(P[k], f.ua);
    t.v[k] = pick3(P[k], f.va);
    const float z = pick3(P[k], w);
    t.z[k] = mirror ? -z : z;
  }
  const double x1 = (double)t.u[1] - (double)t.u[0], y1 = (double)t.v[1] - (double)t.v[0];
  const double x2 = (double)t.u[2] - (double)t.u[0], y2 = (double)t.v[2] - (double)t.v[0];
  t.A2 = __dsub_rn(__dmul_rn(x1, y2), __dmul_rn(y1, x2));
  return t;
}

// Rectangle overlap of the projected bounding box (with margins) and a
// non-degenerate projection: the part of the test shared by both sides.
__device__ inline bool projects_into_face(const CastTri& t, const CastFrame& f) {
  const float umin = fminf(fminf(t.u[0], t.u[1]), t.u[2]);
  const float umax = fmaxf(fmaxf(t.u[0], t.u[1]), t.u[2]);
  const float vmin = fminf(fminf(t.v[0], t.v[1]), t.v[2]);
  const float vmax = fmaxf(fmaxf(t.v[0], t.v[1]), t.v[2]);
  return t.A2 != 0.0 && umax >= -f.hu - f.eu && umin <= f.hu + f.eu && vmax >= -f.hv - f.ev &&
         vmin <= f.hv + f.ev;
}

// Range of the cells whose rays can hit the triangle (conservative).
__device__ inline void cell_range(const CastTri& t, const CastFrame& f, int R, int& i0, int& i1, int& j0,
                                  int& j1) {
  const float umin = fminf(fminf(t.u[0], t.u[1]), t.u[2]);
  const float umax = fmaxf(fmaxf(t.u[0], t.u[1]), t.u[2]);
  const float vmin = fminf(fminf(t.v[0], t.v[1]), t.v[2]);
  const float vmax = fmaxf(fmaxf(t.v[0], t.v[1]), t.v[2]);
  const double hu = f.hu, hv = f.hv;
  // with reciprocals, as the ray-test kernel takes the range of a record (the
  // 1e-6 margins dwarf the difference from dividing)
  i0 = (int)floor(((double)umin - f.eu + hu) * f.idu);
  i1 = (int)floor(((double)umax + f.eu + hu) * f.idu);
  j0 = (int)floor(((double)vmin - f.ev + hv) * f.idv);
  j1 = (int)floor(((double)vmax + f.ev + hv) * f.idv);
  i0 = max(0, min(R - 1, i0));
  i1 = max(0, min(R - 1, i1));
  j0 = max(0, min(R - 1, j0));
  j1 = max(0, min(R - 1, j1));
}


// Load triangle t of mesh M in the box frame.  Returns false (and flags the
// status word) on an out-of-range index.
__device__ inline bool load_tri_local(const MeshDev& M, int t, const BoxRegs& B, float P[3][3],
                                      uint32_t* status) {
  const int32_t* f = M.F + 3 * (int64_t)t;
  const int a = f[0], b = f[1], c = f[2];
  if ((unsigned)a >= (unsigned)M.nv || (unsigned)b >= (unsigned)M.nv || (unsigned)c >= (unsigned)M.nv) {
    atomicOr(status, OBBV_STATUS_BAD_INDEX);
    return false;
  }
  const int idx[3] = {a, b, c};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* p = M.V + 3 * (int64_t)idx[k];
    to_local(B.Q, B.c, p[0], p[1], p[2], P[k]);
  }
  return true;
}
// The kept half prism of cast axis w: the one on the far side of the box from
// the mesh centre cm (the centre of the mesh's bounding box), which holds fewer
// of the mesh's triangles for a box near the surface.  mirror = the box centre
// lies on the -e_w side of cm (the cast then keeps crossings below the slab top).
// One fixed rounding sequence, so boxes sharing a centre and axes (and their
// frame) always choose the same side.
__device__ inline bool cast_mirror(const BoxRegs& B, int w, const float4& cm) {
  const float dx = __fsub_rn(B.c[0], cm.x), dy = __fsub_rn(B.c[1], cm.y), dz = __fsub_rn(B.c[2], cm.z);
  // row w of the axes (w is a run-time index: pick3 keeps it in registers)
  const float c0[3] = {B.Q[0], B.Q[3], B.Q[6]}, c1[3] = {B.Q[1], B.Q[4], B.Q[7]}, c2[3] = {B.Q[2], B.Q[5], B.Q[8]};
  const float q0 = pick3(c0, w), q1 = pick3(c1, w), q2 = pick3(c2, w);
  const float d = __fmaf_rn(q0, dx, __fmaf_rn(q1, dy, __fmul_rn(q2, dz)));
  return d < 0.f;
}

// Whether a world-space box [lo, hi] may hold a triangle that cast axis w of box
// B keeps (the triangle projects into the face rectangle, margins included, and
// reaches above -h_w on the kept side): separating-axis test on the three box
// axes with a margin of 1e-4 of the magnitudes involved -- far above the float32
// rounding of this test and of the kernels' local transforms (both a few units
// of 2^-24 of the same magnitudes) -- so a span the test rejects holds no
// triangle the cull would keep.  Non-finite bounds pass.
__device__ inline bool span_may_cast(const BoxRegs& B, int w, bool mirror, const float4& lo, const float4& hi) {
  if (lo.x > hi.x || lo.y > hi.y || lo.z > hi.z) return false;  // no valid triangle
  // bounds relative to the box centre first (rounding relative to |x - c|, as
  // in the kernels' transforms), then centre and half size
  const float l0 = lo.x - B.c[0], l1 = lo.y - B.c[1], l2 = lo.z - B.c[2];
  const float u0 = hi.x - B.c[0], u1 = hi.y - B.c[1], u2 = hi.z - B.c[2];
  const float m0 = 0.5f * (l0 + u0), m1 = 0.5f * (l1 + u1), m2 = 0.5f * (l2 + u2);
  const float r0 = 0.5f * (u0 - l0), r1 = 0.5f * (u1 - l1), r2 = 0.5f * (u2 - l2);
  const float a0 = fabsf(m0) + r0, a1 = fabsf(m1) + r1, a2 = fabsf(m2) + r2;
  float P[3], rad[3];
#pragma unroll
  for (int row = 0; row < 3; ++row) {
    const float q0 = B.Q[3 * row], q1 = B.Q[3 * row + 1], q2 = B.Q[3 * row + 2];
    P[row] = q0 * m0 + q1 * m1 + q2 * m2;
    rad[row] = fabsf(q0) * r0 + fabsf(q1) * r1 + fabsf(q2) * r2 +
               1e-4f * (fabsf(q0) * a0 + fabsf(q1) * a1 + fabsf(q2) * a2);
  }
  const int ua = (w + 1) % 3, va = (w + 2) % 3;
  const float pu = pick3(P, ua), pv = pick3(P, va), pw = pick3(P, w);
  const float ru = pick3(rad, ua), rv = pick3(rad, va), rw = pick3(rad, w);
  const float mu = pick3(B.h, ua) * 1.0001f, mv = pick3(B.h, va) * 1.0001f, hw = pick3(B.h, w);
  if (pu - ru > mu || pu + ru < -mu || pv - rv > mv || pv + rv < -mv) return false;
  const float zmax = (mirror ? -pw : pw) + rw;
  return !(zmax < -hw * 1.0001f);
}

// Bounds of every span of kSpanTris triangles and of every run of
// kSpansPerItem spans (a whole-mesh cast item): one block of 4 waves per run,
// each wave one span at a time.  Triangles with an out-of-range index are
// flagged and left out; a span with a non-finite vertex gets infinite bounds.
__global__ void __launch_bounds__(256)
k_span_bounds(MeshDev M, float4* __restrict__ spans, float4* __restrict__ runs, uint32_t* status) {
  __shared__ float red[4][6];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int run = blockIdx.x;
  const int64_t n_spans = ((int64_t)M.nt + kSpanTris - 1) / kSpanTris;
  float rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int sp = wave; sp < kSpansPerItem; sp += 4) {
    const int64_t span = (int64_t)run * kSpansPerItem + sp;
    if (span >= n_spans) break;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int k = lane; k < kSpanTris; k += 64) {
      const int64_t t = span * kSpanTris + k;
      if (t >= M.nt) break;
      const int32_t* f = M.F + 3 * t;
      const int idx[3] = {f[0], f[1], f[2]};
      if ((unsigned)idx[0] >= (unsigned)M.nv || (unsigned)idx[1] >= (unsigned)M.nv ||
          (unsigned)idx[2] >= (unsigned)M.nv) {
        atomicOr(status, OBBV_STATUS_BAD_INDEX);
        continue;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float x = M.V[3 * (int64_t)idx[j] + d];
          bad = bad || !isfinite(x);
          lo[d] = fminf(lo[d], x);
          hi[d] = fmaxf(hi[d], x);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = fminf(lo[d], __shfl_xor(lo[d], off));
        hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], off));
      }
    if (__any(bad))
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = -INFINITY;
        hi[d] = INFINITY;
      }
    if (lane == 0) {
      spans[2 * span] = make_float4(lo[0], lo[1], lo[2], 0.f);
      spans[2 * span + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      rlo[d] = fminf(rlo[d], lo[d]);
      rhi[d] = fmaxf(rhi[d], hi[d]);
    }
  }
  if (lane == 0)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[wave][d] = rlo[d];
      red[wave][3 + d] = rhi[d];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    float lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fminf(fminf(red[0][d], red[1][d]), fminf(red[2][d], red[3][d]));
      hi[d] = fmaxf(fmaxf(red[0][3 + d], red[1][3 + d]), fmaxf(red[2][3 + d], red[3][3 + d]));
    }
    runs[2 * run] = make_float4(lo[0], lo[1], lo[2], 0.f);
    runs[2 * run + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
  }
}

// Centre of each mesh's bounding box (xyz, w unused): one block per mesh.
__global__ void __launch_bounds__(256)
k_mesh_centre(const MeshDev* __restrict__ meshes, MeshDev mesh0, int n_meshes, float4* __restrict__ out) {
  __shared__ float red[6][4];
  const int m = blockIdx.x;
  if (m >= n_meshes) return;
  const MeshDev M = meshes ? meshes[m] : mesh0;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int v = threadIdx.x; v < M.nv; v += blockDim.x)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float x = M.V[3 * (int64_t)v + k];
      lo[k] = fminf(lo[k], x);
      hi[k] = fmaxf(hi[k], x);
    }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
    }
    if (lane == 0) {
      red[k][wave] = lo[k];
      red[3 + k][wave] = hi[k];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float c[3];
    for (int k = 0; k < 3; ++k) {
      float a = red[k][0], b = red[3 + k][0];
      for (int v = 1; v < 4; ++v) {
        a = fminf(a, red[k][v]);
        b = fmaxf(b, red[3 + k][v]);
      }
      c[k] = M.nv > 0 ? __fmul_rn(0.5f, __fadd_rn(a, b)) : 0.f;
    }
    out[m] = make_float4(c[0], c[1], c[2], 0.f);
  }
}

// A cast item: up to kCastTris consecutive entries of the triangle list of one
// (box, cast axis), as k_box_chunks tabulates it: bw3 = box * 3 + axis, the
// entry count, and the first entry: an index into the frame lists (first >= 0)
// or mesh triangle -1 - first (first < 0).
struct ItemInfo {
  int64_t first;
  int32_t bw3;
  int32_t count;
};

// Where a box's triangles come from.
struct ListArgs {
  const obbv_box* boxes;
  const int32_t* box_mesh;
  const MeshDev* meshes;  // device mesh table; NULL with a single mesh (then mesh0)
  MeshDev mesh0;
  const float4* list_P;   // nullable: frame lists, frame-local vertex coordinates (3 float4 per triangle)
  uint32_t* status;
};

__device__ inline MeshDev box_mesh_dev(const ListArgs& a, int b) {
  return a.meshes ? a.meshes[a.box_mesh ? a.box_mesh[b] : 0] : a.mesh0;
}

// Entry e of item ii in the box frame, packed as in the frame lists (3 float4:
// vertex 0, 1, 2 coordinates in order, 3 pads); ok = false on a bad index.
struct TriPk {
  float4 x, y, z;
};

__device__ inline TriPk item_tri_pk(const ListArgs& a, const MeshDev& M, const BoxRegs& B, const ItemInfo& ii, int e,
                                    bool& ok) {
  TriPk t;
  if (ii.first >= 0) {
    const float4* q = a.list_P + 3 * (ii.first + e);
    t.x = q[0];
    t.y = q[1];
    t.z = q[2];
    ok = true;
    return t;
  }
  float P[3][3];
  ok = load_tri_local(M, (int)(-1 - ii.first) + e, B, P, a.status);
  t.x = make_float4(P[0][0], P[0][1], P[0][2], P[1][0]);
  t.y = make_float4(P[1][1], P[1][2], P[2][0], P[2][1]);
  t.z = make_float4(P[2][2], 0.f, 0.f, 0.f);
  return t;
}

__device__ inline void unpack_tri(const TriPk& t, float P[3][3]) {
  P[0][0] = t.x.x;
  P[0][1] = t.x.y;
  P[0][2] = t.x.z;
  P[1][0] = t.x.w;
  P[1][1] = t.y.x;
  P[1][2] = t.y.y;
  P[2][0] = t.y.z;
  P[2][1] = t.y.w;
  P[2][2] = t.z.x;
}

// Entry e of item ii in the box frame: from the frame's list (the bits to_local
// gives: same centre, same axes), else transformed from the mesh.  False on an
// out-of-range index.
__device__ inline bool item_tri(const ListArgs& a, const MeshDev& M, const BoxRegs& B, const ItemInfo& ii, int e,
                                float P[3][3]) {
  if (ii.first < 0) return load_tri_local(M, (int)(-1 - ii.first) + e, B, P, a.status);
  const float4* q = a.list_P + 3 * (ii.first + e);
  const float4 x = q[0], y = q[1], z = q[2];
  P[0][0] = x.x;
  P[0][1] = x.y;
  P[0][2] = x.z;
  P[1][0] = x.w;
  P[1][1] = y.x;
  P[1][2] = y.y;
  P[2][0] = y.z;
  P[2][1] = y.w;
  P[2][2] = z.x;
  return true;
}


// A box may use its frame's triangle list only if it has the frame's centre and
// axes (same bits) and lies inside the frame box; otherwise it walks the whole
// mesh (slower, same result).
__device__ inline bool inside_frame(const obbv_box& bx, const obbv_box& fr) {
  const uint32_t* p = reinterpret_cast<const uint32_t*>(&bx);
  const uint32_t* q = reinterpret_cast<const uint32_t*>(&fr);
  bool same = true;
#pragma unroll
  for (int k = 0; k < 12; ++k) same = same && p[k] == q[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) same = same && bx.half[k] <= fr.half[k];  // false on NaN
  return same;
}

// Exclusive scan of one value per thread over a block of kScanBlockThreads;
// returns the exclusive prefix and the block total (all threads).
constexpr int kScanBlockThreads = 1024;
__device__ inline long long block_excl_scan(long long v, long long* wsum, long long& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const long long u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  long long before = 0;
  total = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    if (k < wave) before += wsum[k];
    total += wsum[k];
  }
  __syncthreads();
  return before + inc - v;
}


// Per-wave ballot counts of a 256-thread block, summed in LDS: every block
// writes its own counts (no global atomics on shared counters, which serialise).
constexpr int kCullWaves = kCullThreads / 64;

// Is the triangle kept on the chosen side?  (Mirrored frames flip z, so the
// kept half prism is always "above the slab bottom" in the cast frame.)
__device__ inline bool kept(const CastTri& tr, const CastFrame& f) {
  if (!projects_into_face(tr, f)) return false;
  const float zmax = fmaxf(fmaxf(tr.z[0], tr.z[1]), tr.z[2]);
  return zmax > -f.hw;
}

// Shared frames: boxes with the same centre and axes see every triangle at the
// same local coordinates and keep the same side of every cast (cast_mirror), so
// a triangle can matter to one of them along axis w only if it projects into
// face w of their union (the frame box, with the largest half extents) and lies
// in the frame's kept half prism.  Items are (frame, axis, 256-triangle chunk),
// grouped per (frame, axis).  With item_off NULL the pass writes each item's
// count of such triangles; otherwise it writes their frame-local coordinates at
// list_off[frame * 3 + axis] + item_off[item] + rank (in triangle order).
// The triangles of (frame fr, 256-triangle chunk ch) kept along each axis:
// mk[w] is the wave's ballot, wc[w][wave] its count; P the thread's triangle in
// frame-local coordinates.
__device__ inline void frame_keep(const obbv_box* __restrict__ frames, int fr, int ch, const MeshDev& M,
                                  const float4& cm, uint32_t axis_mask, const float4* __restrict__ spans,
                                  uint32_t* status, float P[3][3], uint64_t mk[3], int32_t (*wc)[kCullWaves]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = ch * kCullThreads + threadIdx.x;
  const BoxRegs B = load_box(frames, fr);
  // the axes whose kept half prism the chunk (one span) may reach
  uint32_t reach = axis_mask;
  if (spans) {
    const float4 lo = spans[2 * ch], hi = spans[2 * ch + 1];
    for (int w = 0; w < 3; ++w)
      if (((reach >> w) & 1u) && !span_may_cast(B, w, cast_mirror(B, w, cm), lo, hi)) reach &= ~(1u << w);
  }
  const bool ok = reach != 0u && box_state(B) == 0 && t < M.nt && load_tri_local(M, t, B, P, status);
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    bool keep = false;
    if (ok && ((reach >> w) & 1u)) {
      const CastFrame f = cast_bounds(B, w);
      keep = kept(cast_tri(P, w, f, cast_mirror(B, w, cm)), f);
    }
    mk[w] = __ballot(keep);
    if (lane == 0) wc[w][wave] = (int)__popcll(mk[w]);
  }
}

__device__ inline void store_tri(float4* q, const float P[3][3]) {
  q[0] = make_float4(P[0][0], P[0][1], P[0][2], P[1][0]);
  q[1] = make_float4(P[1][1], P[1][2], P[2][0], P[2][1]);
  q[2] = make_float4(P[2][2], 0.f, 0.f, 0.f);
}

// Two passes (lists sized exactly): with item_off NULL the pass writes each
// item's count of kept triangles; otherwise it writes their frame-local
// coordinates at list_off[frame * 3 + axis] + item_off[item] + rank (in
// triangle order).
__global__ void __launch_bounds__(kCullThreads)
k_frame_cull(const obbv_box* __restrict__ frames, int n_frames, MeshDev M, const float4* __restrict__ centre,
             uint32_t axis_mask, int nch, int32_t* __restrict__ item_cnt, const int32_t* __restrict__ item_off,
             const int64_t* __restrict__ list_off, float4* __restrict__ list_P, uint32_t* status,
             const float4* __restrict__ spans) {
  __shared__ int32_t wc[3][kCullWaves];
  const int64_t total = (int64_t)n_frames * nch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float4 cm = centre[0];
  for (int64_t fc = blockIdx.x; fc < total; fc += gridDim.x) {
    const int fr = (int)(fc / nch);
    const int ch = (int)(fc - (int64_t)fr * nch);
    float P[3][3];
    uint64_t mk[3];
    frame_keep(frames, fr, ch, M, cm, axis_mask, spans, status, P, mk, wc);
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const int64_t item = ((int64_t)fr * 3 + w) * nch + ch;
      if (!item_off) {
        if (threadIdx.x == 0) {
          int c = 0;
          for (int v = 0; v < kCullWaves; ++v) c += wc[w][v];
          item_cnt[item] = c;
        }
      } else if ((mk[w] >> lane) & 1ull) {
        int pos = item_off[item] + (int)__popcll(mk[w] & ((1ull << lane) - 1ull));
        for (int v = 0; v < wave; ++v) pos += wc[w][v];
        if (pos < item_off[item] + item_cnt[item])
          store_tri(list_P + 3 * (list_off[fr * 3 + w] + pos), P);
        else  // count and write passes disagree: never expected
          atomicOr(status, OBBV_STATUS_BAD_INDEX);
      }
    }
    __syncthreads();
  }
}

// One pass: the kept triangles of every axis are appended to list (frame,
// axis), a segment of seg entries from (frame * 3 + axis) * seg, at positions
// taken from the list's counter list_cnt (zero before the pass).  Entries of a
// list follow the blocks' arrival order; the cast's sums are exact integers, so
// no result depends on it.
__global__ void __launch_bounds__(kCullThreads)
k_frame_list(const obbv_box* __restrict__ frames, int n_frames, MeshDev M, const float4* __restrict__ centre,
             uint32_t axis_mask, int nch, int64_t seg, int32_t* __restrict__ list_cnt, float4* __restrict__ list_P,
             uint32_t* status, const float4* __restrict__ spans) {
  __shared__ int32_t wc[3][kCullWaves];
  __shared__ int32_t base[3];
  const int64_t total = (int64_t)n_frames * nch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float4 cm = centre[0];
  for (int64_t fc = blockIdx.x; fc < total; fc += gridDim.x) {
    const int fr = (int)(fc / nch);
    const int ch = (int)(fc - (int64_t)fr * nch);
    float P[3][3];
    uint64_t mk[3];
    frame_keep(frames, fr, ch, M, cm, axis_mask, spans, status, P, mk, wc);
    __syncthreads();
    if (threadIdx.x < 3) {
      int c = 0;
      for (int v = 0; v < kCullWaves; ++v) c += wc[threadIdx.x][v];
      base[threadIdx.x] = c ? atomicAdd(&list_cnt[fr * 3 + threadIdx.x], c) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      if ((mk[w] >> lane) & 1ull) {
        int pos = base[w] + (int)__popcll(mk[w] & ((1ull << lane) - 1ull));
        for (int v = 0; v < wave; ++v) pos += wc[w][v];
        if (pos < seg)
          store_tri(list_P + 3 * (((int64_t)fr * 3 + w) * seg + pos), P);
        else  // a list holds each triangle once at most: never expected
          atomicOr(status, OBBV_STATUS_BAD_INDEX);
      }
    }
    __syncthreads();
  }
}

// One wave per group of consecutive items [first(g), first(g + 1)): exclusive
// scan of the groups' item counts (column `col` of `ncol`) into item_off, and
// the group total.  Groups are frames (first(g) = g * per) or boxes (first =
// chunk_off).
__device__ inline int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(v, off);
    if (lane >= off) v += u;
  }
  return v;
}

__global__ void k_frame_scan(const int32_t* __restrict__ item_cnt, int n_frames, int per,
                             int32_t* __restrict__ item_off, int32_t* __restrict__ frame_cnt,
                             int64_t* __restrict__ frame_off) {
  const int lane = threadIdx.x & 63;
  const int waves = (int)(gridDim.x * (blockDim.x >> 6));
  for (int g = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6); g < n_frames; g += waves) {
    const int64_t i0 = (int64_t)g * per, i1 = i0 + per;
    int base = 0;
    for (int64_t i = i0; i < i1; i += 64) {
      const int v = i + lane < i1 ? item_cnt[i + lane] : 0;
      const int inc = wave_incl_scan(v, lane);
      if (i + lane < i1) item_off[i + lane] = base + inc - v;
      base += __shfl(inc, 63);
    }
    if (lane == 0) frame_cnt[g] = base;
  }
  if (!frame_off) return;
  // single-block launch: the frames' list offsets as well
  __shared__ long long wsum[kScanBlockThreads / 64];
  __syncthreads();
  long long fb = 0;
  for (int g0 = 0; g0 < n_frames; g0 += (int)blockDim.x) {
    const int g = g0 + (int)threadIdx.x;
    long long total = 0;
    const long long ex = block_excl_scan(g < n_frames ? (long long)frame_cnt[g] : 0ll, wsum, total);
    if (g < n_frames) frame_off[g] = fb + ex;
    fb += total;
  }
  if (threadIdx.x == 0) frame_off[n_frames] = fb;
}





// One block: the cast items of every (box, cast axis) -- its frame's list of
// that axis when the box may use its frame, else the whole mesh; boxes that
// cannot be cast get none --, their offsets chunk_off[0..3 n_boxes], the ray
// grid of every cast, and the per-call counters that must start at zero
// (per-(box, axis) sums, unit queue, finished blocks; the one-pass frame list
// counters once read).
__global__ void __launch_bounds__(kScanBlockThreads)
k_box_chunks(const int32_t* __restrict__ box_mesh, const MeshDev* __restrict__ meshes, MeshDev mesh0, int n_meshes,
             int n_boxes, uint32_t axis_mask, const obbv_box* __restrict__ boxes,
             const obbv_box* __restrict__ frames, const int32_t* __restrict__ box_frame, int n_frames,
             const int64_t* __restrict__ list_off, int32_t* __restrict__ list_cnt, int64_t list_seg,
             int64_t* __restrict__ chunk_off, uint32_t* status,
             const uint32_t* __restrict__ box_key, int R, uint64_t seed, RayFrame* __restrict__ rframe,
             ItemInfo* __restrict__ items, int64_t item_cap, unsigned long long* __restrict__ acc,
             unsigned long long* __restrict__ ctl, const float4* __restrict__ runs,
             const float4* __restrict__ centre, int item_small, int split_below, int nblk) {
  __shared__ long long wsum[kScanBlockThreads / 64];
  __shared__ unsigned long long s_rm[kScanBlockThreads];  // runs kept (the first 64) of a whole-mesh cast
  __shared__ uint8_t s_cul[kScanBlockThreads];            // the pair is a whole-mesh cast with span runs
  if (threadIdx.x < 4) ctl[threadIdx.x] = 0ull;
  for (int e = threadIdx.x; e < 3 * n_boxes; e += blockDim.x) {
    const int b = e / 3;
    rframe[e] = make_ray_frame(load_box(boxes, b), e - 3 * b, box_key ? box_key[b] : (uint32_t)b, R, seed);
    acc[e] = 0ull;
  }
  long long base = 0;
  const int npairs = 3 * n_boxes;
  for (int p0 = 0; p0 < npairs; p0 += kScanBlockThreads) {
    const int pr = p0 + (int)threadIdx.x;
    long long nch = 0, nch_s = 0;  // items of the default size and of item_small entries
    int64_t first = 0, ntri = 0;
    bool list = false, culled = false, mirror = false;
    uint64_t rmask = 0;  // runs kept (the first 64)
    BoxRegs Bx;
    if (pr < npairs) {
      const int b = pr / 3, w = pr - 3 * b;
      const int m = box_mesh ? box_mesh[b] : 0;
      if (m < 0 || m >= n_meshes) {  // out-of-range mesh index: the box sees no triangles
        if (w == 0) atomicOr(status, OBBV_STATUS_BAD_INDEX);
      } else if (((axis_mask >> w) & 1u) && box_state(load_box(boxes, b)) == 0) {
        int64_t n = meshes ? meshes[m].nt : mesh0.nt;
        if (frames) {
          const int f = box_frame[b];
          if (f >= 0 && f < n_frames && inside_frame(boxes[b], frames[f])) {
            if (list_cnt) {
              first = ((int64_t)f * 3 + w) * list_seg;
              n = list_cnt[f * 3 + w];
            } else {
              first = list_off[f * 3 + w];
              n = list_off[f * 3 + w + 1] - first;
            }
            list = true;
          }
        }
        ntri = n;
        nch = (n + kCastTris - 1) / kCastTris;
        nch_s = item_small < kCastTris ? (n + item_small - 1) / item_small : nch;
        if (!list && runs && !meshes) {  // whole mesh: only the runs the kept half prism may reach
          Bx = load_box(boxes, b);
          mirror = cast_mirror(Bx, w, centre[0]);
          culled = true;
        }
      }
    }
    if (runs && !meshes) {
      // the first 64 runs of every whole-mesh cast of these pairs, one (pair,
      // run) test per thread, into bit r of s_rm[pair - p0]
      const long long nr = (mesh0.nt + kCastTris - 1) / kCastTris;
      const int nr64 = (int)min(nr, 64ll);
      const int npc = min(kScanBlockThreads, npairs - p0);
      s_rm[threadIdx.x] = 0ull;
      s_cul[threadIdx.x] = culled ? 1 : 0;
      __syncthreads();
      for (int k = threadIdx.x; k < npc * nr64; k += blockDim.x) {
        const int q = k / nr64, r = k - q * nr64;
        if (!s_cul[q]) continue;
        const int p = p0 + q, b = p / 3, w = p - 3 * b;
        const BoxRegs Bk = load_box(boxes, b);
        if (span_may_cast(Bk, w, cast_mirror(Bk, w, centre[0]), runs[2 * r], runs[2 * r + 1]))
          atomicOr(&s_rm[q], 1ull << r);
      }
      __syncthreads();
      if (culled) {  // items: the kept runs (each cut into pieces of item_small entries)
        const int w = pr - 3 * (pr / 3);
        rmask = s_rm[threadIdx.x];
        long long c = __popcll(rmask);
        for (long long r = 64; r < nr; ++r) c += span_may_cast(Bx, w, mirror, runs[2 * r], runs[2 * r + 1]) ? 1 : 0;
        nch = c;
        nch_s = c;
        if (item_small < kCastTris) {
          long long cs = 0;
          for (long long r = 0; r < nr; ++r)
            if (r < 64 ? ((rmask >> r) & 1ull) != 0 : span_may_cast(Bx, w, mirror, runs[2 * r], runs[2 * r + 1]))
              cs += ((int)min((int64_t)kCastTris, ntri - r * kCastTris) + item_small - 1) / item_small;
          nch_s = cs;
        }
      }
    }
    long long total = 0;
    long long ex = block_excl_scan(nch, wsum, total);
    // a call whose default items give fewer than split_below units takes items
    // of item_small entries instead (more units for the compute units it would
    // leave idle); decided on the whole call, so only with one block of pairs
    int item_tris = kCastTris;
    if (item_small < kCastTris && npairs <= kScanBlockThreads && total * nblk < split_below) {
      item_tris = item_small;
      nch = nch_s;
      ex = block_excl_scan(nch, wsum, total);
    }
    if (pr < npairs) {
      chunk_off[pr] = base + ex;
      if (culled) {
        const int w = pr - 3 * (pr / 3);
        long long c = 0;
        for (long long r = 0; c < nch; ++r) {
          if (r < 64 ? !((rmask >> r) & 1ull) : !span_may_cast(Bx, w, mirror, runs[2 * r], runs[2 * r + 1]))
            continue;
          const int64_t run_n = min((int64_t)kCastTris, ntri - r * kCastTris);
          for (int64_t q = 0; q < run_n && c < nch; q += item_tris) {
            const long long it = base + ex + c++;
            if (it >= item_cap) break;
            ItemInfo ii;
            ii.bw3 = pr;
            ii.count = (int32_t)min((int64_t)item_tris, run_n - q);
            ii.first = -1 - (r * kCastTris + q);
            items[it] = ii;
          }
        }
      } else {
        for (long long c = 0; c < nch; ++c) {
          const long long it = base + ex + c;
          if (it >= item_cap) break;
          ItemInfo ii;
          ii.bw3 = pr;
          ii.count = (int32_t)min((int64_t)item_tris, ntri - c * item_tris);
          ii.first = list ? first + c * item_tris : -1 - c * item_tris;
          items[it] = ii;
        }
      }
    }
    base += total;
  }
  if (threadIdx.x == 0) {
    chunk_off[npairs] = base < item_cap ? base : item_cap;
    if (base > item_cap) atomicOr(status, OBBV_STATUS_OVERFLOW);
  }
  if (list_cnt) {  // one-pass list counters start the next call at zero
    __syncthreads();
    for (int g = threadIdx.x; g < 3 * n_frames; g += blockDim.x) list_cnt[g] = 0;
  }
}

// The test planes of a kept triangle in its cast frame, held in registers.
//   E_k(u, v) = A_k u + B_k v + C_k, k = edge (k -> k+1), oriented so that the
//   inside of the projected triangle is E > 0.  The edge functions of an edge
//   shared by two triangles facing the same way are exact negatives of each
//   other, so a ray with E == 0 exactly is taken by exactly one of them: by the
//   one for which the edge is a top-left edge (A > 0, or A == 0 and B > 0) --
//   the test is watertight.  In bits: E_k passes iff (int)bits(E_k) >= t_k,
//   t_k = 0 for a top-left edge (E >= +0), 1 otherwise (E > 0).
//   y(u, v) = D u + E v + F is the fixed-point depth kMagic + s (w(u, v) + h)
//   2^21 / h (s = crossing sign), clamped to [lo, hi], the triangle's part of the
//   slab; bits(clamped y) - kMagicBits is the crossing's signed inside length.
struct Rec {
  float A0, B0, C0, A1, B1, C1, A2, B2, C2;
  float D, E, F, lo, hi, s;
  int32_t t0, t1, t2;
};

__device__ inline Rec make_rec(const CastTri& t, bool mirror, float hw) {
  const int sa = t.A2 > 0.0 ? 1 : -1;
  const int s = mirror ? -sa : sa;
  float A[3], Bc[3], C[3];
  double Ad[3], Bd[3], Cd[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = k, j = (k + 1) % 3;
    A[k] = __fsub_rn(t.v[i], t.v[j]);
    Bc[k] = __fsub_rn(t.u[j], t.u[i]);
    Ad[k] = __dsub_rn((double)t.v[i], (double)t.v[j]);
    Bd[k] = __dsub_rn((double)t.u[j], (double)t.u[i]);
    Cd[k] = __dsub_rn(__dmul_rn((double)t.u[i], (double)t.v[j]), __dmul_rn((double)t.v[i], (double)t.u[j]));
    C[k] = (float)Cd[k];
    if (sa < 0) {
      A[k] = __fsub_rn(0.0f, A[k]);
      Bc[k] = __fsub_rn(0.0f, Bc[k]);
      C[k] = __fsub_rn(0.0f, C[k]);
    }
  }
  // barycentric weight of vertex 0 is E_1 / A2, of vertex 1 is E_2 / A2, of vertex 2 is E_0 / A2;
  // the fixed-point scale K = s 2^21 / h is folded into the one division
  const double h = hw;
  const double K = (double)s * kHalfQ / h;
  const double KA = K / t.A2;
  const double D = (Ad[1] * t.z[0] + Ad[2] * t.z[1] + Ad[0] * t.z[2]) * KA;
  const double E = (Bd[1] * t.z[0] + Bd[2] * t.z[1] + Bd[0] * t.z[2]) * KA;
  const double F = (Cd[1] * t.z[0] + Cd[2] * t.z[1] + Cd[0] * t.z[2]) * KA;
  const double zmin = fmin(fmin((double)t.z[0], (double)t.z[1]), (double)t.z[2]);
  const double zmax = fmax(fmax((double)t.z[0], (double)t.z[1]), (double)t.z[2]);
  const double zlo = fmin(fmax(-h, zmin), h);
  const double zhi = fmax(fmin(h, zmax), -h);
  double lo = K * (zlo + h) + (double)kMagic;
  double hi = K * (zhi + h) + (double)kMagic;
  if (s < 0) {
    const double tmp = lo;
    lo = hi;
    hi = tmp;
  }
  Rec r;
  r.A0 = A[0];
  r.B0 = Bc[0];
  r.C0 = C[0];
  r.A1 = A[1];
  r.B1 = Bc[1];
  r.C1 = C[1];
  r.A2 = A[2];
  r.B2 = Bc[2];
  r.C2 = C[2];
  r.D = (float)D;
  r.E = (float)E;
  r.F = (float)(F + K * h + (double)kMagic);
  r.lo = (float)lo;
  r.hi = (float)hi;
  r.s = (float)s;
  r.t0 = (A[0] > 0.f || (A[0] == 0.f && Bc[0] > 0.f)) ? 0 : 1;
  r.t1 = (A[1] > 0.f || (A[1] == 0.f && Bc[1] > 0.f)) ? 0 : 1;
  r.t2 = (A[2] > 0.f || (A[2] == 0.f && Bc[2] > 0.f)) ? 0 : 1;
  return r;
}

// One ray-triangle test: 3 edge functions (2 FMA each), the tie rule on their
// bits, the depth plane (2 FMA).  y receives the unclamped fixed-point depth.
__device__ inline bool rec_hit(const Rec& r, float u, float v, float& y) {
  const float e0 = __fmaf_rn(r.A0, u, __fmaf_rn(r.B0, v, r.C0));
  const float e1 = __fmaf_rn(r.A1, u, __fmaf_rn(r.B1, v, r.C1));
  const float e2 = __fmaf_rn(r.A2, u, __fmaf_rn(r.B2, v, r.C2));
  y = __fmaf_rn(r.D, u, __fmaf_rn(r.E, v, r.F));
  return ((int)(__float_as_int(e0) >= r.t0) & (int)(__float_as_int(e1) >= r.t1) &
          (int)(__float_as_int(e2) >= r.t2)) != 0;
}

// Lane src's record and cell range, in every lane of the wave (for the
// wave-wide test).
__device__ inline Rec shfl_rec(const Rec& r, int i0, int i1, int j0, int j1, int src, int& o0, int& o1, int& p0,
                               int& p1) {
  Rec o;
  o.A0 = __shfl(r.A0, src);
  o.B0 = __shfl(r.B0, src);
  o.C0 = __shfl(r.C0, src);
  o.A1 = __shfl(r.A1, src);
  o.B1 = __shfl(r.B1, src);
  o.C1 = __shfl(r.C1, src);
  o.A2 = __shfl(r.A2, src);
  o.B2 = __shfl(r.B2, src);
  o.C2 = __shfl(r.C2, src);
  o.D = __shfl(r.D, src);
  o.E = __shfl(r.E, src);
  o.F = __shfl(r.F, src);
  o.lo = __shfl(r.lo, src);
  o.hi = __shfl(r.hi, src);
  o.s = __shfl(r.s, src);
  o.t0 = __shfl(r.t0, src);
  o.t1 = __shfl(r.t1, src);
  o.t2 = __shfl(r.t2, src);
  o0 = __shfl(i0, src);
  o1 = __shfl(i1, src);
  p0 = __shfl(j0, src);
  p1 = __shfl(j1, src);
  return o;
}

struct CastArgs {
  ListArgs la;
  const ItemInfo* items;
  const int64_t* chunk_off;  // [3 n_boxes + 1] first item of every (box, axis)
  int n_boxes;
  const RayFrame* rframe;    // [n_boxes * 3]
  const float4* centre;      // [n_meshes] mesh centres (cast_mirror)
  unsigned long long* acc;   // [n_boxes * 3] per-(box, axis) sum of q
  unsigned long long* queue; // unit counter, zero at the start of the call
  int R;
  int BC, BR, nbc, nblk;     // ray blocks of BC cells along u by BR cells along v
  int raster_cells;          // records covering more cells of the block are tested wave-wide
  const uint2* jitter;       // nullable: jitter table [keys][3][R][R], every key < its rows
  int32_t* ray_q;            // nullable [n_boxes][3][R][R]
  int32_t* ray_hits;         // nullable [n_boxes][3][R][R]: crossings in the slab + 65536 x beyond it
  int32_t* occ;              // nullable [n_boxes][8][8][8]: sub-slab inside lengths in 2^-19 of a sub-slab
  unsigned long long* test_counter;  // nullable [2 kProfSlots]: tests, bytes
  const float4* spans;       // nullable: span bounds of mesh 0 (single-mesh calls)
};

// Per-ray outputs of one crossing (tests and ray features only).
template <bool STATS, bool OCC>
__device__ inline void note_hit(const CastArgs& a, const Rec& r, float y, int32_t q, int idx, int ci0, int cj0,
                                int bw, int bw3, int32_t* socc) {
  if (STATS) {
    const int dj = idx / bw, di = idx - dj * bw;
    const int i = ci0 + di, j = cj0 + dj;
    const int64_t o = ((int64_t)bw3 * a.R + i) * a.R + j;
    if (a.ray_q) atomicAdd(&a.ray_q[o], q);
    if (a.ray_hits) {
      const float t = (y - kMagic) * r.s;  // position from the slab bottom in 2^-22 of the slab
      const int code = t > 4194304.0f ? 65536 : (t >= 0.0f ? 1 : 0);
      if (code) atomicAdd(&a.ray_hits[o], code);
    }
  }
  if (OCC) {
    // the crossing split over 8 equal sub-slabs (exact integers): the position
    // from the slab bottom in units of 2^-22 of the slab, sub-slab k spans
    // [k 2^19, (k + 1) 2^19]
    const float yq = (float)q * r.s;
    const int dj = idx / bw, i = ci0 + idx - dj * bw, j = cj0 + dj;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int v = (int)(fminf(fmaxf(yq, (float)(k << 19)), (float)((k + 1) << 19)) - (float)(k << 19));
      if (v) atomicAdd(&socc[(i * 8 + j) * 8 + k], r.s > 0.f ? v : -v);
    }
  }
}

// A lane tests its record against the rays of the cells [i0, i1] x [j0, j1]
// (inside the ray block whose first cell is (ci0, cj0), bw cells wide), one flat
// loop over the covered cells.  Returns the sum of the crossings' q.
template <bool STATS, bool OCC, typename Acc>
__device__ inline Acc raster_lane(const CastArgs& a, const Rec& r, int i0, int i1, int j0, int j1, int ci0, int cj0,
                                  int bw, int bw3, const float2* __restrict__ sray, int32_t* socc) {
  const int wdt = i1 - i0 + 1, cells = wdt * (j1 - j0 + 1);
  int idx = (i0 - ci0) + (j0 - cj0) * bw, di = 0;
  Acc sum = 0;
  // two cells per step: both rays are read from LDS before either is tested
  auto test = [&](const float2 p, int at) {
    float y;
    if (rec_hit(r, p.x, p.y, y)) {
      const int32_t q = (int32_t)(__float_as_uint(__builtin_amdgcn_fmed3f(y, r.lo, r.hi)) - kMagicBits);
      sum += q;
      if (STATS || OCC) note_hit<STATS, OCC>(a, r, y, q, at, ci0, cj0, bw, bw3, socc);
    }
  };
  auto step = [&](int& at) {
    ++di;
    const bool wrap = di == wdt;
    at += wrap ? bw - wdt + 1 : 1;
    di = wrap ? 0 : di;
  };
  int t = 0;
  for (; t + 1 < cells; t += 2) {
    int idx1 = idx;
    step(idx1);
    const float2 p0 = sray[idx], p1 = sray[idx1];
    int idx2 = idx1;
    step(idx2);
    test(p0, idx);
    test(p1, idx1);
    idx = idx2;
  }
  if (t < cells) test(sray[idx], idx);
  return sum;
}

// The whole wave tests one record, one covered cell per lane.
template <bool STATS, bool OCC>
__device__ inline int32_t raster_wave(const CastArgs& a, const Rec& r, int i0, int i1, int j0, int j1, int ci0,
                                      int cj0, int bw, int bw3, const float2* __restrict__ sray, int32_t* socc,
                                      int lane) {
  const int wdt = i1 - i0 + 1, cells = wdt * (j1 - j0 + 1);
  int dj = lane / wdt, di = lane - dj * wdt;
  const int q64 = 64 / wdt, r64 = 64 - q64 * wdt;
  int32_t sum = 0;
  for (int t = lane; t < cells; t += 64) {
    const int idx = (i0 - ci0 + di) + (j0 - cj0 + dj) * bw;
    const float2 p = sray[idx];
    float y;
    if (rec_hit(r, p.x, p.y, y)) {
      const int32_t q = (int32_t)(__float_as_uint(__builtin_amdgcn_fmed3f(y, r.lo, r.hi)) - kMagicBits);
      sum += q;
      if (STATS || OCC) note_hit<STATS, OCC>(a, r, y, q, idx, ci0, cj0, bw, bw3, socc);
    }
    di += r64;
    dj += q64;
    if (di >= wdt) {
      di -= wdt;
      ++dj;
    }
  }
  return sum;
}

// Persistent workgroups; each unit = (cast item, cast axis, ray block):
//   A. the item's entries are culled against the kept half prism and the block
//      (each thread's next entry is requested before its current one is culled);
//      survivors are compacted into an LDS list (wave ballots + a workgroup
//      prefix) and their cell ranges merged into one bounding cell range;
//   B. the rays of that range only are generated into LDS;
//   C. each wave draws chunks of 64 survivors from a shared cursor: one
//      survivor per lane, its planes in registers, its covered cells per lane
//      (or, for records covering many cells, by the whole wave, one cell per
//      lane), with no barrier until the unit's sums.
template <bool STATS, bool OCC, bool TAB>
__global__ void __launch_bounds__(kCastThreads) k_cast(CastArgs a) {
  extern __shared__ float2 sray[];  // rays of the survivors' cell range inside the unit's block (u, v)
  __shared__ int32_t sidx[kCastTris];
  __shared__ int32_t s_cursor;  // next survivor of the test phase
  __shared__ int32_t s_wcnt[kCastWaves];
  __shared__ int32_t s_rng[4];
  __shared__ long long s_red[kCastWaves];
  __shared__ long long s_tests[kCastWaves];
  __shared__ int32_t s_read[kCastWaves];  // list entries read per wave (profiling)
  __shared__ unsigned long long s_unit;
  __shared__ int32_t socc[OCC ? 512 : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n_items = a.chunk_off[3 * a.n_boxes];
  const int per_item = a.nblk;
  const unsigned long long n_units = (unsigned long long)n_items * (unsigned long long)per_item;
  for (;;) {
    if (tid == 0) {
      s_unit = atomicAdd(a.queue, 1ull);
      s_cursor = 0;
      s_rng[0] = 0x7fffffff;
      s_rng[1] = -1;
      s_rng[2] = 0x7fffffff;
      s_rng[3] = -1;
    }
    __syncthreads();
    const unsigned long long u = s_unit;
    if (u >= n_units) break;
    const int64_t item = (int64_t)(u / (unsigned long long)per_item);
    const int blk = (int)(u - (unsigned long long)item * per_item);
    const ItemInfo ii = a.items[item];
    const int bw3 = ii.bw3;
    const int b = bw3 / 3, w = bw3 - 3 * b;
    const BoxRegs B = load_box(a.la.boxes, b);
    const MeshDev M = box_mesh_dev(a.la, b);
    const RayFrame rf = a.rframe[bw3];
    const CastFrame f = cast_frame_rf(B, w, rf);
    const bool mirror = cast_mirror(B, w, a.centre[a.la.box_mesh ? a.la.box_mesh[b] : 0]);
    const int bj = blk / a.nbc, bi = blk - bj * a.nbc;
    const int ci0 = bi * a.BC, ci1 = min(a.R, ci0 + a.BC) - 1;
    const int cj0 = bj * a.BR, cj1 = min(a.R, cj0 + a.BR) - 1;
    // A. cull: wave v takes entries v 64 + lane + k kCastThreads and compacts
    // its survivors into its own slice of sidx (no workgroup barrier per step);
    // each lane requests its next two entries ahead of the cull
    constexpr int kSlice = kCastTris / kCastWaves;  // entries a wave culls at most
    int n_mine = 0;                                  // survivors of this wave (uniform in the wave)
    int ri0 = 0x7fffffff, ri1 = -1, rj0 = 0x7fffffff, rj1 = -1;
    // spans of a whole-mesh item that the cast's kept half prism may reach (a
    // wave's 64 entries lie in one span: the test is uniform in the wave)
    uint64_t smask = ~0ull;
    if (a.spans && ii.first < 0) {
      const int64_t sp0 = (-1 - ii.first) / kSpanTris;
      const int nsp = (ii.count + kSpanTris - 1) / kSpanTris;
      const bool reach =
          lane < nsp && span_may_cast(B, w, mirror, a.spans[2 * (sp0 + lane)], a.spans[2 * (sp0 + lane) + 1]);
      smask = __ballot(reach);
    }
    int n_read = 0;
    {
      const int e0 = wave * 64 + lane;
      bool oka = false, okb = false;
      TriPk Ta{}, Tb{};
      if (e0 < ii.count && ((smask >> (e0 / kSpanTris)) & 1ull)) Ta = item_tri_pk(a.la, M, B, ii, e0, oka);
      if (e0 + kCastThreads < ii.count && ((smask >> ((e0 + kCastThreads) / kSpanTris)) & 1ull))
        Tb = item_tri_pk(a.la, M, B, ii, e0 + kCastThreads, okb);
      for (int e = e0; e - lane < ii.count; e += kCastThreads) {
        float P[3][3];
        unpack_tri(Ta, P);
        const bool ok = oka;
        n_read += (e < ii.count && ((smask >> (e / kSpanTris)) & 1ull)) ? 1 : 0;
        Ta = Tb;
        oka = okb;
        okb = false;
        const int en = e + 2 * kCastThreads;
        if (en < ii.count && ((smask >> (en / kSpanTris)) & 1ull)) Tb = item_tri_pk(a.la, M, B, ii, en, okb);
        bool keep = false;
        if (ok) {
          const CastTri tr = cast_tri(P, w, f, mirror);
          if (kept(tr, f)) {
            int i0, i1, j0, j1;
            cell_range(tr, f, a.R, i0, i1, j0, j1);
            keep = i1 >= ci0 && i0 <= ci1 && j1 >= cj0 && j0 <= cj1;
            if (keep) {
              ri0 = min(ri0, max(i0, ci0));
              ri1 = max(ri1, min(i1, ci1));
              rj0 = min(rj0, max(j0, cj0));
              rj1 = max(rj1, min(j1, cj1));
            }
          }
        }
        const uint64_t m = __ballot(keep);
        if (keep) sidx[wave * kSlice + n_mine + (int)__popcll(m & ((1ull << lane) - 1ull))] = e;
        n_mine += (int)__popcll(m);
      }
    }
    if (lane == 0) s_wcnt[wave] = n_mine;
    if (a.test_counter) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) n_read += __shfl_xor(n_read, off);
      if (lane == 0) s_read[wave] = n_read;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      ri0 = min(ri0, __shfl_xor(ri0, off));
      ri1 = max(ri1, __shfl_xor(ri1, off));
      rj0 = min(rj0, __shfl_xor(rj0, off));
      rj1 = max(rj1, __shfl_xor(rj1, off));
    }
    if (lane == 0 && ri1 >= 0) {
      atomicMin(&s_rng[0], ri0);
      atomicMax(&s_rng[1], ri1);
      atomicMin(&s_rng[2], rj0);
      atomicMax(&s_rng[3], rj1);
    }
    __syncthreads();
    // survivors: the waves' slices one after the other
    int n_surv = 0;
#pragma unroll
    for (int v = 0; v < kCastWaves; ++v) n_surv += s_wcnt[v];
    long long acc = 0, tests = 0;
    if (n_surv > 0) {
      // B. the rays of the survivors' cell range: cell (i, j) at
      // (-hu + (i + xi) du, -hv + (j + eta) dv)
      const int ui0 = s_rng[0], uj0 = s_rng[2];
      const int uw = s_rng[1] - ui0 + 1, nray = uw * (s_rng[3] - uj0 + 1);
      // ray k = j uw + i of the range; a thread's rays are kCastThreads apart:
      // (i, j) advance by (si, sj) with a carry (no division per ray)
      const int sj = kCastThreads / uw, si = kCastThreads - sj * uw;
      int rj = tid / uw, ri = tid - rj * uw;
      for (int k0 = tid; k0 < nray; k0 += kRayBatch * kCastThreads) {
        // kRayBatch rays per thread: their jitter is requested (or hashed) before any is used
        double xi[kRayBatch], eta[kRayBatch];
        int ci[kRayBatch], cj[kRayBatch];
#pragma unroll
        for (int q = 0; q < kRayBatch; ++q) {
          // rays past the range read the last one's draws (in bounds, not stored)
          const bool in = k0 + q * kCastThreads < nray;
          ci[q] = ui0 + (in ? ri : uw - 1);
          cj[q] = uj0 + (in ? rj : nray / uw - 1);
          ri += si;
          rj += sj;
          if (ri >= uw) {
            ri -= uw;
            ++rj;
          }
          if (TAB) {
            const uint2 jq = a.jitter[((int64_t)rf.key * 3 + w) * a.R * a.R + (int64_t)cj[q] * a.R + ci[q]];
            xi[q] = (double)jq.x * (1.0 / 16777216.0);
            eta[q] = (double)jq.y * (1.0 / 16777216.0);
          } else {
            const uint64_t z = rf.s0 + (uint64_t)(((uint32_t)ci[q] << 15) + (uint32_t)cj[q]) * (2ull * kGamma);
            xi[q] = u24(mix64(z));
            eta[q] = u24(mix64(z + kGamma));
          }
        }
#pragma unroll
        for (int q = 0; q < kRayBatch; ++q) {
          const int k = k0 + q * kCastThreads;
          if (k < nray)
            sray[k] = make_float2((float)__dadd_rn(-rf.hu, __dmul_rn(__dadd_rn((double)ci[q], xi[q]), rf.du)),
                                  (float)__dadd_rn(-rf.hv, __dmul_rn(__dadd_rn((double)cj[q], eta[q]), rf.dv)));
        }
      }
      if (OCC)
        for (int k = tid; k < 512; k += kCastThreads) socc[k] = 0;
      if (TAB && a.test_counter && tid == 0)
        atomicAdd(&a.test_counter[kProfSlots + (int)(u & (kProfSlots - 1))], (unsigned long long)(8ll * nray));
      __syncthreads();
      // C. each wave takes chunks of 64 survivors from a cursor: a lane tests its
      // survivor over the cells it covers; survivors covering more than
      // raster_cells cells are then tested by the whole wave, one cell per lane
      // (the record broadcast from its lane).  Waves run independently until
      // the sums.
      // The next chunk's triangles are requested before the current chunk is
      // tested.
      auto fetch = [&](int k, TriPk& t) {
        int x = k, v = 0;  // survivor k: entry x of the slice of wave v
        for (int c = s_wcnt[0]; x >= c && v < kCastWaves - 1; c = s_wcnt[++v]) x -= c;
        bool ok;
        t = item_tri_pk(a.la, M, B, ii, sidx[v * kSlice + x], ok);  // succeeded in the cull
      };
      int base = 0;
      if (lane == 0) base = atomicAdd(&s_cursor, 64);
      base = __shfl(base, 0);
      TriPk Tn{};
      if (base + lane < n_surv) fetch(base + lane, Tn);
      while (base < n_surv) {
        const int k = base + lane;
        const bool have = k < n_surv;
        const TriPk Tc = Tn;
        if (lane == 0) base = atomicAdd(&s_cursor, 64);
        base = __shfl(base, 0);
        if (base + lane < n_surv) fetch(base + lane, Tn);
        Rec r{};
        int i0 = 0, i1 = -1, j0 = 0, j1 = -1, cells = 0;
        if (have) {
          float P[3][3];
          unpack_tri(Tc, P);
          const CastTri tr = cast_tri(P, w, f, mirror);
          cell_range(tr, f, a.R, i0, i1, j0, j1);
          i0 = max(i0, ci0);
          i1 = min(i1, ci1);
          j0 = max(j0, cj0);
          j1 = min(j1, cj1);
          r = make_rec(tr, mirror, f.hw);
          cells = (i1 - i0 + 1) * (j1 - j0 + 1);
        }
        const bool wide = have && cells > a.raster_cells;
        if (have && !wide) {
          // a record's crossings share one sign and are at most 2^22 each: an
          // int32 sum holds fewer than 512 of them
          if (cells < 512)
            acc += raster_lane<STATS, OCC, int32_t>(a, r, i0, i1, j0, j1, ui0, uj0, uw, bw3, sray, socc);
          else
            acc += raster_lane<STATS, OCC, long long>(a, r, i0, i1, j0, j1, ui0, uj0, uw, bw3, sray, socc);
          tests += cells;
        }
        for (uint64_t wm = __ballot(wide); wm; wm &= wm - 1) {
          const int src = __ffsll((unsigned long long)wm) - 1;
          int wi0, wi1, wj0, wj1;
          const Rec rw = shfl_rec(r, i0, i1, j0, j1, src, wi0, wi1, wj0, wj1);
          acc += raster_wave<STATS, OCC>(a, rw, wi0, wi1, wj0, wj1, ui0, uj0, uw, bw3, sray, socc, lane);
          tests += lane == 0 ? (long long)(wi1 - wi0 + 1) * (wj1 - wj0 + 1) : 0ll;
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc += __shfl_xor(acc, off);
      tests += __shfl_xor(tests, off);
    }
    if (lane == 0) {
      s_red[wave] = acc;
      s_tests[wave] = tests;
    }
    __syncthreads();
    if (tid == 0) {
      long long sum = 0, nt = 0;
      for (int v = 0; v < kCastWaves; ++v) {
        sum += s_red[v];
        nt += s_tests[v];
      }
      if (sum) atomicAdd(&a.acc[bw3], (unsigned long long)sum);
      if (a.test_counter) {
        long long n_read_all = 0;
        for (int v = 0; v < kCastWaves; ++v) n_read_all += s_read[v];
        const int slot = (int)(u & (kProfSlots - 1));
        atomicAdd(&a.test_counter[slot], (unsigned long long)nt);
        atomicAdd(&a.test_counter[kProfSlots + slot], (unsigned long long)(48ll * n_read_all));
      }
    }
    if (OCC && n_surv > 0) {
      for (int k = tid; k < 512; k += kCastThreads) {
        const int v = socc[k];
        if (v) {
          const int kk = k & 7;
          atomicAdd(&a.occ[(int64_t)b * 512 + (k & ~7) + (mirror ? 7 - kk : kk)], v);
        }
      }
    }
    __syncthreads();
  }
}

// Jitter table of keys [0, n_keys): entry ((key * 3 + w) * R + j) * R + i holds
// the top 24 bits of the u and v draws of cell (i, j) of cast axis w.
__global__ void k_jitter_table(uint64_t seed, int R, int64_t n, uint2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int i = (int)(e % R), j = (int)((e / R) % R);
  const int64_t kw = e / ((int64_t)R * R);
  const int w = (int)(kw % 3);
  const uint32_t key = (uint32_t)(kw / 3);
  const uint64_t c = ray_counter(key, w, i, j);
  out[e] = make_uint2((uint32_t)(splitmix64_at(seed, c) >> 40), (uint32_t)(splitmix64_at(seed, c + 1) >> 40));
}

__global__ void k_or_word(uint32_t* __restrict__ w, uint32_t bits) { atomicOr(w, bits); }

struct Publish {
  int64_t* out;    // nullable: mapped host memory [status, 0, 0, 0, done]
  uint32_t* done;  // blocks finished (zeroed by k_box_chunks: the call's ctl[1])
};

__device__ void finalize_box(const obbv_box* __restrict__ boxes, int b, int R, uint32_t axis_mask,
                             const unsigned long long* __restrict__ acc, double* __restrict__ out_obv,
                             double* __restrict__ out_vin_axis, uint32_t* status);

// float64 OBV per box (and the kept side of every cast when asked); the last
// block to finish publishes the call's status bits to the caller's mapped host
// memory, then out[4] = 1 with a system-scope release: a host that sees it sees
// every output of the call.
__global__ void k_finalize(const obbv_box* __restrict__ boxes, int n_boxes, int R, uint32_t axis_mask,
                           const unsigned long long* __restrict__ acc, const float4* __restrict__ centre,
                           const int32_t* __restrict__ box_mesh, int n_meshes, double* __restrict__ out_obv,
                           double* __restrict__ out_vin_axis, int32_t* __restrict__ out_side, uint32_t* status,
                           Publish pub) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_boxes) {
    finalize_box(boxes, b, R, axis_mask, acc, out_obv, out_vin_axis, status);
    if (out_side) {
      const int m = box_mesh ? box_mesh[b] : 0;
      const BoxRegs B = load_box(boxes, b);
      for (int w = 0; w < 3; ++w)
        out_side[3 * b + w] = (m >= 0 && m < n_meshes && cast_mirror(B, w, centre[m])) ? 1 : 0;
    }
  }
  if (!pub.out) return;
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    if (atomicAdd(pub.done, 1u) == gridDim.x - 1) {
      __threadfence();
      pub.out[0] = (int64_t)atomicOr(status, 0u);
      pub.out[1] = pub.out[2] = pub.out[3] = 0;
      __threadfence_system();
      __hip_atomic_store(pub.out + 4, (int64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

__device__ void finalize_box(const obbv_box* __restrict__ boxes, int b, int R, uint32_t axis_mask,
                             const unsigned long long* __restrict__ acc, double* __restrict__ out_obv,
                             double* __restrict__ out_vin_axis, uint32_t* status) {
  const BoxRegs B = load_box(boxes, b);
  const int st = box_state(B);
  if (st == 2) {
    out_obv[b] = __longlong_as_double(0x7ff8000000000000ll);
    atomicOr(status, OBBV_STATUS_NAN_BOX);
    if (out_vin_axis)
      for (int w = 0; w < 3; ++w) out_vin_axis[3 * b + w] = __longlong_as_double(0x7ff8000000000000ll);
    return;
  }
  const double vbox = 8.0 * (double)B.h[0] * (double)B.h[1] * (double)B.h[2];
  const double denom = kQOne * (double)R * (double)R;
  long long qsum = 0;  // exact: the mean over the cast axes is taken on the integers
  int n = 0;
  for (int w = 0; w < 3; ++w) {
    double vin = 0.0;
    if ((axis_mask >> w) & 1u) {
      const long long q = st == 0 ? (long long)acc[3 * b + w] : 0ll;
      vin = vbox * ((double)q / denom);
      qsum += q;
      ++n;
    }
    if (out_vin_axis) out_vin_axis[3 * b + w] = vin;
  }
  out_obv[b] = vbox - (n ? vbox * ((double)qsum / (denom * n)) : 0.0);
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Pinned host words for totals read back by the host, one block per device and
// scratch-pool set (calls that may run at the same time use different sets).
int64_t* g_pinned[64][kPoolSets] = {};
std::mutex g_pinned_mutex;

int pinned_totals(int pool_base, int64_t** out) {
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  const int set = pool_base / kPoolCount;
  if (dev < 0 || dev >= 64) {
    set_error("device index out of range");
    return OBBV_ERR_UNSUPPORTED;
  }
  OBBV_ARG(set >= 0 && set < kPoolSets, "scratch-pool set out of range");
  std::lock_guard<std::mutex> lock(g_pinned_mutex);
  if (!g_pinned[dev][set]) {
    void* q = nullptr;
    OBBV_HIP(hipHostMalloc(&q, 64, hipHostMallocDefault));
    g_pinned[dev][set] = (int64_t*)q;
  }
  *out = g_pinned[dev][set];
  return OBBV_OK;
}

// Cells above which a record is tested wave-wide: kRasterCells, or
// OBBV_RASTER_CELLS (0..16384) to compare thresholds on a device (same bits).
int raster_cells_choice() {
  const char* e = getenv("OBBV_RASTER_CELLS");
  if (e && *e) {
    const int c = atoi(e);
    if (c >= 0 && c <= kBlockRaysMax) return c;
  }
  return kRasterCells;
}

// Rays per LDS ray block: the call's choice, else OBBV_BLOCK_RAYS, else the default.
int block_rays_choice(int requested) {
  if (requested) return requested;
  const char* e = getenv("OBBV_BLOCK_RAYS");
  if (e && *e) {
    const int c = atoi(e);
    if (c >= 1024 && c <= kBlockRaysMax && (c & (c - 1)) == 0) return c;
  }
  return kBlockRaysDefault;
}

// Span culling of whole-mesh casts: on unless OBBV_SPAN_CULL=0 (same bits either way).
// Frame lists of grouped calls: one pass into fixed segments while they fit in
// 2 GB, else two passes sized exactly; OBBV_FRAME_LISTS=2 takes the two-pass
// build at any size (same bits).
bool frame_lists_two_pass(int64_t bytes_one_pass) {
  const char* e = getenv("OBBV_FRAME_LISTS");
  return bytes_one_pass > ((int64_t)1 << 31) || (e && *e && atoi(e) == 2);
}

bool span_cull_choice() {
  const char* e = getenv("OBBV_SPAN_CULL");
  return !(e && *e && atoi(e) == 0);
}

int64_t n_spans_of(int64_t nt) { return (nt + kSpanTris - 1) / kSpanTris; }
int64_t n_runs_of(int64_t nt) { return (nt + kCastTris - 1) / kCastTris; }
// span bounds table of a single-mesh call: 2 float4 per span and per run
bool spans_apply(int n_meshes, int64_t nt0) { return n_meshes == 1 && nt0 > kCastTris; }
size_t span_table_bytes(int64_t nt) { return 32 * (size_t)(n_spans_of(nt) + n_runs_of(nt)); }

struct BlockGeom {
  int BC, BR, nbc, nblk;
  size_t lds;  // dynamic LDS of the cast kernel (bytes)
};

BlockGeom block_geom(int R, int block_rays) {
  BlockGeom g;
  g.BC = std::min(R, block_rays);
  g.BR = std::min(R, std::max(1, block_rays / g.BC));
  g.nbc = (R + g.BC - 1) / g.BC;
  g.nblk = g.nbc * ((R + g.BR - 1) / g.BR);
  g.lds = (size_t)g.BC * g.BR * sizeof(float2);
  return g;
}

constexpr int kMaxDevicesCast = 64;

template <bool STATS, bool OCC, bool TAB>
int launch_cast(const CastArgs& ca, unsigned grid, size_t lds, hipStream_t s) {
  // per instantiation and device: allow the largest dynamic block (calls on
  // several host threads may both set it; the setting is idempotent)
  static std::atomic<bool> attr_set[kMaxDevicesCast];
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevicesCast || !attr_set[dev].load(std::memory_order_acquire)) {
    OBBV_HIP(hipFuncSetAttribute((const void*)k_cast<STATS, OCC, TAB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(kBlockRaysMax * sizeof(float2))));
    if (dev >= 0 && dev < kMaxDevicesCast) attr_set[dev].store(true, std::memory_order_release);
  }
  hipLaunchKernelGGL((k_cast<STATS, OCC, TAB>), dim3(grid), dim3(kCastThreads), lds, s, ca);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

}  // namespace

// Boxes grouped by shared centre and axes (device arrays; one mesh only).
struct SharedFrames {
  const obbv_box* frames;    // [n_frames] centre, axes and the largest half extents of the group
  const int32_t* box_frame;  // [n_boxes] group of every box
  int32_t n_frames;
};

// Scratch sizes of a call (meta block, items block).
struct CallSizes {
  size_t meta = 0, items = 0;
  int64_t item_cap = 0, units = 0;
};

CallSizes call_sizes(int n_meshes, int n_boxes, int max_nt, int n_frames, int nt0, int nblk, int naxes,
                     int item_tris = kCastTris) {
  CallSizes c;
  c.item_cap = (int64_t)n_boxes * naxes * std::max(1, (max_nt + item_tris - 1) / item_tris);
  c.units = c.item_cap * nblk;
  const int64_t fitems = n_frames ? 3ll * n_frames * ((std::max(nt0, 1) + kCullThreads - 1) / kCullThreads) : 0;
  size_t off = 0;
  auto take = [&](size_t bytes) { off += align_up(bytes); };
  take(sizeof(MeshDev) * n_meshes);
  take(8 * (size_t)(3 * n_boxes + 1));       // chunk_off
  take(sizeof(RayFrame) * 3 * (size_t)n_boxes);
  take(8 * 3 * (size_t)n_boxes);             // acc
  take(16 * (size_t)n_meshes);               // mesh centres
  take(8 * 4);                               // ctl: unit queue, blocks finished
  take(4 * 3 * (size_t)n_frames);            // (frame, axis) list counts
  take(8 * (size_t)(3 * n_frames + 1));      // (frame, axis) list offsets
  take(exclusive_scan_scratch_bytes(3 * n_frames));
  if (spans_apply(n_meshes, nt0)) take(span_table_bytes(nt0));  // span bounds
  c.meta = off;
  c.items = align_up(sizeof(ItemInfo) * (size_t)c.item_cap) + 2 * align_up(4 * (size_t)fitems);
  return c;
}

// Span bounds of a mesh for repeated single-mesh calls (see k_span_bounds):
// bytes of the table (0 when the mesh has one cast item or less) and its launch.
size_t span_table_size(int64_t nt) { return spans_apply(1, nt) ? span_table_bytes(nt) : 0; }
int span_table(const obbv_mesh* m, float4* table, hipStream_t s) {
  const int64_t nt = m->n_triangles;
  if (!spans_apply(1, nt)) return OBBV_OK;
  uint32_t* status = nullptr;
  OBBV_RET(status_word(&status));
  const MeshDev M{m->vertices, m->triangles, m->n_vertices, m->n_triangles};
  hipLaunchKernelGGL(k_span_bounds, dim3((unsigned)n_runs_of(nt)), dim3(256), 0, s, M, table, table + 2 * n_spans_of(nt),
                     status);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}
const float4* span_runs_of(const float4* table, int64_t nt) { return table + 2 * n_spans_of(nt); }

int outer_volume_run(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                     const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                     const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                     int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side, hipStream_t s,
                     int32_t* out_occ, OvExec* ex, const SharedFrames* sf = nullptr) {
  OBBV_ARG(params != nullptr, "params is NULL");
  OBBV_ARG(n_boxes >= 0, "n_boxes < 0");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(meshes != nullptr && n_meshes >= 1, "need at least one mesh");
  OBBV_ARG(boxes != nullptr && out_obv != nullptr, "boxes / out_obv is NULL");
  OBBV_ARG(n_meshes == 1 || box_mesh != nullptr, "box_mesh is required with several meshes");
  OBBV_ARG(params->R >= 1 && params->R <= 32767, "R must be in [1, 32767]");
  OBBV_ARG(params->flags == 0, "flags must be 0");
  OBBV_ARG(params->block_rays == 0 || (params->block_rays >= 1024 && params->block_rays <= kBlockRaysMax &&
                                 (params->block_rays & (params->block_rays - 1)) == 0),
           "block_rays must be 0 or a power of two in [1024, 16384]");
  const int pool_base = ex ? ex->pool_base : 0;
  const uint32_t mask = params->axis_mask ? params->axis_mask : 7u;
  OBBV_ARG(mask <= 7u, "axis_mask has bits above 2");
  OBBV_ARG((int64_t)n_boxes * 6 < (1ll << 31), "too many boxes");
  int max_nt = 0;
  // the mesh table on the host: a fixed array for a few meshes (no allocation)
  MeshDev mh_few[4];
  std::vector<MeshDev> mh_many;
  if (n_meshes > 4) mh_many.resize((size_t)n_meshes);
  MeshDev* mh = n_meshes > 4 ? mh_many.data() : mh_few;
  for (int m = 0; m < n_meshes; ++m) {
    OBBV_ARG(meshes[m].n_triangles >= 0 && meshes[m].n_vertices >= 0, "negative mesh size");
    OBBV_ARG(meshes[m].n_triangles == 0 || (meshes[m].triangles && meshes[m].vertices),
             "mesh pointers are NULL");
    mh[m] = MeshDev{meshes[m].vertices, meshes[m].triangles, meshes[m].n_vertices, meshes[m].n_triangles};
    max_nt = std::max(max_nt, meshes[m].n_triangles);
  }
  const int R = params->R;
  const bool planned = ex && ex->planned;
  OBBV_ARG(!out_occ || (R == 8 && mask == 4u), "occupancy needs R = 8 and axis_mask = 4");
  OBBV_ARG(!sf || (n_meshes == 1 && !planned && sf->n_frames >= 1 && sf->n_frames <= n_boxes),
           "shared frames need one mesh, an unplanned call and 1..n_boxes frames");
  const int n_frames = sf ? sf->n_frames : 0;
  const int naxes = (int)((mask & 1u) + ((mask >> 1) & 1u) + ((mask >> 2) & 1u));
  const BlockGeom bg = block_geom(R, block_rays_choice(params->block_rays));
  const int item_tris = ex && ex->item_tris ? ex->item_tris : kCastTris;
  OBBV_ARG(item_tris % kSpanTris == 0 && kCastTris % item_tris == 0, "item_tris must be a multiple of 256 dividing 4608");
  const CallSizes cs =
      call_sizes(n_meshes, n_boxes, max_nt, n_frames, meshes[0].n_triangles, bg.nblk, naxes, item_tris);

  uint32_t* status = nullptr;
  if (ex && ex->status)
    status = ex->status;
  else
    OBBV_RET(status_word(&status));

  // ---- meta scratch layout (the order of call_sizes) ----
  void* meta_v = nullptr;
  if (planned) {
    if (cs.meta > ex->meta_cap || cs.items > ex->items_cap) {
      set_error("planned scratch too small for this call");
      return OBBV_ERR_WORKSPACE;
    }
    meta_v = ex->meta;
  } else {
    OBBV_RET(pool_get(pool_base + kPoolMeta, cs.meta, &meta_v));
  }
  if (ex) {
    ex->meta_bytes = cs.meta;
    ex->items_bytes = cs.items;
  }
  char* meta = (char*)meta_v;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = meta + off;
    off += align_up(bytes);
    return p;
  };
  MeshDev* d_mesh = (MeshDev*)take(sizeof(MeshDev) * n_meshes);
  int64_t* d_choff = (int64_t*)take(8 * (size_t)(3 * n_boxes + 1));
  RayFrame* d_rframe = (RayFrame*)take(sizeof(RayFrame) * 3 * (size_t)n_boxes);
  unsigned long long* d_acc = (unsigned long long*)take(8 * 3 * (size_t)n_boxes);
  float4* d_centre = (float4*)take(16 * (size_t)n_meshes);
  unsigned long long* d_ctl = (unsigned long long*)take(8 * 4);
  int32_t* d_fcnt = (int32_t*)take(4 * 3 * (size_t)n_frames);
  int64_t* d_foff = (int64_t*)take(8 * (size_t)(3 * n_frames + 1));
  void* d_scan = take(exclusive_scan_scratch_bytes(3 * n_frames));
  const size_t scan_bytes = exclusive_scan_scratch_bytes(3 * n_frames);
  const int64_t nt0 = meshes[0].n_triangles;
  float4* d_spans = spans_apply(n_meshes, nt0) ? (float4*)take(span_table_bytes(nt0)) : nullptr;

  char* items = nullptr;
  if (planned) {
    items = ex->items;
  } else {
    void* iv = nullptr;
    OBBV_RET(pool_get(pool_base + kPoolItems, cs.items, &iv));
    items = (char*)iv;
  }
  ItemInfo* d_items = (ItemInfo*)items;
  const int64_t fitems = n_frames ? 3ll * n_frames * ceil_div(std::max(meshes[0].n_triangles, 1), kCullThreads) : 0;
  int32_t* d_ficnt = (int32_t*)(items + align_up(sizeof(ItemInfo) * (size_t)cs.item_cap));
  int32_t* d_fioff = (int32_t*)((char*)d_ficnt + align_up(4 * (size_t)fitems));

  // the mesh table goes to the device only with several meshes (one mesh travels
  // in the kernel arguments; a plan keeps its table at the start of its meta block)
  if (!planned && n_meshes > 1)
    OBBV_HIP(hipMemcpyAsync(d_mesh, mh, sizeof(MeshDev) * n_meshes, hipMemcpyHostToDevice, s));
  const MeshDev* d_meshes = n_meshes > 1 ? (const MeshDev*)d_mesh : nullptr;

  // mesh centres (the kept side of every cast): given by the caller, or from
  // the meshes' bounding boxes
  const float4* centre = ex && ex->centre ? ex->centre : d_centre;
  if (!(ex && ex->centre)) {
    hipLaunchKernelGGL(k_mesh_centre, dim3(n_meshes), dim3(256), 0, s, d_meshes, mh[0], n_meshes, d_centre);
    OBBV_HIP(hipGetLastError());
  }

  // span bounds: given by the caller (same mesh for every call), or from the mesh
  const float4* spans = nullptr;
  const float4* runs = nullptr;
  if (spans_apply(n_meshes, nt0) && span_cull_choice()) {
    if (ex && ex->spans) {
      spans = ex->spans;
      runs = ex->span_runs;
    } else {
      hipLaunchKernelGGL(k_span_bounds, dim3((unsigned)n_runs_of(nt0)), dim3(256), 0, s, mh[0], d_spans,
                         d_spans + 2 * n_spans_of(nt0), status);
      OBBV_HIP(hipGetLastError());
      spans = d_spans;
      runs = d_spans + 2 * n_spans_of(nt0);
    }
  }

  float4* d_listP = nullptr;
  int32_t* d_lcnt = nullptr;  // one-pass list counters
  int64_t seg = 0;
  if (sf) {  // per (frame, axis): the triangles of the frame's kept half prism
    const int nt = meshes[0].n_triangles;
    const int nch = ceil_div(std::max(nt, 1), kCullThreads);
    const unsigned fgrid = (unsigned)std::min<int64_t>((int64_t)n_frames * nch, 256 * 64);
    const int ngroups = 3 * n_frames;
    if (!frame_lists_two_pass((int64_t)ngroups * std::max(nt, 1) * 48)) {
      // one pass: every list gets room for the whole mesh
      seg = std::max(nt, 1);
      void* cv = nullptr;
      OBBV_RET(pool_get_zeroed(pool_base + kPoolFrameCnt, 4 * (size_t)ngroups, &cv));
      d_lcnt = (int32_t*)cv;
      void* lv = nullptr;
      OBBV_RET(pool_get(pool_base + kPoolLists, (size_t)ngroups * seg * 48, &lv));
      d_listP = (float4*)lv;
      hipLaunchKernelGGL(k_frame_list, dim3(fgrid), dim3(kCullThreads), 0, s, sf->frames, n_frames, mh[0], centre,
                         mask, nch, seg, d_lcnt, d_listP, status, spans);
      OBBV_HIP(hipGetLastError());
    } else {  // large: count, scan, size the lists exactly (one host round trip), write
      hipLaunchKernelGGL(k_frame_cull, dim3(fgrid), dim3(kCullThreads), 0, s, sf->frames, n_frames, mh[0], centre,
                         mask, nch, d_ficnt, (const int32_t*)nullptr, (const int64_t*)nullptr, (float4*)nullptr,
                         status, spans);
      OBBV_HIP(hipGetLastError());
      if ((int64_t)ngroups * nch <= ((int64_t)1 << 20)) {  // one block: item and list offsets
        hipLaunchKernelGGL(k_frame_scan, dim3(1), dim3(kScanBlockThreads), 0, s, (const int32_t*)d_ficnt, ngroups,
                           nch, d_fioff, d_fcnt, d_foff);
        OBBV_HIP(hipGetLastError());
      } else {
        hipLaunchKernelGGL(k_frame_scan, dim3(ceil_div(ngroups, kCullWaves)), dim3(kCullThreads), 0, s,
                           (const int32_t*)d_ficnt, ngroups, nch, d_fioff, d_fcnt, (int64_t*)nullptr);
        OBBV_HIP(hipGetLastError());
        OBBV_RET(exclusive_scan_i32_to_i64(d_fcnt, d_foff, ngroups, d_scan, scan_bytes, s));
      }
      int64_t* pin = nullptr;
      OBBV_RET(pinned_totals(pool_base, &pin));
      OBBV_HIP(hipMemcpyAsync(pin + 3, d_foff + ngroups, 8, hipMemcpyDeviceToHost, s));
      OBBV_HIP(hipStreamSynchronize(s));
      void* lv = nullptr;
      OBBV_RET(pool_get(pool_base + kPoolLists, (size_t)std::max<int64_t>(pin[3], 1) * 48, &lv));
      d_listP = (float4*)lv;
      hipLaunchKernelGGL(k_frame_cull, dim3(fgrid), dim3(kCullThreads), 0, s, sf->frames, n_frames, mh[0], centre,
                         mask, nch, d_ficnt, (const int32_t*)d_fioff, (const int64_t*)d_foff, d_listP, status, spans);
      OBBV_HIP(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(k_box_chunks, dim3(1), dim3(kScanBlockThreads), 0, s, box_mesh, d_meshes, mh[0], n_meshes,
                     n_boxes, mask, boxes, sf ? sf->frames : nullptr, sf ? sf->box_frame : nullptr, n_frames,
                     (const int64_t*)d_foff, d_lcnt, seg, d_choff, status, box_key, R, params->seed, d_rframe, d_items,
                     cs.item_cap, d_acc, d_ctl, runs, centre, item_tris, ex ? ex->split_below : 0, bg.nblk);
  OBBV_HIP(hipGetLastError());

  ListArgs la;
  la.boxes = boxes;
  la.box_mesh = box_mesh;
  la.meshes = d_meshes;
  la.mesh0 = mh[0];
  la.list_P = d_listP;
  la.status = status;
  CastArgs ca;
  ca.la = la;
  ca.items = d_items;
  ca.chunk_off = d_choff;
  ca.n_boxes = n_boxes;
  ca.rframe = d_rframe;
  ca.centre = centre;
  ca.acc = d_acc;
  ca.queue = d_ctl;
  ca.R = R;
  ca.BC = bg.BC;
  ca.BR = bg.BR;
  ca.nbc = bg.nbc;
  ca.nblk = bg.nblk;
  ca.raster_cells = raster_cells_choice();
  ca.jitter = ex && ex->jitter && R == ex->jitter_R && params->seed == ex->jitter_seed ? ex->jitter : nullptr;
  ca.ray_q = out_ray_q;
  ca.ray_hits = out_ray_hits;
  ca.occ = out_occ;
  ca.test_counter = nullptr;
  ca.spans = spans;
  const bool stats = out_ray_q || out_ray_hits;
  if (stats) {
    const size_t per = (size_t)n_boxes * 3 * R * R * 4;
    if (out_ray_q) OBBV_HIP(hipMemsetAsync(out_ray_q, 0, per, s));
    if (out_ray_hits) OBBV_HIP(hipMemsetAsync(out_ray_hits, 0, per, s));
  }
  void* prof_token = nullptr;
  if (profiling_enabled() && !planned) {
    OBBV_RET(profile_counter(&ca.test_counter));
    OBBV_RET(profile_record_begin(s, &prof_token));
  }
  // persistent workgroups: as many as stay resident (LDS bound) across the 256 CUs
  // one 12-wave workgroup per CU (three waves per SIMD); more when the ray block is small
  const size_t lds_static = sizeof(int32_t) * kCastTris + 1024;
  const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(1, (160 * 1024) / (bg.lds + lds_static)));
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cs.units, 256 * per_cu));
  if (out_occ)
    OBBV_RET((launch_cast<false, true, false>(ca, grid, bg.lds, s)));
  else if (stats)
    OBBV_RET((launch_cast<true, false, false>(ca, grid, bg.lds, s)));
  else if (ca.jitter)
    OBBV_RET((launch_cast<false, false, true>(ca, grid, bg.lds, s)));
  else
    OBBV_RET((launch_cast<false, false, false>(ca, grid, bg.lds, s)));
  if (profiling_enabled() && !planned) OBBV_RET(profile_record_end(s, prof_token));
  Publish pub{ex ? ex->publish : nullptr, (uint32_t*)(d_ctl + 1)};
  hipLaunchKernelGGL(k_finalize, dim3(ceil_div(n_boxes, 128)), dim3(128), 0, s, boxes, n_boxes, R, mask,
                     (const unsigned long long*)d_acc, centre, box_mesh, n_meshes, out_obv, out_vin_axis, out_side,
                     status, pub);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

int outer_volume_frames(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key, int32_t n_boxes,
                        const obbv_ov_params* params, const obbv_box* frames, const int32_t* box_frame,
                        int32_t n_frames, double* out_obv, hipStream_t s, OvExec* ex) {
  const SharedFrames sf{frames, box_frame, n_frames};
  return outer_volume_run(mesh, 1, boxes, nullptr, box_key, n_boxes, params, out_obv, nullptr, nullptr, nullptr,
                          nullptr, s, nullptr, ex, &sf);
}

int outer_volume_exec(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key, int32_t n_boxes,
                      const obbv_ov_params* params, double* out_obv, hipStream_t s, OvExec* ex) {
  return outer_volume_run(mesh, 1, boxes, nullptr, box_key, n_boxes, params, out_obv, nullptr, nullptr, nullptr,
                          nullptr, s, nullptr, ex, nullptr);
}

int jitter_table(uint64_t seed, int R, int64_t n_keys, uint2* out, hipStream_t s) {
  OBBV_ARG(R >= 1 && R <= 32767 && n_keys >= 0 && out, "bad jitter table");
  const int64_t n = n_keys * 3 * (int64_t)R * R;
  if (n == 0) return OBBV_OK;
  hipLaunchKernelGGL(k_jitter_table, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, seed, R, n, out);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

int status_or(uint32_t bits, hipStream_t s) {
  uint32_t* w = nullptr;
  OBBV_RET(status_word(&w));
  hipLaunchKernelGGL(k_or_word, dim3(1), dim3(1), 0, s, w, bits);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

int outer_volume_impl(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                      const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                      const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                      int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side, hipStream_t s,
                      int32_t* out_occ) {
  return outer_volume_run(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv, out_vin_axis,
                          out_ray_q, out_ray_hits, out_side, s, out_occ, nullptr);
}

}  // namespace obbv

static int obbv_outer_volume_grouped_body(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                                         int32_t n_boxes, const obbv_ov_params* params, const obbv_box* frames,
                                         const int32_t* box_frame, int32_t n_frames, double* out_obv,
                                         void* stream);
extern "C" int obbv_outer_volume_grouped(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                                         int32_t n_boxes, const obbv_ov_params* params, const obbv_box* frames,
                                         const int32_t* box_frame, int32_t n_frames, double* out_obv,
                                         void* stream) {
  return obbv::guarded([&] { return obbv_outer_volume_grouped_body(mesh, boxes, box_key, n_boxes, params, frames, box_frame, n_frames, out_obv, stream); });
}
static int obbv_outer_volume_grouped_body(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                                         int32_t n_boxes, const obbv_ov_params* params, const obbv_box* frames,
                                         const int32_t* box_frame, int32_t n_frames, double* out_obv,
                                         void* stream) {
  obbv::clear_error();
  OBBV_ARG(mesh && params, "NULL argument");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(frames && box_frame && n_frames >= 1 && n_frames <= n_boxes, "need 1..n_boxes frames");
  return obbv::outer_volume_frames(mesh, boxes, box_key, n_boxes, params, frames, box_frame, n_frames, out_obv,
                                   (hipStream_t)stream, nullptr);
}

static int obbv_outer_volume_ex_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                    const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                    const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                                    int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side,
                                    void* stream);
extern "C" int obbv_outer_volume_ex(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                    const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                    const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                                    int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side,
                                    void* stream) {
  return obbv::guarded([&] { return obbv_outer_volume_ex_body(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv, out_vin_axis, out_ray_q, out_ray_hits, out_side, stream); });
}
static int obbv_outer_volume_ex_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                    const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                    const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                                    int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side,
                                    void* stream) {
  obbv::clear_error();
  return obbv::outer_volume_impl(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv,
                                 out_vin_axis, out_ray_q, out_ray_hits, out_side, (hipStream_t)stream, nullptr);
}

static int obbv_outer_volume_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                 const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                 const obbv_ov_params* params, double* out_obv, void* stream);
extern "C" int obbv_outer_volume(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                 const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                 const obbv_ov_params* params, double* out_obv, void* stream) {
  return obbv::guarded([&] { return obbv_outer_volume_body(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv, stream); });
}
static int obbv_outer_volume_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                 const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                 const obbv_ov_params* params, double* out_obv, void* stream) {
  obbv::clear_error();
  return obbv::outer_volume_impl(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv,
                                 nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream, nullptr);
}

// ---------------------------------------------------------------------------
// allocation-free evaluation: scratch in a fixed device array
// ---------------------------------------------------------------------------
namespace obbv {
namespace {
// 256 bytes of status word, then the call's meta block and cast items.  Each
// device holds its own copy until the process ends.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mutex;
char* g_noalloc_ptr[64] = {};  // device address of `scratch` on each device (host code must not use the name)

int noalloc_scratch(char** out) {
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device index out of range");
    return OBBV_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
      return OBBV_ERR_HIP;
    }
    g_noalloc_ptr[dev] = (char*)p;
  }
  *out = g_noalloc_ptr[dev];
  return OBBV_OK;
}
}  // namespace
}  // namespace obbv

static int obbv_outer_volume_noalloc_body(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                                         int32_t n_boxes, const obbv_ov_params* params, double* out_obv,
                                         uint32_t* out_status, void* stream);
extern "C" int obbv_outer_volume_noalloc(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                                         int32_t n_boxes, const obbv_ov_params* params, double* out_obv,
                                         uint32_t* out_status, void* stream) {
  return obbv::guarded([&] { return obbv_outer_volume_noalloc_body(mesh, boxes, box_key, n_boxes, params, out_obv, out_status, stream); });
}
static int obbv_outer_volume_noalloc_body(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                                         int32_t n_boxes, const obbv_ov_params* params, double* out_obv,
                                         uint32_t* out_status, void* stream) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(mesh && params, "NULL argument");
  OBBV_ARG(n_boxes >= 0, "n_boxes < 0");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(params->R >= 1 && params->R <= 32767, "R must be in [1, 32767]");
  OBBV_ARG(params->block_rays == 0 || (params->block_rays >= 1024 && params->block_rays <= kBlockRaysMax &&
                                       (params->block_rays & (params->block_rays - 1)) == 0),
           "block_rays must be 0 or a power of two in [1024, 16384]");
  const uint32_t mask = params->axis_mask ? params->axis_mask : 7u;
  OBBV_ARG(mask <= 7u, "axis_mask has bits above 2");
  OBBV_ARG(mesh->n_triangles >= 0, "negative mesh size");
  const int naxes = (int)((mask & 1u) + ((mask >> 1) & 1u) + ((mask >> 2) & 1u));
  const BlockGeom bg = block_geom(params->R, block_rays_choice(params->block_rays));
  const CallSizes cs = call_sizes(1, n_boxes, mesh->n_triangles, 0, mesh->n_triangles, bg.nblk, naxes);
  const size_t need = 256 + align_up(cs.meta) + align_up(cs.items);
  if (need > kNoAllocScratchBytes) {
    set_error("obbv_outer_volume_noalloc: the call needs " + std::to_string(need) + " bytes of scratch, more than the " +
              std::to_string(kNoAllocScratchBytes) + " bytes of the fixed array (fewer boxes per call)");
    return OBBV_ERR_WORKSPACE;
  }
  char* base = nullptr;
  OBBV_RET(noalloc_scratch(&base));
  OvExec ex;
  ex.planned = true;
  ex.status = out_status ? out_status : (uint32_t*)base;
  ex.meta = base + 256;
  ex.meta_cap = align_up(cs.meta);
  ex.items = ex.meta + ex.meta_cap;
  ex.items_cap = align_up(cs.items);
  return outer_volume_run(mesh, 1, boxes, nullptr, box_key, n_boxes, params, out_obv, nullptr, nullptr, nullptr,
                          nullptr, (hipStream_t)stream, nullptr, &ex, nullptr);
}

// ---------------------------------------------------------------------------
// surrogate input rows: 15 normalised box parameters + 8 x 8 x 8 occupancy
// ---------------------------------------------------------------------------
namespace obbv {
namespace {
constexpr float kOccUnit = 1.0f / 524288.0f;  // 2^-19: one sub-slab

__global__ void k_features(const obbv_box* __restrict__ boxes, const int32_t* __restrict__ box_mesh, int n_meshes,
                           const float* __restrict__ frame, const int32_t* __restrict__ occ, int n,
                           float* __restrict__ X) {
  const int b = blockIdx.x;
  if (b >= n) return;
  const float* p = reinterpret_cast<const float*>(boxes + b);
  int m = box_mesh ? box_mesh[b] : 0;
  m = (m < 0 || m >= n_meshes) ? 0 : m;
  const float* fr = frame + 4 * m;
  float* x = X + (int64_t)b * 544;
  for (int k = threadIdx.x; k < 544; k += blockDim.x) {
    float v = 0.f;
    if (k < 3)
      v = (p[k] - fr[k]) / fr[3];
    else if (k < 12)
      v = p[k];
    else if (k < 15)
      v = logf(fmaxf(p[k], 1e-30f) / fr[3]);
    else if (k < 527)
      v = (float)occ[(int64_t)b * 512 + (k - 15)] * kOccUnit;
    x[k] = v;
  }
}
}  // namespace
}  // namespace obbv

static int obbv_box_features_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                 const int32_t* box_mesh, int32_t n_boxes, const float* mesh_frame, uint64_t seed,
                                 float* out_X, void* stream);
extern "C" int obbv_box_features(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                 const int32_t* box_mesh, int32_t n_boxes, const float* mesh_frame, uint64_t seed,
                                 float* out_X, void* stream) {
  return obbv::guarded([&] { return obbv_box_features_body(meshes, n_meshes, boxes, box_mesh, n_boxes, mesh_frame, seed, out_X, stream); });
}
static int obbv_box_features_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                 const int32_t* box_mesh, int32_t n_boxes, const float* mesh_frame, uint64_t seed,
                                 float* out_X, void* stream) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(n_boxes >= 0, "n_boxes < 0");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(mesh_frame && out_X && boxes, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  void* q = nullptr;
  OBBV_RET(pool_get(kPoolFeat, (size_t)n_boxes * (512 * 4 + 8), &q));
  int32_t* occ = (int32_t*)q;
  double* obv = (double*)(occ + (size_t)n_boxes * 512);
  OBBV_HIP(hipMemsetAsync(occ, 0, (size_t)n_boxes * 512 * 4, s));
  obbv_ov_params p{8, 4u, seed, 0, 0u};
  OBBV_RET(outer_volume_impl(meshes, n_meshes, boxes, box_mesh, nullptr, n_boxes, &p, obv, nullptr, nullptr, nullptr,
                             nullptr, s, occ));
  hipLaunchKernelGGL(k_features, dim3((unsigned)n_boxes), dim3(128), 0, s, boxes, box_mesh, n_meshes, mesh_frame,
                     (const int32_t*)occ, n_boxes, out_X);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// occupancy volume of a mesh (the ranker samples its inputs from it)
// ---------------------------------------------------------------------------
namespace obbv {
namespace {
// axis-aligned tiling boxes of the bounding box: nb^3 boxes, box (bx, by, bz) at
// index (bz * nb + by) * nb + bx
__global__ void k_tiling_boxes(const float* __restrict__ frame, int nb, obbv_box* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * nb * nb) return;
  const int bx = i % nb, by = (i / nb) % nb, bz = i / (nb * nb);
  float* o = reinterpret_cast<float*>(out + i);
  const int idx[3] = {bx, by, bz};
  for (int k = 0; k < 3; ++k) {
    const float cell = 8.0f * frame[3 + k];
    o[k] = frame[k] + (idx[k] + 0.5f) * cell;  // centre
    o[12 + k] = 0.5f * cell;                     // half extent
  }
  for (int k = 0; k < 9; ++k) o[3 + k] = (k % 4 == 0) ? 1.f : 0.f;
}

// occupancy [box][x][y][z] of the tiling boxes -> volume [z][y][x]
__global__ void k_scatter_volume(const int32_t* __restrict__ occ, int nb, float* __restrict__ vol) {
  const int64_t n = (int64_t)nb * nb * nb * 512;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t box = t / 512;
  const int r = (int)(t % 512);
  const int x = r / 64, y = (r / 8) % 8, z = r % 8;
  const int bx = (int)(box % nb), by = (int)((box / nb) % nb), bz = (int)(box / ((int64_t)nb * nb));
  const int64_t N = 8 * nb;
  vol[((int64_t)(8 * bz + z) * N + (8 * by + y)) * N + (8 * bx + x)] = (float)occ[t] * kOccUnit;
}

}  // namespace
}  // namespace obbv

static int obbv_occupancy_volume_body(const obbv_mesh* mesh, int32_t nb, const float* frame, uint64_t seed,
                                     float* out_volume, void* stream);
extern "C" int obbv_occupancy_volume(const obbv_mesh* mesh, int32_t nb, const float* frame, uint64_t seed,
                                     float* out_volume, void* stream) {
  return obbv::guarded([&] { return obbv_occupancy_volume_body(mesh, nb, frame, seed, out_volume, stream); });
}
static int obbv_occupancy_volume_body(const obbv_mesh* mesh, int32_t nb, const float* frame, uint64_t seed,
                                     float* out_volume, void* stream) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(mesh && frame && out_volume, "NULL argument");
  OBBV_ARG(nb >= 1 && nb <= 64, "nb must be in [1, 64]");
  hipStream_t s = (hipStream_t)stream;
  const int n = nb * nb * nb;
  void* q = nullptr;
  OBBV_RET(pool_get(kPoolFeat, (size_t)n * (512 * 4 + 8 + sizeof(obbv_box)) + 1024, &q));
  int32_t* occ = (int32_t*)q;
  double* obv = (double*)(occ + (size_t)n * 512);
  obbv_box* tb = (obbv_box*)(obv + n);
  OBBV_HIP(hipMemsetAsync(occ, 0, (size_t)n * 512 * 4, s));
  hipLaunchKernelGGL(k_tiling_boxes, dim3(ceil_div(n, 128)), dim3(128), 0, s, frame, nb, tb);
  OBBV_HIP(hipGetLastError());
  obbv_ov_params p{8, 4u, seed, 0, 0u};
  OBBV_RET(outer_volume_impl(mesh, 1, tb, nullptr, nullptr, n, &p, obv, nullptr, nullptr, nullptr, nullptr, s, occ));
  hipLaunchKernelGGL(k_scatter_volume, dim3(ceil_div((int64_t)n * 512, 256)), dim3(256), 0, s,
                     (const int32_t*)occ, nb, out_volume);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// planned evaluations: autotuned ray blocks, fixed scratch, HIP graph replay
// ---------------------------------------------------------------------------
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

namespace obbv {
namespace {

constexpr int kTuneCandidates[3] = {2048, 4096, 8192};

struct OvPlanState {
  std::vector<obbv_mesh> meshes;
  const obbv_box* boxes = nullptr;
  const int32_t* box_mesh = nullptr;
  const uint32_t* box_key = nullptr;
  int32_t n_boxes = 0;
  obbv_ov_params params{};
  double* out_obv = nullptr;
  OvExec ex;
  void* alloc = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  float tuned_ms[3] = {0.f, 0.f, 0.f};
  int64_t item_cap = 0, units = 0;
};

// autotuner cache: (architecture, R, boxes bucket, triangles bucket) -> rays per block
std::map<std::tuple<std::string, int, int, int>, int> g_block_cache;
std::mutex g_block_mutex;

inline int bucket(int64_t x) {
  int b = 0;
  while (x > 1) {
    x >>= 1;
    ++b;
  }
  return b;
}

int time_block(OvPlanState& P, int block, hipStream_t s, float* ms) {
  obbv_ov_params p = P.params;
  p.block_rays = block;
  hipEvent_t a, b;
  OBBV_HIP(hipEventCreate(&a));
  OBBV_HIP(hipEventCreate(&b));
  int rc = outer_volume_impl(P.meshes.data(), (int32_t)P.meshes.size(), P.boxes, P.box_mesh, P.box_key, P.n_boxes,
                             &p, P.out_obv, nullptr, nullptr, nullptr, nullptr, s, nullptr);  // warm
  if (rc == OBBV_OK) rc = hipEventRecord(a, s) == hipSuccess ? OBBV_OK : OBBV_ERR_HIP;
  for (int r = 0; r < 2 && rc == OBBV_OK; ++r)
    rc = outer_volume_impl(P.meshes.data(), (int32_t)P.meshes.size(), P.boxes, P.box_mesh, P.box_key, P.n_boxes, &p,
                           P.out_obv, nullptr, nullptr, nullptr, nullptr, s, nullptr);
  if (rc == OBBV_OK) rc = hipEventRecord(b, s) == hipSuccess ? OBBV_OK : OBBV_ERR_HIP;
  if (rc == OBBV_OK) rc = hipEventSynchronize(b) == hipSuccess ? OBBV_OK : OBBV_ERR_HIP;
  if (rc == OBBV_OK) rc = hipEventElapsedTime(ms, a, b) == hipSuccess ? OBBV_OK : OBBV_ERR_HIP;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // namespace
}  // namespace obbv

static int obbv_ov_plan_create_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                   const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                   const obbv_ov_params* params, double* out_obv, double headroom, void* stream,
                                   obbv_ov_plan** out);
extern "C" int obbv_ov_plan_create(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                   const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                   const obbv_ov_params* params, double* out_obv, double headroom, void* stream,
                                   obbv_ov_plan** out) {
  return obbv::guarded([&] { return obbv_ov_plan_create_body(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv, headroom, stream, out); });
}
static int obbv_ov_plan_create_body(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                   const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                   const obbv_ov_params* params, double* out_obv, double headroom, void* stream,
                                   obbv_ov_plan** out) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(out && meshes && params && boxes && out_obv, "NULL argument");
  OBBV_ARG(n_boxes >= 1 && n_meshes >= 1, "need boxes and meshes");
  OBBV_ARG(headroom >= 1.0, "headroom must be >= 1");
  OBBV_ARG(params->R >= 1 && params->R <= 32767, "R must be in [1, 32767]");
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<OvPlanState> P(new OvPlanState());
  P->meshes.assign(meshes, meshes + n_meshes);
  P->boxes = boxes;
  P->box_mesh = box_mesh;
  P->box_key = box_key;
  P->n_boxes = n_boxes;
  P->params = *params;
  P->out_obv = out_obv;
  int max_nt = 0;
  for (int m = 0; m < n_meshes; ++m) max_nt = std::max(max_nt, meshes[m].n_triangles);
  // autotune the LDS ray block (rays cached per workgroup; larger blocks cull
  // each triangle against fewer blocks, smaller ones keep more workgroups per CU)
  if (P->params.block_rays == 0) {
    int dev = 0;
    OBBV_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    OBBV_HIP(hipGetDeviceProperties(&prop, dev));
    int64_t ntri = 0;
    for (int m = 0; m < n_meshes; ++m) ntri += meshes[m].n_triangles;
    const auto key = std::make_tuple(std::string(prop.gcnArchName), P->params.R, bucket(n_boxes),
                                     bucket(ntri / n_meshes));
    int block = 0;
    {
      std::lock_guard<std::mutex> lock(g_block_mutex);
      auto it = g_block_cache.find(key);
      if (it != g_block_cache.end()) block = it->second;
    }
    if (!block) {
      float best = 0.f;
      for (int c = 0; c < 3; ++c) {
        OBBV_RET(time_block(*P, kTuneCandidates[c], s, &P->tuned_ms[c]));
        if (!block || P->tuned_ms[c] < best) {
          best = P->tuned_ms[c];
          block = kTuneCandidates[c];
        }
      }
      std::lock_guard<std::mutex> lock(g_block_mutex);
      g_block_cache[key] = block;
    }
    P->params.block_rays = block;
  }
  const uint32_t mask = params->axis_mask ? params->axis_mask : 7u;
  const int naxes = (int)((mask & 1u) + ((mask >> 1) & 1u) + ((mask >> 2) & 1u));
  const BlockGeom bg = block_geom(P->params.R, P->params.block_rays);
  const CallSizes cs = call_sizes(n_meshes, n_boxes, max_nt, 0, meshes[0].n_triangles, bg.nblk, naxes);
  P->item_cap = cs.item_cap;
  P->units = cs.units;
  OvExec& ex = P->ex;
  ex.planned = true;
  ex.meta_cap = cs.meta;
  ex.items_cap = cs.items;
  const size_t bytes = align_up(ex.meta_cap) + align_up(ex.items_cap);
  if (hipMalloc(&P->alloc, bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of the planned scratch failed");
    return OBBV_ERR_OOM;
  }
  ex.meta = (char*)P->alloc;
  ex.items = ex.meta + align_up(ex.meta_cap);
  // the mesh table lives at the start of the meta block (outside the graph)
  std::vector<MeshDev> mh((size_t)n_meshes);
  for (int m = 0; m < n_meshes; ++m)
    mh[m] = MeshDev{meshes[m].vertices, meshes[m].triangles, meshes[m].n_vertices, meshes[m].n_triangles};
  OBBV_HIP(hipMemcpy(ex.meta, mh.data(), sizeof(MeshDev) * n_meshes, hipMemcpyHostToDevice));
  // capture one evaluation on a private stream
  hipStream_t cs2 = nullptr;
  OBBV_HIP(hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking));
  OBBV_HIP(hipStreamBeginCapture(cs2, hipStreamCaptureModeThreadLocal));
  int rc = outer_volume_run(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, &P->params, out_obv, nullptr,
                            nullptr, nullptr, nullptr, cs2, nullptr, &ex);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs2, &g);
  (void)hipStreamDestroy(cs2);
  if (rc != OBBV_OK) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipFree(P->alloc);
    return rc;
  }
  if (ec != hipSuccess) {
    (void)hipFree(P->alloc);
    set_error(std::string("graph capture failed: ") + hipGetErrorString(ec));
    return OBBV_ERR_HIP;
  }
  P->graph = g;
  if (hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    (void)hipFree(P->alloc);
    set_error("hipGraphInstantiate failed");
    return OBBV_ERR_HIP;
  }
  (void)s;
  *out = reinterpret_cast<obbv_ov_plan*>(P.release());
  return OBBV_OK;
}

static int obbv_ov_plan_launch_body(obbv_ov_plan* plan, void* stream);
extern "C" int obbv_ov_plan_launch(obbv_ov_plan* plan, void* stream) {
  return obbv::guarded([&] { return obbv_ov_plan_launch_body(plan, stream); });
}
static int obbv_ov_plan_launch_body(obbv_ov_plan* plan, void* stream) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(plan, "NULL plan");
  OvPlanState* P = reinterpret_cast<OvPlanState*>(plan);
  OBBV_HIP(hipGraphLaunch(P->exec, (hipStream_t)stream));
  return OBBV_OK;
}

static int obbv_ov_plan_info_body(obbv_ov_plan* plan, int32_t* out_block_rays, int64_t* out_caps, float* out_tuned_ms);
extern "C" int obbv_ov_plan_info(obbv_ov_plan* plan, int32_t* out_block_rays, int64_t* out_caps, float* out_tuned_ms) {
  return obbv::guarded([&] { return obbv_ov_plan_info_body(plan, out_block_rays, out_caps, out_tuned_ms); });
}
static int obbv_ov_plan_info_body(obbv_ov_plan* plan, int32_t* out_block_rays, int64_t* out_caps, float* out_tuned_ms) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(plan, "NULL plan");
  OvPlanState* P = reinterpret_cast<OvPlanState*>(plan);
  if (out_block_rays) *out_block_rays = P->params.block_rays;
  if (out_caps) {
    out_caps[0] = P->item_cap;
    out_caps[1] = P->units;
    out_caps[2] = (int64_t)(P->ex.meta_cap + P->ex.items_cap);
  }
  if (out_tuned_ms)
    for (int c = 0; c < 3; ++c) out_tuned_ms[c] = P->tuned_ms[c];
  return OBBV_OK;
}

static int obbv_ov_plan_destroy_body(obbv_ov_plan* plan);
extern "C" int obbv_ov_plan_destroy(obbv_ov_plan* plan) {
  return obbv::guarded([&] { return obbv_ov_plan_destroy_body(plan); });
}
static int obbv_ov_plan_destroy_body(obbv_ov_plan* plan) {
  using namespace obbv;
  clear_error();
  if (!plan) return OBBV_OK;
  OvPlanState* P = reinterpret_cast<OvPlanState*>(plan);
  OBBV_HIP(hipDeviceSynchronize());
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->alloc) (void)hipFree(P->alloc);
  delete P;
  return OBBV_OK;
}
