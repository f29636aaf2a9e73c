// Outer volume OBV(X, O) of oriented boxes against a closed mesh
// (Sec. 3, Eq. 4), by jittered parallel rays on each box face and the signed
// crossing sum along each ray (Sec. 4.1, Eq. 9 generalised to a line).
//
// Pipeline per call (all on one stream):
//   [k_frame_cull x 2,   boxes grouped by shared centre and axes: the frame-local
//    k_frame_scan]       coordinates of the triangles each group can see
//   k_box_chunks         work list of (box, 256-triangle chunk) cull items and a
//                        table of them (one block), the ray grid of every cast
//   k_cull_count         per item and cast axis: triangles in the half prism above
//                        the slab bottom and below the slab top, and the ray tiles
//                        each can reach, for both sides (counts summed per block)
//   k_box_sides          keep the half prism with fewer triangles (mirror flag),
//                        take that side's tile counts
//   k_tiles_scan_one     bin, work-item and record offsets (one block for small
//   (or _block/top/add)  calls, else three kernels); unless the scratch is capped
//                        or planned, one host sync for sizes
//   k_write              per kept triangle and ray tile it reaches: a 64-byte test
//                        record copy (edge and depth planes, fixed point, cell
//                        range in the tile) in the tile's bin; the 64-byte ray-test
//                        work items (ray grid, tile, bin range)
//   k_raster             one wave per work item: every record against the rays of
//                        the cells it covers (k_test: against every ray of the tile)
//   k_finalize           float64 OBV per box, publication of the call
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "common.h"

namespace obbv {
namespace {

constexpr int kCullThreads = 256;
constexpr int kTestThreads = 64;
constexpr int kTestChunk = 384;  // records per ray-test work item (measured best of 64..4096)

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

// element k of a 3-vector held in registers (selects, so the vector never
// needs addressable private memory)
__device__ inline float pick3(const float v[3], int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

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

// Workgroup k is dispatched to XCD k % 8; give every XCD a contiguous range of
// logical ids so that tiles of one (box, axis) share that XCD's L2.
__device__ inline int xcd_remap(int bid, int n) {
  const int nx = 8;
  const int q = n / nx, r = n % nx;
  const int x = bid % nx, k = bid / nx;
  return x * q + min(x, r) + k;
}

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
    t.u[k] = P[k][f.ua];
    t.v[k] = P[k][f.va];
    t.z[k] = mirror ? -P[k][w] : P[k][w];
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

// Range of the cells whose rays can hit the triangle (conservative), and the
// range of TE x TE ray tiles holding them.
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

__device__ inline void tile_range(const CastTri& t, const CastFrame& f, int R, int TE, int& ti0,
                                  int& ti1, int& tj0, int& tj1) {
  int i0, i1, j0, j1;
  cell_range(t, f, R, i0, i1, j0, j1);
  ti0 = i0 / TE;
  ti1 = i1 / TE;
  tj0 = j0 / TE;
  tj1 = j1 / TE;
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

// item -> (box, chunk) by binary search over the per-box chunk offsets
__device__ inline int item_box(const int64_t* __restrict__ chunk_off, int n_boxes, int64_t item) {
  int lo = 0, hi = n_boxes;  // chunk_off[lo] <= item < chunk_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// A cull work item (256 triangles of one box's list or of the mesh), as
// k_box_chunks tabulates it: the box, the item's triangle count, and its first
// triangle: an index into the box's frame list (first >= 0) or mesh triangle
// -1 - first (first < 0).
struct ItemInfo {
  int64_t first;
  int32_t b;
  int32_t count;
};

struct CullArgs {
  const ItemInfo* item_info;  // nullable: every item's box and triangles (else a search of chunk_off)
  const obbv_box* boxes;
  const int32_t* box_mesh;
  const MeshDev* meshes;  // device mesh table; NULL with a single mesh (then mesh0)
  MeshDev mesh0;
  const RayFrame* rframe;  // [n_boxes * 3] ray grid of every cast (k_box_chunks)
  const int64_t* chunk_off;
  int n_boxes;
  int R;
  int TE;
  int tpe;  // tiles per face edge
  uint32_t axis_mask;
  uint32_t* status;
  int write_lds;    // write pass: bin slots reserved per tile in LDS (1) or taken one by one (0)
  int64_t rec_cap;  // records and bin entries a planned launch was sized for
  int64_t bin_cap;
  // nullable: the triangles a box can see, one list per shared frame, held as
  // their frame-local vertex coordinates (3 float4 per triangle)
  const float4* list_P;
  const int64_t* list_off;  // [n_frames + 1]
  const int32_t* box_list;  // [n_boxes] frame of every box, -1 = the whole mesh
};

// Number of triangles box b walks.
__device__ inline int box_ntri(const CullArgs& a, int b, const MeshDev& M) {
  const int l = a.list_P ? a.box_list[b] : -1;
  return l < 0 ? M.nt : (int)(a.list_off[l + 1] - a.list_off[l]);
}

// The t-th triangle of box b in the box frame: from its frame's list (the same
// bits to_local gives: same centre, same axes), else transformed from the mesh.
__device__ inline bool cull_tri(const CullArgs& a, int b, const MeshDev& M, const BoxRegs& B, int t,
                                float P[3][3]) {
  const int l = a.list_P ? a.box_list[b] : -1;
  if (l < 0) return t < M.nt && load_tri_local(M, t, B, P, a.status);
  if (t >= (int)(a.list_off[l + 1] - a.list_off[l])) return false;
  const float4* q = a.list_P + 3 * (a.list_off[l] + t);
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

// Triangle `tid` of a tabulated item, in the box frame (false past its end).
__device__ inline bool cull_tri_item(const CullArgs& a, const MeshDev& M, const BoxRegs& B, const ItemInfo& ii,
                                     int tid, float P[3][3]) {
  if (tid >= ii.count) return false;
  if (ii.first < 0) return load_tri_local(M, (int)(-1 - ii.first) + tid, B, P, a.status);
  const float4* q = a.list_P + 3 * (ii.first + tid);
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

// Calls of up to this many boxes get a table of their cull items (k_box_chunks).
constexpr int kItemBoxMax = 2048;

// One block: the number of 256-triangle items of every box (its frame list, or
// the whole mesh), their exclusive scan (chunk_off[0..n_boxes]), the frame use
// of every box, and the per-call counters that must start at zero.
__global__ void __launch_bounds__(kScanBlockThreads)
k_box_chunks(const int32_t* __restrict__ box_mesh, const MeshDev* __restrict__ meshes, MeshDev mesh0, int n_meshes,
             int n_boxes,
             const obbv_box* __restrict__ boxes, const obbv_box* __restrict__ frames,
             const int32_t* __restrict__ box_frame, int n_frames, const int64_t* __restrict__ list_off,
             int32_t* __restrict__ box_list, int64_t* __restrict__ chunk_off, uint32_t* __restrict__ done_counter,
             uint32_t* status, const uint32_t* __restrict__ box_key, int R, uint64_t seed,
             RayFrame* __restrict__ rframe, ItemInfo* __restrict__ item_info) {
  __shared__ long long wsum[kScanBlockThreads / 64];
  // with item_info: every box's first item, first triangle (list index, or -1
  // for the mesh) and triangle count
  __shared__ int32_t sco[kItemBoxMax + 1];
  __shared__ int64_t sfirst[kItemBoxMax];
  __shared__ int32_t sn[kItemBoxMax];
  if (threadIdx.x == 0 && done_counter) *done_counter = 0u;
  for (int e = threadIdx.x; e < 3 * n_boxes; e += blockDim.x) {  // the ray grid of every cast
    const int b = e / 3;
    rframe[e] = make_ray_frame(load_box(boxes, b), e - 3 * b, box_key ? box_key[b] : (uint32_t)b, R, seed);
  }
  long long base = 0;
  for (int b0 = 0; b0 < n_boxes; b0 += kScanBlockThreads) {
    const int b = b0 + (int)threadIdx.x;
    long long nch = 0;
    int64_t first = -1, ntri = 0;
    if (b < n_boxes) {
      const int m = box_mesh ? box_mesh[b] : 0;
      if (m < 0 || m >= n_meshes) {  // out-of-range mesh index: the box sees no triangles
        atomicOr(status, OBBV_STATUS_BAD_INDEX);
        if (box_list) box_list[b] = -1;
      } else {
        int64_t n = meshes ? meshes[m].nt : mesh0.nt;
        if (box_list) {
          const int f = box_frame[b];
          const bool use = f >= 0 && f < n_frames && inside_frame(boxes[b], frames[f]);
          box_list[b] = use ? f : -1;
          if (use) {
            first = list_off[f];
            n = list_off[f + 1] - first;
          }
        }
        ntri = n;
        nch = (n + kCullThreads - 1) / kCullThreads;
      }
    }
    long long total = 0;
    const long long ex = block_excl_scan(nch, wsum, total);
    if (b < n_boxes) {
      chunk_off[b] = base + ex;
      if (item_info) {
        sco[b] = (int32_t)(base + ex);
        sfirst[b] = first;
        sn[b] = (int32_t)ntri;
      }
    }
    base += total;
  }
  if (threadIdx.x == 0) chunk_off[n_boxes] = base;
  if (item_info) {  // every item (the cull passes read it instead of searching chunk_off)
    if (threadIdx.x == 0) sco[n_boxes] = (int32_t)base;
    __syncthreads();
    for (int64_t it = threadIdx.x; it < base; it += blockDim.x) {
      int lo = 0, hi = n_boxes;  // sco[lo] <= it < sco[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sco[mid] <= it)
          lo = mid;
        else
          hi = mid;
      }
      const int64_t t0 = (it - sco[lo]) * (int64_t)kCullThreads;
      ItemInfo ii;
      ii.b = lo;
      ii.count = (int32_t)min((int64_t)kCullThreads, (int64_t)sn[lo] - t0);
      ii.first = sfirst[lo] >= 0 ? sfirst[lo] + t0 : -1 - t0;
      item_info[it] = ii;
    }
  }
}

// Per-wave ballot counts of a 256-thread block, summed in LDS: every block
// writes its own counts (no global atomics on shared counters, which serialise).
constexpr int kCullWaves = kCullThreads / 64;

// Shared frames: boxes with the same centre and axes see every triangle at the
// same local coordinates, and a triangle can matter to one of them only if it
// projects into a face of their union (the frame box, with the largest half
// extents).  Items are (frame, 256-triangle chunk).  With item_off NULL the pass
// writes each item's count of such triangles; otherwise it writes their
// frame-local coordinates at list_off[frame] + item_off[item] + rank (in
// triangle order).
__global__ void __launch_bounds__(kCullThreads)
k_frame_cull(const obbv_box* __restrict__ frames, int n_frames, MeshDev M, uint32_t axis_mask, int nch,
             int32_t* __restrict__ item_cnt, const int32_t* __restrict__ item_off,
             const int64_t* __restrict__ list_off, float4* __restrict__ list_P, uint32_t* status) {
  __shared__ int32_t wc[kCullWaves];
  const int64_t total = (int64_t)n_frames * nch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const int fr = (int)(item / nch);
    const int t = (int)(item - (int64_t)fr * nch) * kCullThreads + threadIdx.x;
    const BoxRegs B = load_box(frames, fr);
    float P[3][3];
    bool keep = false;
    if (box_state(B) == 0 && t < M.nt && load_tri_local(M, t, B, P, status)) {
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        if (!((axis_mask >> w) & 1u)) continue;
        const CastFrame f = cast_bounds(B, w);
        keep = keep || projects_into_face(cast_tri(P, w, f, false), f);
      }
    }
    const uint64_t m = __ballot(keep);
    if (lane == 0) wc[wave] = (int)__popcll(m);
    __syncthreads();
    if (!item_off) {
      if (threadIdx.x == 0) {
        int c = 0;
        for (int v = 0; v < kCullWaves; ++v) c += wc[v];
        item_cnt[item] = c;
      }
    } else if (keep) {
      int pos = item_off[item] + (int)__popcll(m & ((1ull << lane) - 1ull));
      for (int v = 0; v < wave; ++v) pos += wc[v];
      if (pos < item_off[item] + item_cnt[item]) {
        float4* q = list_P + 3 * (list_off[fr] + pos);
        q[0] = make_float4(P[0][0], P[0][1], P[0][2], P[1][0]);
        q[1] = make_float4(P[1][1], P[1][2], P[2][0], P[2][1]);
        q[2] = make_float4(P[2][2], 0.f, 0.f, 0.f);
      } else {  // count and write passes disagree: never expected
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

// Which prism(s) the triangle belongs to, per cast axis.
//   above: projects into the face and reaches above the slab bottom (z_max > -h)
//   below: projects into the face and reaches below the slab top   (z_min <  h)
// Tile counters of one work item (one box, 256 triangles, three axes; both
// sides in the cull pass) are aggregated in LDS when they fit (6 TT resp. 3 TT
// <= kLdsTiles) and flushed with one global atomic per non-zero tile.
constexpr int kLdsTiles = 3 * 1024;

__global__ void __launch_bounds__(kCullThreads)
k_cull_count(CullArgs a, int32_t* __restrict__ item_cnt, int32_t* __restrict__ tile_cnt2) {
  __shared__ int32_t wc[kCullWaves][6];
  __shared__ int32_t cnt[kLdsTiles];
  const int64_t total = a.chunk_off[a.n_boxes];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int TT = a.tpe * a.tpe;
  const bool lds = 6 * TT <= kLdsTiles;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    ItemInfo ii;
    if (a.item_info) {
      ii = a.item_info[item];
    } else {
      ii.b = item_box(a.chunk_off, a.n_boxes, item);
      ii.count = -1;
    }
    const int b = ii.b;
    const BoxRegs B = load_box(a.boxes, b);
    const bool valid = box_state(B) == 0;
    const MeshDev M = a.meshes ? a.meshes[a.box_mesh ? a.box_mesh[b] : 0] : a.mesh0;
    float P[3][3];
    bool ok;
    if (a.item_info) {
      ok = valid && cull_tri_item(a, M, B, ii, threadIdx.x, P);
    } else {
      const int t = (int)(item - a.chunk_off[b]) * kCullThreads + threadIdx.x;
      ok = valid && cull_tri(a, b, M, B, t, P);
    }
    if (lds) {
      for (int k = threadIdx.x; k < 6 * TT; k += kCullThreads) cnt[k] = 0;
      __syncthreads();
    }
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      bool ka = false, kb = false;
      if (ok && ((a.axis_mask >> w) & 1u)) {
        const CastFrame f = cast_frame_rf(B, w, a.rframe[b * 3 + w]);
        const CastTri tr = cast_tri(P, w, f, false);
        if (projects_into_face(tr, f)) {
          const float zmin = fminf(fminf(tr.z[0], tr.z[1]), tr.z[2]);
          const float zmax = fmaxf(fmaxf(tr.z[0], tr.z[1]), tr.z[2]);
          ka = zmax > -f.hw;
          kb = zmin < f.hw;
          if (ka || kb) {  // tile counts of both sides (the mirrored cast negates z only)
            int ti0, ti1, tj0, tj1;
            tile_range(tr, f, a.R, a.TE, ti0, ti1, tj0, tj1);
            for (int tj = tj0; tj <= tj1; ++tj)
              for (int ti = ti0; ti <= ti1; ++ti) {
                const int k = tj * a.tpe + ti;
                if (lds) {
                  if (ka) atomicAdd(&cnt[(2 * w) * TT + k], 1);
                  if (kb) atomicAdd(&cnt[(2 * w + 1) * TT + k], 1);
                } else {
                  const int64_t base = (int64_t)(b * 3 + w) * 2 * TT;
                  if (ka) atomicAdd(&tile_cnt2[base + k], 1);
                  if (kb) atomicAdd(&tile_cnt2[base + TT + k], 1);
                }
              }
          }
        }
      }
      const uint64_t ma = __ballot(ka), mb = __ballot(kb);
      if (lane == 0) {
        wc[wave][2 * w + 0] = (int)__popcll(ma);
        wc[wave][2 * w + 1] = (int)__popcll(mb);
      }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      int c = 0;
      for (int v = 0; v < kCullWaves; ++v) c += wc[v][threadIdx.x];
      item_cnt[6 * item + threadIdx.x] = c;
    }
    if (lds) {  // [axis][side][tile] of this box: the layout of tile_cnt2
      for (int k = threadIdx.x; k < 6 * TT; k += kCullThreads)
        if (cnt[k]) atomicAdd(&tile_cnt2[(int64_t)b * 6 * TT + k], cnt[k]);
    }
    __syncthreads();
  }
}

// One wave per (box, cast axis): the triangle counts of both half prisms, the
// side with fewer triangles (mirror flag), its record count, and that side's
// tile counts.
__global__ void k_box_sides(const int64_t* __restrict__ chunk_off, int n_boxes, const int32_t* __restrict__ item_cnt,
                            int32_t* __restrict__ side, int32_t* __restrict__ rec_cnt, int TT,
                            int32_t* __restrict__ tile_cnt,
                            int32_t* __restrict__ bin_cur, unsigned long long* __restrict__ acc,
                            int32_t* __restrict__ tile_cnt2) {
  const int bw = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (bw >= 3 * n_boxes) return;
  // counters of this (box, axis) that later passes accumulate into
  for (int k = lane; k < TT; k += 64) bin_cur[(int64_t)bw * TT + k] = 0;
  if (lane == 0) acc[bw] = 0ull;
  const int b = bw / 3, w = bw - 3 * b;
  const int64_t i0 = chunk_off[b], i1 = chunk_off[b + 1];
  int up = 0, dn = 0;
  for (int64_t i = i0 + lane; i < i1; i += 64) {
    up += item_cnt[6 * i + 2 * w];
    dn += item_cnt[6 * i + 2 * w + 1];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    up += __shfl_xor(up, off);
    dn += __shfl_xor(dn, off);
  }
  const int mirror = dn < up ? 1 : 0;
  if (lane == 0) {
    side[bw] = mirror;
    rec_cnt[bw] = mirror ? dn : up;
  }
  // the chosen side's tile counts; both sides' counters are left zero for the next call
  int32_t* tc = tile_cnt2 + (int64_t)bw * 2 * TT;
  for (int k = lane; k < TT; k += 64) {
    tile_cnt[(int64_t)bw * TT + k] = tc[mirror * TT + k];
    tc[k] = 0;
    tc[TT + k] = 0;
  }
}

// Offsets of the tile bins and of the test work items in one scan: every
// non-empty bin is cut into chunks of at most `chunk` records (so no wave walks
// a much longer list than the others), and both the bin sizes and the chunk
// counts are scanned together.  Three kernels: per block of kScanBlockThreads
// tiles, one block for the block sums (and the per-(box, axis) record counts),
// then the block offsets.
__global__ void __launch_bounds__(kScanBlockThreads)
k_tiles_scan_block(const int32_t* __restrict__ cnt, int64_t n, int chunk, int64_t* __restrict__ bin_off,
                   int64_t* __restrict__ chunk_off, int64_t* __restrict__ bsum) {
  __shared__ long long wsum[kScanBlockThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kScanBlockThreads + threadIdx.x;
  const int c = i < n ? cnt[i] : 0;
  long long tb = 0, tc = 0;
  const long long eb = block_excl_scan(c, wsum, tb);
  const long long ec = block_excl_scan((c + chunk - 1) / chunk, wsum, tc);
  if (i < n) {
    bin_off[i] = eb;
    chunk_off[i] = ec;
  }
  if (threadIdx.x == 0) {
    bsum[2 * blockIdx.x] = tb;
    bsum[2 * blockIdx.x + 1] = tc;
  }
}

__global__ void __launch_bounds__(kScanBlockThreads)
k_tiles_scan_top(int64_t* __restrict__ bsum, int64_t nb, int64_t n, int64_t* __restrict__ bin_off,
                 int64_t* __restrict__ chunk_off, const int32_t* __restrict__ rec_cnt, int64_t nbw,
                 int64_t* __restrict__ rec_off) {
  __shared__ long long wsum[kScanBlockThreads / 64];
  long long ob = 0, oc = 0;
  for (int64_t j0 = 0; j0 < nb; j0 += kScanBlockThreads) {
    const int64_t j = j0 + threadIdx.x;
    long long tb = 0, tc = 0;
    const long long eb = block_excl_scan(j < nb ? bsum[2 * j] : 0, wsum, tb);
    const long long ec = block_excl_scan(j < nb ? bsum[2 * j + 1] : 0, wsum, tc);
    __syncthreads();  // every thread has read its bsum entries
    if (j < nb) {
      bsum[2 * j] = ob + eb;
      bsum[2 * j + 1] = oc + ec;
    }
    ob += tb;
    oc += tc;
  }
  if (threadIdx.x == 0) {
    bin_off[n] = ob;
    chunk_off[n] = oc;
  }
  long long orr = 0;
  for (int64_t j0 = 0; j0 < nbw; j0 += kScanBlockThreads) {
    const int64_t j = j0 + threadIdx.x;
    long long t = 0;
    const long long e = block_excl_scan(j < nbw ? rec_cnt[j] : 0, wsum, t);
    if (j < nbw) rec_off[j] = orr + e;
    orr += t;
  }
  if (threadIdx.x == 0) rec_off[nbw] = orr;
}

// The same offsets for up to kTilesScanOne tiles in one workgroup (one launch
// instead of three): the counts are staged in LDS (coalesced loads), every
// thread sums a run of consecutive tiles, one block scan of the run sums, then
// every thread writes its run's offsets; then the record offsets of the
// (box, axis) pairs.
constexpr int kTilesScanOne = 16 * 1024;

__global__ void __launch_bounds__(kScanBlockThreads)
k_tiles_scan_one(const int32_t* __restrict__ cnt, int64_t n, int chunk, int64_t* __restrict__ bin_off,
                 int64_t* __restrict__ chunk_off, const int32_t* __restrict__ rec_cnt, int64_t nbw,
                 int64_t* __restrict__ rec_off) {
  __shared__ long long wsum[kScanBlockThreads / 64];
  __shared__ int32_t scnt[kTilesScanOne];
#pragma unroll
  for (int k = 0; k < kTilesScanOne / kScanBlockThreads; ++k) {
    const int i = (int)threadIdx.x + k * kScanBlockThreads;
    scnt[i] = i < n ? cnt[i] : 0;
  }
  __syncthreads();
  const int per = (int)((n + kScanBlockThreads - 1) / kScanBlockThreads);
  const int i0 = min((int)threadIdx.x * per, (int)n), i1 = min(i0 + per, (int)n);
  long long sb = 0, sc = 0;
  for (int i = i0; i < i1; ++i) {
    const int c = scnt[i];
    sb += c;
    sc += (c + chunk - 1) / chunk;
  }
  long long tb = 0, tc = 0;
  long long ob = block_excl_scan(sb, wsum, tb);
  long long oc = block_excl_scan(sc, wsum, tc);
  for (int i = i0; i < i1; ++i) {
    const int c = scnt[i];
    bin_off[i] = ob;
    chunk_off[i] = oc;
    ob += c;
    oc += (c + chunk - 1) / chunk;
  }
  if (threadIdx.x == 0) {
    bin_off[n] = tb;
    chunk_off[n] = tc;
  }
  long long orr = 0;
  for (int64_t j0 = 0; j0 < nbw; j0 += kScanBlockThreads) {
    const int64_t j = j0 + threadIdx.x;
    long long t = 0;
    const long long e = block_excl_scan(j < nbw ? rec_cnt[j] : 0, wsum, t);
    if (j < nbw) rec_off[j] = orr + e;
    orr += t;
  }
  if (threadIdx.x == 0) rec_off[nbw] = orr;
}

__global__ void __launch_bounds__(kScanBlockThreads)
k_tiles_scan_add(int64_t n, const int64_t* __restrict__ bsum, int64_t* __restrict__ bin_off,
                 int64_t* __restrict__ chunk_off) {
  const int64_t i = (int64_t)blockIdx.x * kScanBlockThreads + threadIdx.x;
  if (i >= n || blockIdx.x == 0) return;
  bin_off[i] += bsum[2 * blockIdx.x];
  chunk_off[i] += bsum[2 * blockIdx.x + 1];
}

// Is the triangle kept on the chosen side?  (Mirrored frames flip z, so the
// kept half prism is always "above the slab bottom" in the cast frame.)
__device__ inline bool kept(const CastTri& tr, const CastFrame& f) {
  if (!projects_into_face(tr, f)) return false;
  const float zmax = fmaxf(fmaxf(tr.z[0], tr.z[1]), tr.z[2]);
  return zmax > -f.hw;
}



// The 64-byte test record of a kept triangle in its cast frame.
//   [0..8]   edge functions E_k(u, v) = A_k u + B_k v + C_k, k = edge (k -> k+1),
//            oriented so that the inside of the projected triangle is E >= 0
//   [9..11]  depth plane in fixed point: y(u, v) = D u + E v + F equals
//            kMagic + s (w(u, v) + h) 2^21 / h, s = crossing sign
//   [12..13] clamp of y to the part of the triangle inside the slab
//   [14]     crossing sign s (+1 leaving the solid along +w in the cast frame)
//   [15]     set per bin entry (pack_cells): the triangle's cell range inside the
//            entry's tile
// The edge coefficients of an edge shared by two triangles are exact
// negatives of each other (or equal, when one of them is flipped), so the two
// triangles classify every ray consistently: the test is watertight.
__device__ inline void make_record(const CastTri& t, bool mirror, float hw, float4* __restrict__ out) {
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
  // barycentric weight of vertex 0 is E_1 / A2, of vertex 1 is E_2 / A2, of vertex 2 is E_0 / A2
  const double D = (Ad[1] * t.z[0] + Ad[2] * t.z[1] + Ad[0] * t.z[2]) / t.A2;
  const double E = (Bd[1] * t.z[0] + Bd[2] * t.z[1] + Bd[0] * t.z[2]) / t.A2;
  const double F = (Cd[1] * t.z[0] + Cd[2] * t.z[1] + Cd[0] * t.z[2]) / t.A2;
  const double h = hw;
  const double K = (double)s * kHalfQ / h;
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
  out[0] = make_float4(A[0], Bc[0], C[0], A[1]);
  out[1] = make_float4(Bc[1], C[1], A[2], Bc[2]);
  out[2] = make_float4(C[2], (float)(K * D), (float)(K * E), (float)(K * (F + h) + (double)kMagic));
  out[3] = make_float4((float)lo, (float)hi, (float)s, 0.0f);
}

// Cell range [i0, i1] x [j0, j1] (cell_range) clipped to the tile whose first
// cell is (ci, cj), as four 4-bit offsets from that cell (tiles are at most
// 16 x 16 cells): i0 | i1 << 4 | j0 << 8 | j1 << 12.
__device__ inline uint32_t pack_cells(int i0, int i1, int j0, int j1, int ci, int cj, int TE) {
  const int a0 = max(i0, ci) - ci, a1 = min(i1, ci + TE - 1) - ci;
  const int b0 = max(j0, cj) - cj, b1 = min(j1, cj + TE - 1) - cj;
  return (uint32_t)a0 | ((uint32_t)a1 << 4) | ((uint32_t)b0 << 8) | ((uint32_t)b1 << 12);
}

// Bin slots: every (tile) of the work item first counts its entries in LDS,
// then reserves a contiguous range of its bin with one global atomic; the
// entries then take positions in that range (their order inside a bin does
// not matter: the ray sums are exact integers).  Every entry holds its own copy
// of the record, with the cell range inside its tile.
__global__ void __launch_bounds__(kCullThreads)
k_write(CullArgs a, const int32_t* __restrict__ side, const int64_t* __restrict__ bin_off,
        int32_t* __restrict__ bin_cur, float4* __restrict__ recs, const int64_t* __restrict__ chunk_off,
        int64_t n_tiles, WorkItem* __restrict__ items, int64_t item_cap, int chunk) {
  if (items) {  // the ray-test work items (grid-stride over the tiles)
    const int TT = a.tpe * a.tpe;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles;
         t += (int64_t)gridDim.x * blockDim.x) {
      const int64_t c0 = chunk_off[t], c1 = min(chunk_off[t + 1], item_cap);
      if (c0 >= c1) continue;
      const int64_t b0 = bin_off[t], b1 = bin_off[t + 1];
      const RayFrame& rf = a.rframe[t / TT];
      WorkItem wi;
      wi.hu = rf.hu;
      wi.hv = rf.hv;
      wi.du = rf.du;
      wi.dv = rf.dv;
      wi.s0 = rf.s0;
      wi.g = (int32_t)t;
      wi.key = rf.key;
      wi.pad = 0;
      for (int64_t c = c0; c < c1; ++c) {
        wi.k0 = b0 + (c - c0) * chunk;
        wi.count = (int32_t)(min(b1, wi.k0 + chunk) - wi.k0);
        items[c] = wi;
      }
    }
  }
  // per tile of the item's box (3 TT, dynamic LDS when lds): first bin entry
  // reserved for the item, end of the tile's bin, entries taken so far
  extern __shared__ __align__(8) char wdyn[];
  const int TT = a.tpe * a.tpe;
  const bool lds = a.write_lds && 3 * TT <= kLdsTiles;
  int64_t* base_k = reinterpret_cast<int64_t*>(wdyn);
  int64_t* lim_k = base_k + 3 * TT;
  int32_t* cnt = reinterpret_cast<int32_t*>(lim_k + 3 * TT);
  const int64_t total = a.chunk_off[a.n_boxes];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    ItemInfo ii;
    if (a.item_info) {
      ii = a.item_info[item];
    } else {
      ii.b = item_box(a.chunk_off, a.n_boxes, item);
      ii.count = -1;
    }
    const int b = ii.b;
    const BoxRegs B = load_box(a.boxes, b);
    const bool valid = box_state(B) == 0;
    const MeshDev M = a.meshes ? a.meshes[a.box_mesh ? a.box_mesh[b] : 0] : a.mesh0;
    float P[3][3];
    bool ok;
    if (a.item_info) {
      ok = valid && cull_tri_item(a, M, B, ii, threadIdx.x, P);
    } else {
      const int t = (int)(item - a.chunk_off[b]) * kCullThreads + threadIdx.x;
      ok = valid && cull_tri(a, b, M, B, t, P);
    }
    // pass 1: kept flags, per-wave record counts, and (in LDS) per-tile entry counts
    if (lds)
      for (int k = threadIdx.x; k < 3 * TT; k += kCullThreads) cnt[k] = 0;
    __syncthreads();
    uint32_t keepmask = 0;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      bool keep = false;
      if (ok && ((a.axis_mask >> w) & 1u)) {
        const CastFrame f = cast_frame_rf(B, w, a.rframe[b * 3 + w]);
        const CastTri tr = cast_tri(P, w, f, side[b * 3 + w] != 0);
        keep = kept(tr, f);
        if (keep && lds) {
          int ti0, ti1, tj0, tj1;
          tile_range(tr, f, a.R, a.TE, ti0, ti1, tj0, tj1);
          for (int tj = tj0; tj <= tj1; ++tj)
            for (int ti = ti0; ti <= ti1; ++ti) atomicAdd(&cnt[w * TT + tj * a.tpe + ti], 1);
        }
      }
      keepmask |= keep ? (1u << w) : 0u;
    }
    __syncthreads();
    if (lds) {
      // reserve one range per non-zero tile, with the tile's bin start and end
      for (int k = threadIdx.x; k < 3 * TT; k += kCullThreads) {
        const int c = cnt[k];
        if (c) {
          const int64_t tl = (int64_t)(b * 3 + k / TT) * TT + (k % TT);
          base_k[k] = bin_off[tl] + atomicAdd(&bin_cur[tl], c);
          lim_k[k] = bin_off[tl + 1];
        }
        cnt[k] = 0;
      }
      __syncthreads();
    }
    // pass 2: a record copy per bin entry
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const bool keep = (keepmask >> w) & 1u;
      if (!keep) continue;
      const int bw = b * 3 + w;
      const bool mirror = side[bw] != 0;
      const CastFrame f = cast_frame_rf(B, w, a.rframe[b * 3 + w]);
      const CastTri tr = cast_tri(P, w, f, mirror);
      float4 rec[kRecF4];
      make_record(tr, mirror, f.hw, rec);
      int i0, i1, j0, j1;
      cell_range(tr, f, a.R, i0, i1, j0, j1);
      const int ti0 = i0 / a.TE, ti1 = i1 / a.TE, tj0 = j0 / a.TE, tj1 = j1 / a.TE;
      const int64_t tbase = (int64_t)bw * TT;
      for (int tj = tj0; tj <= tj1; ++tj)
        for (int ti = ti0; ti <= ti1; ++ti) {
          const int64_t tl = tbase + tj * a.tpe + ti;
          const int lt = w * TT + tj * a.tpe + ti;
          int64_t k, lim;
          if (lds) {
            k = base_k[lt] + atomicAdd(&cnt[lt], 1);
            lim = lim_k[lt];
          } else {
            k = bin_off[tl] + atomicAdd(&bin_cur[tl], 1);
            lim = bin_off[tl + 1];
          }
          if (k >= a.bin_cap) {
            atomicOr(a.status, OBBV_STATUS_OVERFLOW);
          } else if (k < lim) {
            float4* o = recs + kRecF4 * k;
            o[0] = rec[0];
            o[1] = rec[1];
            o[2] = rec[2];
            o[3] = make_float4(rec[3].x, rec[3].y, rec[3].z,
                               __uint_as_float(pack_cells(i0, i1, j0, j1, ti * a.TE, tj * a.TE, a.TE)));
          } else {
            atomicOr(a.status, OBBV_STATUS_BAD_INDEX);
          }
        }
    }
    __syncthreads();  // the LDS tile arrays are reused by the next item
  }
}

struct TestArgs {
  const obbv_box* boxes;
  const uint32_t* box_key;
  const int64_t* bin_off;
  const int64_t* chunk_off;  // [nbw * TT + 1] first work item of each tile
  int64_t n_tiles;
  int chunk;
  const float4* recs;        // [bin entries] binned records
  unsigned long long* acc;  // [nbw] per-(box, axis) sum of q
  int32_t* ray_q;           // nullable [nbw][R][R]
  int32_t* ray_hits;        // nullable [nbw][R][R]
  unsigned long long* test_counter;  // nullable [2 kProfSlots]: tests, bytes (slot item % kProfSlots)
  float* occ;                        // nullable [n_boxes][8][8][8]: sub-slab inside fractions (R = 8, axis 2)
  const int32_t* side;               // [nbw] mirrored cast flags
  uint64_t seed;
  int n_boxes;
  int R;
  int tpe;
  uint32_t axis_mask;
  int64_t bin_cap;      // planned launches: bins beyond it were not written
  int64_t item_cap;     // planned launches: work items beyond it are skipped
  const WorkItem* items;     // [work items] every ray-test work item
  int persistent;       // 1: grid-stride over the work items counted on the device
  const uint2* jitter;       // nullable: jitter table [keys][3][R][R] (jitter_table), every key < its rows
  int raster_cells;          // records covering more cells of a tile take the wave-wide path
};

// One wave per TE x TE ray tile of one (box, axis); RPL = (TE/8)^2 rays per lane.
// Every ray is tested against every record in the tile's bin:
//   E_k = A_k u + B_k v + C_k (3 x 2 FMA), inside iff min E_k >= 0,
//   y = D u + E v + F (2 FMA), clamped to the triangle's slab part (med3),
//   acc += inside ? bits(y) : kMagicBits   -- exact integer accumulation.
template <int TE, bool STATS, bool STAGE, bool OCC>
__device__ void test_item(const TestArgs& a, const int64_t item);


template <int TE, bool STATS, bool STAGE, bool OCC>
__global__ void __launch_bounds__(kTestThreads) k_test(TestArgs a) {
  if (!a.persistent) {
    test_item<TE, STATS, STAGE, OCC>(a, xcd_remap(blockIdx.x, gridDim.x));
    return;
  }
  const int64_t total = min(a.chunk_off[a.n_tiles], a.item_cap);
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) test_item<TE, STATS, STAGE, OCC>(a, item);
}

template <int TE, bool STATS, bool STAGE, bool OCC>
__device__ void test_item(const TestArgs& a, const int64_t item) {
  constexpr int NB = TE / 8;
  constexpr int RPL = NB * NB;
  const int TT = a.tpe * a.tpe;
  // tile of this work item: chunk_off[g] <= item < chunk_off[g + 1]
  const int g = a.items[item].g;
  const int bw = g / TT;
  const int tile = g - bw * TT;
  const int b = bw / 3, w = bw - 3 * (bw / 3);
  if (!((a.axis_mask >> w) & 1u)) return;
  const BoxRegs B = load_box(a.boxes, b);
  if (box_state(B) != 0) return;
  const int ua = (w + 1) % 3, va = (w + 2) % 3;
  const double hu = pick3(B.h, ua), hv = pick3(B.h, va);
  const double du = __ddiv_rn(__dmul_rn(2.0, hu), (double)a.R);
  const double dv = __ddiv_rn(__dmul_rn(2.0, hv), (double)a.R);
  const uint32_t key = a.box_key ? a.box_key[b] : (uint32_t)b;
  const int ti = tile % a.tpe, tj = tile / a.tpe;
  const int lane = threadIdx.x;

  float ru[RPL], rv[RPL];
  float occ_acc[OCC ? 8 : 1];
  for (int j = 0; j < (OCC ? 8 : 1); ++j) occ_acc[j] = 0.f;
  uint32_t acc[RPL];
  int hits[RPL];
  bool valid[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = ti * TE + (r % NB) * 8 + (lane & 7);
    const int j = tj * TE + (r / NB) * 8 + (lane >> 3);
    valid[r] = i < a.R && j < a.R;
    acc[r] = 0u;
    hits[r] = 0;
    ru[r] = 0.f;
    rv[r] = 0.f;
    if (valid[r]) {
      const uint64_t n = ray_counter(key, w, i, j);
      const double xi = u24(splitmix64_at(a.seed, n));
      const double eta = u24(splitmix64_at(a.seed, n + 1));
      ru[r] = (float)__dadd_rn(-hu, __dmul_rn(__dadd_rn((double)i, xi), du));
      rv[r] = (float)__dadd_rn(-hv, __dmul_rn(__dadd_rn((double)j, eta), dv));
    }
  }

  const int64_t kb = a.bin_off[g] + (item - a.chunk_off[g]) * a.chunk;
  const int64_t k0 = kb;
  const int64_t k1 = min(a.bin_off[g + 1], kb + a.chunk);
  if (k1 > a.bin_cap) return;  // bins past a planned capacity were not written (flagged)
  auto test_record = [&](const float4 r0, const float4 r1, const float4 r2, const float4 r3) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const float u = ru[r], v = rv[r];
      const float e0 = __fmaf_rn(r0.x, u, __fmaf_rn(r0.y, v, r0.z));
      const float e1 = __fmaf_rn(r0.w, u, __fmaf_rn(r1.x, v, r1.y));
      const float e2 = __fmaf_rn(r1.z, u, __fmaf_rn(r1.w, v, r2.x));
      const float m = fminf(fminf(e0, e1), e2);
      const float y = __fmaf_rn(r2.y, u, __fmaf_rn(r2.z, v, r2.w));
      const float c = __builtin_amdgcn_fmed3f(y, r3.x, r3.y);
      const bool in = m >= 0.0f;
      acc[r] += in ? __float_as_uint(c) : kMagicBits;
      if (STATS) hits[r] += in ? 1 : 0;
      if (OCC && in) {
        // the same crossing split over 8 equal sub-slabs: position from the slab
        // bottom in units of 2^-22 of the slab, sub-slab k spans [k 2^19, (k+1) 2^19]
        const float sg = r3.z;
        const float yq = (c - kMagic) * sg;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          occ_acc[k] += sg * (fminf(fmaxf(yq, (float)(k << 19)), (float)((k + 1) << 19)) - (float)(k << 19));
      }
    }
  };
  if (STAGE) {
    // 64 records at a time: one coalesced record load per lane into LDS, then
    // every lane reads each record from LDS (same address for the whole wave)
    __shared__ float4 srec[kTestThreads * 4];
    for (int64_t base = k0; base < k1; base += kTestThreads) {
      const int n = (int)min((int64_t)kTestThreads, k1 - base);
      if (lane < n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) srec[4 * lane + q] = a.recs[kRecF4 * (base + lane) + q];
      }
      __syncthreads();
      for (int j = 0; j < n; ++j) test_record(srec[4 * j + 0], srec[4 * j + 1], srec[4 * j + 2], srec[4 * j + 3]);
      __syncthreads();
    }
  } else {
    for (int64_t k = k0; k < k1; ++k)
      test_record(a.recs[kRecF4 * k + 0], a.recs[kRecF4 * k + 1], a.recs[kRecF4 * k + 2], a.recs[kRecF4 * k + 3]);
  }
  const uint32_t nbias = (uint32_t)(k1 - k0) * kMagicBits;
  if (a.test_counter && lane == 0) {
    const int ni = min(TE, a.R - ti * TE), nj = min(TE, a.R - tj * TE);
    atomicAdd(&a.test_counter[item & (kProfSlots - 1)], (unsigned long long)((k1 - k0) * (int64_t)(ni * nj)));
    atomicAdd(&a.test_counter[kProfSlots + (item & (kProfSlots - 1))],
              (unsigned long long)(kRecBytes * (k1 - k0) + (int64_t)sizeof(WorkItem)));
  }
  int64_t lane_sum = 0;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int32_t q = valid[r] ? (int32_t)(acc[r] - nbias) : 0;
    lane_sum += q;
    if (STATS && valid[r]) {
      const int i = ti * TE + (r % NB) * 8 + (lane & 7);
      const int j = tj * TE + (r / NB) * 8 + (lane >> 3);
      const int64_t o = ((int64_t)bw * a.R + i) * a.R + j;
      if (a.ray_q) atomicAdd(&a.ray_q[o], q);
      if (a.ray_hits) atomicAdd(&a.ray_hits[o], hits[r]);
    }
  }
  if (OCC && valid[0]) {
    const int i = ti * TE + (lane & 7), j = tj * TE + (lane >> 3);
    const bool mirror = a.side[bw] != 0;
    float* o = a.occ + (((int64_t)b * 8 + i) * 8 + j) * 8;
    for (int k = 0; k < 8; ++k) atomicAdd(&o[mirror ? 7 - k : k], occ_acc[k] * (1.0f / 524288.0f));
  }
  // wave reduction of the 64 lane sums, one 64-bit atomic per wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lane_sum += __shfl_xor(lane_sum, off);
  if (lane == 0 && lane_sum != 0) atomicAdd(&a.acc[bw], (unsigned long long)lane_sum);
}

// Rasterising ray test of 16 x 16-ray tiles.  Each lane takes one record and
// tests only the rays of the cells its projected bounding box covers (the same
// conservative cell range the binning used); a record covering more than
// kRasterCells cells of the tile is tested by the whole wave instead, one covered
// cell per lane.  A crossing inside the triangle adds q = bits(y) - 0x4B400000
// (the fixed-point inside length, as in k_test) to its ray's integer sum in LDS,
// so the sums are exact and independent of the order.
constexpr int kRasterCells = 64;  // default; raster_cells_choice()

__device__ inline bool ray_hit(float u, float v, const float4& r0, const float4& r1, const float4& r2,
                               const float4& r3, int32_t& q) {
  const float e0 = __fmaf_rn(r0.x, u, __fmaf_rn(r0.y, v, r0.z));
  const float e1 = __fmaf_rn(r0.w, u, __fmaf_rn(r1.x, v, r1.y));
  const float e2 = __fmaf_rn(r1.z, u, __fmaf_rn(r1.w, v, r2.x));
  const float mn = fminf(fminf(e0, e1), e2);
  const float y = __fmaf_rn(r2.y, u, __fmaf_rn(r2.z, v, r2.w));
  const float c = __builtin_amdgcn_fmed3f(y, r3.x, r3.y);
  q = (int32_t)(__float_as_uint(c) - kMagicBits);
  return mn >= 0.0f;
}

template <bool STATS, bool TAB>
__device__ void raster_item(const TestArgs& a, const int64_t item) {
  const int TT = a.tpe * a.tpe;
  // the whole item in one request, its (uniform) words moved to scalar
  // registers before any branch (an item exists only for a tile with bin
  // entries, so its axis is one the call casts)
  WorkItem wi;  // ray grid, tile, bin entries
  {
    const uint4* src = reinterpret_cast<const uint4*>(a.items + item);
    uint4 q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = src[k];
    uint32_t d[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      d[4 * k + 0] = __builtin_amdgcn_readfirstlane(q[k].x);
      d[4 * k + 1] = __builtin_amdgcn_readfirstlane(q[k].y);
      d[4 * k + 2] = __builtin_amdgcn_readfirstlane(q[k].z);
      d[4 * k + 3] = __builtin_amdgcn_readfirstlane(q[k].w);
    }
    __builtin_memcpy(&wi, d, sizeof(wi));
  }
  const int g = wi.g;
  const int bw = g / TT;
  const int tile = g - bw * TT;
  const int w = bw - 3 * (bw / 3);
  const int lane = threadIdx.x;
  const int64_t k0 = wi.k0;
  const int64_t k1 = k0 + wi.count;
  if (k1 > a.bin_cap) return;  // bins past a planned capacity were not written (flagged)
  // (boxes whose state is not 0 get no records, hence no ray-test work items)
  const double hu = wi.hu, hv = wi.hv, du = wi.du, dv = wi.dv;
  const int ti = tile % a.tpe, tj = tile / a.tpe;
  const int ci_lo = ti * 16, cj_lo = tj * 16;
  __shared__ float2 sray[256];
  __shared__ int32_t sacc[256];
  __shared__ int32_t shit[STATS ? 256 : 1];
  __shared__ float4 srec[kTestThreads][kRecF4];  // a chunk's records, for the wave-wide path
  bool valid[4];
  // Ray r = lane + 64 k sits in cell (ci_lo + lane % 16, cj_lo + lane / 16 + 4 k):
  // its u draw has state s0 + 2 ((i << 15) + j) GAMMA = z + 8 k GAMMA, where z
  // is the lane's k = 0 state, and its v draw one GAMMA more.
  // With a jitter table (TAB) the two draws of every ray are read from it instead
  // (the same 24-bit values, computed once per key by jitter_table).
  const int i = ci_lo + (lane & 15);
  const uint32_t t0 = ((uint32_t)i << 15) + (uint32_t)(cj_lo + (lane >> 4));
  const uint64_t z0 = wi.s0 + (uint64_t)t0 * (2ull * kGamma);
  uint2 jq[4];
  if (TAB) {  // unconditional, clamped reads: the counters of outstanding loads stay exact
    const uint2* jt = a.jitter + ((int64_t)wi.key * 3 + w) * (int64_t)a.R * a.R;
    const int ic = min(i, a.R - 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) jq[k] = jt[(int64_t)min(cj_lo + (lane >> 4) + 4 * k, a.R - 1) * a.R + ic];
  }
  auto make_ray = [&](int k) {
    const int r = lane + 64 * k;
    const int j = cj_lo + (r >> 4);
    valid[k] = i < a.R && j < a.R;
    float ru = 0.f, rv = 0.f;
    if (valid[k]) {
      double xi, eta;
      if (TAB) {
        xi = (double)jq[k].x * (1.0 / 16777216.0);
        eta = (double)jq[k].y * (1.0 / 16777216.0);
      } else {
        const uint64_t zu = z0 + (uint64_t)k * (8ull * kGamma);
        xi = u24(mix64(zu));
        eta = u24(mix64(zu + kGamma));
      }
      ru = (float)__dadd_rn(-hu, __dmul_rn(__dadd_rn((double)i, xi), du));
      rv = (float)__dadd_rn(-hv, __dmul_rn(__dadd_rn((double)j, eta), dv));
    }
    sray[r] = make_float2(ru, rv);
    sacc[r] = 0;
    if (STATS) shit[r] = 0;
  };
  // The item's first kTestThreads records (contiguous, one 64-byte line each)
  // are requested before the rays are generated.  The load is unconditional
  // (lanes past the item's records read its last one), so the counters of
  // outstanding loads stay exact.  An item holds at least one record.
  const bool have0 = lane < k1 - k0;
  const float4* rp0 = a.recs + kRecF4 * (k0 + min((int64_t)lane, k1 - k0 - 1));
  const float4 p0 = rp0[0], p1 = rp0[1], p2 = rp0[2], p3 = rp0[3];
  __builtin_amdgcn_sched_barrier(0);
  make_ray(0);
  make_ray(1);
  make_ray(2);
  make_ray(3);
  __syncthreads();
  int64_t tests = 0;
  {
    for (int64_t base = k0; base < k1; base += kTestThreads) {
      const int n = (int)min((int64_t)kTestThreads, k1 - base);
      bool have = lane < n, big = false;
      float4 q0, q1, q2, q3;
      if (base == k0) {
        have = have0;
        q0 = p0;
        q1 = p1;
        q2 = p2;
        q3 = p3;
      } else if (have) {
        const float4* rp = a.recs + kRecF4 * (base + lane);
        q0 = rp[0];
        q1 = rp[1];
        q2 = rp[2];
        q3 = rp[3];
      }
      if (have) {
        // the binning's cell range inside this tile, stored with the entry
        const uint32_t pk = __float_as_uint(q3.w);
        const int c0 = ci_lo + (int)(pk & 15u), c1 = ci_lo + (int)((pk >> 4) & 15u);
        const int d0 = cj_lo + (int)((pk >> 8) & 15u), d1 = cj_lo + (int)((pk >> 12) & 15u);
        const int cells = (c1 >= c0 && d1 >= d0) ? (c1 - c0 + 1) * (d1 - d0 + 1) : 0;
        big = cells > a.raster_cells;
        if (!big) {
          tests += cells;
          // one flat loop over the covered cells (row by row), so the wave runs
          // as many iterations as its lane with the most cells
          const int wdt = c1 - c0 + 1;
          int r = (c0 - ci_lo) + 16 * (d0 - cj_lo), di = 0;
          for (int t = 0; t < cells; ++t) {
            const float2 p = sray[r];
            int32_t q;
            if (ray_hit(p.x, p.y, q0, q1, q2, q3, q)) {
              atomicAdd(&sacc[r], q);
              if (STATS) atomicAdd(&shit[r], 1);
            }
            ++di;
            const bool wrap = di == wdt;
            r += wrap ? 17 - wdt : 1;
            di = wrap ? 0 : di;
          }
        }
      }
      // records covering many cells: the whole wave, one covered cell per lane
      // (the record read by every lane from LDS)
      uint64_t bm = __ballot(have && big);
      if (bm) {
        if (have) {
          srec[lane][0] = q0;
          srec[lane][1] = q1;
          srec[lane][2] = q2;
          srec[lane][3] = q3;
        }
        __syncthreads();
      }
      while (bm) {
        const int src = __ffsll((long long)bm) - 1;
        bm &= bm - 1;
        const float4 s0 = srec[src][0], s1 = srec[src][1], s2 = srec[src][2], s3 = srec[src][3];
        const uint32_t pk = __float_as_uint(s3.w);
        const int c0 = (int)(pk & 15u), d0 = (int)((pk >> 8) & 15u);
        const int wdt = (int)((pk >> 4) & 15u) - c0 + 1, cells = wdt * ((int)((pk >> 12) & 15u) - d0 + 1);
        // row of covered cell t: floor((t + 1/2) / wdt), exact for t < 256 with
        // the approximate reciprocal
        const float iw = __builtin_amdgcn_rcpf((float)wdt);
        for (int t = lane; t < cells; t += kTestThreads) {
          const int dj = (int)(((float)t + 0.5f) * iw), di = t - dj * wdt;
          const int r = (c0 + di) + 16 * (d0 + dj);
          const float2 p = sray[r];
          int32_t q;
          if (ray_hit(p.x, p.y, s0, s1, s2, s3, q)) {
            atomicAdd(&sacc[r], q);
            if (STATS) atomicAdd(&shit[r], 1);
          }
        }
        tests += lane == 0 ? (int64_t)cells : 0;
      }
      if (base + kTestThreads < k1) __syncthreads();  // srec is rewritten by the next chunk
    }
  }
  __syncthreads();
  int64_t lane_sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!valid[k]) continue;
    const int r = lane + 64 * k;
    const int32_t q = sacc[r];
    lane_sum += q;
    if (STATS) {
      const int i = ci_lo + (r & 15), j = cj_lo + (r >> 4);
      const int64_t o = ((int64_t)bw * a.R + i) * a.R + j;
      if (a.ray_q) atomicAdd(&a.ray_q[o], q);
      if (a.ray_hits) atomicAdd(&a.ray_hits[o], shit[r]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lane_sum += __shfl_xor(lane_sum, off);
    tests += __shfl_xor(tests, off);
  }
  if (lane == 0 && lane_sum != 0) atomicAdd(&a.acc[bw], (unsigned long long)lane_sum);
  if (lane == 0 && a.test_counter) {
    atomicAdd(&a.test_counter[item & (kProfSlots - 1)], (unsigned long long)tests);
    atomicAdd(&a.test_counter[kProfSlots + (item & (kProfSlots - 1))],
              (unsigned long long)(kRecBytes * (k1 - k0) + (int64_t)sizeof(WorkItem) +
                                   (TAB ? 8 * min(16, a.R - ci_lo) * min(16, a.R - cj_lo) : 0)));
  }
}

template <bool STATS, bool TAB>
__global__ void __launch_bounds__(kTestThreads) k_raster(TestArgs a) {
  if (!a.persistent) {
    raster_item<STATS, TAB>(a, xcd_remap(blockIdx.x, gridDim.x));
    return;
  }
  const int64_t total = min(a.chunk_off[a.n_tiles], a.item_cap);
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    raster_item<STATS, TAB>(a, item);
    __syncthreads();  // LDS of the next item
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
  int64_t* out;  // nullable: mapped host memory [status, records, bin entries, work items, done]
  const int64_t* rec;
  const int64_t* bin;
  const int64_t* items;
  uint32_t* done;  // blocks finished (zeroed by k_box_chunks)
};

__device__ void finalize_box(const obbv_box* __restrict__ boxes, int b, int R, uint32_t axis_mask,
                             const unsigned long long* __restrict__ acc, double* __restrict__ out_obv,
                             double* __restrict__ out_vin_axis, uint32_t* status);

// float64 OBV per box; the last block to finish publishes the call's status bits
// and totals to the caller's mapped host memory, then out[4] = 1 with a
// system-scope release: a host that sees it sees every output of the call.
__global__ void k_finalize(const obbv_box* __restrict__ boxes, int n_boxes, int R, uint32_t axis_mask,
                           const unsigned long long* __restrict__ acc, double* __restrict__ out_obv,
                           double* __restrict__ out_vin_axis, uint32_t* status, Publish pub) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_boxes) finalize_box(boxes, b, R, axis_mask, acc, out_obv, out_vin_axis, status);
  if (!pub.out) return;
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    if (atomicAdd(pub.done, 1u) == gridDim.x - 1) {
      __threadfence();
      pub.out[0] = (int64_t)atomicOr(status, 0u);
      pub.out[1] = *pub.rec;
      pub.out[2] = *pub.bin;
      pub.out[3] = *pub.items;
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

struct HostPinned {
  int64_t* p = nullptr;
};
HostPinned g_pinned[64];

int pinned_totals(int64_t** out) {
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return OBBV_ERR_UNSUPPORTED;
  if (!g_pinned[dev].p) {
    void* q = nullptr;
    OBBV_HIP(hipHostMalloc(&q, 64, hipHostMallocDefault));
    g_pinned[dev].p = (int64_t*)q;
  }
  *out = g_pinned[dev].p;
  return OBBV_OK;
}

}  // namespace

namespace {

bool test_raster_choice();
int test_chunk_choice();
int raster_cells_choice();
int write_lds_choice();

template <int TE>
int launch_test(const TestArgs& ta, int64_t nblocks, bool stats, bool stage, hipStream_t s) {
  const dim3 g((unsigned)nblocks), b(kTestThreads);
  if (TE == 16 && !ta.occ && test_raster_choice()) {
    if (stats)
      hipLaunchKernelGGL((k_raster<true, false>), g, b, 0, s, ta);
    else if (ta.jitter)
      hipLaunchKernelGGL((k_raster<false, true>), g, b, 0, s, ta);
    else
      hipLaunchKernelGGL((k_raster<false, false>), g, b, 0, s, ta);
  } else if (ta.occ && TE == 8)
    hipLaunchKernelGGL((k_test<TE, false, true, true>), g, b, 0, s, ta);
  else if (stats && stage)
    hipLaunchKernelGGL((k_test<TE, true, true, false>), g, b, 0, s, ta);
  else if (stats)
    hipLaunchKernelGGL((k_test<TE, true, false, false>), g, b, 0, s, ta);
  else if (stage)
    hipLaunchKernelGGL((k_test<TE, false, true, false>), g, b, 0, s, ta);
  else
    hipLaunchKernelGGL((k_test<TE, false, false, false>), g, b, 0, s, ta);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

// Record loading of the ray-test loop: 1 = LDS staging (default), 0 = scalar
// loads in batches of four.  OBBV_TEST_STAGE overrides it (used to compare the
// two on a device; staging measured faster).
// Ray tests of 16 x 16 tiles: 1 = rasterising kernel (default), 0 = every ray of
// the tile against every record.  OBBV_TEST_RASTER overrides it.
bool test_raster_choice() {
  const char* e = getenv("OBBV_TEST_RASTER");
  if (e && *e) return atoi(e) != 0;
  return true;
}

// Records per ray-test work item: kTestChunk, or OBBV_TEST_CHUNK (64..4096, a
// multiple of 64) to compare work-item sizes on a device.
int test_chunk_choice() {
  const char* e = getenv("OBBV_TEST_CHUNK");
  if (e && *e) {
    const int c = atoi(e);
    if (c >= 64 && c <= 4096 && c % 64 == 0) return c;
  }
  return kTestChunk;
}

// Cells above which a record of a tile is tested by the whole wave:
// kRasterCells, or OBBV_RASTER_CELLS (0..256) to compare thresholds on a device.
int raster_cells_choice() {
  const char* e = getenv("OBBV_RASTER_CELLS");
  if (e && *e) {
    const int c = atoi(e);
    if (c >= 0 && c <= 256) return c;
  }
  return kRasterCells;
}

// Write pass bin slots: 1 = per-tile ranges reserved from LDS counts (default),
// 0 = one global atomic per entry.  OBBV_WRITE_LDS overrides it.
int write_lds_choice() {
  const char* e = getenv("OBBV_WRITE_LDS");
  if (e && *e) return atoi(e) != 0;
  return 1;
}

bool test_stage_choice() {
  const char* e = getenv("OBBV_TEST_STAGE");
  if (e && *e) return atoi(e) != 0;
  return true;
}

}  // namespace

// Boxes grouped by shared centre and axes (device arrays; one mesh only).
struct SharedFrames {
  const obbv_box* frames;    // [n_frames] centre, axes and the largest half extents of the group
  const int32_t* box_frame;  // [n_boxes] group of every box
  int32_t n_frames;
};

int outer_volume_run(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                     const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                     const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                     int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side, hipStream_t s,
                     float* out_occ, OvExec* ex, const SharedFrames* sf = nullptr) {
  OBBV_ARG(params != nullptr, "params is NULL");
  OBBV_ARG(n_boxes >= 0, "n_boxes < 0");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(meshes != nullptr && n_meshes >= 1, "need at least one mesh");
  OBBV_ARG(boxes != nullptr && out_obv != nullptr, "boxes / out_obv is NULL");
  OBBV_ARG(n_meshes == 1 || box_mesh != nullptr, "box_mesh is required with several meshes");
  OBBV_ARG(params->R >= 1 && params->R <= 32767, "R must be in [1, 32767]");
  OBBV_ARG(params->flags == 0, "flags must be 0");
  const int pool_base = ex ? ex->pool_base : 0;
  OBBV_ARG(params->tile == 0 || params->tile == 8 || params->tile == 16, "tile must be 0, 8 or 16");
  const uint32_t mask = params->axis_mask ? params->axis_mask : 7u;
  OBBV_ARG(mask <= 7u, "axis_mask has bits above 2");
  OBBV_ARG((int64_t)n_boxes * 3 < (1ll << 31) / 2, "too many boxes");
  int max_nt = 0;
  std::vector<MeshDev> mh((size_t)n_meshes);
  for (int m = 0; m < n_meshes; ++m) {
    OBBV_ARG(meshes[m].n_triangles >= 0 && meshes[m].n_vertices >= 0, "negative mesh size");
    OBBV_ARG(meshes[m].n_triangles == 0 || (meshes[m].triangles && meshes[m].vertices),
             "mesh pointers are NULL");
    mh[m] = MeshDev{meshes[m].vertices, meshes[m].triangles, meshes[m].n_vertices, meshes[m].n_triangles};
    max_nt = std::max(max_nt, meshes[m].n_triangles);
  }
  const int R = params->R;
  const int TE = out_occ ? 8 : (params->tile ? params->tile : (R >= 48 ? 16 : 8));
  const bool planned = ex && ex->planned;
  const bool capped = ex && ex->capped && !planned;
  const bool fixed = planned || capped;  // scratch capacities fixed: no host round trip
  OBBV_ARG(!out_occ || (R == 8 && mask == 4u), "occupancy needs R = 8 and axis_mask = 4");
  OBBV_ARG(!sf || (n_meshes == 1 && !planned && sf->n_frames >= 1 && sf->n_frames <= n_boxes),
           "shared frames need one mesh, an unplanned call and 1..n_boxes frames");
  const int n_frames = sf ? sf->n_frames : 0;
  const int tpe = ceil_div(R, TE);
  const int64_t TT = (int64_t)tpe * tpe;
  const int64_t nbw = (int64_t)n_boxes * 3;
  OBBV_ARG(nbw * TT < (1ll << 31), "R too large for this many boxes in one call");

  uint32_t* status = nullptr;
  OBBV_RET(status_word(&status));
  if (ex && ex->status) status = ex->status;

  // ---- meta scratch layout ----
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t o_mesh = take(sizeof(MeshDev) * n_meshes);
  const size_t o_done = take(4);
  const size_t o_blist = take(4 * (size_t)(sf ? n_boxes : 0));
  const size_t o_choff = take(8 * (size_t)(n_boxes + 1));
  const size_t o_side = take(4 * (size_t)nbw);
  const size_t o_reccnt = take(4 * (size_t)nbw);
  const size_t o_recoff = take(8 * (size_t)(nbw + 1));
  const size_t o_binoff = take(8 * (size_t)(nbw * TT + 1));
  const size_t o_chunkoff = take(8 * (size_t)(nbw * TT + 1));
  const size_t o_tilecnt = take(4 * (size_t)(nbw * TT));  // written by k_box_sides
  const size_t o_tc2 = take(8 * (size_t)(nbw * TT));  // a plan's two-sided tile counters (unused otherwise)
  const size_t o_bincur = take(4 * (size_t)(nbw * TT));   // zeroed by k_box_sides
  const size_t o_acc = take(8 * (size_t)nbw);             // zeroed by k_box_sides
  const size_t o_rframe = take(sizeof(RayFrame) * (size_t)nbw);  // written by k_box_sides
  const size_t o_fcnt = take(4 * (size_t)n_frames);
  const size_t o_foff = take(8 * (size_t)(n_frames + 1));
  const size_t scan_bytes =
      std::max({exclusive_scan_scratch_bytes(n_frames), (size_t)16 * (ceil_div(nbw * TT, kScanBlockThreads) + 1)});
  const size_t o_scan = take(scan_bytes);
  void* meta_v = nullptr;
  if (planned) {
    if (off > ex->meta_cap) {
      set_error("planned scratch too small for this call");
      return OBBV_ERR_WORKSPACE;
    }
    meta_v = ex->meta;
  } else {
    OBBV_RET(pool_get(pool_base + kPoolMeta, off, &meta_v));
  }
  if (ex) ex->meta_bytes = off;
  char* meta = (char*)meta_v;
  MeshDev* d_mesh = (MeshDev*)(meta + o_mesh);
  uint32_t* d_done = (uint32_t*)(meta + o_done);
  int64_t* d_choff = (int64_t*)(meta + o_choff);
  int32_t* d_side = (int32_t*)(meta + o_side);
  int32_t* d_reccnt = (int32_t*)(meta + o_reccnt);
  int64_t* d_recoff = (int64_t*)(meta + o_recoff);
  int64_t* d_binoff = (int64_t*)(meta + o_binoff);
  int64_t* d_chunkoff = (int64_t*)(meta + o_chunkoff);
  int32_t* d_tilecnt = (int32_t*)(meta + o_tilecnt);
  int32_t* d_bincur = (int32_t*)(meta + o_bincur);
  unsigned long long* d_acc = (unsigned long long*)(meta + o_acc);
  RayFrame* d_rframe = (RayFrame*)(meta + o_rframe);
  int32_t* d_blist = sf ? (int32_t*)(meta + o_blist) : nullptr;
  int32_t* d_fcnt = (int32_t*)(meta + o_fcnt);
  int64_t* d_foff = (int64_t*)(meta + o_foff);
  void* d_scan = meta + o_scan;

  // per-item counts and offsets of the cull passes (every entry is written)
  const int64_t items_bound = (int64_t)n_boxes * ceil_div(std::max(max_nt, 1), kCullThreads);
  const int64_t fitems = sf ? (int64_t)n_frames * ceil_div(std::max(meshes[0].n_triangles, 1), kCullThreads) : 0;
  const size_t items_bytes = align_up(24 * (size_t)items_bound) + align_up(sizeof(ItemInfo) * (size_t)items_bound) +
                             2 * align_up(4 * (size_t)fitems);
  char* items = nullptr;
  if (planned) {
    if (items_bytes > ex->items_cap) {
      set_error("planned scratch too small for this call");
      return OBBV_ERR_WORKSPACE;
    }
    items = ex->items;
  } else {
    void* iv = nullptr;
    OBBV_RET(pool_get(pool_base + kPoolItems, items_bytes, &iv));
    items = (char*)iv;
  }
  if (ex) ex->items_bytes = items_bytes;
  int32_t* d_icnt = (int32_t*)items;
  ItemInfo* d_iteminfo = (ItemInfo*)(items + align_up(24 * (size_t)items_bound));  // [items_bound] every cull item
  int32_t* d_ficnt = (int32_t*)((char*)d_iteminfo + align_up(sizeof(ItemInfo) * (size_t)items_bound));
  int32_t* d_fioff = (int32_t*)((char*)d_ficnt + align_up(4 * (size_t)fitems));

  // the mesh table goes to the device only with several meshes (one mesh travels
  // in the kernel arguments)
  if (!planned && n_meshes > 1)
    OBBV_HIP(hipMemcpyAsync(d_mesh, mh.data(), sizeof(MeshDev) * n_meshes, hipMemcpyHostToDevice, s));
  const MeshDev* d_meshes = n_meshes > 1 ? (const MeshDev*)d_mesh : nullptr;

  float4* d_listP = nullptr;
  if (sf) {  // candidate triangles of every shared frame
    const int nt = meshes[0].n_triangles;
    const int nch = ceil_div(std::max(nt, 1), kCullThreads);
    const unsigned fgrid = (unsigned)std::min<int64_t>((int64_t)n_frames * nch, 256 * 16);
    hipLaunchKernelGGL(k_frame_cull, dim3(fgrid), dim3(kCullThreads), 0, s, sf->frames, n_frames, mh[0], mask,
                       nch, d_ficnt, (const int32_t*)nullptr, (const int64_t*)nullptr, (float4*)nullptr, status);
    OBBV_HIP(hipGetLastError());
    if ((int64_t)n_frames * nch <= ((int64_t)1 << 20)) {  // one block: item and frame offsets
      hipLaunchKernelGGL(k_frame_scan, dim3(1), dim3(kScanBlockThreads), 0, s, (const int32_t*)d_ficnt, n_frames,
                         nch, d_fioff, d_fcnt, d_foff);
      OBBV_HIP(hipGetLastError());
    } else {
      hipLaunchKernelGGL(k_frame_scan, dim3(ceil_div(n_frames, kCullWaves)), dim3(kCullThreads), 0, s,
                         (const int32_t*)d_ficnt, n_frames, nch, d_fioff, d_fcnt, (int64_t*)nullptr);
      OBBV_HIP(hipGetLastError());
      OBBV_RET(exclusive_scan_i32_to_i64(d_fcnt, d_foff, n_frames, d_scan, scan_bytes, s));
    }
    int64_t bound = (int64_t)n_frames * nt;
    if (bound * 48 > ((int64_t)1 << 31)) {  // large: size the lists exactly (one host round trip)
      int64_t* pin = nullptr;
      OBBV_RET(pinned_totals(&pin));
      OBBV_HIP(hipMemcpyAsync(pin + 3, d_foff + n_frames, 8, hipMemcpyDeviceToHost, s));
      OBBV_HIP(hipStreamSynchronize(s));
      bound = pin[3];
    }
    void* lv = nullptr;
    OBBV_RET(pool_get(pool_base + kPoolLists, (size_t)std::max<int64_t>(bound, 1) * 48, &lv));
    d_listP = (float4*)lv;
    hipLaunchKernelGGL(k_frame_cull, dim3(fgrid), dim3(kCullThreads), 0, s, sf->frames, n_frames, mh[0], mask,
                       nch, d_ficnt, (const int32_t*)d_fioff, (const int64_t*)d_foff, d_listP, status);
    OBBV_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_box_chunks, dim3(1), dim3(kScanBlockThreads), 0, s, box_mesh, d_meshes, mh[0],
                     n_meshes, n_boxes, boxes, sf ? sf->frames : nullptr, sf ? sf->box_frame : nullptr, n_frames,
                     (const int64_t*)d_foff, d_blist, d_choff, d_done, status, box_key, R, params->seed, d_rframe,
                     n_boxes <= kItemBoxMax && items_bound < ((int64_t)1 << 31) ? d_iteminfo : (ItemInfo*)nullptr);
  OBBV_HIP(hipGetLastError());

  CullArgs ca;
  ca.item_info = n_boxes <= kItemBoxMax && items_bound < ((int64_t)1 << 31) ? d_iteminfo : nullptr;
  ca.write_lds = write_lds_choice();
  ca.boxes = boxes;
  ca.box_mesh = box_mesh;
  ca.meshes = d_meshes;
  ca.mesh0 = mh[0];
  ca.rframe = d_rframe;
  ca.chunk_off = d_choff;
  ca.n_boxes = n_boxes;
  ca.R = R;
  ca.TE = TE;
  ca.tpe = tpe;
  ca.axis_mask = mask;
  ca.status = status;
  ca.rec_cap = fixed ? ex->rec_cap : INT64_MAX;
  ca.bin_cap = fixed ? ex->bin_cap : INT64_MAX;
  ca.list_P = d_listP;
  ca.list_off = sf ? d_foff : nullptr;
  ca.box_list = d_blist;
  const unsigned cull_grid = (unsigned)std::min<int64_t>(items_bound, 256 * 16);

  // both sides' tile counters: zero on entry, left zero by k_box_sides (a plan
  // keeps its own block in the meta scratch, zeroed at creation)
  int32_t* d_tc2 = nullptr;
  if (planned) {
    d_tc2 = (int32_t*)(meta + o_tc2);
  } else {
    void* tcv = nullptr;
    OBBV_RET(pool_get_zeroed(pool_base + kPoolTileCnt2, 8 * (size_t)nbw * TT, &tcv));
    d_tc2 = (int32_t*)tcv;
  }
  hipLaunchKernelGGL(k_cull_count, dim3(cull_grid), dim3(kCullThreads), 0, s, ca, d_icnt, d_tc2);
  OBBV_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_box_sides, dim3(ceil_div(nbw, kCullWaves)), dim3(kCullThreads), 0, s,
                     (const int64_t*)d_choff, n_boxes, (const int32_t*)d_icnt, d_side, d_reccnt, (int)TT,
                     d_tilecnt, d_bincur, d_acc, d_tc2);
  OBBV_HIP(hipGetLastError());
  // bin and work-item offsets of the tiles, record offsets of the (box, axis) pairs
  const int chunk = test_chunk_choice();
  if (nbw * TT <= kTilesScanOne) {
    hipLaunchKernelGGL(k_tiles_scan_one, dim3(1), dim3(kScanBlockThreads), 0, s, (const int32_t*)d_tilecnt, nbw * TT,
                       chunk, d_binoff, d_chunkoff, (const int32_t*)d_reccnt, nbw, d_recoff);
    OBBV_HIP(hipGetLastError());
  } else {
    const int64_t nt_all = nbw * TT;
    const int64_t nb = ceil_div(nt_all, kScanBlockThreads);
    int64_t* bsum = (int64_t*)d_scan;
    hipLaunchKernelGGL(k_tiles_scan_block, dim3((unsigned)nb), dim3(kScanBlockThreads), 0, s,
                       (const int32_t*)d_tilecnt, nt_all, chunk, d_binoff, d_chunkoff, bsum);
    OBBV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tiles_scan_top, dim3(1), dim3(kScanBlockThreads), 0, s, bsum, nb, nt_all, d_binoff,
                       d_chunkoff, (const int32_t*)d_reccnt, nbw, d_recoff);
    OBBV_HIP(hipGetLastError());
    if (nb > 1) {
      hipLaunchKernelGGL(k_tiles_scan_add, dim3((unsigned)nb), dim3(kScanBlockThreads), 0, s, nt_all,
                         (const int64_t*)bsum, d_binoff, d_chunkoff);
      OBBV_HIP(hipGetLastError());
    }
  }

  int64_t n_rec, n_bin, n_items;
  if (fixed) {  // no host round trip: capacities were fixed beforehand
    n_rec = ex->rec_cap;
    n_bin = ex->bin_cap;
    n_items = ex->item_cap;
  } else {
    int64_t* pin = nullptr;
    OBBV_RET(pinned_totals(&pin));
    OBBV_HIP(hipMemcpyAsync(pin + 0, d_recoff + nbw, 8, hipMemcpyDeviceToHost, s));
    OBBV_HIP(hipMemcpyAsync(pin + 1, d_binoff + nbw * TT, 8, hipMemcpyDeviceToHost, s));
    OBBV_HIP(hipMemcpyAsync(pin + 2, d_chunkoff + nbw * TT, 8, hipMemcpyDeviceToHost, s));
    OBBV_HIP(hipStreamSynchronize(s));
    n_rec = pin[0];
    n_bin = pin[1];
    n_items = pin[2];
    if (ex) {
      ex->n_rec = n_rec;
      ex->n_bin = n_bin;
      ex->n_items = n_items;
    }
  }
  OBBV_ARG(n_items < (1ll << 31), "too many ray-test work items in one call; split the boxes");
  OBBV_ARG(n_rec < (1ll << 31), "more than 2^31 triangle records in one call; split the boxes");

  if (n_rec > 0) {
    void* recs_v = nullptr;
    if (fixed)
      recs_v = ex->recs;
    else
      OBBV_RET(pool_get(pool_base + kPoolRecords, (size_t)std::max<int64_t>(n_bin, 1) * kRecBytes, &recs_v));
    WorkItem* itile = nullptr;
    if (fixed) {
      itile = ex->itile;
    } else {
      void* tv = nullptr;
      OBBV_RET(pool_get(pool_base + kPoolTiles, (size_t)std::max<int64_t>(n_items, 1) * sizeof(WorkItem), &tv));
      itile = (WorkItem*)tv;
    }
    const size_t write_lds = ca.write_lds && 3 * TT <= kLdsTiles ? (size_t)(3 * TT) * 20 : 0;
    hipLaunchKernelGGL(k_write, dim3(cull_grid), dim3(kCullThreads), write_lds, s, ca, d_side, d_binoff, d_bincur,
                       (float4*)recs_v, (const int64_t*)d_chunkoff, nbw * TT,
                       n_items > 0 ? itile : (WorkItem*)nullptr, n_items, chunk);
    OBBV_HIP(hipGetLastError());
    TestArgs ta;
    ta.boxes = boxes;
    ta.box_key = box_key;
    ta.bin_off = d_binoff;
    ta.chunk_off = d_chunkoff;
    ta.n_tiles = nbw * TT;
    ta.chunk = chunk;
    ta.raster_cells = raster_cells_choice();
    ta.recs = (const float4*)recs_v;
    ta.acc = d_acc;
    ta.ray_q = out_ray_q;
    ta.ray_hits = out_ray_hits;
    ta.test_counter = nullptr;
    ta.occ = out_occ;
    ta.side = d_side;
    ta.bin_cap = fixed ? ex->bin_cap : INT64_MAX;
    ta.item_cap = fixed ? ex->item_cap : INT64_MAX;
    ta.items = itile;
    ta.persistent = fixed ? 1 : 0;
    ta.jitter = ex && ex->jitter && R == ex->jitter_R && params->seed == ex->jitter_seed ? ex->jitter : nullptr;
    void* prof_token = nullptr;
    if (profiling_enabled() && !planned) {
      OBBV_RET(profile_counter(&ta.test_counter));
      OBBV_RET(profile_record_begin(s, &prof_token));
    }
    ta.seed = params->seed;
    ta.n_boxes = n_boxes;
    ta.R = R;
    ta.tpe = tpe;
    ta.axis_mask = mask;
    const bool stats = out_ray_q || out_ray_hits;
    if (stats) {
      const size_t per = (size_t)nbw * R * R * 4;
      if (out_ray_q) OBBV_HIP(hipMemsetAsync(out_ray_q, 0, per, s));
      if (out_ray_hits) OBBV_HIP(hipMemsetAsync(out_ray_hits, 0, per, s));
    }
    if (n_items > 0) {
      const bool stage = test_stage_choice();
      const int64_t grid = fixed ? std::min<int64_t>(n_items, 256 * 32) : n_items;
      if (TE == 8)
        OBBV_RET(launch_test<8>(ta, grid, stats, stage, s));
      else
        OBBV_RET(launch_test<16>(ta, grid, stats, stage, s));
    }
    if (profiling_enabled() && !planned) OBBV_RET(profile_record_end(s, prof_token));
  } else if (out_ray_q || out_ray_hits) {
    const size_t per = (size_t)nbw * R * R * 4;
    if (out_ray_q) OBBV_HIP(hipMemsetAsync(out_ray_q, 0, per, s));
    if (out_ray_hits) OBBV_HIP(hipMemsetAsync(out_ray_hits, 0, per, s));
  }
  if (out_side) OBBV_HIP(hipMemcpyAsync(out_side, d_side, 4 * nbw, hipMemcpyDeviceToDevice, s));
  Publish pub{ex ? ex->publish : nullptr, d_recoff + nbw, d_binoff + nbw * TT, d_chunkoff + nbw * TT, d_done};
  hipLaunchKernelGGL(k_finalize, dim3(ceil_div(n_boxes, 128)), dim3(128), 0, s, boxes, n_boxes, R, mask,
                     (const unsigned long long*)d_acc, out_obv, out_vin_axis, status, pub);
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
                      float* out_occ) {
  return outer_volume_run(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv, out_vin_axis,
                          out_ray_q, out_ray_hits, out_side, s, out_occ, nullptr);
}

}  // namespace obbv

extern "C" int obbv_outer_volume_grouped(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
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

extern "C" int obbv_outer_volume_ex(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                    const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                    const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                                    int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side,
                                    void* stream) {
  obbv::clear_error();
  return obbv::outer_volume_impl(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv,
                                 out_vin_axis, out_ray_q, out_ray_hits, out_side, (hipStream_t)stream, nullptr);
}

extern "C" int obbv_outer_volume(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                 const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                 const obbv_ov_params* params, double* out_obv, void* stream) {
  obbv::clear_error();
  return obbv::outer_volume_impl(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, params, out_obv,
                                 nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream, nullptr);
}

// ---------------------------------------------------------------------------
// surrogate input rows: 15 normalised box parameters + 8 x 8 x 8 occupancy
// ---------------------------------------------------------------------------
namespace obbv {
namespace {
__global__ void k_features(const obbv_box* __restrict__ boxes, const int32_t* __restrict__ box_mesh, int n_meshes,
                           const float* __restrict__ frame, const float* __restrict__ occ, int n,
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
      v = occ[(int64_t)b * 512 + (k - 15)];
    x[k] = v;
  }
}
}  // namespace
}  // namespace obbv

extern "C" int obbv_box_features(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
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
  float* occ = (float*)q;
  double* obv = (double*)(occ + (size_t)n_boxes * 512);
  OBBV_HIP(hipMemsetAsync(occ, 0, (size_t)n_boxes * 512 * 4, s));
  obbv_ov_params p{8, 4u, seed, 8, 0u};
  OBBV_RET(outer_volume_impl(meshes, n_meshes, boxes, box_mesh, nullptr, n_boxes, &p, obv, nullptr, nullptr, nullptr,
                             nullptr, s, occ));
  hipLaunchKernelGGL(k_features, dim3((unsigned)n_boxes), dim3(128), 0, s, boxes, box_mesh, n_meshes, mesh_frame, occ,
                     n_boxes, out_X);
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
__global__ void k_scatter_volume(const float* __restrict__ occ, int nb, float* __restrict__ vol) {
  const int64_t n = (int64_t)nb * nb * nb * 512;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t box = t / 512;
  const int r = (int)(t % 512);
  const int x = r / 64, y = (r / 8) % 8, z = r % 8;
  const int bx = (int)(box % nb), by = (int)((box / nb) % nb), bz = (int)(box / ((int64_t)nb * nb));
  const int64_t N = 8 * nb;
  vol[((int64_t)(8 * bz + z) * N + (8 * by + y)) * N + (8 * bx + x)] = occ[t];
}

}  // namespace
}  // namespace obbv

extern "C" int obbv_occupancy_volume(const obbv_mesh* mesh, int32_t nb, const float* frame, uint64_t seed,
                                     float* out_volume, void* stream) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(mesh && frame && out_volume, "NULL argument");
  OBBV_ARG(nb >= 1 && nb <= 64, "nb must be in [1, 64]");
  hipStream_t s = (hipStream_t)stream;
  const int n = nb * nb * nb;
  void* q = nullptr;
  OBBV_RET(pool_get(kPoolFeat, (size_t)n * (512 * 4 + 8 + sizeof(obbv_box)) + 1024, &q));
  float* occ = (float*)q;
  double* obv = (double*)(occ + (size_t)n * 512);
  obbv_box* tb = (obbv_box*)(obv + n);
  OBBV_HIP(hipMemsetAsync(occ, 0, (size_t)n * 512 * 4, s));
  hipLaunchKernelGGL(k_tiling_boxes, dim3(ceil_div(n, 128)), dim3(128), 0, s, frame, nb, tb);
  OBBV_HIP(hipGetLastError());
  obbv_ov_params p{8, 4u, seed, 8, 0u};
  OBBV_RET(outer_volume_impl(mesh, 1, tb, nullptr, nullptr, n, &p, obv, nullptr, nullptr, nullptr, nullptr, s, occ));
  hipLaunchKernelGGL(k_scatter_volume, dim3(ceil_div((int64_t)n * 512, 256)), dim3(256), 0, s, occ, nb, out_volume);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// planned evaluations: autotuned tile size, fixed scratch, HIP graph replay
// ---------------------------------------------------------------------------
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

namespace obbv {
namespace {

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
  float tuned_ms[2] = {0.f, 0.f};
};

// autotuner cache: (device, R, boxes bucket, triangles bucket) -> tile edge
std::map<std::tuple<int, int, int, int>, int> g_tile_cache;
std::mutex g_tile_mutex;

inline int bucket(int64_t x) {
  int b = 0;
  while (x > 1) {
    x >>= 1;
    ++b;
  }
  return b;
}

int time_tile(OvPlanState& P, int tile, hipStream_t s, float* ms) {
  obbv_ov_params p = P.params;
  p.tile = tile;
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

extern "C" int obbv_ov_plan_create(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                                   const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                                   const obbv_ov_params* params, double* out_obv, double headroom, void* stream,
                                   obbv_ov_plan** out) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(out && meshes && params && boxes && out_obv, "NULL argument");
  OBBV_ARG(n_boxes >= 1 && n_meshes >= 1, "need boxes and meshes");
  OBBV_ARG(headroom >= 1.0, "headroom must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<OvPlanState> P(new OvPlanState());
  P->meshes.assign(meshes, meshes + n_meshes);
  P->boxes = boxes;
  P->box_mesh = box_mesh;
  P->box_key = box_key;
  P->n_boxes = n_boxes;
  P->params = *params;
  P->out_obv = out_obv;
  // autotune the ray tile edge (8: one ray per lane, 16: four rays per lane)
  if (P->params.tile == 0) {
    int dev = 0;
    OBBV_HIP(hipGetDevice(&dev));
    int64_t ntri = 0;
    for (int m = 0; m < n_meshes; ++m) ntri += meshes[m].n_triangles;
    const auto key = std::make_tuple(dev, P->params.R, bucket(n_boxes), bucket(ntri / n_meshes));
    int tile = 0;
    {
      std::lock_guard<std::mutex> lock(g_tile_mutex);
      auto it = g_tile_cache.find(key);
      if (it != g_tile_cache.end()) tile = it->second;
    }
    if (!tile) {
      OBBV_RET(time_tile(*P, 8, s, &P->tuned_ms[0]));
      OBBV_RET(time_tile(*P, 16, s, &P->tuned_ms[1]));
      tile = P->tuned_ms[0] <= P->tuned_ms[1] ? 8 : 16;
      std::lock_guard<std::mutex> lock(g_tile_mutex);
      g_tile_cache[key] = tile;
    }
    P->params.tile = tile;
  }
  // size the scratch with one synchronous evaluation
  OvExec probe;
  OBBV_RET(outer_volume_run(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, &P->params, out_obv, nullptr,
                            nullptr, nullptr, nullptr, s, nullptr, &probe));
  OBBV_HIP(hipStreamSynchronize(s));
  OvExec& ex = P->ex;
  ex.planned = true;
  ex.meta_cap = probe.meta_bytes;
  ex.rec_cap = (int64_t)std::ceil((double)probe.n_rec * headroom) + 1024;
  ex.bin_cap = (int64_t)std::ceil((double)probe.n_bin * headroom) + 4096;
  ex.item_cap = (int64_t)std::ceil((double)probe.n_items * headroom) + 64;
  ex.items_cap = probe.items_bytes;
  const size_t bytes = align_up(ex.meta_cap) + align_up((size_t)ex.bin_cap * kRecBytes) + align_up(ex.items_cap) +
                       align_up((size_t)ex.item_cap * sizeof(WorkItem));
  if (hipMalloc(&P->alloc, bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of the planned scratch failed");
    return OBBV_ERR_OOM;
  }
  OBBV_HIP(hipMemset(P->alloc, 0, bytes));  // counters that every launch leaves zero start zero
  ex.meta = (char*)P->alloc;
  ex.recs = (float4*)(ex.meta + align_up(ex.meta_cap));
  ex.items = (char*)ex.recs + align_up((size_t)ex.bin_cap * kRecBytes);
  ex.itile = (WorkItem*)(ex.items + align_up(ex.items_cap));
  // the mesh table lives at the start of the meta block (outside the graph)
  std::vector<MeshDev> mh((size_t)n_meshes);
  for (int m = 0; m < n_meshes; ++m)
    mh[m] = MeshDev{meshes[m].vertices, meshes[m].triangles, meshes[m].n_vertices, meshes[m].n_triangles};
  OBBV_HIP(hipMemcpy(ex.meta, mh.data(), sizeof(MeshDev) * n_meshes, hipMemcpyHostToDevice));
  uint32_t* st = nullptr;
  OBBV_RET(status_word(&st));
  // capture one evaluation on a private stream
  hipStream_t cs = nullptr;
  OBBV_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  OBBV_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int rc = outer_volume_run(meshes, n_meshes, boxes, box_mesh, box_key, n_boxes, &P->params, out_obv, nullptr,
                            nullptr, nullptr, nullptr, cs, nullptr, &ex);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
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
  *out = reinterpret_cast<obbv_ov_plan*>(P.release());
  return OBBV_OK;
}

extern "C" int obbv_ov_plan_launch(obbv_ov_plan* plan, void* stream) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(plan, "NULL plan");
  OvPlanState* P = reinterpret_cast<OvPlanState*>(plan);
  OBBV_HIP(hipGraphLaunch(P->exec, (hipStream_t)stream));
  return OBBV_OK;
}

extern "C" int obbv_ov_plan_info(obbv_ov_plan* plan, int32_t* out_tile, int64_t* out_caps, float* out_tuned_ms) {
  using namespace obbv;
  clear_error();
  OBBV_ARG(plan, "NULL plan");
  OvPlanState* P = reinterpret_cast<OvPlanState*>(plan);
  if (out_tile) *out_tile = P->params.tile;
  if (out_caps) {
    out_caps[0] = P->ex.rec_cap;
    out_caps[1] = P->ex.bin_cap;
    out_caps[2] = P->ex.item_cap;
  }
  if (out_tuned_ms) {
    out_tuned_ms[0] = P->tuned_ms[0];
    out_tuned_ms[1] = P->tuned_ms[1];
  }
  return OBBV_OK;
}

extern "C" int obbv_ov_plan_destroy(obbv_ov_plan* plan) {
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
