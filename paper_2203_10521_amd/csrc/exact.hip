// Exact outer volume of oriented boxes (Sec. 3, Eq. 4), the evaluator without
// quadrature: along one local axis w of a box, the divergence theorem turns the
// solid's volume inside the box into a sum over triangles of the integral, over
// the triangle's projection clipped to the box face, of the clamped inside
// length.  Per (box, triangle), in float64: the projected triangle is clipped to
// the face rectangle (Sutherland-Hodgman, depth carried along the clipped
// edges), split by the slab planes w = +h and w = -h; the piece above the slab
// counts its area times the slab height 2h, the piece inside the slab the
// integral of (w + h), the piece below nothing; the sign is the orientation of
// the projected triangle.  Sums run in a fixed order (bitwise deterministic).
#include <algorithm>

#include "common.h"

// Built with -ffp-contract=off (build.py): every operation rounds on its own,
// in the order the oracle follows.

namespace obbv {
namespace {

constexpr int kExactThreads = 256;
constexpr int kExactPerThread = 16;                             // triangles of a thread in one block
constexpr int kExactChunk = kExactThreads * kExactPerThread;  // triangles of one block
constexpr int kPolyMax = 10;  // a triangle clipped by 4 planes has <= 7 vertices, then <= 9

struct P3 {
  double u, v, w;
};

// The affine functions the polygons are clipped by (each >= 0 is kept):
// 0: x + h, 1: h - x, 2: x - h, of coordinate c (0 = u, 1 = v, 2 = w).
__device__ inline double plane(const P3& p, int c, int kind, double h) {
  const double x = c == 0 ? p.u : (c == 1 ? p.v : p.w);
  return kind == 0 ? __dadd_rn(x, h) : (kind == 1 ? __dsub_rn(h, x) : __dsub_rn(x, h));
}

// Sutherland-Hodgman: the part of the convex polygon in[0..n) where the plane
// function is >= 0; new vertices interpolate all three coordinates.
__device__ inline int clip(const P3* in, int n, P3* out, int c, int kind, double h) {
  int m = 0;
  for (int k = 0; k < n; ++k) {
    const P3 p = in[k], q = in[k + 1 < n ? k + 1 : 0];
    const double gp = plane(p, c, kind, h), gq = plane(q, c, kind, h);
    if (gp >= 0.0) out[m++] = p;
    if ((gp > 0.0 && gq < 0.0) || (gp < 0.0 && gq > 0.0)) {
      const double t = __ddiv_rn(gp, __dsub_rn(gp, gq));
      out[m].u = __dadd_rn(p.u, __dmul_rn(t, __dsub_rn(q.u, p.u)));
      out[m].v = __dadd_rn(p.v, __dmul_rn(t, __dsub_rn(q.v, p.v)));
      out[m].w = __dadd_rn(p.w, __dmul_rn(t, __dsub_rn(q.w, p.w)));
      ++m;
    }
  }
  return m;
}

// twice the signed area of the projection of (p, q, r) on (u, v)
__device__ inline double area2(const P3& p, const P3& q, const P3& r) {
  return __dsub_rn(__dmul_rn(__dsub_rn(q.u, p.u), __dsub_rn(r.v, p.v)),
                   __dmul_rn(__dsub_rn(q.v, p.v), __dsub_rn(r.u, p.u)));
}

// (area, integral of w) of a convex planar polygon by a fan from vertex 0
__device__ inline void fan(const P3* poly, int n, double& area, double& wint) {
  area = 0.0;
  wint = 0.0;
  for (int k = 1; k + 1 < n; ++k) {
    const double a = __ddiv_rn(fabs(area2(poly[0], poly[k], poly[k + 1])), 2.0);
    area = __dadd_rn(area, a);
    wint = __dadd_rn(wint, __ddiv_rn(__dmul_rn(a, __dadd_rn(__dadd_rn(poly[0].w, poly[k].w), poly[k + 1].w)), 3.0));
  }
}

// The signed inside-length integral of one triangle (cast-frame coordinates).
__device__ double triangle_inside(const P3& a, const P3& b, const P3& c, double hu, double hv, double hw) {
  const double s2 = area2(a, b, c);
  if (s2 == 0.0) return 0.0;
  P3 A[kPolyMax], B[kPolyMax];
  A[0] = a;
  A[1] = b;
  A[2] = c;
  int n = clip(A, 3, B, 0, 0, hu);
  if (n < 3) return 0.0;
  n = clip(B, n, A, 0, 1, hu);
  if (n < 3) return 0.0;
  n = clip(A, n, B, 1, 0, hv);
  if (n < 3) return 0.0;
  n = clip(B, n, A, 1, 1, hv);
  if (n < 3) return 0.0;
  double total = 0.0, area, wint;
  bool on_top = true;
  for (int k = 0; k < n; ++k) on_top = on_top && A[k].w == hw;
  if (on_top) {  // in the plane w = +h: one piece, inside over the whole slab
    fan(A, n, area, wint);
    total = __dmul_rn(__dmul_rn(2.0, hw), area);
  } else {
    P3 C[kPolyMax];
    const int nt = clip(A, n, B, 2, 2, hw);  // above the slab
    if (nt >= 3) {
      fan(B, nt, area, wint);
      total = __dadd_rn(total, __dmul_rn(__dmul_rn(2.0, hw), area));
    }
    int nm = clip(A, n, C, 2, 1, hw);  // below the top ...
    if (nm >= 3) {
      nm = clip(C, nm, B, 2, 0, hw);  // ... and above the bottom
      if (nm >= 3) {
        fan(B, nm, area, wint);
        total = __dadd_rn(total, __dadd_rn(wint, __dmul_rn(hw, area)));
      }
    }
  }
  return s2 > 0.0 ? total : -total;
}

struct ExactBox {
  double c[3], Q[9], h[3];
  bool ok;
};

__device__ inline ExactBox exact_box(const obbv_box* __restrict__ boxes, int b) {
  ExactBox B;
  const float* p = reinterpret_cast<const float*>(boxes + b);
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    B.c[k] = p[k];
    ok = ok && isfinite(p[k]);
  }
  for (int k = 0; k < 9; ++k) {
    B.Q[k] = p[3 + k];
    ok = ok && isfinite(p[3 + k]);
  }
  for (int k = 0; k < 3; ++k) {
    B.h[k] = p[12 + k];
    ok = ok && isfinite(p[12 + k]) && p[12 + k] >= 0.f;
  }
  B.ok = ok;
  return B;
}

// Partial inside volumes: block (chunk, box) sums the contributions of its
// kExactChunk triangles (each thread its 16 in index order, then a fixed tree
// over the block) into part[box * n_chunks + chunk].
__global__ void __launch_bounds__(kExactThreads)
k_exact_partial(const obbv_box* __restrict__ boxes, int axis, MeshDev M, int n_chunks, double* __restrict__ part,
                uint32_t* status) {
  __shared__ double red[kExactThreads];
  const int chunk = blockIdx.x, b = blockIdx.y;
  const ExactBox B = exact_box(boxes, b);
  const int ua = (axis + 1) % 3, va = (axis + 2) % 3;
  const double hu = B.h[ua], hv = B.h[va], hw = B.h[axis];
  double sum = 0.0;
  // a flat box holds no volume: its OBV is 0 (not the rounding of degenerate pieces)
  if (B.ok && hu > 0.0 && hv > 0.0 && hw > 0.0) {
    for (int k = 0; k < kExactPerThread; ++k) {
      const int64_t t = (int64_t)chunk * kExactChunk + (int64_t)k * kExactThreads + threadIdx.x;
      if (t >= M.nt) break;
      const int32_t* f = M.F + 3 * t;
      const int i0 = f[0], i1 = f[1], i2 = f[2];
      if ((unsigned)i0 >= (unsigned)M.nv || (unsigned)i1 >= (unsigned)M.nv || (unsigned)i2 >= (unsigned)M.nv) {
        atomicOr(status, OBBV_STATUS_BAD_INDEX);
        continue;
      }
      const int vi[3] = {i0, i1, i2};
      P3 P[3];
      double lo_u = INFINITY, hi_u = -INFINITY, lo_v = INFINITY, hi_v = -INFINITY, hi_w = -INFINITY;
      for (int q = 0; q < 3; ++q) {
        const float* x = M.V + 3 * (int64_t)vi[q];
        const double d0 = __dsub_rn((double)x[0], B.c[0]), d1 = __dsub_rn((double)x[1], B.c[1]),
                     d2 = __dsub_rn((double)x[2], B.c[2]);
        double l[3];
        for (int r = 0; r < 3; ++r)
          l[r] = __dadd_rn(__dadd_rn(__dmul_rn(d0, B.Q[3 * r]), __dmul_rn(d1, B.Q[3 * r + 1])),
                           __dmul_rn(d2, B.Q[3 * r + 2]));
        P[q].u = l[ua];
        P[q].v = l[va];
        P[q].w = l[axis];
        lo_u = fmin(lo_u, P[q].u);
        hi_u = fmax(hi_u, P[q].u);
        lo_v = fmin(lo_v, P[q].v);
        hi_v = fmax(hi_v, P[q].v);
        hi_w = fmax(hi_w, P[q].w);
      }
      // triangles off the face or below the slab contribute exactly nothing
      if (hi_u >= -hu && lo_u <= hu && hi_v >= -hv && lo_v <= hv && hi_w > -hw)
        sum = __dadd_rn(sum, triangle_inside(P[0], P[1], P[2], hu, hv, hw));
    }
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int off = kExactThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = __dadd_rn(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)b * n_chunks + chunk] = red[0];
}

// OBV of every box: V_box minus its partial sums taken in chunk order.
__global__ void k_exact_final(const obbv_box* __restrict__ boxes, int n_boxes, int n_chunks,
                              const double* __restrict__ part, double* __restrict__ out_obv, uint32_t* status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_boxes) return;
  const ExactBox B = exact_box(boxes, b);
  if (!B.ok) {
    out_obv[b] = __longlong_as_double(0x7ff8000000000000ll);
    atomicOr(status, OBBV_STATUS_NAN_BOX);
    return;
  }
  double inside = 0.0;
  for (int c = 0; c < n_chunks; ++c) inside = __dadd_rn(inside, part[(int64_t)b * n_chunks + c]);
  const double vbox = __dmul_rn(__dmul_rn(__dmul_rn(8.0, B.h[0]), B.h[1]), B.h[2]);
  out_obv[b] = __dsub_rn(vbox, inside);
}

}  // namespace

int outer_volume_exact(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t axis,
                       double* out_obv, hipStream_t s) {
  OBBV_ARG(mesh && (n_boxes == 0 || (boxes && out_obv)), "NULL argument");
  OBBV_ARG(n_boxes >= 0, "n_boxes < 0");
  OBBV_ARG(axis >= 0 && axis <= 2, "axis must be 0, 1 or 2");
  OBBV_ARG(mesh->n_triangles >= 0 && mesh->n_vertices >= 0, "negative mesh size");
  OBBV_ARG(mesh->n_triangles == 0 || (mesh->triangles && mesh->vertices), "mesh pointers are NULL");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(n_boxes <= 65535, "at most 65,535 boxes per exact call");
  uint32_t* status = nullptr;
  OBBV_RET(status_word(&status));
  const MeshDev M{mesh->vertices, mesh->triangles, mesh->n_vertices, mesh->n_triangles};
  const int n_chunks = std::max(1, ceil_div(M.nt, kExactChunk));
  void* p = nullptr;
  OBBV_RET(pool_get(kPoolExact, sizeof(double) * (size_t)n_boxes * n_chunks, &p));
  double* part = (double*)p;
  hipLaunchKernelGGL(k_exact_partial, dim3((unsigned)n_chunks, (unsigned)n_boxes), dim3(kExactThreads), 0, s, boxes,
                     axis, M, n_chunks, part, status);
  OBBV_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_exact_final, dim3((unsigned)ceil_div(n_boxes, 128)), dim3(128), 0, s, boxes, n_boxes, n_chunks,
                     (const double*)part, out_obv, status);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

}  // namespace obbv

static int obbv_outer_volume_exact_body(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t axis,
                                       double* out_obv, void* stream);
extern "C" int obbv_outer_volume_exact(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t axis,
                                       double* out_obv, void* stream) {
  return obbv::guarded([&] { return obbv_outer_volume_exact_body(mesh, boxes, n_boxes, axis, out_obv, stream); });
}
static int obbv_outer_volume_exact_body(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t axis,
                                       double* out_obv, void* stream) {
  obbv::clear_error();
  return obbv::outer_volume_exact(mesh, boxes, n_boxes, axis, out_obv, (hipStream_t)stream);
}
