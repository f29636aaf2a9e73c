// The paper's central-projection estimator of the outer volume (Sec. 4.1,
// Eq. 9-10), the variant of the hot step that casts from the box centre: rays
// through the pixel centres of a 6 x m x m cube map in the box frame, one cone
// of directions per pixel (its exact solid angle W).  Along the ray t d the box
// is left at t_e = min_k h_k / |d_k|; a crossing of the mesh at t > 0 counts
// s = +1 when the ray leaves the solid (outward normal . d > 0), -1 when it
// enters; the cone's outer volume is (r_e^3 - sum_k s_k min(r_k, r_e)^3) W / 3
// with r = t |d| (the crossings beyond the box count as reaching it).
// Crossings come from a watertight test (the ray's largest axis made z,
// vertices sheared onto the ray, three 2-D edge functions; Woop, Benthin and
// Wald 2013) with one owner for points on a shared edge (an oriented edge
// function equal to 0 passes only on a top-left edge).  float64 throughout,
// one fixed order of operations; sums in a fixed order.
#include <algorithm>
#include <cstdlib>

#include "common.h"

// Built with -ffp-contract=off (build.py): every operation rounds on its own,
// in the order the oracle follows.

namespace obbv {
namespace {

constexpr int kCentralThreads = 256;  // rays of a block
constexpr int kCentralTile = 256;     // triangles staged in LDS per step

__device__ inline double cube(double x) { return __dmul_rn(__dmul_rn(x, x), x); }

// the solid angle helper of a pixel corner: atan(a b / sqrt(1 + a^2 + b^2))
__device__ inline double corner(double a, double b) {
  return atan(__ddiv_rn(__dmul_rn(a, b), sqrt(__dadd_rn(__dadd_rn(1.0, __dmul_rn(a, a)), __dmul_rn(b, b)))));
}

// edge p -> q of a counter-clockwise 2-D triangle owns its points when it runs
// left horizontally or downwards
__device__ inline bool topleft(double px, double py, double qx, double qy) {
  const double dx = __dsub_rn(qx, px), dy = __dsub_rn(qy, py);
  return dy < 0.0 || (dy == 0.0 && dx < 0.0);
}

__device__ inline double pick(const double v[3], int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

__global__ void __launch_bounds__(kCentralThreads)
k_central_partial(const obbv_box* __restrict__ boxes, MeshDev M, int m, int n_chunks, int cull,
                  double* __restrict__ part, uint32_t* status) {
  __shared__ double sT[12][kCentralTile];  // A, B, C (box frame), outward normal
  __shared__ int32_t sIdx[kCentralTile];   // the tile's triangles that may be hit, in triangle order
  __shared__ int32_t sWc[kCentralTile / 64];
  __shared__ double red[kCentralThreads];
  const int chunk = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const float* bp = reinterpret_cast<const float*>(boxes + b);
  double c[3], Q[9], h[3];
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    c[k] = bp[k];
    ok = ok && isfinite(bp[k]);
  }
  for (int k = 0; k < 9; ++k) {
    Q[k] = bp[3 + k];
    ok = ok && isfinite(bp[3 + k]);
  }
  for (int k = 0; k < 3; ++k) {
    h[k] = bp[12 + k];
    ok = ok && isfinite(bp[12 + k]) && bp[12 + k] >= 0.f;
  }
  const int n_rays = 6 * m * m;
  const int p = chunk * kCentralThreads + tid;
  const bool ray = ok && p < n_rays;
  // the pixel's direction, solid angle, exit depth and shear
  double d[3] = {0.0, 0.0, 0.0}, W = 0.0, re = 0.0, dn = 1.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
  int kx = 0, ky = 1, kz = 2;
  if (ray) {
    const int face = p / (m * m), rem = p - face * m * m;
    const int i = rem / m, j = rem - (rem / m) * m;
    const double md = (double)m;
    const double a = __dadd_rn(-1.0, __ddiv_rn(__dadd_rn(2.0 * i, 1.0), md));
    const double bb = __dadd_rn(-1.0, __ddiv_rn(__dadd_rn(2.0 * j, 1.0), md));
    const double a0 = __dadd_rn(-1.0, __ddiv_rn(2.0 * i, md)), a1 = __dadd_rn(-1.0, __ddiv_rn(2.0 * (i + 1), md));
    const double b0 = __dadd_rn(-1.0, __ddiv_rn(2.0 * j, md)), b1 = __dadd_rn(-1.0, __ddiv_rn(2.0 * (j + 1), md));
    W = __dadd_rn(__dsub_rn(__dsub_rn(corner(a1, b1), corner(a0, b1)), corner(a1, b0)), corner(a0, b0));
    const int axis = face / 2;
    d[axis] = (face & 1) ? -1.0 : 1.0;
    d[(axis + 1) % 3] = a;
    d[(axis + 2) % 3] = bb;
    double te = INFINITY;
    for (int k = 0; k < 3; ++k)
      if (d[k] != 0.0) te = fmin(te, __ddiv_rn(h[k], fabs(d[k])));
    dn = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(d[0], d[0]), __dmul_rn(d[1], d[1])), __dmul_rn(d[2], d[2])));
    re = __dmul_rn(te, dn);
    kz = 0;
    if (fabs(d[1]) > fabs(d[kz])) kz = 1;
    if (fabs(d[2]) > fabs(d[kz])) kz = 2;
    kx = (kz + 1) % 3;
    ky = (kz + 2) % 3;
    if (d[kz] < 0.0) {
      const int t = kx;
      kx = ky;
      ky = t;
    }
    Sx = __ddiv_rn(pick(d, kx), pick(d, kz));
    Sy = __ddiv_rn(pick(d, ky), pick(d, kz));
    Sz = __ddiv_rn(1.0, pick(d, kz));
  }
  // The block's rays lie in the pyramid of directions over its pixels of one
  // face (a in [a_lo, a_hi] along face axis + 1, b in [b_lo, b_hi] along axis
  // + 2, sigma = +-x[axis] > 0), half a pixel inside its sides.  A triangle
  // whose three vertices lie beyond one side (or behind the centre) by more
  // than 1e-9 of their coordinates holds no point of any ray at t > 0, so it
  // adds no crossing and is skipped: the sum is unchanged, bit for bit.
  // Blocks spanning two faces cull nothing.
  const int p0 = chunk * kCentralThreads, p1 = min(p0 + kCentralThreads, n_rays) - 1;
  const int mm = m * m;
  const bool pyr = cull != 0 && ok && p0 / mm == p1 / mm;
  const int pface = p0 / mm, paxis = pface / 2;
  const double psg = (pface & 1) ? -1.0 : 1.0;
  double a_lo = 0.0, a_hi = 0.0, b_lo = 0.0, b_hi = 0.0;
  if (pyr) {
    const int r0 = p0 - pface * mm, r1 = p1 - pface * mm;
    const int i0 = r0 / m, i1 = r1 / m;
    const int j0 = i0 == i1 ? r0 - i0 * m : 0, j1 = i0 == i1 ? r1 - i1 * m : m - 1;
    const double md = (double)m;
    a_lo = __dadd_rn(-1.0, __ddiv_rn(2.0 * i0, md));
    a_hi = __dadd_rn(-1.0, __ddiv_rn(2.0 * (i1 + 1), md));
    b_lo = __dadd_rn(-1.0, __ddiv_rn(2.0 * j0, md));
    b_hi = __dadd_rn(-1.0, __ddiv_rn(2.0 * (j1 + 1), md));
  }
  double sum = 0.0;  // sum_k s_k min(r_k, r_e)^3, crossings in triangle order
  for (int t0 = 0; t0 < M.nt; t0 += kCentralTile) {
    __syncthreads();
    {
      const int t = t0 + tid;
      int good = 0;
      if (ok && t < M.nt) {
        const int32_t* f = M.F + 3 * (int64_t)t;
        const int vi[3] = {f[0], f[1], f[2]};
        if ((unsigned)vi[0] >= (unsigned)M.nv || (unsigned)vi[1] >= (unsigned)M.nv ||
            (unsigned)vi[2] >= (unsigned)M.nv) {
          atomicOr(status, OBBV_STATUS_BAD_INDEX);
        } else {
          double L[3][3];
          for (int q = 0; q < 3; ++q) {
            const float* x = M.V + 3 * (int64_t)vi[q];
            const double d0 = __dsub_rn((double)x[0], c[0]), d1 = __dsub_rn((double)x[1], c[1]),
                         d2 = __dsub_rn((double)x[2], c[2]);
            for (int r = 0; r < 3; ++r)
              L[q][r] = __dadd_rn(__dadd_rn(__dmul_rn(Q[3 * r], d0), __dmul_rn(Q[3 * r + 1], d1)),
                                  __dmul_rn(Q[3 * r + 2], d2));
          }
          for (int q = 0; q < 3; ++q)
            for (int r = 0; r < 3; ++r) sT[3 * q + r][tid] = L[q][r];
          const double e1[3] = {__dsub_rn(L[1][0], L[0][0]), __dsub_rn(L[1][1], L[0][1]), __dsub_rn(L[1][2], L[0][2])};
          const double e2[3] = {__dsub_rn(L[2][0], L[0][0]), __dsub_rn(L[2][1], L[0][1]), __dsub_rn(L[2][2], L[0][2])};
          sT[9][tid] = __dsub_rn(__dmul_rn(e1[1], e2[2]), __dmul_rn(e1[2], e2[1]));
          sT[10][tid] = __dsub_rn(__dmul_rn(e1[2], e2[0]), __dmul_rn(e1[0], e2[2]));
          sT[11][tid] = __dsub_rn(__dmul_rn(e1[0], e2[1]), __dmul_rn(e1[1], e2[0]));
          good = 1;
          if (pyr) {
            // sides of the pyramid (value > 0: outside), and behind the centre
            int out = 0x1f;
            for (int q = 0; q < 3; ++q) {
              const double sg = __dmul_rn(psg, pick(L[q], paxis));
              const double xa = pick(L[q], (paxis + 1) % 3), xb = pick(L[q], (paxis + 2) % 3);
              const double tol = __dmul_rn(1e-9, __dadd_rn(__dadd_rn(fabs(sg), fabs(xa)), fabs(xb)));
              int o = 0;
              if (-sg > tol) o |= 1;
              if (__dsub_rn(xa, __dmul_rn(a_hi, sg)) > tol) o |= 2;
              if (__dsub_rn(__dmul_rn(a_lo, sg), xa) > tol) o |= 4;
              if (__dsub_rn(xb, __dmul_rn(b_hi, sg)) > tol) o |= 8;
              if (__dsub_rn(__dmul_rn(b_lo, sg), xb) > tol) o |= 16;
              out &= o;
            }
            if (out) good = 0;
          }
        }
      }
      // compact the tile's kept triangles, in triangle order
      const uint64_t mk = __ballot(good != 0);
      const int lane = tid & 63, wv = tid >> 6;
      if (lane == 0) sWc[wv] = (int)__popcll(mk);
      __syncthreads();
      int pos = (int)__popcll(mk & ((1ull << lane) - 1ull));
      for (int v = 0; v < wv; ++v) pos += sWc[v];
      if (good) sIdx[pos] = tid;
    }
    __syncthreads();
    if (!ray) continue;
    int nk = 0;
    for (int v = 0; v < kCentralTile / 64; ++v) nk += sWc[v];
    for (int kk = 0; kk < nk; ++kk) {
      const int k = sIdx[kk];
      const double Akz = sT[kz][k], Bkz = sT[3 + kz][k], Ckz = sT[6 + kz][k];
      const double Ax = __dsub_rn(sT[kx][k], __dmul_rn(Sx, Akz)), Ay = __dsub_rn(sT[ky][k], __dmul_rn(Sy, Akz));
      const double Bx = __dsub_rn(sT[3 + kx][k], __dmul_rn(Sx, Bkz)), By = __dsub_rn(sT[3 + ky][k], __dmul_rn(Sy, Bkz));
      const double Cx = __dsub_rn(sT[6 + kx][k], __dmul_rn(Sx, Ckz)), Cy = __dsub_rn(sT[6 + ky][k], __dmul_rn(Sy, Ckz));
      const double U = __dsub_rn(__dmul_rn(Cx, By), __dmul_rn(Cy, Bx));
      const double V = __dsub_rn(__dmul_rn(Ax, Cy), __dmul_rn(Ay, Cx));
      const double Wf = __dsub_rn(__dmul_rn(Bx, Ay), __dmul_rn(By, Ax));
      const double det = __dadd_rn(__dadd_rn(U, V), Wf);
      if (det == 0.0) continue;
      const bool flip = det < 0.0;
      const double Uo = flip ? -U : U, Vo = flip ? -V : V, Wo = flip ? -Wf : Wf;
      const bool tlU = flip ? topleft(Cx, Cy, Bx, By) : topleft(Bx, By, Cx, Cy);
      const bool tlV = flip ? topleft(Ax, Ay, Cx, Cy) : topleft(Cx, Cy, Ax, Ay);
      const bool tlW = flip ? topleft(Bx, By, Ax, Ay) : topleft(Ax, Ay, Bx, By);
      if (!((Uo > 0.0 || (Uo == 0.0 && tlU)) && (Vo > 0.0 || (Vo == 0.0 && tlV)) && (Wo > 0.0 || (Wo == 0.0 && tlW))))
        continue;
      const double tnum = __dadd_rn(__dadd_rn(__dmul_rn(U, __dmul_rn(Sz, Akz)), __dmul_rn(V, __dmul_rn(Sz, Bkz))),
                                    __dmul_rn(Wf, __dmul_rn(Sz, Ckz)));
      const double t = __ddiv_rn(tnum, det);
      if (!(t > 0.0)) continue;
      const double nd = __dadd_rn(__dadd_rn(__dmul_rn(sT[9][k], d[0]), __dmul_rn(sT[10][k], d[1])),
                                  __dmul_rn(sT[11][k], d[2]));
      if (nd == 0.0) continue;
      const double cu = cube(fmin(__dmul_rn(t, dn), re));
      sum = __dadd_rn(sum, nd > 0.0 ? cu : -cu);
    }
  }
  red[tid] = ray ? __ddiv_rn(__dmul_rn(__dsub_rn(cube(re), sum), W), 3.0) : 0.0;
  __syncthreads();
  for (int off = kCentralThreads / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] = __dadd_rn(red[tid], red[tid + off]);
    __syncthreads();
  }
  if (tid == 0) part[(int64_t)b * n_chunks + chunk] = red[0];
}

__global__ void k_central_final(const obbv_box* __restrict__ boxes, int n_boxes, int n_chunks,
                                const double* __restrict__ part, double* __restrict__ out_obv, uint32_t* status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_boxes) return;
  const float* bp = reinterpret_cast<const float*>(boxes + b);
  bool ok = true;
  for (int k = 0; k < 15; ++k) ok = ok && isfinite(bp[k]);
  for (int k = 12; k < 15; ++k) ok = ok && bp[k] >= 0.f;
  if (!ok) {
    out_obv[b] = __longlong_as_double(0x7ff8000000000000ll);
    atomicOr(status, OBBV_STATUS_NAN_BOX);
    return;
  }
  double v = 0.0;
  for (int c = 0; c < n_chunks; ++c) v = __dadd_rn(v, part[(int64_t)b * n_chunks + c]);
  out_obv[b] = v;
}

}  // namespace

int outer_volume_central(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t m, double* out_obv,
                         hipStream_t s) {
  OBBV_ARG(mesh && (n_boxes == 0 || (boxes && out_obv)), "NULL argument");
  OBBV_ARG(n_boxes >= 0, "n_boxes < 0");
  OBBV_ARG(m >= 1 && m <= 256, "m must be in [1, 256]");
  OBBV_ARG(mesh->n_triangles >= 0 && mesh->n_vertices >= 0, "negative mesh size");
  OBBV_ARG(mesh->n_triangles == 0 || (mesh->triangles && mesh->vertices), "mesh pointers are NULL");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(n_boxes <= 65535, "at most 65,535 boxes per central-projection call");
  uint32_t* status = nullptr;
  OBBV_RET(status_word(&status));
  const MeshDev M{mesh->vertices, mesh->triangles, mesh->n_vertices, mesh->n_triangles};
  const int n_chunks = ceil_div(6 * m * m, kCentralThreads);
  void* p = nullptr;
  OBBV_RET(pool_get(kPoolCentral, sizeof(double) * (size_t)n_boxes * n_chunks, &p));
  double* part = (double*)p;
  // OBBV_CENTRAL_CULL=0 tests every triangle against every ray (same bits)
  const char* e = getenv("OBBV_CENTRAL_CULL");
  const int cull = (e && *e && atoi(e) == 0) ? 0 : 1;
  hipLaunchKernelGGL(k_central_partial, dim3((unsigned)n_chunks, (unsigned)n_boxes), dim3(kCentralThreads), 0, s,
                     boxes, M, m, n_chunks, cull, part, status);
  OBBV_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_central_final, dim3((unsigned)ceil_div(n_boxes, 128)), dim3(128), 0, s, boxes, n_boxes,
                     n_chunks, (const double*)part, out_obv, status);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

}  // namespace obbv

static int obbv_outer_volume_central_body(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t m,
                                         double* out_obv, void* stream);
extern "C" int obbv_outer_volume_central(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t m,
                                         double* out_obv, void* stream) {
  return obbv::guarded([&] { return obbv_outer_volume_central_body(mesh, boxes, n_boxes, m, out_obv, stream); });
}
static int obbv_outer_volume_central_body(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t m,
                                         double* out_obv, void* stream) {
  obbv::clear_error();
  return obbv::outer_volume_central(mesh, boxes, n_boxes, m, out_obv, (hipStream_t)stream);
}
