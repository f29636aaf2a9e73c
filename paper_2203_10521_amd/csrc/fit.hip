// Covariance OBB per triangle cluster.
//
// The box of a cluster is fixed by its centre and axes, its extents by
// enclosing the cluster (Sec. 4.2.1); the axes are the principal directions of
// the cluster's surface (area-weighted covariance of the triangles, the PCA
// split named among top-down builders in Sec. 2).
//
// Every sum is exact and so independent of the order in which threads add: a
// cluster's terms are converted to 64-bit fixed point with a power-of-two scale
// 2^k chosen per cluster so that its total stays below 2^62 (k from per-cluster
// maxima, themselves order-independent), and summed with integer atomics.
//
//   k_fit_bounds  per triangle: count_c += 1, max area, max |vertex coordinate|
//   k_fit_mean    per triangle: S_c += A_T, M_c += A_T m_T (fixed point; terms at
//                 most max area, resp. max area x max |coordinate|)
//   k_fit_dev     per triangle: max over its vertices of |v_d - mu_c,d|
//   k_fit_cov     per triangle: C_c += A_T E_T[(x - mu)(x - mu)^T] with
//                 E_T[y y^T] = (9 m m^T + p p^T + q q^T + r r^T) / 12 (centred
//                 vertices; terms at most area x max deviation^2)
//   k_fit_eig     per cluster: C / S, float64 cyclic Jacobi, axes by decreasing
//                 eigenvalue, largest |component| of e0 and e1 positive, e2 = e0 x e1
//   k_fit_extent  per triangle: min / max of the vertex projections (ordered-integer atomics)
//   k_fit_box     per cluster: centre = axes^T mid, half = (max - min) / 2
#include <algorithm>
#include <cmath>

#include "common.h"

namespace obbv {
namespace {

constexpr int kFitThreads = 256;

struct FitScratch {
  int32_t* cnt;    // [n]
  uint64_t* amax;  // [n] ordered keys: largest triangle area
  uint64_t* cmax;  // [n] largest |vertex coordinate|
  uint64_t* dmax;  // [n] largest |vertex coordinate - mean|
  long long* S;    // [n]     fixed point, scale 2^kS
  long long* M;    // [n][3]  scale 2^kM
  long long* C;    // [n][6]  xx yy zz xy xz yz, scale 2^kC
  uint64_t* lo;    // [n][3] ordered keys
  uint64_t* hi;    // [n][3]
};

// order-preserving map of a double to uint64 (for atomic min / max)
__device__ inline uint64_t ordered_key(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double from_ordered_key(uint64_t k) {
  const uint64_t u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double((long long)u);
}

// Exponent k of the fixed-point scale of a sum whose total magnitude is below
// `bound`: bound * 2^k <= 2^62, so the 64-bit sum cannot overflow.
__device__ inline int fx_exp(double bound) {
  if (!(bound > 0.0) || !isfinite(bound)) return 0;
  int e;
  (void)frexp(bound, &e);  // bound < 2^e
  return 62 - e;
}
__device__ inline long long to_fx(double v, int k) { return __double2ll_rn(ldexp(v, k)); }
__device__ inline double from_fx(long long q, int k) { return ldexp((double)q, -k); }

struct ClusterScales {
  int kS, kM, kC;
};

// bound_S = count x max area, bound_M = bound_S x max |coordinate|,
// bound_C = bound_S x max deviation^2 (kC is valid after k_fit_dev)
__device__ inline ClusterScales cluster_scales(const FitScratch& s, int c) {
  const double n = (double)s.cnt[c];
  const double a = from_ordered_key(s.amax[c]);
  const double x = from_ordered_key(s.cmax[c]);
  const double d = from_ordered_key(s.dmax[c]);
  ClusterScales k;
  k.kS = fx_exp(n * a);
  k.kM = fx_exp(n * a * x);
  k.kC = fx_exp(n * a * d * d);
  return k;
}

// Adds vals[0..N) of every lane into base[N * cluster + k]: lanes with the same
// cluster are summed across the wave first, then one lane per cluster does the
// atomics (triangles of one cluster are mostly contiguous, so a wave usually
// holds one or two clusters).  Lanes with c < 0 contribute nothing.  Integer
// sums: the same result in any order.
template <int N>
__device__ inline void wave_cluster_add(long long* base, int c, const long long (&vals)[N]) {
  const int lane = threadIdx.x & 63;
  uint64_t todo = __ballot(c >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lc = __shfl(c, leader);
    const bool mine = c == lc;
    const uint64_t mask = __ballot(mine);
    for (int k = 0; k < N; ++k) {
      long long v = mine ? vals[k] : 0ll;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == leader) atomicAdd((unsigned long long*)&base[N * lc + k], (unsigned long long)v);
    }
    todo &= ~mask;
  }
}

// Largest key of the lanes of each cluster into base[cluster].
__device__ inline void wave_cluster_max(uint64_t* base, int c, uint64_t key) {
  const int lane = threadIdx.x & 63;
  uint64_t todo = __ballot(c >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lc = __shfl(c, leader);
    const bool mine = c == lc;
    const uint64_t mask = __ballot(mine);
    unsigned long long v = mine ? key : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long v2 = __shfl_xor(v, off);
      v = v2 > v ? v2 : v;
    }
    if (lane == leader) atomicMax((unsigned long long*)&base[lc], v);
    todo &= ~mask;
  }
}

template <int N>
__device__ inline void wave_cluster_minmax(uint64_t* lo, uint64_t* hi, int c, const uint64_t (&kl)[N],
                                           const uint64_t (&kh)[N]) {
  const int lane = threadIdx.x & 63;
  uint64_t todo = __ballot(c >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lc = __shfl(c, leader);
    const bool mine = c == lc;
    const uint64_t mask = __ballot(mine);
    for (int k = 0; k < N; ++k) {
      unsigned long long a = mine ? kl[k] : ~0ull, b = mine ? kh[k] : 0ull;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long a2 = __shfl_xor(a, off), b2 = __shfl_xor(b, off);
        a = a2 < a ? a2 : a;
        b = b2 > b ? b2 : b;
      }
      if (lane == leader) {
        atomicMin((unsigned long long*)&lo[N * lc + k], a);
        atomicMax((unsigned long long*)&hi[N * lc + k], b);
      }
    }
    todo &= ~mask;
  }
}

__device__ inline bool tri_cluster_of(const int32_t* __restrict__ cl, int t, int n, int& c) {
  c = cl[t];
  return c >= 0 && c < n;
}

__device__ inline bool load_tri(const MeshDev& M, int t, double p[3][3], uint32_t* status) {
  const int32_t* f = M.F + 3 * (int64_t)t;
  int idx[3] = {f[0], f[1], f[2]};
  for (int k = 0; k < 3; ++k)
    if ((unsigned)idx[k] >= (unsigned)M.nv) {
      atomicOr(status, OBBV_STATUS_BAD_INDEX);
      return false;
    }
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) p[k][d] = (double)M.V[3 * (int64_t)idx[k] + d];
  return true;
}

__device__ inline double tri_area(const double p[3][3]) {
  const double a0 = p[1][0] - p[0][0], a1 = p[1][1] - p[0][1], a2 = p[1][2] - p[0][2];
  const double b0 = p[2][0] - p[0][0], b1 = p[2][1] - p[0][1], b2 = p[2][2] - p[0][2];
  const double c0 = a1 * b2 - a2 * b1, c1 = a2 * b0 - a0 * b2, c2 = a0 * b1 - a1 * b0;
  return 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
}

__device__ inline void tri_mean(const double p[3][3], double m[3]) {
  for (int d = 0; d < 3; ++d) m[d] = (p[0][d] + p[1][d] + p[2][d]) / 3.0;
}

__global__ void __launch_bounds__(kFitThreads)
k_fit_bounds(MeshDev M, const int32_t* __restrict__ cl, int n, FitScratch s, uint32_t* status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  double p[3][3];
  if (t < M.nt && tri_cluster_of(cl, t, n, c) && !load_tri(M, t, p, status)) c = -1;
  if (t >= M.nt) c = -1;
  uint64_t ka = 0, kx = 0;
  if (c >= 0) {
    double x = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) x = fmax(x, fabs(p[k][d]));
    ka = ordered_key(tri_area(p));
    kx = ordered_key(x);
    atomicAdd(&s.cnt[c], 1);
  }
  wave_cluster_max(s.amax, c, ka);
  wave_cluster_max(s.cmax, c, kx);
}

__global__ void __launch_bounds__(kFitThreads)
k_fit_mean(MeshDev M, const int32_t* __restrict__ cl, int n, FitScratch s, uint32_t* status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  double p[3][3];
  if (t < M.nt && tri_cluster_of(cl, t, n, c) && !load_tri(M, t, p, status)) c = -1;
  if (t >= M.nt) c = -1;
  long long a1[1] = {0}, m3[3] = {0, 0, 0};
  if (c >= 0) {
    const ClusterScales k = cluster_scales(s, c);
    const double A = tri_area(p);
    double m[3];
    tri_mean(p, m);
    a1[0] = to_fx(A, k.kS);
    for (int d = 0; d < 3; ++d) m3[d] = to_fx(A * m[d], k.kM);
  }
  wave_cluster_add<1>(s.S, c, a1);
  wave_cluster_add<3>(s.M, c, m3);
}

// area and mean of cluster c (float64 of the exact sums); false when the area is 0
__device__ inline bool cluster_mean(const FitScratch& s, int c, double& S, double mu[3]) {
  if (s.cnt[c] <= 0) return false;
  const ClusterScales k = cluster_scales(s, c);
  S = from_fx(s.S[c], k.kS);
  if (!(S > 0.0)) return false;
  for (int d = 0; d < 3; ++d) mu[d] = from_fx(s.M[3 * c + d], k.kM) / S;
  return true;
}

__global__ void __launch_bounds__(kFitThreads)
k_fit_dev(MeshDev M, const int32_t* __restrict__ cl, int n, FitScratch s, uint32_t* status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  double p[3][3], mu[3], S;
  if (t < M.nt && tri_cluster_of(cl, t, n, c) && !load_tri(M, t, p, status)) c = -1;
  if (t >= M.nt) c = -1;
  if (c >= 0 && !cluster_mean(s, c, S, mu)) c = -1;
  uint64_t kd = 0;
  if (c >= 0) {
    double x = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) x = fmax(x, fabs(p[k][d] - mu[d]));
    kd = ordered_key(x);
  }
  wave_cluster_max(s.dmax, c, kd);
}

__global__ void __launch_bounds__(kFitThreads)
k_fit_cov(MeshDev M, const int32_t* __restrict__ cl, int n, FitScratch s, uint32_t* status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  double p[3][3], mu[3], S;
  if (t < M.nt && tri_cluster_of(cl, t, n, c) && !load_tri(M, t, p, status)) c = -1;
  if (t >= M.nt) c = -1;
  if (c >= 0 && !cluster_mean(s, c, S, mu)) c = -1;
  long long acc[6] = {0, 0, 0, 0, 0, 0};
  if (c >= 0) {
    const int kC = cluster_scales(s, c).kC;
    const double A = tri_area(p);
    double m[3];
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) p[k][d] -= mu[d];
    tri_mean(p, m);
    const int ii[6] = {0, 1, 2, 0, 0, 1};
    const int jj[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; ++e) {
      const int i = ii[e], j = jj[e];
      acc[e] = to_fx(A * ((9.0 * m[i] * m[j] + p[0][i] * p[0][j] + p[1][i] * p[1][j] + p[2][i] * p[2][j]) / 12.0),
                     kC);
    }
  }
  wave_cluster_add<6>(s.C, c, acc);
}

// Cyclic Jacobi on a symmetric 3x3 matrix a (float64, in place); v = eigenvectors (columns).
__device__ inline void jacobi3(double a[3][3], double v[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    const double diag = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]);
    if (off <= 1e-300 || off <= 1e-18 * diag) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        // rotation angle that zeroes a[p][q]
        const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double t;
        if (fabs(theta) > 1e150)
          t = 0.5 / theta;
        else
          t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        // a <- J^T a J with J = identity except J[p][p] = J[q][q] = c, J[p][q] = sn, J[q][p] = -sn
        for (int k = 0; k < 3; ++k) {
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - sn * vkq;
          v[k][q] = sn * vkp + c * vkq;
        }
      }
  }
}

__global__ void k_fit_eig(int n, FitScratch s, obbv_box* __restrict__ out, double* __restrict__ eig) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float* o = reinterpret_cast<float*>(out + c);
  double S = 0.0, mu[3];
  if (!cluster_mean(s, c, S, mu)) {
    for (int k = 0; k < 15; ++k) o[k] = 0.f;
    o[3] = o[7] = o[11] = 1.f;
    if (eig)
      for (int k = 0; k < 3; ++k) eig[3 * c + k] = 0.0;
    return;
  }
  const int kC = cluster_scales(s, c).kC;
  double C6[6];
  for (int e = 0; e < 6; ++e) C6[e] = from_fx(s.C[6 * c + e], kC);
  double a[3][3] = {{C6[0] / S, C6[3] / S, C6[4] / S},
                    {C6[3] / S, C6[1] / S, C6[5] / S},
                    {C6[4] / S, C6[5] / S, C6[2] / S}};
  double v[3][3];
  jacobi3(a, v);
  double lam[3] = {a[0][0], a[1][1], a[2][2]};
  int ord[3] = {0, 1, 2};
  // decreasing eigenvalue (stable insertion sort)
  for (int i = 1; i < 3; ++i)
    for (int j = i; j > 0 && lam[ord[j]] > lam[ord[j - 1]]; --j) {
      const int tmp = ord[j];
      ord[j] = ord[j - 1];
      ord[j - 1] = tmp;
    }
  double e[2][3];
  for (int r = 0; r < 2; ++r) {
    int kmax = 0;
    for (int k = 0; k < 3; ++k) {
      e[r][k] = v[k][ord[r]];
      if (fabs(e[r][k]) > fabs(e[r][kmax])) kmax = k;
    }
    if (e[r][kmax] < 0.0)
      for (int k = 0; k < 3; ++k) e[r][k] = -e[r][k];
  }
  const double e2[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1], e[0][2] * e[1][0] - e[0][0] * e[1][2],
                        e[0][0] * e[1][1] - e[0][1] * e[1][0]};
  for (int k = 0; k < 3; ++k) {
    o[3 + k] = (float)e[0][k];
    o[6 + k] = (float)e[1][k];
    o[9 + k] = (float)e2[k];
  }
  if (eig)
    for (int k = 0; k < 3; ++k) eig[3 * c + k] = lam[ord[k]];
}

__global__ void __launch_bounds__(kFitThreads)
k_fit_extent(MeshDev M, const int32_t* __restrict__ cl, int n, const obbv_box* __restrict__ boxes, FitScratch s,
             uint32_t* status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  double p[3][3];
  if (t < M.nt && tri_cluster_of(cl, t, n, c) && !load_tri(M, t, p, status)) c = -1;
  if (t >= M.nt) c = -1;
  uint64_t kl[3] = {~0ull, ~0ull, ~0ull}, kh[3] = {0ull, 0ull, 0ull};
  if (c >= 0) {
    const float* ax = reinterpret_cast<const float*>(boxes + c) + 3;
    for (int r = 0; r < 3; ++r) {
      double lo = 1e300, hi = -1e300;
      for (int k = 0; k < 3; ++k) {
        const double x =
            (double)ax[3 * r] * p[k][0] + (double)ax[3 * r + 1] * p[k][1] + (double)ax[3 * r + 2] * p[k][2];
        lo = fmin(lo, x);
        hi = fmax(hi, x);
      }
      kl[r] = ordered_key(lo);
      kh[r] = ordered_key(hi);
    }
  }
  wave_cluster_minmax<3>(s.lo, s.hi, c, kl, kh);
}

__global__ void k_fit_box(int n, FitScratch s, obbv_box* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double S, mu[3];
  if (!cluster_mean(s, c, S, mu)) return;
  float* o = reinterpret_cast<float*>(out + c);
  double mid[3];
  for (int r = 0; r < 3; ++r) {
    const double lo = from_ordered_key(s.lo[3 * c + r]);
    const double hi = from_ordered_key(s.hi[3 * c + r]);
    mid[r] = 0.5 * (lo + hi);
    o[12 + r] = __double2float_ru(0.5 * (hi - lo));
  }
  for (int k = 0; k < 3; ++k) {
    double x = 0.0;
    for (int r = 0; r < 3; ++r) x += (double)o[3 + 3 * r + k] * mid[r];
    o[k] = (float)x;
  }
}

}  // namespace

int fit_impl(const obbv_mesh* mesh, const int32_t* tri_cluster, int32_t n_clusters, obbv_box* out_boxes,
             double* out_eigvals, hipStream_t st) {
  OBBV_ARG(mesh != nullptr, "mesh is NULL");
  OBBV_ARG(n_clusters >= 0, "n_clusters < 0");
  if (n_clusters == 0) return OBBV_OK;
  OBBV_ARG(out_boxes != nullptr, "out_boxes is NULL");
  OBBV_ARG(mesh->n_triangles >= 0 && mesh->n_vertices >= 0, "negative mesh size");
  OBBV_ARG(mesh->n_triangles == 0 || (mesh->triangles && mesh->vertices && tri_cluster),
           "mesh or tri_cluster pointer is NULL");
  uint32_t* status = nullptr;
  OBBV_RET(status_word(&status));
  const size_t n = (size_t)n_clusters;
  // cnt (8-byte slots) | amax | cmax | dmax | S | M[3] | C[6] | lo[3] | hi[3]
  const size_t zeroed = n * 8 * (1 + 3 + 1 + 3 + 6);
  const size_t bytes = zeroed + n * 8 * 6;
  void* p = nullptr;
  OBBV_RET(pool_get(kPoolFit, bytes, &p));
  FitScratch s;
  s.cnt = (int32_t*)p;
  s.amax = (uint64_t*)((char*)p + n * 8);
  s.cmax = s.amax + n;
  s.dmax = s.cmax + n;
  s.S = (long long*)(s.dmax + n);
  s.M = s.S + n;
  s.C = s.M + 3 * n;
  s.lo = (uint64_t*)(s.C + 6 * n);
  s.hi = s.lo + 3 * n;
  // counts and sums start at 0; so do the maxima (key 0 is below the key of every
  // non-negative double)
  OBBV_HIP(hipMemsetAsync(p, 0, zeroed, st));
  OBBV_HIP(hipMemsetAsync(s.lo, 0xFF, n * 8 * 3, st));
  OBBV_HIP(hipMemsetAsync(s.hi, 0x00, n * 8 * 3, st));
  MeshDev M{mesh->vertices, mesh->triangles, mesh->n_vertices, mesh->n_triangles};
  const unsigned gt = (unsigned)ceil_div(std::max(M.nt, 1), kFitThreads);
  const unsigned gc = (unsigned)ceil_div(n_clusters, 128);
  if (M.nt > 0) {
    hipLaunchKernelGGL(k_fit_bounds, dim3(gt), dim3(kFitThreads), 0, st, M, tri_cluster, n_clusters, s, status);
    OBBV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fit_mean, dim3(gt), dim3(kFitThreads), 0, st, M, tri_cluster, n_clusters, s, status);
    OBBV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fit_dev, dim3(gt), dim3(kFitThreads), 0, st, M, tri_cluster, n_clusters, s, status);
    OBBV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fit_cov, dim3(gt), dim3(kFitThreads), 0, st, M, tri_cluster, n_clusters, s, status);
    OBBV_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fit_eig, dim3(gc), dim3(128), 0, st, n_clusters, s, out_boxes, out_eigvals);
  OBBV_HIP(hipGetLastError());
  if (M.nt > 0) {
    hipLaunchKernelGGL(k_fit_extent, dim3(gt), dim3(kFitThreads), 0, st, M, tri_cluster, n_clusters,
                       out_boxes, s, status);
    OBBV_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fit_box, dim3(gc), dim3(128), 0, st, n_clusters, s, out_boxes);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

}  // namespace obbv

static int obbv_fit_body(const obbv_mesh* mesh, const int32_t* tri_cluster, int32_t n_clusters,
                        obbv_box* out_boxes, double* out_eigvals, void* stream);
extern "C" int obbv_fit(const obbv_mesh* mesh, const int32_t* tri_cluster, int32_t n_clusters,
                        obbv_box* out_boxes, double* out_eigvals, void* stream) {
  return obbv::guarded([&] { return obbv_fit_body(mesh, tri_cluster, n_clusters, out_boxes, out_eigvals, stream); });
}
static int obbv_fit_body(const obbv_mesh* mesh, const int32_t* tri_cluster, int32_t n_clusters,
                        obbv_box* out_boxes, double* out_eigvals, void* stream) {
  obbv::clear_error();
  return obbv::fit_impl(mesh, tri_cluster, n_clusters, out_boxes, out_eigvals, (hipStream_t)stream);
}
