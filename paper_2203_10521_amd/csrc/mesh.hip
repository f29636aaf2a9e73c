// Mesh staging checks on the device (the solid-mesh requirement of Sec. 6):
// every index in range, every directed edge once with its reverse once (closed
// and consistently oriented), and a positive enclosed volume.
//
//   k_edge_insert  per directed edge (a, b): the undirected key (min, max) goes
//                  into an open-addressing table (linear probing, 64-bit CAS);
//                  the entry counts the edge's two directions separately
//   k_edge_check   per table entry: directed edges without exactly one reverse,
//                  and repeats of a directed edge
//   k_coord_max    largest |vertex coordinate| (bounds the volume terms)
//   k_volume       per triangle det[a, b, c] as 64-bit fixed point with one
//                  power-of-two scale for the mesh, summed exactly: the volume
//                  does not depend on thread order
#include <cstring>

#include "common.h"

namespace obbv {
namespace {

constexpr int kMeshThreads = 256;
constexpr uint64_t kEmptyKey = ~0ull;

__global__ void __launch_bounds__(kMeshThreads)
k_edge_insert(const int32_t* __restrict__ F, int64_t nt, int32_t nv, uint64_t* __restrict__ keys,
              int32_t* __restrict__ cnt, uint64_t mask, int32_t* __restrict__ report) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nt) return;
  const int64_t t = e / 3;
  const int k = (int)(e - 3 * t);
  const int32_t a = F[3 * t + k], b = F[3 * t + (k + 1) % 3];
  // each index is the start of exactly one directed edge: count it there
  if (a < 0 || a >= nv) atomicAdd(&report[2], 1);
  if (a < 0 || a >= nv || b < 0 || b >= nv) return;
  const bool fwd = a < b;
  const uint64_t key = fwd ? (((uint64_t)a << 32) | (uint32_t)b) : (((uint64_t)b << 32) | (uint32_t)a);
  uint64_t slot = mix64(key) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&keys[slot], (unsigned long long)kEmptyKey, (unsigned long long)key);
    if (prev == kEmptyKey || prev == key) {
      atomicAdd(&cnt[2 * slot + (fwd ? 0 : 1)], 1);
      return;
    }
    slot = (slot + 1) & mask;
  }
}

__device__ inline int block_sum(int v, int* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  int s = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

__global__ void __launch_bounds__(kMeshThreads)
k_edge_check(const uint64_t* __restrict__ keys, const int32_t* __restrict__ cnt, uint64_t cap,
             int32_t* __restrict__ report) {
  __shared__ int sh[kMeshThreads / 64];
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int unmatched = 0, repeated = 0;
  if (s < cap && keys[s] != kEmptyKey) {
    const int f = cnt[2 * s], r = cnt[2 * s + 1];
    // an occurrence of (a, b) is matched when (b, a) occurs exactly once
    unmatched = (r != 1 ? f : 0) + (f != 1 ? r : 0);
    repeated = (f > 1 ? f - 1 : 0) + (r > 1 ? r - 1 : 0);
  }
  unmatched = block_sum(unmatched, sh);
  repeated = block_sum(repeated, sh);
  if (threadIdx.x == 0) {
    if (unmatched) atomicAdd(&report[0], unmatched);
    if (repeated) atomicAdd(&report[1], repeated);
  }
}

// |x| of a non-negative float orders like its bits
__global__ void __launch_bounds__(kMeshThreads)
k_coord_max(const float* __restrict__ V, int64_t n, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t m = i < n ? __float_as_uint(fabsf(V[i])) : 0u;
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(m, off);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// exponent k with bound * 2^k <= 2^62
__device__ inline int fx_exp(double bound) {
  if (!(bound > 0.0) || !isfinite(bound)) return 0;
  int e;
  (void)frexp(bound, &e);
  return 62 - e;
}

__global__ void __launch_bounds__(kMeshThreads)
k_volume(const float* __restrict__ V, const int32_t* __restrict__ F, int64_t nt, const uint32_t* __restrict__ cmax,
         unsigned long long* __restrict__ sum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // |det[a, b, c]| <= |a| |b| |c| <= (sqrt(3) max |coordinate|)^3 per triangle
  const double c = (double)__uint_as_float(*cmax);
  const int k = fx_exp((double)nt * 5.196152422706632 * c * c * c);
  long long q = 0;
  if (t < nt) {
    const float* a = V + 3 * (int64_t)F[3 * t + 0];
    const float* b = V + 3 * (int64_t)F[3 * t + 1];
    const float* d = V + 3 * (int64_t)F[3 * t + 2];
    const double bc0 = (double)b[1] * d[2] - (double)b[2] * d[1];
    const double bc1 = (double)b[2] * d[0] - (double)b[0] * d[2];
    const double bc2 = (double)b[0] * d[1] - (double)b[1] * d[0];
    q = __double2ll_rn(ldexp((double)a[0] * bc0 + (double)a[1] * bc1 + (double)a[2] * bc2, k));
  }
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
  if ((threadIdx.x & 63) == 0 && q) atomicAdd(sum, (unsigned long long)q);
}

}  // namespace
}  // namespace obbv

using namespace obbv;

static int obbv_validate_mesh_body(const obbv_mesh* mesh, int32_t* out_report, double* out_volume,
                                  void* stream);
extern "C" int obbv_validate_mesh(const obbv_mesh* mesh, int32_t* out_report, double* out_volume,
                                  void* stream) {
  return obbv::guarded([&] { return obbv_validate_mesh_body(mesh, out_report, out_volume, stream); });
}
static int obbv_validate_mesh_body(const obbv_mesh* mesh, int32_t* out_report, double* out_volume,
                                  void* stream) {
  clear_error();
  OBBV_ARG(mesh != nullptr, "mesh is NULL");
  OBBV_ARG(mesh->n_triangles >= 0 && mesh->n_vertices >= 0, "negative mesh size");
  OBBV_ARG(mesh->n_triangles == 0 || (mesh->triangles && mesh->vertices), "mesh pointers are NULL");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nt = mesh->n_triangles, nv = mesh->n_vertices;
  int32_t report[4] = {0, 0, 0, 0};
  double vol = 0.0;
  if (nt > 0) {
    // a table of at least twice the directed-edge count: probing always ends
    uint64_t cap = 1024;
    while (cap < (uint64_t)(6 * nt)) cap <<= 1;
    // keys [cap] | counts [2 cap] | report [4] | coordinate max | volume sum
    const size_t bytes = cap * 8 + cap * 8 + 64;
    void* p = nullptr;
    OBBV_RET(pool_get(kPoolMesh, bytes, &p));
    uint64_t* keys = (uint64_t*)p;
    int32_t* cnt = (int32_t*)(keys + cap);
    int32_t* rep = cnt + 2 * cap;
    uint32_t* cmax = (uint32_t*)(rep + 4);
    unsigned long long* vsum = (unsigned long long*)(rep + 8);
    OBBV_HIP(hipMemsetAsync(keys, 0xFF, cap * 8, s));
    OBBV_HIP(hipMemsetAsync(cnt, 0, cap * 8 + 64, s));
    const unsigned ge = (unsigned)ceil_div(3 * nt, kMeshThreads);
    hipLaunchKernelGGL(k_edge_insert, dim3(ge), dim3(kMeshThreads), 0, s, mesh->triangles, nt, (int32_t)nv, keys, cnt,
                       cap - 1, rep);
    OBBV_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_edge_check, dim3((unsigned)ceil_div((int64_t)cap, kMeshThreads)), dim3(kMeshThreads), 0, s,
                       keys, cnt, cap, rep);
    OBBV_HIP(hipGetLastError());
    int32_t host_rep[4];
    OBBV_HIP(hipMemcpyAsync(host_rep, rep, 16, hipMemcpyDeviceToHost, s));
    OBBV_HIP(hipStreamSynchronize(s));
    std::memcpy(report, host_rep, sizeof(report));
    if (report[2] == 0) {
      hipLaunchKernelGGL(k_coord_max, dim3((unsigned)ceil_div(3 * nv, kMeshThreads)), dim3(kMeshThreads), 0, s,
                         mesh->vertices, 3 * nv, cmax);
      OBBV_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_volume, dim3((unsigned)ceil_div(nt, kMeshThreads)), dim3(kMeshThreads), 0, s,
                         mesh->vertices, mesh->triangles, nt, cmax, vsum);
      OBBV_HIP(hipGetLastError());
      uint32_t hc = 0;
      long long hs = 0;
      OBBV_HIP(hipMemcpyAsync(&hc, cmax, 4, hipMemcpyDeviceToHost, s));
      OBBV_HIP(hipMemcpyAsync(&hs, vsum, 8, hipMemcpyDeviceToHost, s));
      OBBV_HIP(hipStreamSynchronize(s));
      float c;
      std::memcpy(&c, &hc, 4);
      const double bound = (double)nt * 5.196152422706632 * (double)c * (double)c * (double)c;
      int k = 0;
      if (bound > 0.0 && std::isfinite(bound)) {
        int e;
        (void)std::frexp(bound, &e);
        k = 62 - e;
      }
      vol = std::ldexp((double)hs, -k) / 6.0;
    }
  }
  if (out_report) std::memcpy(out_report, report, sizeof(report));
  if (out_volume) *out_volume = vol;
  if (report[2]) {
    set_error("triangle index out of range");
    return OBBV_ERR_INVALID_ARG;
  }
  if (report[1]) {
    set_error("a directed edge occurs more than once (inconsistent orientation)");
    return OBBV_ERR_MESH_NOT_ORIENTED;
  }
  if (report[0]) {
    set_error("a directed edge has no reverse edge (mesh not closed)");
    return OBBV_ERR_MESH_NOT_CLOSED;
  }
  if (nt > 0 && !(vol > 0.0)) {
    set_error("enclosed volume is not positive (triangles not outward oriented)");
    return OBBV_ERR_MESH_NOT_ORIENTED;
  }
  return OBBV_OK;
}
