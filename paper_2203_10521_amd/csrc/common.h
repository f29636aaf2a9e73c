// Internal helpers of libobbv (device and host).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>

#include "obbv.h"

namespace obbv {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

#define OBBV_HIP(call)                                                          \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::obbv::set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return OBBV_ERR_HIP;                                                      \
    }                                                                           \
  } while (0)

#define OBBV_ARG(cond, msg)                                                     \
  do {                                                                          \
    if (!(cond)) {                                                              \
      ::obbv::set_error(std::string("invalid argument: ") + (msg));             \
      return OBBV_ERR_INVALID_ARG;                                              \
    }                                                                           \
  } while (0)

// Runs the body of a C entry point: a C++ exception (a failed host
// allocation, a thread that could not start) becomes an error code and a
// message, so that no exception crosses the C ABI.
template <class F>
int guarded(F&& body) noexcept {
  const char* msg = "internal error";
  int code = OBBV_ERR_INTERNAL;
  try {
    return body();
  } catch (const std::bad_alloc&) {
    msg = "host memory allocation failed";
    code = OBBV_ERR_OOM;
  } catch (const std::exception& e) {
    try {
      set_error(std::string("internal error: ") + e.what());
      return OBBV_ERR_INTERNAL;
    } catch (...) {
    }
  } catch (...) {
  }
  try {
    set_error(msg);
  } catch (...) {
  }
  return code;
}

#define OBBV_RET(call)                                                          \
  do {                                                                          \
    int r_ = (call);                                                            \
    if (r_ != OBBV_OK) return r_;                                               \
  } while (0)

// ---------------------------------------------------------------------------
// per-device scratch: a few independently growing buffers and the status word
// ---------------------------------------------------------------------------
enum PoolSlot {
  kPoolMeta = 0,   // per-call counters, offsets, ray grids, per-(box, axis) sums
  kPoolFit = 1,
  kPoolMlp = 2,
  kPoolFeat = 3,
  kPoolLists = 4,  // frame lists of grouped calls
  kPoolItems = 5,  // cast items
  kPoolRank = 6,
  kPoolMesh = 7,   // mesh validation: edge table and counters
  kPoolFrameCnt = 8,  // (frame, axis) list counters of one-pass grouped calls (zero between calls)
  kPoolExact = 9,     // per-(box, triangle chunk) partial sums of the exact evaluator
  kPoolCentral = 10,  // per-(box, ray chunk) partial sums of the central-projection estimator
  kPoolCount = 11
};
// Sets of the slots: calls that may run at the same time on different streams
// take their scratch from different sets (slot + set * kPoolCount).
constexpr int kPoolSets = 8;

// Ensures slot `slot` (< kPoolCount * kPoolSets) of the current device holds at
// least `bytes` and returns it.  Growing frees the old block (hipFree waits for
// the device), so call it only where no queued kernel still reads that slot.
int pool_get(int slot, size_t bytes, void** out);
// As pool_get; a new (grown) block is zeroed before it is returned.
int pool_get_zeroed(int slot, size_t bytes, void** out);

// How one outer-volume evaluation is executed.  Default: scratch comes from the
// library pool.  planned: scratch fixed beforehand (meta / items blocks of the
// caller), no host round trip, capturable into a HIP graph.  `status`
// (nullable, device) replaces the library status word for the call; with
// `publish` (nullable, pinned host memory mapped for the device) the call's
// last kernel writes there the status bits ([0]) and then a done word ([4] = 1),
// so the caller can spin on host memory instead of waiting on the stream.
struct OvExec {
  bool planned = false;
  char* meta = nullptr;
  size_t meta_cap = 0, meta_bytes = 0;
  char* items = nullptr;  // cast items of the call
  size_t items_cap = 0, items_bytes = 0;
  uint32_t* status = nullptr;
  int64_t* publish = nullptr;
  int pool_base = 0;  // slot offset of the pool set the call's pooled scratch comes from
  // nullable: jitter table (jitter_table) covering every key of the call, built
  // for this R and seed; the cast kernel then reads the draws from it
  const uint2* jitter = nullptr;
  int jitter_R = 0;
  uint64_t jitter_seed = 0;
  // nullable: device float4 [n_meshes] centre of each mesh's bounding box (the
  // kept side of every cast); computed by the call when absent
  const float4* centre = nullptr;
  // nullable: span bounds of the (single) mesh (span_table), reused from call to
  // call; computed by the call when absent
  const float4* spans = nullptr;
  const float4* span_runs = nullptr;
  // smaller cast items for calls that run alone: a call whose default items
  // would give fewer than split_below cast units takes items of item_tris
  // entries (a multiple of 256 dividing the default) instead, so that it
  // leaves fewer compute units idle; 0 = never.  The results do not change.
  int item_tris = 0;
  int split_below = 0;
};
// Span bounds table of a mesh for repeated single-mesh outer-volume calls:
// its size in bytes (0: the mesh needs none), its computation (stream ordered)
// and the run bounds inside it.
size_t span_table_size(int64_t nt);
int span_table(const obbv_mesh* m, float4* table, hipStream_t s);
const float4* span_runs_of(const float4* table, int64_t nt);
// Jitter table of keys [0, n_keys) for ray grids of R x R cells (stream ordered).
int jitter_table(uint64_t seed, int R, int64_t n_keys, uint2* out, hipStream_t s);
int status_word(uint32_t** out);   // device pointer of this device's status word

// measurement hooks (obbv_profile_enable / obbv_profile_read)
bool profiling_enabled();
// device counters: tests in slots [0, kProfSlots), bytes in [kProfSlots,
// 2 kProfSlots); a count is the sum of its slots, and a wave adds to one slot,
// so the waves of a launch do not serialise on one address
constexpr int kProfSlots = 256;
int profile_counter(unsigned long long** out);
int profile_record_begin(hipStream_t s, void** token);            // event before the cast kernel
int profile_record_end(hipStream_t s, void* token);               // event after the cast kernel

// ---------------------------------------------------------------------------
// constants of the fixed-point ray integration
// ---------------------------------------------------------------------------
// A ray's inside length of the slab [-h, h] is carried as q = L / (2h) * 2^22.
// Each crossing's contribution is produced directly as a float in [2^23, 2^24]
// whose bit pattern is kMagicBits + q_k (the float rounds to an integer there),
// so per-ray sums are exact integer adds and independent of crossing order.
constexpr float kMagic = 12582912.0f;      // 1.5 * 2^23
constexpr uint32_t kMagicBits = 0x4B400000u;
constexpr double kQOne = 4194304.0;        // 2^22 <-> the full slab length 2h
constexpr double kHalfQ = 2097152.0;       // 2^21 <-> h

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output n of the stream with
// seed s is mix64(s + (n + 1) * GAMMA), mix64 = their variant-13 finaliser.
// ---------------------------------------------------------------------------
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t n) {
  return mix64(seed + (n + 1ull) * kGamma);
}

// top 24 bits as a double in [0, 1): exact
__host__ __device__ inline double u24(uint64_t x) {
  return (double)(x >> 40) * (1.0 / 16777216.0);
}

// counter of the u jitter of cell (i, j) of cast axis w of box `key`;
// the v jitter uses counter + 1
__host__ __device__ inline uint64_t ray_counter(uint32_t key, int w, int i, int j) {
  return 2ull * (((uint64_t)key << 32) | ((uint64_t)w << 30) | ((uint64_t)i << 15) |
                 (uint64_t)j);
}

// ---------------------------------------------------------------------------
// device view of a mesh
// ---------------------------------------------------------------------------
struct MeshDev {
  const float* V;
  const int32_t* F;
  int32_t nv;
  int32_t nt;
};

// Box-local coordinates x' = Q (x - c) with one fixed rounding sequence, so a
// vertex shared by several triangles maps to bit-identical local coordinates
// (the watertightness of the ray test relies on this).
__device__ inline void to_local(const float* __restrict__ Q, const float* __restrict__ c,
                                float x, float y, float z, float out[3]) {
  const float dx = __fsub_rn(x, c[0]);
  const float dy = __fsub_rn(y, c[1]);
  const float dz = __fsub_rn(z, c[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    out[k] = __fmaf_rn(Q[3 * k + 0], dx, __fmaf_rn(Q[3 * k + 1], dy, __fmul_rn(Q[3 * k + 2], dz)));
}

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// exclusive scan of n int32 counts into n + 1 int64 offsets (offsets[n] = total)
int exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* scratch,
                              size_t scratch_bytes, hipStream_t s);
size_t exclusive_scan_scratch_bytes(int64_t n);

}  // namespace obbv
