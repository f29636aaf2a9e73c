// Internal helpers of libobbv (device and host).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
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

#define OBBV_RET(call)                                                          \
  do {                                                                          \
    int r_ = (call);                                                            \
    if (r_ != OBBV_OK) return r_;                                               \
  } while (0)

// ---------------------------------------------------------------------------
// per-device scratch: a few independently growing buffers and the status word
// ---------------------------------------------------------------------------
enum PoolSlot {
  kPoolMeta = 0,
  kPoolRecords = 1,  // binned records
  kPoolFit = 2,
  kPoolMlp = 3,
  kPoolFeat = 4,
  kPoolLists = 5,
  kPoolItems = 6,
  kPoolTiles = 7,
  kPoolRank = 8,
  kPoolTileCnt2 = 9,  // zero between calls (each call leaves what it used zero)
  kPoolCount = 10
};
// Two sets of the slots: calls that may run at the same time on different
// streams take their scratch from different sets (slot + set * kPoolCount).
constexpr int kPoolSets = 2;

// Ensures slot `slot` (< kPoolCount * kPoolSets) of the current device holds at
// least `bytes` and returns it.  Growing frees the old block (hipFree waits for
// the device), so call it only where no queued kernel still reads that slot.
int pool_get(int slot, size_t bytes, void** out);
// As pool_get; a new (grown) block is zeroed before it is returned.
int pool_get_zeroed(int slot, size_t bytes, void** out);

// A binned ray-test record, one per bin entry: 4 float4 = 64 bytes (edge
// planes, depth plane, clamp, sign, and the record's cell range inside the tile
// of its bin).  A tile's entries are contiguous, so a ray-test wave reads one
// aligned 64-byte line per record with no index indirection.
constexpr int kRecF4 = 4;
constexpr int kRecBytes = 16 * kRecF4;

// A ray-test work item (64 bytes, written by the write pass): up to a chunk of
// one ray tile's bin entries and the ray grid of the tile's (box, axis) cast,
// so a ray-test wave needs no further table before its rays and records.
struct WorkItem {
  double hu, hv, du, dv;  // half extents of the cast face and cell sizes (u, v)
  uint64_t s0;            // SplitMix64 state of the u draw of cell (0, 0)
  int64_t k0;             // first bin entry
  int32_t count;          // bin entries (at least one)
  int32_t g;              // tile: ((box * 3 + axis) * tiles per face + tile)
  uint32_t key;           // the box's jitter key
  int32_t pad;
};
static_assert(sizeof(WorkItem) == 64, "WorkItem layout");

// How one outer-volume evaluation is executed.  Default: scratch is sized from
// the device counts (one host round trip).  planned: fixed scratch, no round
// trip, capturable into a HIP graph.  capped: fixed record / bin / work-item
// capacities for a caller that checks the actual totals afterwards and repeats
// the call if they exceed the capacities.  `status` (nullable, device) replaces
// the library status word for the call; with `publish` (nullable, pinned host
// memory mapped for the device) the call's last kernel writes there the status
// bits ([0], uint32) and the totals ([1..3], int64: records, bin entries, work
// items), so the caller reads them after a stream synchronisation without a
// copy command.
struct OvExec {
  bool planned = false;
  bool capped = false;
  char* meta = nullptr;
  size_t meta_cap = 0, meta_bytes = 0;
  float4* recs = nullptr;                     // [bin_cap] binned records (kRecF4 float4 each)
  int64_t rec_cap = 0, bin_cap = 0, item_cap = 0;  // records counted per call, bin entries, work items
  int64_t n_rec = 0, n_bin = 0, n_items = 0;  // counts of the last synchronous run
  char* items = nullptr;                      // per-cull-item counts and offsets
  size_t items_cap = 0, items_bytes = 0;
  WorkItem* itile = nullptr;                  // [item_cap] ray-test work items
  uint32_t* status = nullptr;
  int64_t* publish = nullptr;
  int pool_base = 0;  // slot offset of the pool set the call's pooled scratch comes from
  // nullable: jitter table (jitter_table) covering every key of the call, built
  // for this R and seed; the ray-test kernel then reads the draws from it
  const uint2* jitter = nullptr;
  int jitter_R = 0;
  uint64_t jitter_seed = 0;
};
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
int profile_record_begin(hipStream_t s, void** token);            // event before k_test
int profile_record_end(hipStream_t s, void* token);               // event after k_test

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
