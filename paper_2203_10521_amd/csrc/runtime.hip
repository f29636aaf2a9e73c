// Host runtime of libobbv: errors, per-device scratch pool, status word,
// device exclusive scan, mesh validation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace obbv {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// ---------------------------------------------------------------------------
// scratch pool
// ---------------------------------------------------------------------------
namespace {
constexpr int kMaxDevices = 64;
struct DevicePool {
  void* ptr[kPoolCount * kPoolSets] = {};
  size_t cap[kPoolCount * kPoolSets] = {};
  uint32_t* status = nullptr;
};
DevicePool g_pools[kMaxDevices];
std::mutex g_pool_mutex;
}  // namespace

static int pool_get_impl(int slot, size_t bytes, void** out, bool zero);

int pool_get(int slot, size_t bytes, void** out) { return pool_get_impl(slot, bytes, out, false); }

int pool_get_zeroed(int slot, size_t bytes, void** out) { return pool_get_impl(slot, bytes, out, true); }

static int pool_get_impl(int slot, size_t bytes, void** out, bool zero) {
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of range");
    return OBBV_ERR_UNSUPPORTED;
  }
  if (slot < 0 || slot >= kPoolCount * kPoolSets) {
    set_error("scratch slot out of range");
    return OBBV_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  DevicePool& p = g_pools[dev];
  if (bytes == 0) bytes = 256;
  if (p.cap[slot] < bytes) {
    if (p.ptr[slot]) {
      // kernels of earlier calls may still read the old block
      OBBV_HIP(hipDeviceSynchronize());
      OBBV_HIP(hipFree(p.ptr[slot]));
      p.ptr[slot] = nullptr;
      p.cap[slot] = 0;
    }
    size_t want = std::max(bytes + bytes / 4, (size_t)1 << 20);
    void* q = nullptr;
    if (hipMalloc(&q, want) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of " + std::to_string(want) + " bytes of scratch failed");
      return OBBV_ERR_OOM;
    }
    if (zero && hipMemset(q, 0, want) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(q);
      set_error("hipMemset of new scratch failed");
      return OBBV_ERR_HIP;
    }
    p.ptr[slot] = q;
    p.cap[slot] = want;
  }
  *out = p.ptr[slot];
  return OBBV_OK;
}

int status_word(uint32_t** out) {
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of range");
    return OBBV_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  DevicePool& p = g_pools[dev];
  if (!p.status) {
    void* q = nullptr;
    OBBV_HIP(hipMalloc(&q, 256));
    OBBV_HIP(hipMemset(q, 0, 256));
    p.status = (uint32_t*)q;
  }
  *out = p.status;
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan int32 -> int64 (two kernels per level, recursive on block sums;
// out[n] = total)
// ---------------------------------------------------------------------------
namespace {
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;  // elements per block

template <typename T>
__global__ void __launch_bounds__(kScanThreads)
k_scan_block(const T* __restrict__ in, int64_t* __restrict__ out, int64_t* __restrict__ sums,
             int64_t n, int64_t* __restrict__ total_out) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < n ? (int64_t)in[idx] : 0;
    run += v[k];
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread totals
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int64_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t excl = sh[threadIdx.x] - run;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) out[idx] = excl;
    excl += v[k];
  }
  if (threadIdx.x == kScanThreads - 1 && sums) sums[blockIdx.x] = sh[threadIdx.x];
  if (threadIdx.x == kScanThreads - 1 && total_out) *total_out = sh[threadIdx.x];  // single-block level
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_add(int64_t* __restrict__ out, const int64_t* __restrict__ offs, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  const int64_t add = offs[blockIdx.x];
  for (int k = threadIdx.x; k < kScanBlock; k += kScanThreads) {
    const int64_t idx = base + k;
    if (idx < n) out[idx] += add;
  }
}

__global__ void k_zero_i64(int64_t* __restrict__ p) { *p = 0; }

// Exclusive scan of one level; the single-block top level also writes the
// grand total to total_out.
template <typename T>
int scan_level(const T* in, int64_t* out, int64_t n, int64_t* scratch, hipStream_t s, int64_t* total_out) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_block<T>, dim3(1), dim3(kScanThreads), 0, s, in, out,
                       (int64_t*)nullptr, n, total_out);
    OBBV_HIP(hipGetLastError());
    return OBBV_OK;
  }
  int64_t* sums = scratch;
  int64_t* sums_scan = scratch + nb;
  hipLaunchKernelGGL(k_scan_block<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, sums,
                     n, (int64_t*)nullptr);
  OBBV_HIP(hipGetLastError());
  OBBV_RET(scan_level<int64_t>(sums, sums_scan, nb, scratch + 2 * nb, s, total_out));
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, sums_scan, n);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}
}  // namespace

size_t exclusive_scan_scratch_bytes(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (m > kScanBlock) {
    m = (m + kScanBlock - 1) / kScanBlock;
    total += 2 * (size_t)m;
  }
  return (total + 8) * sizeof(int64_t);
}

int exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* scratch,
                              size_t scratch_bytes, hipStream_t s) {
  if (n <= 0) {  // a kernel, not a memset node, so the call stays capturable
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, out);
    OBBV_HIP(hipGetLastError());
    return OBBV_OK;
  }
  if (scratch_bytes < exclusive_scan_scratch_bytes(n)) {
    set_error("scan scratch too small");
    return OBBV_ERR_WORKSPACE;
  }
  OBBV_RET(scan_level<int32_t>(in, out, n, (int64_t*)scratch, s, out + n));
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// measurement: event pairs around k_test launches, device test counter
// ---------------------------------------------------------------------------
namespace {
struct ProfState {
  bool enabled = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<hipEvent_t> spare;  // events of earlier reads, reused
  unsigned long long* counter = nullptr;  // [2 kProfSlots]
  int counter_dev = -1;
};
ProfState g_prof;
std::mutex g_prof_mutex;
}  // namespace

bool profiling_enabled() { return g_prof.enabled; }

int profile_counter(unsigned long long** out) {
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  if (!g_prof.counter || g_prof.counter_dev != dev) {
    void* q = nullptr;
    OBBV_HIP(hipMalloc(&q, 2 * kProfSlots * 8));
    OBBV_HIP(hipMemset(q, 0, 2 * kProfSlots * 8));
    g_prof.counter = (unsigned long long*)q;
    g_prof.counter_dev = dev;
  }
  *out = g_prof.counter;
  return OBBV_OK;
}

int profile_record_begin(hipStream_t s, void** token) {
  hipEvent_t ev[2];
  {
    std::lock_guard<std::mutex> lock(g_prof_mutex);
    for (int k = 0; k < 2; ++k) {
      if (g_prof.spare.empty()) {
        OBBV_HIP(hipEventCreate(&ev[k]));
      } else {
        ev[k] = g_prof.spare.back();
        g_prof.spare.pop_back();
      }
    }
  }
  hipEvent_t a = ev[0], b = ev[1];
  OBBV_HIP(hipEventRecord(a, s));
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  g_prof.events.emplace_back(a, b);
  *token = (void*)(g_prof.events.size() - 1);
  return OBBV_OK;
}

int profile_record_end(hipStream_t s, void* token) {
  hipEvent_t b;
  {
    std::lock_guard<std::mutex> lock(g_prof_mutex);
    b = g_prof.events[(size_t)token].second;
  }
  OBBV_HIP(hipEventRecord(b, s));
  return OBBV_OK;
}

}  // namespace obbv

using namespace obbv;

static int obbv_profile_enable_body(int enable);
extern "C" int obbv_profile_enable(int enable) {
  return obbv::guarded([&] { return obbv_profile_enable_body(enable); });
}
static int obbv_profile_enable_body(int enable) {
  clear_error();
  g_prof.enabled = enable != 0;
  if (g_prof.enabled) {
    unsigned long long* c = nullptr;
    OBBV_RET(profile_counter(&c));
  }
  return OBBV_OK;
}

static int obbv_profile_read_body(double* out_test_ms, int64_t* out_launches, int64_t* out_tests,
                                 int64_t* out_bytes, double* out_busy_ms);
extern "C" int obbv_profile_read(double* out_test_ms, int64_t* out_launches, int64_t* out_tests,
                                 int64_t* out_bytes, double* out_busy_ms) {
  return obbv::guarded([&] { return obbv_profile_read_body(out_test_ms, out_launches, out_tests, out_bytes, out_busy_ms); });
}
static int obbv_profile_read_body(double* out_test_ms, int64_t* out_launches, int64_t* out_tests,
                                 int64_t* out_bytes, double* out_busy_ms) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_prof_mutex);
  double total = 0.0;
  // launch intervals from the first launch's start event, merged into the busy time
  std::vector<std::pair<double, double>> iv;
  iv.reserve(g_prof.events.size());
  for (auto& e : g_prof.events) {
    OBBV_HIP(hipEventSynchronize(e.second));
    float ms = 0.f, t0 = 0.f;
    OBBV_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    OBBV_HIP(hipEventElapsedTime(&t0, g_prof.events.front().first, e.first));
    total += ms;
    iv.emplace_back((double)t0, (double)t0 + (double)ms);
  }
  for (auto& e : g_prof.events) {
    g_prof.spare.push_back(e.first);
    g_prof.spare.push_back(e.second);
  }
  std::sort(iv.begin(), iv.end());
  double busy = 0.0, lo = 0.0, hi = -1.0;
  for (const auto& x : iv) {
    if (x.first > hi) {
      if (hi > lo) busy += hi - lo;
      lo = x.first;
      hi = x.second;
    } else {
      hi = std::max(hi, x.second);
    }
  }
  if (hi > lo) busy += hi - lo;
  const int64_t n = (int64_t)g_prof.events.size();
  g_prof.events.clear();
  unsigned long long tests = 0, bytes = 0;
  if (g_prof.counter) {
    OBBV_HIP(hipDeviceSynchronize());
    unsigned long long slots[2 * kProfSlots];
    OBBV_HIP(hipMemcpy(slots, g_prof.counter, sizeof(slots), hipMemcpyDeviceToHost));
    for (int k = 0; k < kProfSlots; ++k) {
      tests += slots[k];
      bytes += slots[kProfSlots + k];
    }
    OBBV_HIP(hipMemset(g_prof.counter, 0, sizeof(slots)));
  }
  if (out_test_ms) *out_test_ms = total;
  if (out_launches) *out_launches = n;
  if (out_tests) *out_tests = (int64_t)tests;
  if (out_bytes) *out_bytes = (int64_t)bytes;
  if (out_busy_ms) *out_busy_ms = busy;
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// C ABI: library
// ---------------------------------------------------------------------------
extern "C" const char* obbv_version(void) { return "obbv 0.1.0 (gfx950)"; }

extern "C" const char* obbv_last_error(void) { return g_last_error.c_str(); }

static int obbv_status_body(void* stream, uint32_t* out_flags);
extern "C" int obbv_status(void* stream, uint32_t* out_flags) {
  return obbv::guarded([&] { return obbv_status_body(stream, out_flags); });
}
static int obbv_status_body(void* stream, uint32_t* out_flags) {
  clear_error();
  hipStream_t s = (hipStream_t)stream;
  uint32_t* st = nullptr;
  OBBV_RET(status_word(&st));
  uint32_t host = 0;
  OBBV_HIP(hipMemcpyAsync(&host, st, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  OBBV_HIP(hipMemsetAsync(st, 0, sizeof(uint32_t), s));
  OBBV_HIP(hipStreamSynchronize(s));
  if (out_flags) *out_flags = host;
  return OBBV_OK;
}

static int obbv_release_body(void);
extern "C" int obbv_release(void) {
  return obbv::guarded([&] { return obbv_release_body(); });
}
static int obbv_release_body(void) {
  clear_error();
  int cur = 0;
  OBBV_HIP(hipGetDevice(&cur));
  std::lock_guard<std::mutex> lock(g_pool_mutex);
  for (int d = 0; d < kMaxDevices; ++d) {
    DevicePool& p = g_pools[d];
    bool any = p.status != nullptr;
    for (int k = 0; k < kPoolCount * kPoolSets; ++k) any = any || p.ptr[k];
    if (!any) continue;
    OBBV_HIP(hipSetDevice(d));
    for (int k = 0; k < kPoolCount * kPoolSets; ++k) {
      if (p.ptr[k]) OBBV_HIP(hipFree(p.ptr[k]));
      p.ptr[k] = nullptr;
      p.cap[k] = 0;
    }
    if (p.status) OBBV_HIP(hipFree(p.status));
    p.status = nullptr;
  }
  OBBV_HIP(hipSetDevice(cur));
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// C ABI: mesh validation (synchronous, host side)
// ---------------------------------------------------------------------------
