// Same-layer Lloyd clustering (Sec. 4.2.1) and the multigrid-like hierarchy
// (Sec. 4.2.2) on top of the outer-volume kernels.
//
// The flood's decisions need a priority queue and mesh adjacency; they run on
// the host.  Every outer-volume value they need -- grown candidate boxes of a
// round of every group of a level, union boxes, parameter-update candidates --
// is evaluated by one batched obbv outer-volume launch sequence per round, so the
// device sees a few large batches per round instead of one box at a time.
//
// Reading of the paper (shared with the CPU oracle):
//   * a box has fixed centre c and axes Q during the partition; its half extents
//     enclose its elements symmetrically: h = max |Q (v - c)| over the vertices;
//   * boxes are stored as float32: centre and axes rounded to nearest, half
//     extents rounded up;
//   * key of an element = distance from its centroid to the nearest centre of its
//     group; each box starts from the element nearest its centre;
//   * a round pops the K smallest-key frontier elements of every group; for each
//     (element, box) the grown box is evaluated unless it equals the current box;
//     dOBV = |OBV(grown) - OBV(current)| (Eq. 12); argmin with ties to the nearer
//     centre, then the lower index (Eq. 13); boxes grow to the union of what they
//     received; unreachable elements are assigned one by one at the end;
//   * parameter update: tight box for the axes, +-delta rotations about each
//     local axis, gradient, line search at {8, 4, 2, 1, 0.5} delta along -g,
//     keep the best if it lowers OBV.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <numeric>
#include <queue>
#include <string>
#include <stdexcept>
#include <exception>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace obbv {

int outer_volume_impl(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                      const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                      const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                      int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side, hipStream_t s,
                      int32_t* out_occ);
int outer_volume_frames(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key, int32_t n_boxes,
                        const obbv_ov_params* params, const obbv_box* frames, const int32_t* box_frame,
                        int32_t n_frames, double* out_obv, hipStream_t s, OvExec* ex);
int outer_volume_exec(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key, int32_t n_boxes,
                      const obbv_ov_params* params, double* out_obv, hipStream_t s, OvExec* ex);
int status_or(uint32_t bits, hipStream_t s);
int fit_impl(const obbv_mesh* mesh, const int32_t* tri_cluster, int32_t n_clusters, obbv_box* out_boxes,
             double* out_eigvals, hipStream_t st);
int mlp_forward_impl(const float* params, const float* X, int32_t n, float* out_f, hipStream_t s);
int mlp_pack_impl(const float* params, short* packed, hipStream_t s);
int64_t mlp_packed_entries();
int mlp_rank_packed(const float* params, const short* packed, const float* volume, int32_t N, const float* frame,
                    const obbv_box* boxes, int32_t n, void* scratch, float* out_f, hipStream_t s,
                    unsigned long long* tag, unsigned seq, const obbv_box* host_boxes);
size_t mlp_rank_scratch_bytes(int32_t n);

namespace {

struct HBox {
  float c[3];
  float Q[9];
  float h[3];
};

// Wall-clock accounting of the Lloyd driver, printed to stderr when the
// environment variable OBBV_LLOYD_TIMING is set (measurement only).
struct WallTimer {
  double s = 0.0;
  std::chrono::steady_clock::time_point t0;
  void start() { t0 = std::chrono::steady_clock::now(); }
  void stop() { s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

// Upload of a call's staging area: the device reads the mapped pinned host
// buffer directly (one launch in the stream, no runtime copy).
__global__ void k_stage(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// host-side sections of the flood rounds (measurement only)
struct FloodTimers {
  WallTimer pops, extents, cands, rank_post, exact_post, decide, grow, pred_pack, pred_launch, pred_wait;
};
static thread_local FloodTimers g_ft;  // per host thread (floods may run on two)

inline float f32_up(double x) {
  float y = (float)x;
  if ((double)y < x) y = nextafterf(y, INFINITY);
  return y;
}

inline bool same_h(const float a[3], const float b[3]) { return a[0] == b[0] && a[1] == b[1] && a[2] == b[2]; }

// ---------------------------------------------------------------------------
// batched outer-volume evaluation on the device
// ---------------------------------------------------------------------------
struct Evaluator {
  obbv_mesh mesh{};
  obbv_ov_params params{};
  // centre of the mesh's bounding box (the kept side of every cast), staged
  // with every call so the device need not compute it
  float centre[4] = {0.f, 0.f, 0.f, 0.f};
  bool have_centre = false;
  void set_centre(const std::vector<float>& V) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (size_t i = 0; i < V.size(); i += 3)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::fmin(lo[k], V[i + k]);
        hi[k] = std::fmax(hi[k], V[i + k]);
      }
    for (int k = 0; k < 3; ++k) centre[k] = V.empty() ? 0.f : 0.5f * (lo[k] + hi[k]);
    centre[3] = 0.f;
    have_centre = true;
  }
  hipStream_t stream = nullptr;
  char* dbuf = nullptr;  // device: boxes, keys, frames, box frames, control words, results
  char* hbuf = nullptr;  // pinned host staging of the same layout
  char* hdev = nullptr;  // hbuf as mapped for the device (results are written there)
  size_t cap = 0;
  WallTimer t_prep, t_dev;
  int64_t evals = 0;
  int64_t calls = 0;
  std::vector<HBox> fr;  // frames of the current call (host)
  // frame grouping buffers, reused from call to call: an open-addressing table
  // of (centre, axes) keys, each box's key group, and the boxes by group
  std::vector<int32_t> gslot, gfirst, gid, gcount, gstart, gmem;
  std::vector<int32_t> box_frame;
  // optional uniform sample (reservoir) of the evaluated (box, outer volume) pairs
  int64_t smp_cap = 0, smp_seen = 0;
  std::vector<HBox> smp_box;
  std::vector<double> smp_val;

  void record(const std::vector<HBox>& boxes, const std::vector<double>& vals) {
    for (size_t i = 0; i < boxes.size(); ++i) {
      const int64_t k = smp_seen++;
      if ((int64_t)smp_box.size() < smp_cap) {
        smp_box.push_back(boxes[i]);
        smp_val.push_back(vals[i]);
      } else {
        const uint64_t j = splitmix64_at(0x5DEECE66Dull, (uint64_t)k) % (uint64_t)(k + 1);
        if ((int64_t)j < smp_cap) {
          smp_box[j] = boxes[i];
          smp_val[j] = vals[i];
        }
      }
    }
  }

  // span bounds of the mesh (reused by every call; the mesh does not change
  // during the state's life); the judge's evaluator borrows the table
  float4* spans = nullptr;
  bool spans_done = false, owns_spans = false;
  int ensure_spans() {
    if (spans_done) return OBBV_OK;
    spans_done = true;
    const size_t bytes = span_table_size(mesh.n_triangles);
    if (!bytes) return OBBV_OK;
    if (hipMalloc((void**)&spans, bytes) != hipSuccess) {
      (void)hipGetLastError();
      spans = nullptr;  // every call then computes its own
      return OBBV_OK;
    }
    owns_spans = true;
    return span_table(&mesh, spans, stream);
  }

  ~Evaluator() {
    if (owns_spans && spans) (void)hipFree(spans);
    if (jtab) (void)hipFree(jtab);
    if (dbuf) (void)hipFree(dbuf);
    if (hbuf) (void)hipHostFree(hbuf);
  }

  static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

  // the evaluation between begin() and finish()
  const std::vector<HBox>* cur_boxes = nullptr;
  size_t cur_n = 0, cur_nf = 0, o_box = 0, o_key = 0, o_frame = 0, o_bf = 0, o_ctl = 0, o_out = 0;
  bool cur_shared = false, in_flight = false;
  int pool_base = 0;  // pool set of the outer-volume scratch (one per concurrent stream)
  int item_tris = 0;    // smaller cast items for its calls with few units (0: never)
  int split_below = 0;  // the unit count below which a call takes them

  // `overlap` (nullable) runs on the host while the device evaluates
  int eval(const std::vector<HBox>& boxes, const std::vector<uint32_t>& keys, std::vector<double>& out,
           const std::function<void()>* overlap = nullptr) {
    OBBV_RET(begin(boxes, keys));
    if (overlap) (*overlap)();
    return finish(out);
  }

  // the device has published the enqueued evaluation (k_finalize's done word)
  bool published() const {
    return __atomic_load_n((const int64_t*)(hbuf + o_ctl + 64) + 4, __ATOMIC_ACQUIRE) != 0;
  }
  // the enqueued evaluation has finished (no wait)
  bool ready() const { return !in_flight || published(); }

  // Jitter table of the keys [0, jkeys) at this R and seed (device), so the
  // ray-test kernel reads the draws instead of recomputing them in every call.
  uint2* jtab = nullptr;
  int64_t jkeys = 0;
  int jR = 0;
  uint64_t jseed = 0;
  bool jtab_use = false;
  static constexpr int64_t kJitterTableBytes = (int64_t)256 << 20;
  // OBBV_JITTER_TABLE=0 turns the table off (the kernel then computes every
  // draw), so the two paths can be compared bit for bit
  const bool jtab_allowed = [] {
    const char* e = getenv("OBBV_JITTER_TABLE");
    return !(e && *e && atoi(e) == 0);
  }();

  int ensure_jitter(const std::vector<uint32_t>& keys) {
    uint32_t kmax = 0;
    for (uint32_t k : keys) kmax = std::max(kmax, k);
    const int R = params.R;
    const int64_t per_key = 3 * (int64_t)R * R * (int64_t)sizeof(uint2);
    const int64_t want = ((int64_t)kmax + 64) / 64 * 64;
    jtab_use = jtab_allowed && want * per_key <= kJitterTableBytes;
    if (!jtab_use) return OBBV_OK;
    if (jtab && want <= jkeys && jR == R && jseed == params.seed) return OBBV_OK;
    if (jtab) {
      OBBV_HIP(hipStreamSynchronize(stream));
      OBBV_HIP(hipFree(jtab));
      jtab = nullptr;
      jkeys = 0;
    }
    if (hipMalloc((void**)&jtab, (size_t)(want * per_key)) != hipSuccess) {
      (void)hipGetLastError();
      jtab = nullptr;
      jtab_use = false;  // evaluate without the table
      return OBBV_OK;
    }
    OBBV_RET(jitter_table(params.seed, R, want, jtab, stream));
    jkeys = want;
    jR = R;
    jseed = params.seed;
    return OBBV_OK;
  }

  int run_call(OvExec* ex) {
    ex->pool_base = pool_base;
    ex->item_tris = item_tris;
    ex->split_below = item_tris ? split_below : 0;
    if (jtab_use) {
      ex->jitter = jtab;
      ex->jitter_R = jR;
      ex->jitter_seed = jseed;
    }
    double* hout = (double*)(hdev + o_out);  // results go straight to pinned host memory
    if (cur_shared)
      return outer_volume_frames(&mesh, (const obbv_box*)(dbuf + o_box), (const uint32_t*)(dbuf + o_key),
                                 (int32_t)cur_n, &params, (const obbv_box*)(dbuf + o_frame),
                                 (const int32_t*)(dbuf + o_bf), (int32_t)cur_nf, hout, stream, ex);
    return outer_volume_exec(&mesh, (const obbv_box*)(dbuf + o_box), (const uint32_t*)(dbuf + o_key),
                             (int32_t)cur_n, &params, hout, stream, ex);
  }

  // Stages the boxes and enqueues their evaluation on `stream`; finish() waits
  // and returns the values.  `boxes` must stay unchanged until finish().
  int begin(const std::vector<HBox>& boxes, const std::vector<uint32_t>& keys) {
    if (in_flight) {
      set_error("internal: evaluation started while another is in flight");
      return OBBV_ERR_INVALID_ARG;
    }
    const size_t n = boxes.size();
    cur_boxes = &boxes;
    cur_n = n;
    in_flight = false;
    if (n == 0) return OBBV_OK;
    t_prep.start();
    // Candidates of one box share its centre and axes: group them into frames so
    // that the mesh is culled and transformed once per frame (against the union
    // of its boxes).  Boxes of one centre and axes are split into size classes
    // (a frame grows while the sum of its half extents stays within 1.6 times
    // that of its smallest box), so small candidates do not walk the triangles
    // of far-grown ones.
    box_frame.resize(n);
    fr.clear();
    {
      // key groups in order of first appearance, boxes in index order within
      // a group (an open-addressing table over the 48 bytes of centre and axes)
      size_t tsize = 16;
      while (tsize < 2 * n) tsize <<= 1;
      gslot.assign(tsize, -1);  // group of a table slot
      gfirst.clear();           // first box of each group
      gid.resize(n);
      auto same_key = [&](size_t x, size_t y) {
        return std::memcmp(boxes[x].c, boxes[y].c, 12) == 0 && std::memcmp(boxes[x].Q, boxes[y].Q, 36) == 0;
      };
      for (size_t i = 0; i < n; ++i) {
        uint32_t w[12];
        std::memcpy(w, boxes[i].c, 12);
        std::memcpy(w + 3, boxes[i].Q, 36);
        uint64_t h = 0x9E3779B97F4A7C15ull;
        for (int k = 0; k < 12; ++k) h = (h ^ w[k]) * 0xFF51AFD7ED558CCDull;
        size_t t = (size_t)(h ^ (h >> 29)) & (tsize - 1);
        while (gslot[t] >= 0 && !same_key((size_t)gfirst[gslot[t]], i)) t = (t + 1) & (tsize - 1);
        if (gslot[t] < 0) {
          gslot[t] = (int32_t)gfirst.size();
          gfirst.push_back((int32_t)i);
        }
        gid[i] = gslot[t];
      }
      const size_t ng = gfirst.size();
      gcount.assign(ng, 0);
      for (size_t i = 0; i < n; ++i) ++gcount[gid[i]];
      gstart.resize(ng + 1);
      gstart[0] = 0;
      for (size_t g = 0; g < ng; ++g) gstart[g + 1] = gstart[g] + gcount[g];
      gmem.resize(n);
      for (size_t g = 0; g < ng; ++g) gcount[g] = gstart[g];
      for (size_t i = 0; i < n; ++i) gmem[gcount[gid[i]]++] = (int32_t)i;
      auto size_of = [](const float h[3]) { return (double)h[0] + (double)h[1] + (double)h[2]; };
      for (size_t g = 0; g < ng; ++g) {
        int32_t* m0 = gmem.data() + gstart[g];
        int32_t* m1 = gmem.data() + gstart[g + 1];
        std::stable_sort(m0, m1, [&](int32_t x, int32_t y) { return size_of(boxes[x].h) < size_of(boxes[y].h); });
        double limit = -1.0;
        for (const int32_t* it = m0; it != m1; ++it) {
          const int32_t i = *it;
          const double si = size_of(boxes[i].h);
          if (fr.empty() || limit < 0.0 || !(si <= limit)) {  // NaN sizes start their own frame
            fr.push_back(boxes[i]);
            limit = 1.6 * si;
          } else {
            HBox& f = fr.back();
            for (int r = 0; r < 3; ++r) f.h[r] = std::fmax(f.h[r], boxes[i].h[r]);
          }
          box_frame[i] = (int32_t)fr.size() - 1;
        }
      }
    }
    const size_t nf = fr.size();
    const bool shared = 2 * nf <= n;
    cur_nf = nf;
    cur_shared = shared;
    o_box = 0;
    o_key = al(n * sizeof(obbv_box));
    o_frame = o_key + al(n * 4);
    o_bf = o_frame + al(nf * sizeof(obbv_box));
    o_ctl = o_bf + al(n * 4);
    o_out = o_ctl + 256;
    const size_t need = o_out + al(n * 8);
    if (need > cap) {
      if (dbuf) {
        OBBV_HIP(hipStreamSynchronize(stream));
        OBBV_HIP(hipFree(dbuf));
        OBBV_HIP(hipHostFree(hbuf));
        dbuf = hbuf = hdev = nullptr;
        cap = 0;
      }
      const size_t want = std::max(need * 2, (size_t)1 << 16);
      if (hipMalloc((void**)&dbuf, want) != hipSuccess) {
        (void)hipGetLastError();
        dbuf = nullptr;
        set_error("hipMalloc failed for the Lloyd evaluation buffer");
        return OBBV_ERR_OOM;
      }
      if (hipHostMalloc((void**)&hbuf, want, hipHostMallocDefault) != hipSuccess ||
          hipHostGetDevicePointer((void**)&hdev, hbuf, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(dbuf);
        if (hbuf) (void)hipHostFree(hbuf);
        dbuf = hbuf = hdev = nullptr;
        set_error("hipHostMalloc failed for the Lloyd evaluation buffer");
        return OBBV_ERR_OOM;
      }
      cap = want;
    }
    auto put = [](obbv_box* d, const HBox& b) {
      std::memcpy(d->center, b.c, 12);
      std::memcpy(d->axes, b.Q, 36);
      std::memcpy(d->half, b.h, 12);
    };
    obbv_box* hb = (obbv_box*)(hbuf + o_box);
    for (size_t i = 0; i < n; ++i) put(hb + i, boxes[i]);
    std::memcpy(hbuf + o_key, keys.data(), n * 4);
    if (shared) {
      obbv_box* hf = (obbv_box*)(hbuf + o_frame);
      for (size_t f = 0; f < nf; ++f) put(hf + f, fr[f]);
      std::memcpy(hbuf + o_bf, box_frame.data(), n * 4);
    }
    // control words: the call's private status word (device, zeroed by the
    // upload); the published status bits and totals (host, written by the device)
    std::memset(hbuf + o_ctl, 0, 256);
    std::memcpy(hbuf + o_ctl + 192, centre, 16);
    t_prep.stop();
    t_dev.start();
    OBBV_RET(ensure_jitter(keys));
    OBBV_RET(ensure_spans());
    {
      const int64_t n16 = (int64_t)(o_out / 16);  // o_out is a multiple of 256
      const unsigned grid = (unsigned)std::min<int64_t>((n16 + 255) / 256, 64);
      hipLaunchKernelGGL(k_stage, dim3(grid), dim3(256), 0, stream, (const uint4*)hdev, (uint4*)dbuf, n16);
      OBBV_HIP(hipGetLastError());
    }
    {  // one pass, no host round trip; finish() spins on the published done word
      OvExec ex;
      ex.status = (uint32_t*)(dbuf + o_ctl);
      ex.publish = (int64_t*)(hdev + o_ctl + 64);
      ex.centre = have_centre ? (const float4*)(dbuf + o_ctl + 192) : nullptr;
      ex.spans = spans;
      ex.span_runs = spans ? span_runs_of(spans, mesh.n_triangles) : nullptr;
      OBBV_RET(run_call(&ex));
      in_flight = true;
    }
    return OBBV_OK;
  }

  int finish(std::vector<double>& out) {
    const size_t n = cur_n;
    out.assign(n, 0.0);
    if (n == 0) return OBBV_OK;
    if (in_flight) {
      in_flight = false;
      // spin on the published done word (no runtime wake-up latency, the host
      // stays warm); after 10 s without it, wait on the stream, which reports a
      // failed launch
      auto t0 = std::chrono::steady_clock::now();
      for (uint64_t spin = 0; !published(); ++spin) {
        if ((spin & 4095) == 4095 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > 10.0) {
          OBBV_HIP(hipStreamSynchronize(stream));
          if (!published()) {
            set_error("outer-volume call finished without publishing");
            return OBBV_ERR_HIP;
          }
          break;
        }
        __builtin_ia32_pause();
      }
      const int64_t* hpub = (const int64_t*)(hbuf + o_ctl + 64);
      const uint32_t st = (uint32_t)hpub[0];
      if (st) OBBV_RET(status_or(st, stream));
    }
    t_dev.stop();
    std::memcpy(out.data(), hbuf + o_out, n * 8);
    evals += (int64_t)n;
    ++calls;
    if (smp_cap > 0) record(*cur_boxes, out);
    return OBBV_OK;
  }
};

// ---------------------------------------------------------------------------
// learned ranker: sampled occupancy features + MLP, batched on the device
// ---------------------------------------------------------------------------
struct Predictor {
  obbv_surrogate cfg{};
  bool on = false;
  hipStream_t stream = nullptr;
  bool paused = false;  // the judge found the ranker off: exact evaluation until the next iteration
  int judge_set = 1;    // pool set of the judge's exact evaluations
  int64_t cfg_gen = 0;  // configuration generation (flood-part predictors follow the state's)
  WallTimer t_pred;
  double err_sum = 0.0;
  int64_t err_n = 0, predicted = 0, fallbacks = 0, calls = 0;
  static constexpr int kWindow = 256;

  // Rolling mean |predicted - exact| outer fraction over the last kWindow verified
  // candidates; above cfg.max_error (once 64 are in) the ranker pauses.
  std::vector<double> window;
  size_t wpos = 0;
  void judge(double err) {
    if ((int)window.size() < kWindow) {
      window.push_back(err);
    } else {
      err_sum -= window[wpos];
      window[wpos] = err;
      wpos = (wpos + 1) % kWindow;
    }
    err_sum += err;
    err_n = (int64_t)window.size();
    if (err_n >= 64 && err_sum / (double)err_n > (double)cfg.max_error) {
      paused = true;
      ++fallbacks;
      window.clear();
      wpos = 0;
      err_sum = 0.0;
      err_n = 0;
    }
  }

  char* hbuf = nullptr;  // pinned staging: boxes in, predictions out (written by the device)
  char* hdev = nullptr;
  size_t hcap = 0;
  short* packed = nullptr;  // bfloat16 transposed weights of cfg.mlp_params
  bool packed_ready = false;
  char* dbuf = nullptr;  // device: bfloat16 input rows and occupancy sums
  size_t dcap = 0;
  unsigned sig_seq = 0;  // call number, in the tag of every prediction word

  // Judge: every judge_every-th ranked round, a sample of the round's candidates
  // is evaluated exactly on a stream of its own (scratch from the second pool
  // set) while the flood goes on; the errors enter the judge when it finishes.
  Evaluator jev;
  hipStream_t jstream = nullptr;
  std::vector<HBox> jboxes;
  std::vector<uint32_t> jkeys;
  std::vector<float> jpred;
  std::vector<double> jvals;
  int64_t judged_evals = 0;
  double jerr_sum = 0.0, jerr_max = 0.0;  // all judged errors (measurement)

  int judge_begin(const Evaluator& ev, const std::vector<HBox>& cb, const std::vector<uint32_t>& ck,
                  const std::vector<float>& fp, size_t n) {
    if (n == 0 || jev.in_flight) return OBBV_OK;
    if (!jstream) {
      OBBV_HIP(hipStreamCreateWithFlags(&jstream, hipStreamNonBlocking));
      jev.stream = jstream;
      jev.pool_base = judge_set * kPoolCount;
    }
    jev.mesh = ev.mesh;
    jev.params = ev.params;
    jev.spans = ev.spans;  // borrowed (the judge never frees it)
    jev.spans_done = true;
    std::memcpy(jev.centre, ev.centre, 16);
    jev.have_centre = ev.have_centre;
    const size_t stride = (n + kWindow - 1) / kWindow;  // at most one window per judged round
    jboxes.clear();
    jkeys.clear();
    jpred.clear();
    for (size_t z = 0; z < n; z += stride) {
      jboxes.push_back(cb[z]);
      jkeys.push_back(ck[z]);
      jpred.push_back(fp[z]);
    }
    return jev.begin(jboxes, jkeys);
  }

  // Takes the finished judge evaluation (waits for it with `wait`).
  int judge_poll(bool wait) {
    if (!jev.in_flight && jev.cur_n == 0) return OBBV_OK;
    if (!wait && !jev.ready()) return OBBV_OK;
    OBBV_RET(jev.finish(jvals));
    jev.cur_n = 0;
    judged_evals += (int64_t)jvals.size();
    for (size_t x = 0; x < jvals.size(); ++x) {
      const HBox& bx = jboxes[x];
      const double vb = 8.0 * (double)bx.h[0] * (double)bx.h[1] * (double)bx.h[2];
      if (vb > 0.0) {
        const double err = std::fabs((double)jpred[x] - jvals[x] / vb);
        jerr_sum += err;
        jerr_max = std::max(jerr_max, err);
        judge(err);
      }
    }
    return OBBV_OK;
  }

  ~Predictor() {
    if (jstream) {
      (void)hipStreamSynchronize(jstream);
      (void)hipStreamDestroy(jstream);
    }
    if (stream) (void)hipStreamSynchronize(stream);
    if (dbuf) (void)hipFree(dbuf);
    if (hbuf) (void)hipHostFree(hbuf);
    if (packed) (void)hipFree(packed);
  }

  // Predicted outer fractions of `boxes`: the boxes are staged in mapped pinned
  // memory (and, for a few, in the kernel arguments), one launch (two for many
  // boxes) samples their inputs and runs the network, and every prediction
  // lands in mapped memory as one 64-bit word tagged with the call number, which
  // the host spins on (no completion counter or flag on the device).
  int predict(const std::vector<HBox>& boxes_a, const std::vector<HBox>& boxes_b, std::vector<float>& out,
              const std::function<void()>* overlap = nullptr) {
    const size_t na = boxes_a.size(), n = na + boxes_b.size();
    out.assign(n, 0.f);
    if (n == 0) return OBBV_OK;
    t_pred.start();
    const size_t o_f = (n * sizeof(obbv_box) + 255) & ~(size_t)255;
    const size_t hneed = o_f + n * 8;
    if (hneed > hcap) {
      OBBV_HIP(hipStreamSynchronize(stream));
      if (hbuf) OBBV_HIP(hipHostFree(hbuf));
      hbuf = hdev = nullptr;
      hcap = 0;
      const size_t hwant = std::max(hneed * 2, (size_t)1 << 16);
      if (hipHostMalloc((void**)&hbuf, hwant, hipHostMallocDefault) != hipSuccess ||
          hipHostGetDevicePointer((void**)&hdev, hbuf, 0) != hipSuccess) {
        (void)hipGetLastError();
        set_error("allocation failed for the ranker buffers");
        return OBBV_ERR_OOM;
      }
      std::memset(hbuf, 0, hwant);  // no stale tag in the prediction words
      hcap = hwant;
    }
    const size_t dneed = mlp_rank_scratch_bytes((int32_t)n);
    if (dneed > dcap) {
      OBBV_HIP(hipStreamSynchronize(stream));
      if (dbuf) OBBV_HIP(hipFree(dbuf));
      dbuf = nullptr;
      dcap = 0;
      const size_t want = std::max(dneed * 2, (size_t)1 << 20);
      if (hipMalloc((void**)&dbuf, want) != hipSuccess) {
        (void)hipGetLastError();
        dbuf = nullptr;
        set_error("allocation failed for the ranker inputs");
        return OBBV_ERR_OOM;
      }
      dcap = want;
    }
    g_ft.pred_pack.start();
    obbv_box* hb = (obbv_box*)hbuf;
    for (size_t i = 0; i < n; ++i) {
      const HBox& bx = i < na ? boxes_a[i] : boxes_b[i - na];
      std::memcpy(hb[i].center, bx.c, 12);
      std::memcpy(hb[i].axes, bx.Q, 36);
      std::memcpy(hb[i].half, bx.h, 12);
    }
    g_ft.pred_pack.stop();
    if (!packed) {
      if (hipMalloc((void**)&packed, (size_t)mlp_packed_entries() * 2) != hipSuccess) {
        (void)hipGetLastError();
        packed = nullptr;
        set_error("allocation failed for the ranker weights");
        return OBBV_ERR_OOM;
      }
    }
    if (!packed_ready) {
      OBBV_RET(mlp_pack_impl(cfg.mlp_params, packed, stream));
      packed_ready = true;
    }
    // a tag no word holds yet (words of earlier calls carry smaller numbers, a
    // fresh buffer zeros)
    const unsigned seq = ++sig_seq == 0u ? ++sig_seq : sig_seq;
    uint64_t* words = reinterpret_cast<uint64_t*>(hbuf + o_f);
    g_ft.pred_launch.start();
    OBBV_RET(mlp_rank_packed(cfg.mlp_params, packed, cfg.volume, cfg.N, cfg.frame, (const obbv_box*)hdev, (int32_t)n,
                             dbuf, nullptr, stream, reinterpret_cast<unsigned long long*>(hdev + o_f), seq, hb));
    g_ft.pred_launch.stop();
    if (overlap) (*overlap)();  // host work for later rounds while the device ranks
    g_ft.pred_wait.start();
    // spin on the tagged words, in order (no runtime wake-up latency); after 10 s
    // without them, wait on the stream, which reports a failed launch
    auto t0 = std::chrono::steady_clock::now();
    uint64_t spin = 0;
    for (size_t i = 0; i < n; ++i) {
      uint64_t w;
      while (((w = __atomic_load_n(&words[i], __ATOMIC_ACQUIRE)) >> 32) != seq) {
        if ((++spin & 4095) == 0 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > 10.0) {
          OBBV_HIP(hipStreamSynchronize(stream));
          if ((__atomic_load_n(&words[i], __ATOMIC_ACQUIRE) >> 32) != seq) {
            set_error("ranker kernels finished without writing every prediction");
            return OBBV_ERR_HIP;
          }
        }
        __builtin_ia32_pause();
      }
      const uint32_t bits = (uint32_t)w;
      std::memcpy(&out[i], &bits, 4);
    }
    g_ft.pred_wait.stop();
    predicted += (int64_t)n;
    ++calls;
    t_pred.stop();
    return OBBV_OK;
  }
};

// ---------------------------------------------------------------------------
// host copy of the mesh: vertices, triangles, centroids, edge adjacency
// ---------------------------------------------------------------------------
struct HostMesh {
  std::vector<float> V;
  std::vector<int32_t> F;
  int nv = 0, nt = 0;
  std::vector<double> cen;            // [nt][3]
  std::vector<int32_t> adj_off, adj;  // CSR of edge-adjacent triangles (sorted)

  int load(const obbv_mesh* m, hipStream_t s) {
    nv = m->n_vertices;
    nt = m->n_triangles;
    V.resize((size_t)nv * 3);
    F.resize((size_t)nt * 3);
    if (nv) OBBV_HIP(hipMemcpyAsync(V.data(), m->vertices, V.size() * 4, hipMemcpyDeviceToHost, s));
    if (nt) OBBV_HIP(hipMemcpyAsync(F.data(), m->triangles, F.size() * 4, hipMemcpyDeviceToHost, s));
    OBBV_HIP(hipStreamSynchronize(s));
    for (int32_t x : F)
      if (x < 0 || x >= nv) {
        set_error("triangle index out of range");
        return OBBV_ERR_INVALID_ARG;
      }
    cen.resize((size_t)nt * 3);
    for (int t = 0; t < nt; ++t)
      for (int d = 0; d < 3; ++d) {
        const double a = V[3 * F[3 * t + 0] + d], b = V[3 * F[3 * t + 1] + d], c = V[3 * F[3 * t + 2] + d];
        cen[3 * t + d] = ((a + b) + c) / 3.0;
      }
    // adjacency through sorted undirected edge keys
    std::vector<std::pair<uint64_t, int32_t>> e;
    e.reserve((size_t)nt * 3);
    for (int t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k) {
        uint32_t a = (uint32_t)F[3 * t + k], b = (uint32_t)F[3 * t + (k + 1) % 3];
        if (a > b) std::swap(a, b);
        e.emplace_back(((uint64_t)a << 32) | b, t);
      }
    std::sort(e.begin(), e.end());
    std::vector<std::vector<int32_t>> nb((size_t)nt);
    for (size_t i = 0; i < e.size();) {
      size_t j = i;
      while (j < e.size() && e[j].first == e[i].first) ++j;
      for (size_t x = i; x < j; ++x)
        for (size_t y = i; y < j; ++y)
          if (e[x].second != e[y].second) nb[e[x].second].push_back(e[y].second);
      i = j;
    }
    adj_off.assign((size_t)nt + 1, 0);
    for (int t = 0; t < nt; ++t) {
      auto& v = nb[t];
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      adj_off[t + 1] = adj_off[t] + (int32_t)v.size();
    }
    adj.resize(adj_off[nt]);
    for (int t = 0; t < nt; ++t) std::copy(nb[t].begin(), nb[t].end(), adj.begin() + adj_off[t]);
    return OBBV_OK;
  }

  // local coordinates Q (v - c), summed in axis order (float64)
  inline void local(int vi, const float c[3], const double Q[9], double out[3]) const {
    const double p0 = (double)V[3 * vi + 0] - (double)c[0];
    const double p1 = (double)V[3 * vi + 1] - (double)c[1];
    const double p2 = (double)V[3 * vi + 2] - (double)c[2];
    for (int r = 0; r < 3; ++r) out[r] = (p0 * Q[3 * r + 0] + p1 * Q[3 * r + 1]) + p2 * Q[3 * r + 2];
  }
};

// ---------------------------------------------------------------------------
// flood elements: single triangles, or units made of several triangles
// ---------------------------------------------------------------------------
struct Elements {
  int n = 0;
  std::vector<int32_t> tri_off, tris;  // CSR: triangles of each element
  std::vector<double> cen;             // [n][3] element centroid
  std::vector<int32_t> adj_off, adj;   // CSR: adjacent elements
  std::vector<int64_t> vtx_off;        // CSR into vtx (3 doubles per vertex)
  std::vector<double> vtx;             // the vertices of each element's triangles

  // float64 copies of the vertices of every element's triangles, element by
  // element (the extent test of a candidate reads one contiguous run)
  void build_vertices(const HostMesh& M) {
    vtx_off.assign((size_t)n + 1, 0);
    vtx.clear();
    vtx.reserve((size_t)tris.size() * 9);
    for (int e = 0; e < n; ++e) {
      for (int x = tri_off[e]; x < tri_off[e + 1]; ++x)
        for (int k = 0; k < 3; ++k) {
          const int vi = M.F[3 * tris[x] + k];
          for (int d = 0; d < 3; ++d) vtx.push_back((double)M.V[3 * vi + d]);
        }
      vtx_off[e + 1] = (int64_t)vtx.size();
    }
  }

  static Elements triangles(const HostMesh& M) {
    Elements E;
    E.n = M.nt;
    E.tri_off.resize((size_t)M.nt + 1);
    E.tris.resize((size_t)M.nt);
    for (int t = 0; t <= M.nt; ++t) E.tri_off[t] = t;
    std::iota(E.tris.begin(), E.tris.end(), 0);
    E.cen = M.cen;
    E.adj_off = M.adj_off;
    E.adj = M.adj;
    E.build_vertices(M);
    return E;
  }
};

// element_extent with the box centre and axes already in float64 (the same
// arithmetic, from the element's contiguous vertex copies)
inline void element_extent_fast(const Elements& E, int e, const double c[3], const double Q[9], double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  for (int64_t x = E.vtx_off[e]; x < E.vtx_off[e + 1]; x += 3) {
    const double p0 = E.vtx[x] - c[0], p1 = E.vtx[x + 1] - c[1], p2 = E.vtx[x + 2] - c[2];
    for (int r = 0; r < 3; ++r)
      out[r] = std::max(out[r], std::fabs((p0 * Q[3 * r + 0] + p1 * Q[3 * r + 1]) + p2 * Q[3 * r + 2]));
  }
}

// per-axis max over the element's vertices of |Q (v - c)|
void element_extent(const HostMesh& M, const Elements& E, int e, const HBox& b, double out[3]) {
  double Q[9];
  for (int k = 0; k < 9; ++k) Q[k] = b.Q[k];
  out[0] = out[1] = out[2] = 0.0;
  for (int x = E.tri_off[e]; x < E.tri_off[e + 1]; ++x) {
    const int t = E.tris[x];
    for (int k = 0; k < 3; ++k) {
      double p[3];
      M.local(M.F[3 * t + k], b.c, Q, p);
      for (int r = 0; r < 3; ++r) out[r] = std::max(out[r], std::fabs(p[r]));
    }
  }
}

inline double dist3(const double* a, const float* c) {
  const double d0 = a[0] - (double)c[0], d1 = a[1] - (double)c[1], d2 = a[2] - (double)c[2];
  return std::sqrt((d0 * d0 + d1 * d1) + d2 * d2);
}

// ---------------------------------------------------------------------------
// one partition step for many groups in lockstep
// ---------------------------------------------------------------------------
struct Group {
  std::vector<int32_t> elems;  // sorted element ids
  std::vector<int32_t> boxes;  // global box ids; local index = position
};

struct Counters {
  int64_t evals = 0, rounds = 0, trivial = 0, moves = 0;
};

struct PartitionIO {
  std::vector<HBox>* boxes;        // in: centres / axes; out: grown boxes
  std::vector<double>* obv;        // out: OBV of the grown boxes
  std::vector<uint32_t>* slot;     // jitter key per box
  std::vector<int32_t>* elem_box;  // out: box of each element (-1 = none)
};

int flood_partition(const HostMesh& M, const Elements& E, const std::vector<Group>& groups, PartitionIO io,
                    int K, Evaluator& ev, Counters& cnt, Predictor* pred) {
  std::vector<HBox>& boxes = *io.boxes;
  std::vector<double>& obv = *io.obv;
  std::vector<int32_t>& eb = *io.elem_box;
  const std::vector<uint32_t>& slot = *io.slot;
  const int G = (int)groups.size();
  eb.assign((size_t)E.n, -1);
  std::vector<int32_t> elem_group((size_t)E.n, -1);
  for (int g = 0; g < G; ++g)
    for (int e : groups[g].elems) elem_group[e] = g;
  using QE = std::pair<double, int32_t>;
  std::vector<std::priority_queue<QE, std::vector<QE>, std::greater<QE>>> heap((size_t)G);
  std::vector<char> queued((size_t)E.n, 0);
  std::vector<double> key((size_t)E.n, 0.0);

  // keys, seeds, initial boxes
  std::vector<HBox> req_boxes;
  std::vector<uint32_t> req_keys;
  std::vector<int32_t> req_box;
  for (int g = 0; g < G; ++g) {
    const Group& gr = groups[g];
    const int b = (int)gr.boxes.size();
    if (gr.elems.empty() || b == 0) continue;
    for (int e : gr.elems) {
      double k = INFINITY;
      for (int i = 0; i < b; ++i) k = std::min(k, dist3(&E.cen[3 * e], boxes[gr.boxes[i]].c));
      key[e] = k;
    }
    std::vector<char> chosen;  // small: membership via eb
    for (int i = 0; i < b && i < (int)gr.elems.size(); ++i) {
      const int bi = gr.boxes[i];
      int best = -1;
      double bd = INFINITY;
      for (int e : gr.elems) {
        if (eb[e] >= 0) continue;
        const double d = dist3(&E.cen[3 * e], boxes[bi].c);
        if (d < bd || (d == bd && e < best)) {
          bd = d;
          best = e;
        }
      }
      eb[best] = bi;
      double ext[3];
      element_extent(M, E, best, boxes[bi], ext);
      for (int r = 0; r < 3; ++r) boxes[bi].h[r] = f32_up(ext[r]);
      req_boxes.push_back(boxes[bi]);
      req_keys.push_back(slot[bi]);
      req_box.push_back(bi);
    }
  }
  std::vector<double> vals;
  OBBV_RET(ev.eval(req_boxes, req_keys, vals));
  cnt.evals += (int64_t)vals.size();
  for (size_t x = 0; x < vals.size(); ++x) obv[req_box[x]] = vals[x];
  for (int g = 0; g < G; ++g)
    for (int e : groups[g].elems)
      if (eb[e] >= 0) queued[e] = 1;
  auto push_neighbours = [&](int e) {
    const int g = elem_group[e];
    for (int x = E.adj_off[e]; x < E.adj_off[e + 1]; ++x) {
      const int n = E.adj[x];
      if (elem_group[n] == g && eb[n] < 0 && !queued[n]) {
        queued[n] = 1;
        heap[g].push({key[n], n});
      }
    }
  };
  for (int g = 0; g < G; ++g)
    for (int e : groups[g].elems)
      if (eb[e] >= 0) push_neighbours(e);

  // Boxes that grew at the end of a round to a size none of their evaluated
  // candidates had: their outer volume is evaluated with the next round that
  // evaluates candidates (one device call per round; the values are the same).
  std::vector<int32_t> stale;
  std::vector<char> is_stale(boxes.size(), 0);
  int64_t round_no = 0;
  auto flush_stale = [&]() -> int {
    if (stale.empty()) return OBBV_OK;
    req_boxes.clear();
    req_keys.clear();
    for (int bi : stale) {
      req_boxes.push_back(boxes[bi]);
      req_keys.push_back(slot[bi]);
    }
    OBBV_RET(ev.eval(req_boxes, req_keys, vals));
    cnt.evals += (int64_t)vals.size();
    for (size_t x = 0; x < stale.size(); ++x) {
      obv[stale[x]] = vals[x];
      is_stale[stale[x]] = 0;
    }
    stale.clear();
    return OBBV_OK;
  };

  // one decision round over the given pops of every group
  struct Cand {
    int e, g, li;  // element, group, local box index
    float h[3];
    bool trivial;
    double val;
  };
  // round buffers, reused from round to round
  std::vector<Cand> cands;
  std::vector<HBox> cb;        // candidate boxes to evaluate
  std::vector<uint32_t> ck;    // their jitter keys
  std::vector<int32_t> cidx;   // their candidate indices
  std::vector<double> dpred;   // predicted change per candidate
  std::vector<char> predicted_c, evaluated, keep;
  std::vector<float> fcand, fp;
  std::vector<HBox> pb, rb;
  std::vector<uint32_t> rk;
  std::vector<int32_t> ri, cur_of((size_t)boxes.size(), -1), touched;
  std::vector<uint64_t> rmask;  // containment mask of each pop of the round
  std::vector<char> in_touched(boxes.size(), 0);
  std::vector<std::vector<std::pair<double, size_t>>> per_box((size_t)boxes.size());
  std::vector<std::vector<int32_t>> got((size_t)boxes.size());  // candidate index per receiving box
  // Centres and axes of every group's boxes in float64.  Only the half extents
  // change during the flood, so an element's extent in a box frame does not
  // depend on the decisions: the extents of a round's pops are computed while
  // the device works on the round before.
  std::vector<std::vector<double>> gbc((size_t)G), gbQ((size_t)G);
  for (int g = 0; g < G; ++g) {
    const Group& gr = groups[g];
    gbc[g].resize(gr.boxes.size() * 3);
    gbQ[g].resize(gr.boxes.size() * 9);
    for (size_t i = 0; i < gr.boxes.size(); ++i) {
      const HBox& bx = boxes[gr.boxes[i]];
      for (int k = 0; k < 3; ++k) gbc[g][3 * i + k] = bx.c[k];
      for (int k = 0; k < 9; ++k) gbQ[g][9 * i + k] = bx.Q[k];
    }
  }
  // Containment masks: bit i of a pop's mask is set when box i of its group
  // already contains the element (extent <= half extent on every axis).  Boxes
  // only grow during the flood, so a set bit stays true; a clear bit can turn
  // true only for a box that grew after the mask was taken, and the round
  // re-tests exactly those boxes.  Groups of more than 64 boxes go without, and
  // OBBV_FLOOD_MASKS=0 turns the masks off (every pop then builds its candidate
  // boxes), so the two paths can be compared bit for bit.
  size_t max_group = 0;
  for (int g = 0; g < G; ++g) max_group = std::max(max_group, groups[g].boxes.size());
  const char* masks_env = getenv("OBBV_FLOOD_MASKS");
  const bool use_mask = max_group <= 64 && !(masks_env && *masks_env && atoi(masks_env) == 0);
  // the round in which each box last grew (-1: not during this flood)
  std::vector<int64_t> grown_at(boxes.size(), -1);
  auto contains = [](const double* ext, const float h[3]) {
    return ext[0] <= (double)h[0] && ext[1] <= (double)h[1] && ext[2] <= (double)h[2];
  };
  // extents [pop][box of its group][3] and the pops' containment masks, pops in
  // group order
  auto pop_extents = [&](const std::vector<std::vector<int32_t>>& pops, std::vector<double>& out,
                         std::vector<uint64_t>& mask) {
    g_ft.extents.start();
    size_t total = 0, npop = 0;
    for (int g = 0; g < G; ++g) {
      total += pops[g].size() * groups[g].boxes.size();
      npop += pops[g].size();
    }
    out.resize(total * 3);
    mask.assign(npop, 0);
    size_t x = 0, p = 0;
    for (int g = 0; g < G; ++g) {
      const size_t b = groups[g].boxes.size();
      for (int e : pops[g]) {
        uint64_t m = 0;
        for (size_t i = 0; i < b; ++i, x += 3) {
          element_extent_fast(E, e, &gbc[g][3 * i], &gbQ[g][9 * i], &out[x]);
          if (use_mask && contains(&out[x], boxes[groups[g].boxes[i]].h)) m |= 1ull << i;
        }
        mask[p++] = m;
      }
    }
    g_ft.extents.stop();
  };
  // `overlap` (the next round's pops and their extents) runs once per round,
  // while the device works if the round makes a device call, else at its end
  auto round = [&](const std::vector<std::vector<int32_t>>& pops, const std::vector<double>& pext,
                   const std::vector<uint64_t>& pmask, const std::function<void()>& overlap) -> int {
    bool overlapped = false;
    const std::function<void()> overlap_once = [&]() {
      if (!overlapped) {
        overlapped = true;
        overlap();
      }
    };
    g_ft.cands.start();
    const int64_t rno = cnt.rounds;
    size_t total = 0;
    for (int g = 0; g < G; ++g) total += pops[g].size() * groups[g].boxes.size();
    cands.resize(total);  // at most this many entries are written below
    // appended (their capacity is kept from round to round: no re-initialised
    // elements)
    cb.clear();
    ck.clear();
    cidx.clear();
    size_t nc = 0, px = 0, p = 0, npop = 0;
    for (int g = 0; g < G; ++g) npop += pops[g].size();
    rmask.assign(npop, 0);
    // a box that already contains the element has dOBV = 0, the minimum: then the
    // element's other candidates need no evaluation.  Such a pop (a non-zero
    // containment mask, after re-testing the boxes that grew in the previous
    // round) takes no candidate entries: its decision is taken from the mask.
    for (int g = 0; g < G; ++g) {
      const Group& gr = groups[g];
      const int b = (int)gr.boxes.size();
      uint64_t regrown = 0;
      if (use_mask)
        for (int i = 0; i < b; ++i) regrown |= grown_at[gr.boxes[i]] == rno - 1 ? 1ull << i : 0ull;
      for (int e : pops[g]) {
        if (use_mask) {
          uint64_t m = pmask[p];
          for (uint64_t t = regrown & ~m; t; t &= t - 1) {
            const int i = __builtin_ctzll(t);
            if (contains(&pext[3 * (px + i)], boxes[gr.boxes[i]].h)) m |= 1ull << i;
          }
          rmask[p] = m;
          if (m) {
            cnt.trivial += __builtin_popcountll(m);
            px += b;
            ++p;
            continue;
          }
        }
        ++p;
        const size_t first = nc;
        bool any_trivial = false;
        for (int i = 0; i < b; ++i) {
          const HBox& bx = boxes[gr.boxes[i]];
          const double* ext = &pext[3 * px++];
          Cand& c = cands[nc++];
          c.e = e;
          c.g = g;
          c.li = i;
          // an axis the element does not widen keeps the box's (float) extent
          for (int r = 0; r < 3; ++r) c.h[r] = ext[r] <= (double)bx.h[r] ? bx.h[r] : f32_up(ext[r]);
          c.trivial = same_h(c.h, bx.h);
          c.val = 0.0;
          if (c.trivial) {
            ++cnt.trivial;
            any_trivial = true;
          }
        }
        if (any_trivial) continue;
        for (int i = 0; i < b; ++i) {
          cb.push_back(boxes[gr.boxes[i]]);
          std::memcpy(cb.back().h, cands[first + i].h, 12);
          ck.push_back(slot[gr.boxes[i]]);
          cidx.push_back((int32_t)(first + i));
        }
      }
    }
    g_ft.cands.stop();
    // Learned ranking.  The ranker predicts the outer fraction of every candidate
    // and of the current boxes; the predicted change of a move is
    // f(grown) V(grown) - f(current) V(current) (the two predictions share most of
    // their error).  For every receiving box only the verify_top candidates with
    // the smallest predicted change are evaluated exactly; the other candidates
    // are decided on the prediction.
    dpred.assign(nc, 0.0);
    predicted_c.assign(nc, 0);
    fcand.clear();  // prediction of each kept candidate (judge)
    const bool ranked = pred && pred->on && !pred->paused && !cidx.empty();
    const bool judge_round = ranked && round_no % std::max(1, pred->cfg.judge_every) == 0;
    ++round_no;
    if (ranked) {
      pb.clear();  // the current boxes, predicted after the candidates
      for (int32_t x : cidx) {
        const int bi = groups[cands[x].g].boxes[cands[x].li];
        if (cur_of[bi] < 0) {
          cur_of[bi] = (int32_t)(cb.size() + pb.size());
          pb.push_back(boxes[bi]);
        }
      }
      OBBV_RET(pred->predict(cb, pb, fp, &overlap_once));
      if (judge_round) {
        // the previous judge evaluation enters the judge now (waiting for it if
        // needed), then this round's sample is sent: the judged rounds and the
        // round at which their errors count are fixed, whatever the timing
        const int64_t before = pred->judged_evals;
        OBBV_RET(pred->judge_poll(true));
        cnt.evals += pred->judged_evals - before;
        OBBV_RET(pred->judge_begin(ev, cb, ck, fp, cidx.size()));
      }
      g_ft.rank_post.start();
      const size_t top = (size_t)std::max(0, pred->cfg.verify_top);
      const bool rank_top = top > 0;
      for (size_t z = 0; z < cidx.size(); ++z) {
        const Cand& c = cands[cidx[z]];
        const int bi = groups[c.g].boxes[c.li];
        const HBox& cu = boxes[bi];
        const double vg = 8.0 * (double)c.h[0] * (double)c.h[1] * (double)c.h[2];
        const double vc = 8.0 * (double)cu.h[0] * (double)cu.h[1] * (double)cu.h[2];
        const double d = (double)fp[z] * vg - (double)fp[cur_of[bi]] * vc;
        dpred[cidx[z]] = std::max(d, 0.0);
        predicted_c[cidx[z]] = 1;
        if (rank_top) per_box[bi].push_back({dpred[cidx[z]], z});
      }
      for (int32_t x : cidx) cur_of[groups[cands[x].g].boxes[cands[x].li]] = -1;
      // the verify_top smallest predicted changes of every receiving box are
      // evaluated exactly
      keep.assign(cidx.size(), 0);
      if (rank_top)
        for (auto& v : per_box) {
          if (v.empty()) continue;
          std::sort(v.begin(), v.end());
          for (size_t q = 0; q < std::min(top, v.size()); ++q) keep[v[q].second] = 1;
          v.clear();
        }
      rb.clear();
      rk.clear();
      ri.clear();
      for (size_t z = 0; z < cidx.size(); ++z)
        if (keep[z]) {
          rb.push_back(cb[z]);
          rk.push_back(ck[z]);
          ri.push_back(cidx[z]);
          fcand.push_back(fp[z]);
        }
      cb.swap(rb);
      ck.swap(rk);
      cidx.swap(ri);
      g_ft.rank_post.stop();
    }
    // one device call, if any candidate needs an exact value: the stale boxes
    // (their exact volumes enter the exact changes), then the candidates
    const size_t ns = cb.empty() ? 0 : stale.size();
    req_boxes.clear();
    req_keys.clear();
    vals.clear();
    if (!cb.empty()) {
      for (int bi : stale) {
        req_boxes.push_back(boxes[bi]);
        req_keys.push_back(slot[bi]);
      }
      req_boxes.insert(req_boxes.end(), cb.begin(), cb.end());
      req_keys.insert(req_keys.end(), ck.begin(), ck.end());
      OBBV_RET(ev.eval(req_boxes, req_keys, vals, &overlap_once));
      cnt.evals += (int64_t)vals.size();
      for (size_t x = 0; x < ns; ++x) {
        obv[stale[x]] = vals[x];
        is_stale[stale[x]] = 0;
      }
      stale.clear();
    }
    g_ft.exact_post.start();
    evaluated.assign(nc, 0);
    for (size_t x = 0; x < cidx.size(); ++x) {
      cands[cidx[x]].val = vals[ns + x];
      evaluated[cidx[x]] = 1;
    }
    if (!fcand.empty()) {  // the exact kernel judges the ranker
      for (size_t x = 0; x < cidx.size(); ++x) {
        const HBox& bx = req_boxes[ns + x];
        const double vb = 8.0 * (double)bx.h[0] * (double)bx.h[1] * (double)bx.h[2];
        if (vb > 0.0) pred->judge(std::fabs((double)fcand[x] - vals[ns + x] / vb));
      }
    }
    g_ft.exact_post.stop();
    // decisions
    g_ft.decide.start();
    touched.clear();
    size_t ci = 0;
    p = 0;
    for (int g = 0; g < G; ++g) {
      const Group& gr = groups[g];
      const int b = (int)gr.boxes.size();
      for (int e : pops[g]) {
        const uint64_t m = rmask[p++];
        if (m) {  // the containing box nearest the element (first on ties) takes it, unchanged
          int best = -1;
          double bdist = 0.0;
          for (uint64_t t = m; t; t &= t - 1) {
            const int i = __builtin_ctzll(t);
            const double dd = dist3(&E.cen[3 * e], boxes[gr.boxes[i]].c);
            if (best < 0 || dd < bdist) {
              best = i;
              bdist = dd;
            }
          }
          const int bi = gr.boxes[best];
          eb[e] = bi;
          ++cnt.moves;
          if (!in_touched[bi]) {
            in_touched[bi] = 1;
            touched.push_back(bi);
          }
          continue;
        }
        int best = -1;
        double bd = 0.0, bdist = 0.0;
        for (int i = 0; i < b; ++i) {
          const Cand& c = cands[ci + i];
          const int bi = gr.boxes[i];
          double d;
          if (c.trivial)
            d = 0.0;
          else if (evaluated[ci + i])
            d = std::fabs(c.val - obv[bi]);
          else if (predicted_c[ci + i])
            d = dpred[ci + i];
          else
            continue;  // another box contains the element
          const double dd = dist3(&E.cen[3 * e], boxes[bi].c);
          if (best < 0 || d < bd || (d == bd && (dd < bdist || (dd == bdist && i < best)))) {
            best = i;
            bd = d;
            bdist = dd;
          }
        }
        const int bi = gr.boxes[best];
        eb[e] = bi;
        ++cnt.moves;
        if (!in_touched[bi]) {
          in_touched[bi] = 1;
          touched.push_back(bi);
        }
        got[bi].push_back((int32_t)(ci + best));
        ci += b;
      }
    }
    g_ft.decide.stop();
    // grow the receiving boxes to the union
    g_ft.grow.start();
    for (int bi : touched) {
      in_touched[bi] = 0;
      // a box that took only elements it contained keeps its size
      if (got[bi].empty()) continue;
      float hn[3];
      std::memcpy(hn, cands[got[bi][0]].h, 12);
      for (size_t x = 1; x < got[bi].size(); ++x)
        for (int r = 0; r < 3; ++r) hn[r] = std::max(hn[r], cands[got[bi][x]].h[r]);
      if (!same_h(hn, boxes[bi].h)) {
        std::memcpy(boxes[bi].h, hn, 12);
        grown_at[bi] = rno;
        bool found = false;
        for (int cx : got[bi])
          if (evaluated[cx] && same_h(cands[cx].h, hn)) {
            obv[bi] = cands[cx].val;
            found = true;
            break;
          }
        if (!found && !is_stale[bi]) {
          is_stale[bi] = 1;
          stale.push_back(bi);
        }
      }
      got[bi].clear();
    }
    g_ft.grow.stop();
    overlap_once();
    return OBBV_OK;
  };

  // The pop sequence does not depend on the decisions (a popped element's
  // neighbours enter the frontier whichever box takes it, and only unassigned
  // elements are ever in the frontier), so the next round's pops are taken while
  // the device works on the current round.
  std::vector<std::vector<int32_t>> pops((size_t)G), next((size_t)G);
  auto take_pops = [&](std::vector<std::vector<int32_t>>& out) -> bool {
    g_ft.pops.start();
    bool any = false;
    for (int g = 0; g < G; ++g) {
      out[g].clear();
      while (!heap[g].empty() && (int)out[g].size() < K) {
        const int e = heap[g].top().second;
        heap[g].pop();
        if (eb[e] < 0) out[g].push_back(e);
      }
      any = any || !out[g].empty();
    }
    g_ft.pops.stop();
    return any;
  };
  bool any_next = false;
  std::vector<double> ext, next_ext;
  std::vector<uint64_t> pmask, next_mask;
  const std::function<void()> advance = [&]() {
    g_ft.pops.start();
    for (int g = 0; g < G; ++g)
      for (int e : pops[g]) push_neighbours(e);
    g_ft.pops.stop();
    any_next = take_pops(next);
    pop_extents(next, next_ext, next_mask);
  };
  bool any = take_pops(pops);
  pop_extents(pops, ext, pmask);
  while (any) {
    ++cnt.rounds;
    OBBV_RET(round(pops, ext, pmask, advance));
    pops.swap(next);
    ext.swap(next_ext);
    pmask.swap(next_mask);
    any = any_next;
  }
  // elements no flood reached: one by one, in index order, all groups in lockstep
  std::vector<std::vector<int32_t>> left((size_t)G);
  size_t maxleft = 0;
  for (int g = 0; g < G; ++g) {
    if (groups[g].boxes.empty()) continue;
    for (int e : groups[g].elems)
      if (eb[e] < 0) left[g].push_back(e);
    maxleft = std::max(maxleft, left[g].size());
  }
  for (size_t p = 0; p < maxleft; ++p) {
    for (int g = 0; g < G; ++g) {
      pops[g].clear();
      if (p < left[g].size()) pops[g].push_back(left[g][p]);
    }
    ++cnt.rounds;
    pop_extents(pops, ext, pmask);
    OBBV_RET(round(pops, ext, pmask, [] {}));
  }
  if (pred && pred->on) {
    const int64_t before = pred->judged_evals;
    OBBV_RET(pred->judge_poll(true));
    cnt.evals += pred->judged_evals - before;
  }
  return flush_stale();
}

// ---------------------------------------------------------------------------
// parameter update
// ---------------------------------------------------------------------------
void mat3_mul(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = (A[3 * i + 0] * B[0 + j] + A[3 * i + 1] * B[3 + j]) + A[3 * i + 2] * B[6 + j];
}

void rot_local(int k, double th, double R[9]) {
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  const int a = (k + 1) % 3, b = (k + 2) % 3;
  const double c = std::cos(th), s = std::sin(th);
  R[3 * a + a] = c;
  R[3 * a + b] = -s;
  R[3 * b + a] = s;
  R[3 * b + b] = c;
}

void rodrigues(const double r[3], double R[9]) {
  const double th = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  if (th == 0.0) return;
  const double k[3] = {r[0] / th, r[1] / th, r[2] / th};
  const double Kx[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
  double K2[9];
  mat3_mul(Kx, Kx, K2);
  const double s = std::sin(th), c1 = 1.0 - std::cos(th);
  for (int i = 0; i < 9; ++i) R[i] = (R[i] + s * Kx[i]) + c1 * K2[i];
}

// tightest box with axes Q (rounded to float32) around the given vertices
HBox tight_box(const HostMesh& M, const std::vector<int32_t>& verts, const double Qd[9]) {
  HBox b;
  double Q[9];
  for (int k = 0; k < 9; ++k) {
    b.Q[k] = (float)Qd[k];
    Q[k] = (double)b.Q[k];
  }
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  const float zero[3] = {0.f, 0.f, 0.f};
  for (int v : verts) {
    double p[3];
    M.local(v, zero, Q, p);
    for (int r = 0; r < 3; ++r) {
      lo[r] = std::min(lo[r], p[r]);
      hi[r] = std::max(hi[r], p[r]);
    }
  }
  double mid[3];
  for (int r = 0; r < 3; ++r) mid[r] = 0.5 * (lo[r] + hi[r]);
  for (int k = 0; k < 3; ++k) b.c[k] = (float)((Q[0 + k] * mid[0] + Q[3 + k] * mid[1]) + Q[6 + k] * mid[2]);
  double ext[3] = {0, 0, 0};
  for (int v : verts) {
    double p[3];
    M.local(v, b.c, Q, p);
    for (int r = 0; r < 3; ++r) ext[r] = std::max(ext[r], std::fabs(p[r]));
  }
  for (int r = 0; r < 3; ++r) b.h[r] = f32_up(ext[r]);
  return b;
}

// fn(i) for i in [0, n) on up to eight host threads (each i independent)
template <class Fn>
void parallel_for(size_t n, Fn fn) {
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nt = std::min<size_t>({n, (size_t)8, hw});
  if (nt <= 1) {
    for (size_t i = 0; i < n; ++i) fn(i);
    return;
  }
  // an exception of any share (or a thread that cannot start) is rethrown
  // here once every started thread has been joined
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  std::exception_ptr err;
  std::mutex mu;
  auto run = [&](size_t t) {
    try {
      for (size_t i = t; i < n; i += nt) fn(i);
    } catch (...) {
      std::lock_guard<std::mutex> lock(mu);
      if (!err) err = std::current_exception();
    }
  };
  try {
    for (size_t t = 1; t < nt; ++t) th.emplace_back(run, t);
  } catch (...) {
    std::lock_guard<std::mutex> lock(mu);
    if (!err) err = std::current_exception();
  }
  run(0);
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

// Update every box with a non-empty vertex set; returns the accepted OBV per box.
int update_boxes(const HostMesh& M, const std::vector<std::vector<int32_t>>& verts, std::vector<HBox>& boxes,
                 std::vector<double>& obv, const std::vector<uint32_t>& slot, const std::vector<int32_t>& which,
                 double delta, Evaluator& ev, Counters& cnt) {
  const double steps[5] = {8.0, 4.0, 2.0, 1.0, 0.5};
  // the current axes and the six +-delta rotations of every box: 7 tight boxes
  // each (independent, computed on several host threads)
  std::vector<HBox> req(which.size() * 7);
  std::vector<uint32_t> keys(which.size() * 7);
  parallel_for(req.size(), [&](size_t x) {
    const int bi = which[x / 7], m = (int)(x % 7);
    double Q[9];
    for (int k = 0; k < 9; ++k) Q[k] = (double)boxes[bi].Q[k];
    if (m == 0) {
      req[x] = tight_box(M, verts[bi], Q);
    } else {
      const int k = (m - 1) / 2, sg = (m - 1) % 2;
      double R[9], Q2[9];
      rot_local(k, sg == 0 ? delta : -delta, R);
      mat3_mul(R, Q, Q2);
      req[x] = tight_box(M, verts[bi], Q2);
    }
    keys[x] = slot[bi];
  });
  std::vector<double> v1;
  OBBV_RET(ev.eval(req, keys, v1));
  cnt.evals += (int64_t)v1.size();
  // a line search along the descent direction: 5 rotations per box whose
  // finite-difference gradient is non-zero
  std::vector<int32_t> has_line;
  std::vector<std::pair<int32_t, int32_t>> tasks;  // (index into which, step)
  std::vector<std::array<double, 3>> dir(which.size());
  for (size_t x = 0; x < which.size(); ++x) {
    const double* v = &v1[7 * x];
    double g[3];
    for (int k = 0; k < 3; ++k) g[k] = (v[1 + 2 * k] - v[2 + 2 * k]) / (2.0 * delta);
    const double gn = std::sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
    if (gn == 0.0) {
      has_line.push_back(0);
      continue;
    }
    has_line.push_back(1);
    dir[x] = {-g[0] / gn, -g[1] / gn, -g[2] / gn};
    for (int si = 0; si < 5; ++si) tasks.push_back({(int32_t)x, si});
  }
  std::vector<HBox> req2(tasks.size());
  std::vector<uint32_t> keys2(tasks.size());
  parallel_for(tasks.size(), [&](size_t y) {
    const size_t x = (size_t)tasks[y].first;
    const double s = steps[tasks[y].second];
    double Q[9];
    for (int k = 0; k < 9; ++k) Q[k] = (double)boxes[which[x]].Q[k];
    const double r[3] = {s * delta * dir[x][0], s * delta * dir[x][1], s * delta * dir[x][2]};
    double R[9], Q2[9];
    rodrigues(r, R);
    mat3_mul(R, Q, Q2);
    req2[y] = tight_box(M, verts[which[x]], Q2);
    keys2[y] = slot[which[x]];
  });
  std::vector<double> v2;
  OBBV_RET(ev.eval(req2, keys2, v2));
  cnt.evals += (int64_t)v2.size();
  size_t li = 0;
  for (size_t x = 0; x < which.size(); ++x) {
    const int bi = which[x];
    HBox best = req[7 * x];
    double bv = v1[7 * x];
    if (has_line[x]) {
      int j = 0;
      for (int s = 1; s < 5; ++s)
        if (v2[li + s] < v2[li + j]) j = s;
      if (v2[li + j] < bv) {
        best = req2[li + j];
        bv = v2[li + j];
      }
      li += 5;
    }
    boxes[bi] = best;
    obv[bi] = bv;
  }
  return OBBV_OK;
}

std::vector<int32_t> vertex_set(const HostMesh& M, const std::vector<int32_t>& tris, std::vector<char>& mark) {
  std::vector<int32_t> v;
  for (int t : tris)
    for (int k = 0; k < 3; ++k) {
      const int x = M.F[3 * t + k];
      if (!mark[x]) {
        mark[x] = 1;
        v.push_back(x);
      }
    }
  for (int x : v) mark[x] = 0;
  std::sort(v.begin(), v.end());
  return v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Lloyd state behind the C ABI
// ---------------------------------------------------------------------------
struct LloydState {
  HostMesh M;
  Elements E;
  Evaluator ev;
  int K = 32;
  double delta = 0.02;
  std::vector<Group> groups;
  std::vector<HBox> boxes;
  std::vector<double> obv;
  std::vector<uint32_t> slot;
  std::vector<int32_t> tri_box;
  Counters cnt;
  double layer_error = 0.0;
  Predictor pred;
  WallTimer t_flood, t_update, t_life;
  int64_t n_calls0 = 0;
  // more evaluators, each on a stream and scratch set of its own, for floods
  // whose groups are split over several host threads
  // pool sets: 0 the flood's evaluator, 1-3 the other parts' evaluators, 4 the
  // judge of the state's predictor, 5-7 the judges of the other parts' predictors
  static constexpr int kFloodParts = 4;
  static_assert(2 * kFloodParts <= kPoolSets, "a pool set per evaluator and per judge");
  Evaluator evx[kFloodParts - 1];
  Predictor predx[kFloodParts - 1];
  hipStream_t streamx[kFloodParts - 1] = {};

  int ensure_evx(int parts) {
    OBBV_RET(ev.ensure_spans());
    hipEvent_t e;
    OBBV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t r = hipEventRecord(e, ev.stream);
    for (int k = 0; k < parts - 1 && r == hipSuccess; ++k) {
      Evaluator& x = evx[k];
      if (!streamx[k]) {
        r = hipStreamCreateWithFlags(&streamx[k], hipStreamNonBlocking);
        if (r != hipSuccess) break;
        x.stream = streamx[k];
        x.pool_base = (k + 1) * kPoolCount;
      }
      x.mesh = ev.mesh;
      x.params = ev.params;
      x.spans = ev.spans;  // borrowed (made once, never replaced)
      x.spans_done = true;
      std::memcpy(x.centre, ev.centre, 16);
      x.have_centre = ev.have_centre;
      // the stream starts after the work enqueued so far on the first
      r = hipStreamWaitEvent(streamx[k], e, 0);
    }
    (void)hipEventDestroy(e);
    OBBV_HIP(r);
    return OBBV_OK;
  }

  LloydState() {
    t_life.start();
    pred.judge_set = kFloodParts;
    for (int k = 0; k < kFloodParts - 1; ++k) predx[k].judge_set = kFloodParts + 1 + k;
  }
  ~LloydState() {
    for (int k = 0; k < kFloodParts - 1; ++k)
      if (streamx[k]) {
        (void)hipStreamSynchronize(streamx[k]);
        predx[k].stream = nullptr;  // its destructor runs after the stream is gone
        (void)hipStreamDestroy(streamx[k]);
      }
    if (!getenv("OBBV_LLOYD_TIMING")) return;
    t_life.stop();
    fprintf(stderr,
            "[obbv lloyd] wall %.3f s: flood %.3f s (%lld rounds, %lld ranked), parameter update %.3f s; "
            "outer-volume calls %lld (host prep %.3f s, device incl. launches %.3f s); "
            "ranker %.3f s\n",
            t_life.s, t_flood.s, (long long)cnt.rounds, (long long)pred.calls, t_update.s, (long long)ev.calls,
            ev.t_prep.s, ev.t_dev.s, pred.t_pred.s);
    const FloodTimers& f = g_ft;
    fprintf(stderr,
            "[obbv lloyd] flood host: pops %.3f s, pop extents %.3f s, candidates %.3f s, ranker post %.3f s, "
            "exact post %.3f s, decisions %.3f s, growth %.3f s; ranker: pack %.3f s, launch %.3f s, wait %.3f s\n",
            f.pops.s, f.extents.s, f.cands.s, f.rank_post.s, f.exact_post.s, f.decide.s, f.grow.s, f.pred_pack.s, f.pred_launch.s,
            f.pred_wait.s);
    if (pred.judged_evals > 0)
      fprintf(stderr, "[obbv lloyd] judge: %lld candidates, mean |f - exact| %.5f, max %.5f, fallbacks %lld\n",
              (long long)pred.judged_evals, pred.jerr_sum / (double)pred.judged_evals, pred.jerr_max,
              (long long)pred.fallbacks);
    g_ft = FloodTimers();
  }
};

// Host threads a flood of independent groups is split over (OBBV_FLOOD_STREAMS,
// 1 to 4, default 4: the device's hardware queues per process).  The bits do not depend on it: the flood of a group
// reads and writes only its own elements and boxes, and a box's outer volume
// does not depend on the call that evaluates it.
static int flood_streams_choice() {
  const char* e = getenv("OBBV_FLOOD_STREAMS");
  if (e && *e) return std::max(1, std::min(LloydState::kFloodParts, atoi(e)));
  return LloydState::kFloodParts;
}

// The calls of a flood that runs on one stream run alone on the device; those
// with few cast units take smaller cast items: OBBV_ALONE_ITEM_TRIS entries (0:
// never; else 768, 1536 or 2304), by default 1536.  The bits do not depend on it.
static int alone_item_tris() {
  const char* e = getenv("OBBV_ALONE_ITEM_TRIS");
  if (e && *e) {
    const int v = atoi(e);
    if (v == 0 || v == 768 || v == 1536 || v == 2304) return v;
  }
  return 1536;
}

// ... and the cast-unit count below which such a call takes them:
// OBBV_ALONE_SPLIT_BELOW, by default 128.
static int alone_split_below() {
  const char* e = getenv("OBBV_ALONE_SPLIT_BELOW");
  if (e && *e) return std::max(0, atoi(e));
  return 128;
}

// The flood of `groups`: with two groups or more, the groups are split into
// parts of about equal element counts (largest group
// first, into the lightest part; groups keep their order inside a part),
// flooded on host threads with an evaluator (stream, scratch set) each, so that
// one part's device work overlaps another's host work and fills the CUs
// another's calls leave idle.
static int flood_split(LloydState& S, const std::vector<Group>& groups, PartitionIO io) {
  const int parts = std::min<int>(flood_streams_choice(), (int)groups.size());
  if (parts < 2 || S.ev.smp_cap != 0) {
    // a flood on one stream: its calls run alone on the device, so those with
    // few cast units take smaller items (more units for idle compute units)
    S.ev.item_tris = alone_item_tris();
    S.ev.split_below = alone_split_below();
    const int rc = flood_partition(S.M, S.E, groups, io, S.K, S.ev, S.cnt, &S.pred);
    S.ev.item_tris = 0;
    return rc;
  }
  std::vector<int> order(groups.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return groups[a].elems.size() > groups[b].elems.size(); });
  std::vector<int> part_of(groups.size(), 0);
  std::vector<size_t> load((size_t)parts, 0);
  for (int g : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    part_of[g] = k;
    load[k] += groups[g].elems.size();
  }
  std::vector<std::vector<Group>> pg((size_t)parts);
  for (size_t g = 0; g < groups.size(); ++g) pg[part_of[g]].push_back(groups[g]);
  OBBV_RET(S.ensure_evx(parts));
  const int nx = parts - 1;
  // with the ranker on, every part has a predictor of its own (same network and
  // settings; its own stream, staging, judge window and judge scratch set)
  for (int k = 0; k < nx && S.pred.on; ++k) {
    Predictor& P = S.predx[k];
    if (P.cfg_gen != S.pred.cfg_gen) {
      P.cfg = S.pred.cfg;
      P.cfg_gen = S.pred.cfg_gen;
      P.packed_ready = false;
      P.window.clear();
      P.wpos = 0;
      P.err_sum = 0.0;
      P.err_n = 0;
    }
    P.on = true;
    P.paused = S.pred.paused;
    P.stream = S.streamx[k];
  }
  std::vector<std::vector<int32_t>> ebx((size_t)nx);
  std::vector<Counters> cx((size_t)nx);
  std::vector<int> rcx((size_t)nx, OBBV_OK);
  std::vector<std::string> errx((size_t)nx);
  int dev = 0;
  OBBV_HIP(hipGetDevice(&dev));
  std::vector<std::thread> th;
  struct Joiner {  // every started thread is joined, also when this frame unwinds
    std::vector<std::thread>& t;
    ~Joiner() {
      for (std::thread& x : t)
        if (x.joinable()) x.join();
    }
  } joiner{th};
  for (int k = 0; k < nx; ++k)
    th.emplace_back([&, k] {
      try {  // nothing may leave a thread: a failure becomes the part's return code
        if (hipSetDevice(dev) != hipSuccess) {
          rcx[k] = OBBV_ERR_HIP;
          errx[k] = "hipSetDevice failed in a flood thread";
          return;
        }
        PartitionIO iok{io.boxes, io.obv, io.slot, &ebx[k]};
        rcx[k] = flood_partition(S.M, S.E, pg[k + 1], iok, S.K, S.evx[k], cx[k], S.pred.on ? &S.predx[k] : nullptr);
        if (rcx[k] != OBBV_OK) errx[k] = obbv_last_error();
      } catch (const std::bad_alloc&) {
        rcx[k] = OBBV_ERR_OOM;
      } catch (...) {
        rcx[k] = OBBV_ERR_INTERNAL;
      }
    });
  const int rc0 = flood_partition(S.M, S.E, pg[0], io, S.K, S.ev, S.cnt, &S.pred);
  for (std::thread& t : th) t.join();  // (an exception above is joined by `joiner`)
  for (int k = 0; k < nx; ++k)
    if (rcx[k] != OBBV_OK) {
      if (!errx[k].empty())
        set_error(errx[k]);
      else
        set_error(rcx[k] == OBBV_ERR_OOM ? "flood thread: host memory allocation failed" : "flood thread: internal error");
      return rcx[k];
    }
  OBBV_RET(rc0);
  std::vector<int32_t>& eb = *io.elem_box;
  for (int k = 0; k < nx; ++k) {
    for (const Group& g : pg[k + 1])
      for (int e : g.elems) eb[e] = ebx[k][e];
    S.cnt.evals += cx[k].evals;
    S.cnt.rounds += cx[k].rounds;
    S.cnt.trivial += cx[k].trivial;
    S.cnt.moves += cx[k].moves;
    S.ev.calls += S.evx[k].calls;
    S.evx[k].calls = 0;
    Predictor& P = S.predx[k];
    S.pred.predicted += P.predicted;
    S.pred.fallbacks += P.fallbacks;
    S.pred.calls += P.calls;
    S.pred.judged_evals += P.judged_evals;
    S.pred.jerr_sum += P.jerr_sum;
    S.pred.jerr_max = std::max(S.pred.jerr_max, P.jerr_max);
    S.pred.t_pred.s += P.t_pred.s;
    P.predicted = P.fallbacks = P.calls = P.judged_evals = 0;
    P.jerr_sum = P.jerr_max = P.t_pred.s = 0.0;
  }
  return OBBV_OK;
}

// One Lloyd iteration (partition + parameter update) of every group.
static int lloyd_iterate(LloydState& S) {
  S.pred.paused = false;  // a judge fallback lasts for one iteration
  std::vector<int32_t> eb;
  PartitionIO io{&S.boxes, &S.obv, &S.slot, &eb};
  // groups with a single box: every element goes to it, the update fits the tight box
  std::vector<Group> flood_groups;
  for (const Group& g : S.groups)
    if (g.boxes.size() > 1) flood_groups.push_back(g);
  S.t_flood.start();
  OBBV_RET(flood_split(S, flood_groups, io));
  S.t_flood.stop();
  for (const Group& g : S.groups)
    if (g.boxes.size() == 1)
      for (int e : g.elems) eb[e] = g.boxes[0];
  // triangles of each box
  std::vector<std::vector<int32_t>> tris(S.boxes.size());
  S.tri_box.assign((size_t)S.M.nt, -1);
  for (int e = 0; e < S.E.n; ++e)
    if (eb[e] >= 0)
      for (int x = S.E.tri_off[e]; x < S.E.tri_off[e + 1]; ++x) {
        tris[eb[e]].push_back(S.E.tris[x]);
        S.tri_box[S.E.tris[x]] = eb[e];
      }
  std::vector<std::vector<int32_t>> verts(S.boxes.size());
  std::vector<char> mark((size_t)S.M.nv, 0);
  std::vector<int32_t> which;
  for (size_t b = 0; b < S.boxes.size(); ++b)
    if (!tris[b].empty()) {
      verts[b] = vertex_set(S.M, tris[b], mark);
      which.push_back((int32_t)b);
    }
  S.t_update.start();
  OBBV_RET(update_boxes(S.M, verts, S.boxes, S.obv, S.slot, which, S.delta, S.ev, S.cnt));
  S.t_update.stop();
  S.layer_error = 0.0;
  for (size_t b = 0; b < S.boxes.size(); ++b) S.layer_error += tris[b].empty() ? 0.0 : S.obv[b];
  return OBBV_OK;
}

// One adjustment of every group with two boxes or more (Sec. 4.2.1, third
// step): the least important box (fewest triangles; ties: larger outer volume,
// then higher index) moves to the centroid of the triangle farthest from the
// centre of the group's box with the largest outer volume (ties: lower index;
// farthest: ties to the lower triangle), with that box's axes; one Lloyd
// iteration of the adjusted groups follows, and each group keeps its result
// only if its error (sum of its boxes' outer volumes) drops.
static int lloyd_adjust(LloydState& S, int32_t* out_accepted) {
  const int G = (int)S.groups.size();
  std::vector<int64_t> cnt(S.boxes.size(), 0);
  for (int t = 0; t < S.M.nt; ++t)
    if (S.tri_box[t] >= 0) ++cnt[S.tri_box[t]];
  const std::vector<HBox> boxes0 = S.boxes;
  const std::vector<double> obv0 = S.obv;
  const std::vector<int32_t> tri_box0 = S.tri_box;
  std::vector<int> state(G, -1);  // -1 not adjusted, 0 undone, 1 kept
  std::vector<double> e0(G, 0.0);
  std::vector<Group> adjusted;
  for (int g = 0; g < G; ++g) {
    const Group& gr = S.groups[g];
    const int b = (int)gr.boxes.size();
    if (b < 2 || gr.elems.empty()) continue;
    for (int bi : gr.boxes) e0[g] += cnt[bi] > 0 ? S.obv[bi] : 0.0;
    int j = 0;
    for (int i = 1; i < b; ++i) {
      const int bi = gr.boxes[i], bj = gr.boxes[j];
      if (cnt[bi] < cnt[bj] || (cnt[bi] == cnt[bj] && (S.obv[bi] > S.obv[bj] || (S.obv[bi] == S.obv[bj]))))
        j = i;
    }
    int w = -1;
    for (int i = 0; i < b; ++i)
      if (i != j && (w < 0 || S.obv[gr.boxes[i]] > S.obv[gr.boxes[w]])) w = i;
    const int bw = gr.boxes[w];
    if (cnt[bw] == 0) continue;
    int far = -1;
    double fd = -1.0;
    for (int e : gr.elems) {
      if (S.tri_box[e] != bw) continue;  // elements are the group's triangles
      const double d = dist3(&S.M.cen[3 * (size_t)e], S.boxes[bw].c);
      if (d > fd || (d == fd && e < far)) {
        fd = d;
        far = e;
      }
    }
    HBox& bj = S.boxes[gr.boxes[j]];
    for (int k = 0; k < 3; ++k) bj.c[k] = (float)S.M.cen[3 * (size_t)far + k];
    std::memcpy(bj.Q, S.boxes[bw].Q, 36);
    state[g] = 0;
    adjusted.push_back(gr);
  }
  if (!adjusted.empty()) {
    std::vector<Group> all;
    all.swap(S.groups);
    S.groups = adjusted;
    const int rc = lloyd_iterate(S);
    S.groups.swap(all);
    OBBV_RET(rc);
    // triangles of the groups that were not adjusted keep their boxes
    for (int g = 0; g < G; ++g)
      if (state[g] < 0)
        for (int e : S.groups[g].elems) S.tri_box[e] = tri_box0[e];
    for (int g = 0; g < G; ++g) {
      if (state[g] < 0) continue;
      const Group& gr = S.groups[g];
      std::fill(cnt.begin(), cnt.end(), 0);
      for (int e : gr.elems)
        if (S.tri_box[e] >= 0) ++cnt[S.tri_box[e]];
      double e1 = 0.0;
      for (int bi : gr.boxes) e1 += cnt[bi] > 0 ? S.obv[bi] : 0.0;
      if (e1 < e0[g]) {
        state[g] = 1;
        continue;
      }
      for (int bi : gr.boxes) {
        S.boxes[bi] = boxes0[bi];
        S.obv[bi] = obv0[bi];
      }
      for (int e : gr.elems) S.tri_box[e] = tri_box0[e];
    }
    // boxes of groups that were not adjusted are untouched by the iteration
    S.layer_error = 0.0;
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int t = 0; t < S.M.nt; ++t)
      if (S.tri_box[t] >= 0) ++cnt[S.tri_box[t]];
    for (size_t bi = 0; bi < S.boxes.size(); ++bi) S.layer_error += cnt[bi] > 0 ? S.obv[bi] : 0.0;
  }
  if (out_accepted)
    for (int g = 0; g < G; ++g) out_accepted[g] = state[g];
  return OBBV_OK;
}

}  // namespace obbv

using namespace obbv;

static int obbv_lloyd_create_body(const obbv_mesh* mesh, const obbv_lloyd_params* p, obbv_lloyd** out);
extern "C" int obbv_lloyd_create(const obbv_mesh* mesh, const obbv_lloyd_params* p, obbv_lloyd** out) {
  return obbv::guarded([&] { return obbv_lloyd_create_body(mesh, p, out); });
}
static int obbv_lloyd_create_body(const obbv_mesh* mesh, const obbv_lloyd_params* p, obbv_lloyd** out) {
  clear_error();
  OBBV_ARG(mesh && p && out, "NULL argument");
  OBBV_ARG(p->R >= 1 && p->R <= 32767, "R must be in [1, 32767]");
  OBBV_ARG(p->pops_per_round >= 1, "pops_per_round must be >= 1");
  OBBV_ARG(p->delta > 0.0, "delta must be positive");
  OBBV_ARG(mesh->n_triangles > 0 && mesh->triangles && mesh->vertices, "empty mesh");
  LloydState* S = new LloydState();
  S->ev.mesh = *mesh;
  S->ev.params.R = p->R;
  S->ev.params.axis_mask = 7;
  S->ev.params.seed = p->seed;
  S->ev.params.block_rays = p->block_rays;
  S->ev.params.flags = 0;
  S->ev.stream = nullptr;
  S->K = p->pops_per_round;
  S->delta = p->delta;
  int rc = S->M.load(mesh, nullptr);
  if (rc != OBBV_OK) {
    delete S;
    return rc;
  }
  S->ev.set_centre(S->M.V);
  S->E = Elements::triangles(S->M);
  *out = reinterpret_cast<obbv_lloyd*>(S);
  return OBBV_OK;
}

static int obbv_lloyd_set_groups_body(obbv_lloyd* st, int32_t n_boxes, const int32_t* tri_group,
                                     const int32_t* box_group, const float* boxes, const uint32_t* box_slot);
extern "C" int obbv_lloyd_set_groups(obbv_lloyd* st, int32_t n_boxes, const int32_t* tri_group,
                                     const int32_t* box_group, const float* boxes, const uint32_t* box_slot) {
  return obbv::guarded([&] { return obbv_lloyd_set_groups_body(st, n_boxes, tri_group, box_group, boxes, box_slot); });
}
static int obbv_lloyd_set_groups_body(obbv_lloyd* st, int32_t n_boxes, const int32_t* tri_group,
                                     const int32_t* box_group, const float* boxes, const uint32_t* box_slot) {
  clear_error();
  OBBV_ARG(st && tri_group && box_group && boxes, "NULL argument");
  OBBV_ARG(n_boxes >= 1, "n_boxes must be >= 1");
  LloydState& S = *reinterpret_cast<LloydState*>(st);
  int32_t ng = 0;
  for (int b = 0; b < n_boxes; ++b) {
    OBBV_ARG(box_group[b] >= 0, "box_group must be >= 0");
    ng = std::max(ng, box_group[b] + 1);
  }
  S.groups.assign((size_t)ng, Group{});
  for (int b = 0; b < n_boxes; ++b) S.groups[box_group[b]].boxes.push_back(b);
  for (int t = 0; t < S.M.nt; ++t) {
    const int g = tri_group[t];
    OBBV_ARG(g < ng, "tri_group beyond the last group");
    if (g >= 0) S.groups[g].elems.push_back(t);
  }
  S.boxes.resize((size_t)n_boxes);
  S.obv.assign((size_t)n_boxes, 0.0);
  S.slot.resize((size_t)n_boxes);
  for (int b = 0; b < n_boxes; ++b) {
    std::memcpy(S.boxes[b].c, boxes + 15 * b, 12);
    std::memcpy(S.boxes[b].Q, boxes + 15 * b + 3, 36);
    std::memcpy(S.boxes[b].h, boxes + 15 * b + 12, 12);
    S.slot[b] = box_slot ? box_slot[b] : (uint32_t)b;
  }
  S.tri_box.assign((size_t)S.M.nt, -1);
  return OBBV_OK;
}

static int obbv_lloyd_step_body(obbv_lloyd* st, void* stream);
extern "C" int obbv_lloyd_step(obbv_lloyd* st, void* stream) {
  return obbv::guarded([&] { return obbv_lloyd_step_body(st, stream); });
}
static int obbv_lloyd_step_body(obbv_lloyd* st, void* stream) {
  clear_error();
  OBBV_ARG(st, "NULL state");
  LloydState& S = *reinterpret_cast<LloydState*>(st);
  OBBV_ARG(!S.groups.empty(), "obbv_lloyd_set_groups was not called");
  S.ev.stream = (hipStream_t)stream;
  S.pred.stream = (hipStream_t)stream;
  return lloyd_iterate(S);
}

static int obbv_lloyd_adjust_body(obbv_lloyd* st, int32_t* out_accepted, void* stream);
extern "C" int obbv_lloyd_adjust(obbv_lloyd* st, int32_t* out_accepted, void* stream) {
  return obbv::guarded([&] { return obbv_lloyd_adjust_body(st, out_accepted, stream); });
}
static int obbv_lloyd_adjust_body(obbv_lloyd* st, int32_t* out_accepted, void* stream) {
  clear_error();
  OBBV_ARG(st, "NULL state");
  LloydState& S = *reinterpret_cast<LloydState*>(st);
  OBBV_ARG(!S.groups.empty(), "obbv_lloyd_set_groups was not called");
  S.ev.stream = (hipStream_t)stream;
  S.pred.stream = (hipStream_t)stream;
  return lloyd_adjust(S, out_accepted);
}

static int obbv_lloyd_set_surrogate_body(obbv_lloyd* st, const obbv_surrogate* sur);
extern "C" int obbv_lloyd_set_surrogate(obbv_lloyd* st, const obbv_surrogate* sur) {
  return obbv::guarded([&] { return obbv_lloyd_set_surrogate_body(st, sur); });
}
static int obbv_lloyd_set_surrogate_body(obbv_lloyd* st, const obbv_surrogate* sur) {
  clear_error();
  OBBV_ARG(st, "NULL state");
  LloydState& S = *reinterpret_cast<LloydState*>(st);
  if (!sur) {
    S.pred.on = false;
    return OBBV_OK;
  }
  OBBV_ARG(sur->mlp_params && sur->volume && sur->frame, "surrogate arrays are NULL");
  OBBV_ARG(sur->N >= 1 && sur->verify_top >= 0 && sur->judge_every >= 1, "bad surrogate sizes");
  S.pred.cfg = *sur;
  S.pred.packed_ready = false;
  ++S.pred.cfg_gen;
  S.pred.on = true;
  S.pred.paused = false;
  S.pred.window.clear();
  S.pred.wpos = 0;
  S.pred.err_sum = 0.0;
  S.pred.err_n = 0;
  return OBBV_OK;
}

static int obbv_lloyd_get_body(obbv_lloyd* st, int32_t* tri_box, float* boxes, double* obv, double* layer_error,
                              int64_t* counters);
extern "C" int obbv_lloyd_get(obbv_lloyd* st, int32_t* tri_box, float* boxes, double* obv, double* layer_error,
                              int64_t* counters) {
  return obbv::guarded([&] { return obbv_lloyd_get_body(st, tri_box, boxes, obv, layer_error, counters); });
}
static int obbv_lloyd_get_body(obbv_lloyd* st, int32_t* tri_box, float* boxes, double* obv, double* layer_error,
                              int64_t* counters) {
  // counters: [0] evaluations, [1] rounds, [2] no-evaluation candidates, [3] moves,
  // [4] ranker predictions, [5] ranker fallbacks
  clear_error();
  OBBV_ARG(st, "NULL state");
  LloydState& S = *reinterpret_cast<LloydState*>(st);
  if (tri_box) std::memcpy(tri_box, S.tri_box.data(), 4 * (size_t)S.M.nt);
  if (boxes)
    for (size_t b = 0; b < S.boxes.size(); ++b) {
      std::memcpy(boxes + 15 * b, S.boxes[b].c, 12);
      std::memcpy(boxes + 15 * b + 3, S.boxes[b].Q, 36);
      std::memcpy(boxes + 15 * b + 12, S.boxes[b].h, 12);
    }
  if (obv) std::memcpy(obv, S.obv.data(), 8 * S.obv.size());
  if (layer_error) *layer_error = S.layer_error;
  if (counters) {
    counters[0] = S.cnt.evals;
    counters[1] = S.cnt.rounds;
    counters[2] = S.cnt.trivial;
    counters[3] = S.cnt.moves;
    counters[4] = S.pred.predicted;
    counters[5] = S.pred.fallbacks;
  }
  return OBBV_OK;
}

static int obbv_lloyd_record_body(obbv_lloyd* st, int64_t cap);
extern "C" int obbv_lloyd_record(obbv_lloyd* st, int64_t cap) {
  return obbv::guarded([&] { return obbv_lloyd_record_body(st, cap); });
}
static int obbv_lloyd_record_body(obbv_lloyd* st, int64_t cap) {
  clear_error();
  OBBV_ARG(st, "NULL state");
  OBBV_ARG(cap >= 0, "cap must be >= 0");
  LloydState& S = *reinterpret_cast<LloydState*>(st);
  S.ev.smp_cap = cap;
  S.ev.smp_seen = 0;
  S.ev.smp_box.clear();
  S.ev.smp_val.clear();
  return OBBV_OK;
}

static int obbv_lloyd_take_records_body(obbv_lloyd* st, int64_t max_n, float* boxes, double* obv, int64_t* n_out);
extern "C" int obbv_lloyd_take_records(obbv_lloyd* st, int64_t max_n, float* boxes, double* obv, int64_t* n_out) {
  return obbv::guarded([&] { return obbv_lloyd_take_records_body(st, max_n, boxes, obv, n_out); });
}
static int obbv_lloyd_take_records_body(obbv_lloyd* st, int64_t max_n, float* boxes, double* obv, int64_t* n_out) {
  clear_error();
  OBBV_ARG(st && n_out, "NULL argument");
  LloydState& S = *reinterpret_cast<LloydState*>(st);
  const int64_t n = std::min<int64_t>(max_n, (int64_t)S.ev.smp_box.size());
  OBBV_ARG(n == 0 || (boxes && obv), "NULL output arrays");
  for (int64_t i = 0; i < n; ++i) {
    std::memcpy(boxes + 15 * i, S.ev.smp_box[i].c, 12);
    std::memcpy(boxes + 15 * i + 3, S.ev.smp_box[i].Q, 36);
    std::memcpy(boxes + 15 * i + 12, S.ev.smp_box[i].h, 12);
    obv[i] = S.ev.smp_val[i];
  }
  *n_out = n;
  S.ev.smp_seen = 0;
  S.ev.smp_box.clear();
  S.ev.smp_val.clear();
  return OBBV_OK;
}

static int obbv_lloyd_destroy_body(obbv_lloyd* st);
extern "C" int obbv_lloyd_destroy(obbv_lloyd* st) {
  return obbv::guarded([&] { return obbv_lloyd_destroy_body(st); });
}
static int obbv_lloyd_destroy_body(obbv_lloyd* st) {
  clear_error();
  delete reinterpret_cast<LloydState*>(st);
  return OBBV_OK;
}

// ---------------------------------------------------------------------------
// hierarchy: top-down levels, then multigrid-like up / down sweeps (Sec. 4.2.2)
// ---------------------------------------------------------------------------
namespace obbv {
namespace {

constexpr uint64_t kSeedSalt = 0x243F6A8885A308D3ull;

struct Level {
  std::vector<HBox> box;
  std::vector<double> obv;
  std::vector<int32_t> parent;    // level-local index of the parent node (-1 at the root)
  std::vector<uint32_t> slot;     // global node id = jitter key
  std::vector<int32_t> tri_node;  // [nt] level-local node of every triangle
};

struct Tree {
  int L = 1, b = 1;
  std::vector<Level> lv;
  double error() const {  // Eq. 7 with omega = layers to the leaves (leaf = 1)
    double e = 0.0;
    for (int l = 0; l < L; ++l) {
      double s = 0.0;
      for (size_t j = 0; j < lv[l].obv.size(); ++j) s += lv[l].obv[j];
      e += (double)(L - l) * s;
    }
    return e;
  }
};

// seed triangles of group (level, parent): draws from SplitMix64, duplicates rejected
std::vector<int32_t> random_seeds(const std::vector<int32_t>& G, int count, uint64_t seed, int level, int parent) {
  std::vector<int32_t> out;
  uint64_t draw = 0;
  while ((int)out.size() < count) {
    const uint64_t n = ((uint64_t)level << 48) | ((uint64_t)parent << 20) | draw++;
    const int32_t t = G[(size_t)(splitmix64_at(seed ^ kSeedSalt, n) % (uint64_t)G.size())];
    if (std::find(out.begin(), out.end(), t) == out.end()) out.push_back(t);
  }
  return out;
}

// run `iters` Lloyd iterations of level l with its current parents; children of a
// parent are the level-l nodes pointing at it
int solve_level(LloydState& S, Tree& T, int l, int iters) {
  Level& C = T.lv[l];
  const Level& P = T.lv[l - 1];
  const int np = (int)P.box.size();
  S.groups.assign((size_t)np, Group{});
  for (int t = 0; t < S.M.nt; ++t) S.groups[P.tri_node[t]].elems.push_back(t);
  for (int j = 0; j < (int)C.box.size(); ++j)
    if (C.parent[j] >= 0 && C.box[j].h[0] >= 0.f) S.groups[C.parent[j]].boxes.push_back(j);
  // a group keeps at most as many boxes as it has triangles
  for (auto& g : S.groups)
    if (g.boxes.size() > g.elems.size()) g.boxes.resize(g.elems.size());
  S.E = Elements::triangles(S.M);
  S.boxes = C.box;
  S.obv = C.obv;
  S.slot = C.slot;
  for (int it = 0; it < iters; ++it) OBBV_RET(lloyd_iterate(S));
  C.box = S.boxes;
  // nodes that kept no triangles become empty boxes
  std::vector<char> used(C.box.size(), 0);
  for (int t = 0; t < S.M.nt; ++t)
    if (S.tri_box[t] >= 0) used[S.tri_box[t]] = 1;
  for (size_t j = 0; j < C.box.size(); ++j) {
    C.obv[j] = used[j] ? S.obv[j] : 0.0;
    if (!used[j]) C.box[j].h[0] = C.box[j].h[1] = C.box[j].h[2] = 0.f;
  }
  for (int t = 0; t < S.M.nt; ++t) C.tri_node[t] = S.tri_box[t];
  return OBBV_OK;
}

// bottom-up merge of level l: the level-(l+1) boxes are the units of a Lloyd
// iteration that re-groups them under the level-l boxes of each grandparent
int merge_level(LloydState& S, Tree& T, int l) {
  Level& A = T.lv[l];          // merged level
  Level& U = T.lv[l + 1];      // units
  const Level& G = T.lv[l - 1];
  const int nu = (int)U.box.size();
  // elements = units with triangles
  Elements E;
  std::vector<int32_t> unit_of_elem, elem_of_unit((size_t)nu, -1);
  std::vector<std::vector<int32_t>> ut((size_t)nu);
  for (int t = 0; t < S.M.nt; ++t)
    if (U.tri_node[t] >= 0) ut[U.tri_node[t]].push_back(t);
  E.tri_off.push_back(0);
  for (int u = 0; u < nu; ++u) {
    if (ut[u].empty()) continue;
    elem_of_unit[u] = E.n++;
    unit_of_elem.push_back(u);
    for (int t : ut[u]) E.tris.push_back(t);
    E.tri_off.push_back((int32_t)E.tris.size());
    for (int k = 0; k < 3; ++k) E.cen.push_back((double)U.box[u].c[k]);
  }
  E.build_vertices(S.M);
  // unit adjacency: a mesh edge joins triangles of the two units
  std::vector<std::vector<int32_t>> nb((size_t)E.n);
  for (int t = 0; t < S.M.nt; ++t) {
    const int a = U.tri_node[t] >= 0 ? elem_of_unit[U.tri_node[t]] : -1;
    if (a < 0) continue;
    for (int x = S.M.adj_off[t]; x < S.M.adj_off[t + 1]; ++x) {
      const int u2 = U.tri_node[S.M.adj[x]];
      const int c = u2 >= 0 ? elem_of_unit[u2] : -1;
      if (c >= 0 && c != a) nb[a].push_back(c);
    }
  }
  E.adj_off.assign((size_t)E.n + 1, 0);
  for (int e = 0; e < E.n; ++e) {
    std::sort(nb[e].begin(), nb[e].end());
    nb[e].erase(std::unique(nb[e].begin(), nb[e].end()), nb[e].end());
    E.adj_off[e + 1] = E.adj_off[e] + (int32_t)nb[e].size();
    for (int c : nb[e]) E.adj.push_back(c);
  }
  // groups: grandparents; their boxes are the level-l nodes under them
  const int ng = (int)G.box.size();
  S.groups.assign((size_t)ng, Group{});
  for (int e = 0; e < E.n; ++e) {
    const int u = unit_of_elem[e];
    const int a = U.parent[u];
    S.groups[A.parent[a]].elems.push_back(e);
  }
  for (int j = 0; j < (int)A.box.size(); ++j)
    if (A.parent[j] >= 0 && A.obv.size() && (A.box[j].h[0] > 0.f || A.box[j].h[1] > 0.f))
      S.groups[A.parent[j]].boxes.push_back(j);
  for (auto& g : S.groups)
    if (g.boxes.size() > g.elems.size()) g.boxes.resize(g.elems.size());
  S.E = std::move(E);
  S.boxes = A.box;
  S.obv = A.obv;
  S.slot = A.slot;
  std::vector<int32_t> eb;
  PartitionIO io{&S.boxes, &S.obv, &S.slot, &eb};
  std::vector<Group> fg;
  for (const Group& g : S.groups)
    if (g.boxes.size() > 1) fg.push_back(g);
  S.pred.paused = false;
  OBBV_RET(flood_split(S, fg, io));
  for (const Group& g : S.groups)
    if (g.boxes.size() == 1)
      for (int e : g.elems) eb[e] = g.boxes[0];
  // new parents of the units, triangles of the merged boxes, box update
  std::vector<std::vector<int32_t>> tris(A.box.size());
  for (int e = 0; e < S.E.n; ++e) {
    if (eb[e] < 0) continue;
    U.parent[unit_of_elem[e]] = eb[e];
    for (int x = S.E.tri_off[e]; x < S.E.tri_off[e + 1]; ++x) tris[eb[e]].push_back(S.E.tris[x]);
  }
  std::vector<std::vector<int32_t>> verts(A.box.size());
  std::vector<char> mark((size_t)S.M.nv, 0);
  std::vector<int32_t> which;
  for (size_t j = 0; j < A.box.size(); ++j)
    if (!tris[j].empty()) {
      verts[j] = vertex_set(S.M, tris[j], mark);
      which.push_back((int32_t)j);
    }
  S.t_update.start();
  OBBV_RET(update_boxes(S.M, verts, S.boxes, S.obv, S.slot, which, S.delta, S.ev, S.cnt));
  S.t_update.stop();
  A.box = S.boxes;
  for (size_t j = 0; j < A.box.size(); ++j) {
    A.obv[j] = tris[j].empty() ? 0.0 : S.obv[j];
    if (tris[j].empty()) A.box[j].h[0] = A.box[j].h[1] = A.box[j].h[2] = 0.f;
  }
  for (int t = 0; t < S.M.nt; ++t) A.tri_node[t] = U.tri_node[t] >= 0 ? U.parent[U.tri_node[t]] : -1;
  return OBBV_OK;
}

}  // namespace
}  // namespace obbv

static int obbv_build_hierarchy_body(const obbv_mesh* mesh, const obbv_hier_params* p, float* out_boxes,
                                    double* out_obv, int32_t* out_parent, int32_t* out_tri_node, double* out_e,
                                    int64_t* out_counters, void* stream);
extern "C" int obbv_build_hierarchy(const obbv_mesh* mesh, const obbv_hier_params* p, float* out_boxes,
                                    double* out_obv, int32_t* out_parent, int32_t* out_tri_node, double* out_e,
                                    int64_t* out_counters, void* stream) {
  return obbv::guarded([&] { return obbv_build_hierarchy_body(mesh, p, out_boxes, out_obv, out_parent, out_tri_node, out_e, out_counters, stream); });
}
static int obbv_build_hierarchy_body(const obbv_mesh* mesh, const obbv_hier_params* p, float* out_boxes,
                                    double* out_obv, int32_t* out_parent, int32_t* out_tri_node, double* out_e,
                                    int64_t* out_counters, void* stream) {
  clear_error();
  OBBV_ARG(mesh && p, "NULL argument");
  OBBV_ARG(p->levels >= 1 && p->levels <= 12, "levels must be in [1, 12]");
  OBBV_ARG(p->branching >= 1, "branching must be >= 1");
  OBBV_ARG(p->iters >= 1 && p->sweeps >= 0, "iters >= 1 and sweeps >= 0");
  int64_t n_nodes = 0, w = 1;
  for (int l = 0; l < p->levels; ++l, w *= p->branching) n_nodes += w;
  OBBV_ARG(n_nodes < (1 << 24), "too many nodes");
  obbv_lloyd_params lp{p->R, p->block_rays, p->seed, p->pops_per_round, 0, p->delta};
  OBBV_ARG(p->reserved == 0, "reserved must be 0");
  obbv_lloyd* handle = nullptr;
  OBBV_RET(obbv_lloyd_create(mesh, &lp, &handle));
  std::unique_ptr<LloydState> S(reinterpret_cast<LloydState*>(handle));
  hipStream_t s = (hipStream_t)stream;
  S->ev.stream = s;
  S->pred.stream = s;
  if (p->surrogate) OBBV_RET(obbv_lloyd_set_surrogate(handle, p->surrogate));
  const int nt = S->M.nt;
  Tree T;
  T.L = p->levels;
  T.b = p->branching;
  T.lv.resize((size_t)T.L);
  // root: covariance fit of all triangles, then parameter updates
  {
    Level& R0 = T.lv[0];
    int32_t* dcl = nullptr;
    obbv_box* dbox = nullptr;
    OBBV_HIP(hipMalloc(&dcl, 4 * (size_t)nt));
    OBBV_HIP(hipMalloc(&dbox, sizeof(obbv_box)));
    OBBV_HIP(hipMemsetAsync(dcl, 0, 4 * (size_t)nt, s));
    int rc = fit_impl(mesh, dcl, 1, dbox, nullptr, s);
    obbv_box hb;
    if (rc == OBBV_OK) rc = hipMemcpyAsync(&hb, dbox, sizeof(hb), hipMemcpyDeviceToHost, s) == hipSuccess ? 0 : OBBV_ERR_HIP;
    if (rc == OBBV_OK) rc = hipStreamSynchronize(s) == hipSuccess ? 0 : OBBV_ERR_HIP;
    (void)hipFree(dcl);
    (void)hipFree(dbox);
    OBBV_RET(rc);
    HBox rb;
    std::memcpy(rb.c, hb.center, 12);
    std::memcpy(rb.Q, hb.axes, 36);
    std::memcpy(rb.h, hb.half, 12);
    R0.box = {rb};
    R0.obv = {0.0};
    R0.parent = {-1};
    R0.slot = {0u};
    R0.tri_node.assign((size_t)nt, 0);
    S->groups.assign(1, Group{});
    for (int t = 0; t < nt; ++t) S->groups[0].elems.push_back(t);
    S->groups[0].boxes = {0};
    S->boxes = R0.box;
    S->obv = R0.obv;
    S->slot = R0.slot;
    for (int it = 0; it < p->iters; ++it) OBBV_RET(lloyd_iterate(*S));
    R0.box = S->boxes;
    R0.obv = S->obv;
  }
  // top-down: each level splits every parent's triangles among `branching` children
  uint32_t node_base = 1;
  for (int l = 1; l < T.L; ++l) {
    const Level& P = T.lv[l - 1];
    Level& C = T.lv[l];
    const int np = (int)P.box.size();
    const int nc = np * T.b;
    C.box.assign((size_t)nc, HBox{});
    C.obv.assign((size_t)nc, 0.0);
    C.parent.assign((size_t)nc, -1);
    C.slot.resize((size_t)nc);
    C.tri_node.assign((size_t)nt, -1);
    std::vector<std::vector<int32_t>> G((size_t)np);
    for (int t = 0; t < nt; ++t) G[P.tri_node[t]].push_back(t);
    for (int q = 0; q < np; ++q) {
      const int nseed = std::min<int>(T.b, (int)G[q].size());
      std::vector<int32_t> seeds = nseed ? random_seeds(G[q], nseed, p->seed, l, q) : std::vector<int32_t>{};
      for (int k = 0; k < T.b; ++k) {
        const int j = q * T.b + k;
        C.parent[j] = q;
        C.slot[j] = node_base + (uint32_t)j;
        HBox& bx = C.box[j];
        std::memcpy(bx.Q, P.box[q].Q, 36);
        if (k < nseed) {
          for (int d = 0; d < 3; ++d) bx.c[d] = (float)S->M.cen[3 * seeds[k] + d];
          bx.h[0] = bx.h[1] = bx.h[2] = 0.f;
        } else {  // more children than triangles: an empty node
          std::memcpy(bx.c, P.box[q].c, 12);
          bx.h[0] = bx.h[1] = bx.h[2] = -1.f;
        }
      }
    }
    OBBV_RET(solve_level(*S, T, l, p->iters));
    for (auto& bx : C.box)
      if (bx.h[0] < 0.f) bx.h[0] = bx.h[1] = bx.h[2] = 0.f;
    node_base += (uint32_t)nc;
  }
  double e = T.error();
  if (out_e) out_e[0] = e;
  // sweeps: bottom-up merges while Eq. 7 improves, then top-down re-solves
  for (int sw = 0; sw < p->sweeps; ++sw) {
    int top = T.L;  // highest level changed by the up pass
    for (int l = T.L - 2; l >= 1; --l) {
      const Tree saved = T;
      OBBV_RET(merge_level(*S, T, l));
      const double e2 = T.error();
      if (e2 < e) {
        e = e2;
        top = l;
      } else {
        T = saved;
        break;
      }
    }
    for (int l = std::max(1, top + 1); l < T.L; ++l) {
      const Tree saved = T;
      OBBV_RET(solve_level(*S, T, l, p->iters));
      const double e2 = T.error();
      if (e2 < e)
        e = e2;
      else
        T = saved;
    }
    if (out_e) out_e[1 + sw] = e;
  }
  // outputs, level-major global node numbering
  int64_t g0 = 0;
  for (int l = 0; l < T.L; ++l) {
    const Level& Lv = T.lv[l];
    const int64_t pbase = l > 0 ? g0 - (int64_t)T.lv[l - 1].box.size() : 0;
    for (size_t j = 0; j < Lv.box.size(); ++j) {
      const int64_t g = g0 + (int64_t)j;
      if (out_boxes) {
        std::memcpy(out_boxes + 15 * g, Lv.box[j].c, 12);
        std::memcpy(out_boxes + 15 * g + 3, Lv.box[j].Q, 36);
        std::memcpy(out_boxes + 15 * g + 12, Lv.box[j].h, 12);
      }
      if (out_obv) out_obv[g] = Lv.obv[j];
      if (out_parent) out_parent[g] = Lv.parent[j] >= 0 ? (int32_t)(pbase + Lv.parent[j]) : -1;
    }
    if (out_tri_node)
      for (int t = 0; t < nt; ++t)
        out_tri_node[(int64_t)l * nt + t] = Lv.tri_node[t] >= 0 ? (int32_t)(g0 + Lv.tri_node[t]) : -1;
    g0 += (int64_t)Lv.box.size();
  }
  if (out_counters) {
    out_counters[0] = S->cnt.evals;
    out_counters[1] = S->cnt.rounds;
    out_counters[2] = S->cnt.trivial;
    out_counters[3] = S->cnt.moves;
    out_counters[4] = S->pred.predicted;
    out_counters[5] = S->pred.fallbacks;
  }
  return OBBV_OK;
}
