// Surrogate ranker MLP: 544 -> 256 (ReLU) -> 256 (ReLU) -> 1, trained on (box,
// outer fraction) pairs from the exact outer-volume kernel.  The output corrects
// the occupancy estimate: f = (1 - mean occupancy) + sigmoid(z) - 1/2.
//
// Every matrix product runs on MFMA (v_mfma_f32_32x32x8bf16_1k in training,
// v_mfma_f32_32x32x16_bf16 in the fused inference tile): operands are
// rounded to bfloat16 (round to nearest even) as they are loaded, products are
// accumulated in float32.  Activations, gradients and the master weights stay in
// float32 memory; the bfloat16 rounding points are the inputs, the weights, the
// hidden activations and the back-propagated gradients entering each product.
//
// Parameter vector (float32, kMlpParams entries):
//   W1 [544][256] | b1 [256] | W2 [256][256] | b2 [256] | w3 [256] | b3 [1]
// (W[i][o] multiplies input i into output o).
#include <cmath>

#include <cstring>

#include "common.h"
#include "box_features.h"

namespace obbv {
namespace {

constexpr int kIn = 544, kH = 256;
constexpr int64_t oW1 = 0, ob1 = oW1 + (int64_t)kIn * kH, oW2 = ob1 + kH, ob2 = oW2 + (int64_t)kH * kH,
                  ow3 = ob2 + kH, ob3 = ow3 + kH, kParams = ob3 + 1;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ inline short f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ inline float bf(float x) { return __uint_as_float(((uint32_t)(uint16_t)f2bf(x)) << 16); }

// C[m, n] (+)= sum_k bf16(A[m, k]) bf16(B[k, n]) with arbitrary element strides;
// with `bias` (forward layers) C[m, n] = max(sum + bias[n], 0) instead.
// One wave per 32 x 32 tile of C; M, N multiples of 32, K a multiple of 8.
// MFMA 32x32x8 operand layout: lane l holds A[l % 32][4 (l / 32) + j] and
// B[4 (l / 32) + j][l % 32], j = 0..3; result register r of lane l is
// C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
__global__ void __launch_bounds__(64)
k_gemm(const float* __restrict__ A, int64_t sam, int64_t sak, const float* __restrict__ B, int64_t sbk,
       int64_t sbn, float* __restrict__ C, int64_t scm, int64_t scn, int M, int N, int K, int accumulate,
       const float* __restrict__ bias) {
  const int tiles_n = N / 32;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - (blockIdx.x / tiles_n) * tiles_n;
  const int lane = threadIdx.x;
  const int r = lane & 31, kq = (lane >> 5) * 4;
  const int64_t m = (int64_t)tm * 32 + r, n = (int64_t)tn * 32 + r;
  v16f acc;
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 8) {
    v4s a, b;
    for (int j = 0; j < 4; ++j) {
      const int64_t k = k0 + kq + j;
      a[j] = f2bf(A[m * sam + k * sak]);
      b[j] = f2bf(B[k * sbk + n * sbn]);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  for (int rr = 0; rr < 16; ++rr) {
    const int64_t row = (int64_t)tm * 32 + 8 * (rr / 4) + 4 * (lane >> 5) + (rr % 4);
    const int64_t col = (int64_t)tn * 32 + (lane & 31);
    float* c = C + row * scm + col * scn;
    if (bias)
      *c = fmaxf(acc[rr] + bias[col], 0.f);
    else
      *c = accumulate ? *c + acc[rr] : acc[rr];
  }
}

int gemm(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C, int64_t scm,
         int64_t scn, int M, int N, int K, bool accumulate, hipStream_t s, const float* bias_relu = nullptr) {
  if (M % 32 || N % 32 || K % 8) {
    set_error("MLP product sizes must be multiples of 32 (M, N) and 8 (K)");
    return OBBV_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_gemm, dim3((unsigned)((M / 32) * (N / 32))), dim3(64), 0, s, A, sam, sak, B, sbk, sbn, C, scm,
                     scn, M, N, K, accumulate ? 1 : 0, bias_relu);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

// z = bf16(H2) . bf16(w3) + b3; the output corrects the occupancy estimate
// h = 1 - mean(X[15..526]): f = h + sigmoid(z) - 1/2; with targets: dz and the loss
__global__ void k_head(const float* __restrict__ H2, const float* __restrict__ P, const float* __restrict__ X, int n,
                       float* __restrict__ f, const float* __restrict__ t, float* __restrict__ dz,
                       float* __restrict__ loss) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const float* hr = H2 + (int64_t)row * kH;
  float z = 0.f;
  for (int c = 0; c < kH; ++c) z = fmaf(bf(hr[c]), bf(P[ow3 + c]), z);
  z += P[ob3];
  const float* x = X + (int64_t)row * kIn;
  float occ = 0.f;
  for (int c = 15; c < 527; ++c) occ += x[c];
  const float sig = 1.f / (1.f + expf(-z));
  const float fr = (1.f - occ / 512.f) + sig - 0.5f;
  f[row] = fr;
  if (t) {
    const float e = fr - t[row];
    dz[row] = 2.f * e * sig * (1.f - sig) / (float)n;
    atomicAdd(loss, e * e / (float)n);
  }
}

// dw3[c] = sum_r bf16(H2[r][c]) bf16(dz[r]); db3 = sum_r dz[r]  (one thread per column)
__global__ void k_dw3(const float* __restrict__ H2, const float* __restrict__ dz, int n, float* __restrict__ G) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > kH) return;
  float acc = 0.f;
  if (c < kH) {
    for (int r = 0; r < n; ++r) acc = fmaf(bf(H2[(int64_t)r * kH + c]), bf(dz[r]), acc);
    G[ow3 + c] = acc;
  } else {
    for (int r = 0; r < n; ++r) acc += dz[r];
    G[ob3] = acc;
  }
}

// dH2[r][c] = bf16(dz[r]) bf16(w3[c]) [H2 > 0]
__global__ void k_dh2(const float* __restrict__ dz, const float* __restrict__ P, const float* __restrict__ H2, int n,
                      float* __restrict__ dH2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * kH) return;
  const int r = (int)(i / kH), c = (int)(i % kH);
  dH2[i] = H2[i] > 0.f ? bf(dz[r]) * bf(P[ow3 + c]) : 0.f;
}

__global__ void k_relu_mask(float* __restrict__ G, const float* __restrict__ H, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(H[i] > 0.f)) G[i] = 0.f;
}

// out[c] = sum_r X[r][c]  (unrounded gradient sums for the biases)
__global__ void k_colsum(const float* __restrict__ X, int n, int w, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= w) return;
  float acc = 0.f;
  for (int r = 0; r < n; ++r) acc += X[(int64_t)r * w + c];
  out[c] = acc;
}

// Adam (Kingma and Ba, 2015) with bias correction, float32 master weights
__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ G,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Fused inference: the network on 32 rows per workgroup, on the 32 x 32 x 16
// bfloat16 MFMA (v_mfma_f32_32x32x16_bf16): lane l holds A[l % 32][8 (l / 32) + j]
// and B[8 (l / 32) + j][l % 32], j = 0..7, of each K-step of 16; the result
// layout is that of the 32 x 32 x 8 form.  The weights are pre-packed as bfloat16
// in the order the lanes consume them: for output unit n, lane half q and K-step
// k, entry (((n / 32) (K / 16) + k) 64 + 32 q + n % 32) 8 + j holds
// W[16 k + 8 q + j][n], so the 64 lanes of the wave that computes columns
// 32 (n / 32) .. read one contiguous kilobyte per K-step (16 cache lines per
// load instruction instead of 64).
constexpr int64_t kPacked = (int64_t)kIn * kH + (int64_t)kH * kH;  // bf16 entries
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline v16f mfma16(const v8s a, const v8s b, const v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

__global__ void k_mlp_pack(const float* __restrict__ P, short* __restrict__ W) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPacked) return;
  const bool first = i < (int64_t)kIn * kH;
  const int K = first ? kIn : kH;
  const int64_t e = first ? i : i - (int64_t)kIn * kH;
  const int j = (int)(e & 7);
  const int64_t rest = e >> 3;
  const int ln = (int)(rest & 63);  // lane: 32 q + n % 32
  const int64_t tk = rest >> 6;     // (n / 32) (K / 16) + k
  const int k = (int)(tk % (K / 16));
  const int n = 32 * (int)(tk / (K / 16)) + (ln & 31), q = ln >> 5;
  const int in = 16 * k + 8 * q + j;
  W[i] = f2bf(P[(first ? oW1 : oW2) + (int64_t)in * kH + n]);
}

constexpr int kFusedRows = 32;
static_assert(kFeatIn == kIn, "feature rows and the first layer disagree");
// LDS row pitches of the tile (bfloat16 entries): 8 more than the row, so the
// 32 rows a K-step reads fall in different banks (a pitch of 256 entries put
// every row in the same one)
constexpr int kInPitch = kIn + 8, kHPitch = kH + 8;

// The network on one tile of kFusedRows rows, by one workgroup of kRowThreads.
// Layers 1 and 2: bfloat16 rows sx [32][kInPitch] -> sh1 (bfloat16 [32][kHPitch]) -> the
// second hidden layer in registers.  Eight waves, wave w computes the 32 x 32
// output tile of columns 32 w .. 32 w + 31.  A wave's weight operands for both
// layers (544 + 256 contiguous bytes per lane) are issued before the rows are
// staged, so the layers wait on one memory latency instead of one per K-step.
// Head: each lane forms bf16(h2) bf16(w3) for its column and 16 rows; the 32
// columns of a wave are summed by an xor butterfly (1, 2, 4, 8, 16) within each
// half-wave, the eight wave sums in order, then the bias:
// f = (1 - occ / 512) + sigmoid(z) - 1/2.  `stage` fills sx and socc.  Every
// thread of the block calls this (barriers).
constexpr int kRowThreads = 512;

// `pre` runs before any weight is requested (a stage whose own loads should
// return first issues them there); kLateW2: the second layer's weights are
// requested after the rows are staged (a stage that holds many registers of
// its own), else with the first layer's.  kOneRow: only row 0 of the tile is a
// real row (the other rows' values are never written out, so they are left
// uncomputed where the layers allow; row 0 takes the same arithmetic).  The
// tile's outputs are f[row0 + t] for t < rows, or, with `tag`, the 64-bit words
// tag[row0 + t] = seq << 32 | bits(f) (one system-scope store each, so a host
// that reads a word with this call's seq in it has the value as well).
template <bool kLateW2 = false, bool kOneRow = false, class Stage, class Pre>
__device__ void mlp_tile(const float* __restrict__ P, const short* __restrict__ W, Stage stage, Pre pre, short* sx,
                         short* sh1, float* zp, const float* socc, int64_t row0, int rows, float* __restrict__ f,
                         unsigned long long* __restrict__ tag = nullptr, unsigned seq = 0u) {
  pre();
  __builtin_amdgcn_sched_barrier(0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = 32 * wave + (lane & 31);
  // this lane's biases and head weight, requested with the weights
  const float bias1 = P[ob1 + c], bias2 = P[ob2 + c], w3 = bf(P[ow3 + c]), bias3 = P[ob3];
  const int r = lane & 31, kq = (lane >> 5) * 8;
  // this wave's operands: K-step k of lane l at v8s index (wave (K / 16) + k) 64 + l
  const v8s* w1 = reinterpret_cast<const v8s*>(W) + (int64_t)wave * (kIn / 16) * 64 + lane;
  const v8s* w2 = reinterpret_cast<const v8s*>(W + (int64_t)kIn * kH) + (int64_t)wave * (kH / 16) * 64 + lane;
  v8s b1[kIn / 16], b2[kH / 16];
  for (int k = 0; k < kIn / 16; ++k) b1[k] = w1[64 * k];
  if (!kLateW2)
    for (int k = 0; k < kH / 16; ++k) b2[k] = w2[64 * k];
  __builtin_amdgcn_sched_barrier(0);  // the weight loads are in flight before the rows are staged
  stage();
  __syncthreads();
  if (kLateW2) {
    for (int k = 0; k < kH / 16; ++k) b2[k] = w2[64 * k];
    __builtin_amdgcn_sched_barrier(0);
  }
  {
    v16f acc;
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    for (int k = 0; k < kIn / 16; ++k) {
      const v8s x = *reinterpret_cast<const v8s*>(&sx[r * kInPitch + 16 * k + kq]);
      acc = mfma16(x, b1[k], acc);
    }
    if (kOneRow) {
      if (lane < 32) sh1[c] = f2bf(fmaxf(acc[0] + bias1, 0.f));
    } else {
      for (int rr = 0; rr < 16; ++rr) {
        const int row = 8 * (rr / 4) + 4 * (lane >> 5) + (rr % 4);
        sh1[row * kHPitch + c] = f2bf(fmaxf(acc[rr] + bias1, 0.f));
      }
    }
  }
  __syncthreads();
  v16f acc;
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k = 0; k < kH / 16; ++k) {
    const v8s h = *reinterpret_cast<const v8s*>(&sh1[r * kHPitch + 16 * k + kq]);
    acc = mfma16(h, b2[k], acc);
  }
  if (kOneRow) {  // row 0 sits in acc[0] of lanes 0..31
    float v = bf(fmaxf(acc[0] + bias2, 0.f)) * w3;
    for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) zp[wave * kFusedRows] = v;
  } else {
    float v[16];
    for (int rr = 0; rr < 16; ++rr) v[rr] = bf(fmaxf(acc[rr] + bias2, 0.f)) * w3;
    for (int o = 1; o < 32; o <<= 1)
      for (int rr = 0; rr < 16; ++rr) v[rr] += __shfl_xor(v[rr], o, 64);
    if ((lane & 31) == 0)
      for (int rr = 0; rr < 16; ++rr) zp[wave * kFusedRows + 8 * (rr / 4) + 4 * (lane >> 5) + (rr % 4)] = v[rr];
  }
  __syncthreads();
  if ((int)threadIdx.x < rows) {
    float z = 0.f;
    for (int w = 0; w < kRowThreads / 64; ++w) z += zp[w * kFusedRows + threadIdx.x];
    z += bias3;
    const float sig = 1.f / (1.f + expf(-z));
    const float out = (1.f - socc[threadIdx.x] / 512.f) + sig - 0.5f;
    if (tag)
      __hip_atomic_store(&tag[row0 + threadIdx.x], ((unsigned long long)seq << 32) | __float_as_uint(out),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    else
      f[row0 + threadIdx.x] = out;
  }
}

// Network outputs of 32 rows per workgroup.  kFloat: float32 rows X [n][kIn]
// (n a multiple of 32), rounded to bfloat16 and their occupancy sums taken here;
// otherwise bfloat16 rows Xb [n][kIn] with their sums in occ [n] (rows >= n read
// as zero); with `tag` the outputs go out as tagged words (mlp_tile).
template <bool kFloat>
__global__ void __launch_bounds__(kRowThreads)
k_mlp_rows(const float* __restrict__ P, const short* __restrict__ W, const float* __restrict__ X,
           const short* __restrict__ Xb, const float* __restrict__ occ, int n, float* __restrict__ f,
           unsigned long long* tag, unsigned seq) {
  __shared__ short sx[kFusedRows * kInPitch];
  __shared__ short sh1[kFusedRows * kHPitch];
  __shared__ float zp[(kRowThreads / 64) * kFusedRows];
  __shared__ float socc[kFusedRows];
  const int64_t row0 = (int64_t)blockIdx.x * kFusedRows;
  auto stage = [&]() {
    if constexpr (kFloat) {
      for (int i = threadIdx.x; i < kFusedRows * kIn; i += blockDim.x) {
        const int rw = i / kIn;
        sx[rw * kInPitch + (i - rw * kIn)] = f2bf(X[row0 * kIn + i]);
      }
      const int wave = threadIdx.x >> 6;
      for (int rw = wave; rw < kFusedRows; rw += kRowThreads / 64) {
        const float* x = X + (row0 + rw) * kIn;
        const float o = occ_sum_wave([&](int k) { return x[k]; });
        if ((threadIdx.x & 63) == 0) socc[rw] = o;
      }
    } else {
      typedef int v4i __attribute__((ext_vector_type(4)));
      constexpr int kChunks = kIn / 8;  // 16-byte pieces of a row
      for (int i = threadIdx.x; i < kFusedRows * kChunks; i += blockDim.x) {
        const int rw = i / kChunks, c = i - rw * kChunks;
        v4i q = {0, 0, 0, 0};
        if (row0 + rw < n) q = *reinterpret_cast<const v4i*>(Xb + (row0 + rw) * kIn + 8 * c);
        *reinterpret_cast<v4i*>(&sx[rw * kInPitch + 8 * c]) = q;
      }
      if (threadIdx.x < kFusedRows) socc[threadIdx.x] = row0 + threadIdx.x < n ? occ[row0 + threadIdx.x] : 0.f;
    }
  };
  mlp_tile(P, W, stage, [] {}, sx, sh1, zp, socc, row0, (int)min((int64_t)kFusedRows, n - row0), f, tag, seq);
}

// ranker input rows from the occupancy volume, one workgroup per box
__global__ void k_sample_features(const float* __restrict__ vol, int N, const float* __restrict__ frame,
                                  const obbv_box* __restrict__ boxes, int n, float* __restrict__ X) {
  const int b = blockIdx.x;
  if (b >= n) return;
  const float* p = reinterpret_cast<const float*>(boxes + b);
  float* x = X + (int64_t)b * kFeatIn;
  for (int k = threadIdx.x; k < kFeatIn; k += blockDim.x) x[k] = box_feature(k, p, frame, vol, N);
}

// Ranker inputs of one box per workgroup (256 threads), for k_mlp_rows<false>:
// bfloat16 row Xb [b][kIn] and the occupancy sum occ [b].  Thread t computes
// inputs t, t + 256, t + 512 with their 24 volume reads issued together; the
// float values equal k_sample_features' and the sum is occ_sum_wave's.  The box
// may sit in mapped host memory: it is read once.
constexpr int kRankPerThread = (kIn + 255) / 256;

__global__ void __launch_bounds__(256)
k_rank_inputs(const float* __restrict__ vol, int N, const float* __restrict__ frame,
              const obbv_box* __restrict__ boxes, int n, short* __restrict__ Xb, float* __restrict__ occ) {
  __shared__ float sbox[16];
  __shared__ float sf[kIn];
  const int64_t b = blockIdx.x;
  if (b >= n) return;
  if (threadIdx.x < 15) sbox[threadIdx.x] = reinterpret_cast<const float*>(boxes)[b * 15 + threadIdx.x];
  __syncthreads();
  OccSample smp[kRankPerThread];
  float v[kRankPerThread][8];
  for (int m = 0; m < kRankPerThread; ++m) {  // no branches: every read in flight together
    const int r = min(max((int)threadIdx.x + 256 * m - kFeatOcc0, 0), kFeatOccN - 1);
    smp[m] = occ_sample_at(r, sbox, frame);
    for (int c = 0; c < 8; ++c) v[m][c] = occ_corner(vol, N, smp[m], c);
  }
  for (int m = 0; m < kRankPerThread; ++m) {
    const int k = threadIdx.x + 256 * m;
    if (k >= kIn) break;
    float x = 0.f;
    if (k < kFeatOcc0) x = box_param_feature(k, sbox, frame);
    else if (k < kFeatOcc0 + kFeatOccN) x = occ_blend(smp[m], v[m]);
    sf[k] = x;
    Xb[b * kIn + k] = f2bf(x);
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const float o = occ_sum_wave([&](int k) { return sf[k]; });
    if (threadIdx.x == 0) occ[b] = o;
  }
}

// Ranking of kRankRows boxes per workgroup in one launch: the workgroup computes
// its boxes' inputs as k_rank_inputs does (the same float values, bfloat16 row
// and occupancy sum) straight into the tile's LDS rows, the other rows of the
// 32-row tile are zero, and the network runs as in k_mlp_rows, so the outputs
// are bitwise those of k_rank_inputs + k_mlp_rows<false>.  The volume reads are
// requested first, then the first layer's weights.  A workgroup's volume gathers
// (4,352 per box) and weight loads (401 KB) pass one CU's load pipeline, so few
// boxes per workgroup spread the gathers over more CUs.  With `tag` the outputs
// go out as tagged words (mlp_tile): no completion counter or flag, so a
// workgroup ends right after its own store.
// Up to kArgBoxes boxes can travel in the kernel arguments (no read of mapped
// host memory on the critical path).
constexpr int kArgBoxes = 32;
struct RankArgBoxes {
  float v[kArgBoxes * 15];
};

template <int kRankRows>
__global__ void __launch_bounds__(kRowThreads)
k_rank_fused(const float* __restrict__ P, const short* __restrict__ W, const float* __restrict__ vol, int N,
             const float* __restrict__ frame, const obbv_box* __restrict__ boxes, RankArgBoxes ab, int use_ab,
             int n, float* __restrict__ f, unsigned long long* tag, unsigned seq) {
  __shared__ __align__(16) short sx[kFusedRows * kInPitch];
  __shared__ short sh1[kFusedRows * kHPitch];
  __shared__ float zp[(kRowThreads / 64) * kFusedRows];
  __shared__ float socc[kFusedRows];
  __shared__ float sbox[kRankRows][16];
  __shared__ float sf[kRankRows][kIn];
  constexpr int kRankFusedPer = (kRankRows * kIn + kRowThreads - 1) / kRowThreads;
  const int64_t row0 = (int64_t)blockIdx.x * kRankRows;
  const int rows = (int)min((int64_t)kRankRows, n - row0);
  OccSample smp[kRankFusedPer];
  float v[kRankFusedPer][8];
  // before the weights: the tile's boxes (from the arguments, or from `boxes`,
  // which may sit in mapped host memory: each read once; rows past the last
  // box take the first box and are discarded), then every volume read of the
  // inputs, so these return first
  auto pre = [&]() {
    if (threadIdx.x < kRankRows * 15) {
      const int rw = threadIdx.x / 15, e = threadIdx.x - 15 * (threadIdx.x / 15);
      const int64_t at = (row0 + (rw < rows ? rw : 0)) * 15 + e;
      sbox[rw][e] = use_ab ? ab.v[at] : reinterpret_cast<const float*>(boxes)[at];
    }
    __syncthreads();
    for (int m = 0; m < kRankFusedPer; ++m) {  // no branches: every read in flight together
      const int idx = min((int)threadIdx.x + kRowThreads * m, kRankRows * kIn - 1);
      const int rw = idx / kIn, k = idx - rw * kIn;
      const int r = min(max(k - kFeatOcc0, 0), kFeatOccN - 1);
      smp[m] = occ_sample_at(r, sbox[rw], frame);
      for (int c = 0; c < 8; ++c) v[m][c] = occ_corner(vol, N, smp[m], c);
    }
  };
  auto stage = [&]() {
    // rows kRankRows.. of the tile are zero
    typedef int v4i __attribute__((ext_vector_type(4)));
    constexpr int kChunks = kInPitch / 8;
    for (int i = threadIdx.x; i < (kFusedRows - kRankRows) * kChunks; i += kRowThreads)
      *reinterpret_cast<v4i*>(&sx[kRankRows * kInPitch + 8 * i]) = v4i{0, 0, 0, 0};
    for (int m = 0; m < kRankFusedPer; ++m) {
      const int idx = threadIdx.x + kRowThreads * m;
      if (idx >= kRankRows * kIn) break;
      const int rw = idx / kIn, k = idx - rw * kIn;
      float x = 0.f;
      if (k < kFeatOcc0) x = box_param_feature(k, sbox[rw], frame);
      else if (k < kFeatOcc0 + kFeatOccN) x = occ_blend(smp[m], v[m]);
      sf[rw][k] = x;
      sx[rw * kInPitch + k] = rw < rows ? f2bf(x) : (short)0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    if (wave < kRankRows) {
      const float o = occ_sum_wave([&](int k) { return sf[wave][k]; });
      if ((threadIdx.x & 63) == 0) socc[wave] = o;
    }
  };
  // the second layer's weights after the stage: requested with the first
  // layer's, they delay the volume gathers in the CU's load pipeline
  mlp_tile<true, kRankRows == 1>(P, W, stage, pre, sx, sh1, zp, socc, row0, rows, f, tag, seq);
}

struct MlpScratch {
  float* H1;
  float* H2;
  float* f;
  float* dz;
  float* dH2;
  float* dH1;
  float* G;
  float* loss;
};

int mlp_scratch(int n, MlpScratch& S) {
  const size_t bytes = ((size_t)n * kH * 4 + (size_t)n * 2 + (size_t)kParams + 64) * sizeof(float);
  void* p = nullptr;
  OBBV_RET(pool_get(kPoolMlp, bytes, &p));
  float* q = (float*)p;
  S.H1 = q;
  q += (size_t)n * kH;
  S.H2 = q;
  q += (size_t)n * kH;
  S.dH2 = q;
  q += (size_t)n * kH;
  S.dH1 = q;
  q += (size_t)n * kH;
  S.f = q;
  q += n;
  S.dz = q;
  q += n;
  S.loss = q;
  q += 16;
  S.G = q;
  return OBBV_OK;
}

inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int forward(const float* P, const float* X, int n, MlpScratch& S, float* out_f, const float* t, hipStream_t s) {
  OBBV_RET(gemm(X, kIn, 1, P + oW1, kH, 1, S.H1, kH, 1, n, kH, kIn, false, s, P + ob1));
  OBBV_RET(gemm(S.H1, kH, 1, P + oW2, kH, 1, S.H2, kH, 1, n, kH, kH, false, s, P + ob2));
  if (t) OBBV_HIP(hipMemsetAsync(S.loss, 0, 4, s));
  hipLaunchKernelGGL(k_head, dim3(blocks(n, 256)), dim3(256), 0, s, S.H2, P, X, n, out_f, t, S.dz, S.loss);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

}  // namespace

int mlp_pack_impl(const float* params, short* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((unsigned)((kPacked + 255) / 256)), dim3(256), 0, s, params, packed);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

int64_t mlp_packed_entries() { return kPacked; }

int mlp_infer_packed(const float* params, const short* packed, const float* X, int32_t n, float* out_f,
                     hipStream_t s) {
  OBBV_ARG(n >= 0 && n % kFusedRows == 0, "n must be a non-negative multiple of 32");
  if (n == 0) return OBBV_OK;
  hipLaunchKernelGGL(k_mlp_rows<true>, dim3((unsigned)(n / kFusedRows)), dim3(kRowThreads), 0, s, params, packed, X,
                     (const short*)nullptr, (const float*)nullptr, n, out_f, (unsigned long long*)nullptr, 0u);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

// Rankings of at most kRankOneBoxMax boxes take the one-launch kernel with one
// box per workgroup, of at most kRankFusedMax with four; every workgroup reads
// the 401 KB of weights, so larger calls take the two launches.
constexpr int kRankOneBoxMax = 256;
constexpr int kRankFusedMax = 1024;

// scratch of mlp_rank_packed: Xb [n][kIn] bfloat16 | occ [n]
size_t mlp_rank_scratch_bytes(int32_t n) { return (((size_t)n * kIn * 2 + 255) & ~(size_t)255) + (size_t)n * 4; }

int mlp_rank_packed(const float* params, const short* packed, const float* volume, int32_t N, const float* frame,
                    const obbv_box* boxes, int32_t n, void* scratch, float* out_f, hipStream_t s,
                    unsigned long long* tag, unsigned seq, const obbv_box* host_boxes) {
  OBBV_ARG(n >= 0 && N >= 1, "bad size");
  if (n == 0) return OBBV_OK;
  RankArgBoxes ab;
  const int use_ab = host_boxes && n <= kArgBoxes;
  if (use_ab) std::memcpy(ab.v, host_boxes, (size_t)n * sizeof(obbv_box));
  if (n <= kRankOneBoxMax) {  // one launch, one box per workgroup
    hipLaunchKernelGGL(k_rank_fused<1>, dim3((unsigned)n), dim3(kRowThreads), 0, s, params, packed, volume, N, frame,
                       boxes, ab, use_ab, n, out_f, tag, seq);
    OBBV_HIP(hipGetLastError());
    return OBBV_OK;
  }
  if (n <= kRankFusedMax) {  // one launch, four boxes per workgroup
    hipLaunchKernelGGL(k_rank_fused<4>, dim3((unsigned)((n + 3) / 4)), dim3(kRowThreads), 0, s, params, packed, volume,
                       N, frame, boxes, ab, use_ab, n, out_f, tag, seq);
    OBBV_HIP(hipGetLastError());
    return OBBV_OK;
  }
  short* Xb = (short*)scratch;
  float* occ = (float*)((char*)scratch + (((size_t)n * kIn * 2 + 255) & ~(size_t)255));
  hipLaunchKernelGGL(k_rank_inputs, dim3((unsigned)n), dim3(256), 0, s, volume, N, frame, boxes, n, Xb, occ);
  hipLaunchKernelGGL(k_mlp_rows<false>, dim3((unsigned)((n + kFusedRows - 1) / kFusedRows)), dim3(kRowThreads), 0, s,
                     params, packed, (const float*)nullptr, (const short*)Xb, (const float*)occ, n, out_f, tag, seq);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

int mlp_forward_impl(const float* params, const float* X, int32_t n, float* out_f, hipStream_t s) {
  OBBV_ARG(params && X && out_f, "NULL argument");
  OBBV_ARG(n >= 0 && n % 32 == 0, "n must be a non-negative multiple of 32");
  if (n == 0) return OBBV_OK;
  void* pv = nullptr;
  OBBV_RET(pool_get(kPoolMlp, (size_t)kPacked * 2, &pv));
  OBBV_RET(mlp_pack_impl(params, (short*)pv, s));
  return mlp_infer_packed(params, (const short*)pv, X, n, out_f, s);
}

}  // namespace obbv

using namespace obbv;

static int obbv_mlp_forward_body(const float* params, const float* X, int32_t n, float* out_f, void* stream);
extern "C" int obbv_mlp_forward(const float* params, const float* X, int32_t n, float* out_f, void* stream) {
  return obbv::guarded([&] { return obbv_mlp_forward_body(params, X, n, out_f, stream); });
}
static int obbv_mlp_forward_body(const float* params, const float* X, int32_t n, float* out_f, void* stream) {
  clear_error();
  return mlp_forward_impl(params, X, n, out_f, (hipStream_t)stream);
}

static int obbv_sample_features_body(const float* volume, int32_t N, const float* frame, const obbv_box* boxes,
                                    int32_t n_boxes, float* out_X, void* stream);
extern "C" int obbv_sample_features(const float* volume, int32_t N, const float* frame, const obbv_box* boxes,
                                    int32_t n_boxes, float* out_X, void* stream) {
  return obbv::guarded([&] { return obbv_sample_features_body(volume, N, frame, boxes, n_boxes, out_X, stream); });
}
static int obbv_sample_features_body(const float* volume, int32_t N, const float* frame, const obbv_box* boxes,
                                    int32_t n_boxes, float* out_X, void* stream) {
  clear_error();
  OBBV_ARG(n_boxes >= 0 && N >= 1, "bad size");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(volume && frame && boxes && out_X, "NULL argument");
  hipLaunchKernelGGL(k_sample_features, dim3((unsigned)n_boxes), dim3(128), 0, (hipStream_t)stream, volume, N, frame,
                     boxes, n_boxes, out_X);
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

static int obbv_mlp_rank_boxes_body(const float* params, const float* volume, int32_t N, const float* frame,
                                   const obbv_box* boxes, int32_t n_boxes, float* out_f, void* stream);
extern "C" int obbv_mlp_rank_boxes(const float* params, const float* volume, int32_t N, const float* frame,
                                   const obbv_box* boxes, int32_t n_boxes, float* out_f, void* stream) {
  return obbv::guarded([&] { return obbv_mlp_rank_boxes_body(params, volume, N, frame, boxes, n_boxes, out_f, stream); });
}
static int obbv_mlp_rank_boxes_body(const float* params, const float* volume, int32_t N, const float* frame,
                                   const obbv_box* boxes, int32_t n_boxes, float* out_f, void* stream) {
  clear_error();
  OBBV_ARG(n_boxes >= 0 && N >= 1, "bad size");
  if (n_boxes == 0) return OBBV_OK;
  OBBV_ARG(params && volume && frame && boxes && out_f, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  void* pv = nullptr;
  void* sc = nullptr;
  OBBV_RET(pool_get(kPoolMlp, (size_t)kPacked * 2, &pv));
  OBBV_RET(pool_get(kPoolRank, mlp_rank_scratch_bytes(n_boxes), &sc));
  OBBV_RET(mlp_pack_impl(params, (short*)pv, s));
  return mlp_rank_packed(params, (const short*)pv, volume, N, frame, boxes, n_boxes, sc, out_f, s, nullptr, 0u, nullptr);
}

static int obbv_mlp_train_step_body(float* params, float* adam_m, float* adam_v, int32_t step, const float* X,
                                   const float* target, int32_t n, float lr, float* out_loss, float* out_grad,
                                   void* stream);
extern "C" int obbv_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, const float* X,
                                   const float* target, int32_t n, float lr, float* out_loss, float* out_grad,
                                   void* stream) {
  return obbv::guarded([&] { return obbv_mlp_train_step_body(params, adam_m, adam_v, step, X, target, n, lr, out_loss, out_grad, stream); });
}
static int obbv_mlp_train_step_body(float* params, float* adam_m, float* adam_v, int32_t step, const float* X,
                                   const float* target, int32_t n, float lr, float* out_loss, float* out_grad,
                                   void* stream) {
  clear_error();
  OBBV_ARG(params && adam_m && adam_v && X && target, "NULL argument");
  OBBV_ARG(n > 0 && n % 32 == 0, "n must be a positive multiple of 32");
  OBBV_ARG(step >= 1, "step counts from 1");
  hipStream_t s = (hipStream_t)stream;
  MlpScratch S;
  OBBV_RET(mlp_scratch(n, S));
  OBBV_RET(forward(params, X, n, S, S.f, target, s));
  float* G = out_grad ? out_grad : S.G;
  const float* P = params;
  // head
  hipLaunchKernelGGL(k_dw3, dim3(blocks(kH + 1, 64)), dim3(64), 0, s, S.H2, S.dz, n, G);
  hipLaunchKernelGGL(k_dh2, dim3(blocks((int64_t)n * kH, 256)), dim3(256), 0, s, S.dz, P, S.H2, n, S.dH2);
  OBBV_HIP(hipGetLastError());
  // layer 2: dW2 = H1^T dH2, db2 = colsum dH2, dH1 = (dH2 W2^T) [H1 > 0]
  OBBV_RET(gemm(S.H1, 1, kH, S.dH2, kH, 1, G + oW2, kH, 1, kH, kH, n, false, s));
  hipLaunchKernelGGL(k_colsum, dim3(blocks(kH, 64)), dim3(64), 0, s, S.dH2, n, kH, G + ob2);
  OBBV_RET(gemm(S.dH2, kH, 1, P + oW2, 1, kH, S.dH1, kH, 1, n, kH, kH, false, s));
  hipLaunchKernelGGL(k_relu_mask, dim3(blocks((int64_t)n * kH, 256)), dim3(256), 0, s, S.dH1, S.H1, (int64_t)n * kH);
  // layer 1: dW1 = X^T dH1, db1 = colsum dH1
  OBBV_RET(gemm(X, 1, kIn, S.dH1, kH, 1, G + oW1, kH, 1, kIn, kH, n, false, s));
  hipLaunchKernelGGL(k_colsum, dim3(blocks(kH, 64)), dim3(64), 0, s, S.dH1, n, kH, G + ob1);
  OBBV_HIP(hipGetLastError());
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  if (lr > 0.f)
    hipLaunchKernelGGL(k_adam, dim3(blocks(kParams, 256)), dim3(256), 0, s, params, adam_m, adam_v, G, kParams, lr,
                       b1, b2, 1e-8f, c1, c2);
  if (out_loss) OBBV_HIP(hipMemcpyAsync(out_loss, S.loss, 4, hipMemcpyDeviceToDevice, s));
  OBBV_HIP(hipGetLastError());
  return OBBV_OK;
}

extern "C" int64_t obbv_mlp_param_count(void) { return kParams; }
