// Surrogate ranker MLP: 544 -> 256 (ReLU) -> 256 (ReLU) -> 1, trained on (box,
// outer fraction) pairs from the exact outer-volume kernel.  The output corrects
// the occupancy estimate: f = (1 - mean occupancy) + sigmoid(z) - 1/2.
//
// Every matrix product runs on MFMA (v_mfma_f32_32x32x8bf16_1k): operands are
// rounded to bfloat16 (round to nearest even) as they are loaded, products are
// accumulated in float32.  Activations, gradients and the master weights stay in
// float32 memory; the bfloat16 rounding points are the inputs, the weights, the
// hidden activations and the back-propagated gradients entering each product.
//
// Parameter vector (float32, kMlpParams entries):
//   W1 [544][256] | b1 [256] | W2 [256][256] | b2 [256] | w3 [256] | b3 [1]
// (W[i][o] multiplies input i into output o).
#include <cmath>

#include "common.h"

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
// Fused inference: the three layers of 32 rows in one workgroup.  The weights
// are pre-packed as bfloat16 and transposed ([out][in]) so that the four
// consecutive inputs a lane feeds one MFMA step are one 8-byte load; the input
// rows and the first hidden layer sit in LDS as bfloat16, the second hidden
// layer in float32.  Same rounding points, operands and accumulation order as
// the layer-by-layer path, hence the same bits.
// ---------------------------------------------------------------------------
constexpr int64_t kPacked = (int64_t)kIn * kH + (int64_t)kH * kH;  // bf16 entries

__global__ void k_mlp_pack(const float* __restrict__ P, short* __restrict__ W) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPacked) return;
  if (i < (int64_t)kIn * kH) {
    const int o = (int)(i / kIn), k = (int)(i - (int64_t)o * kIn);
    W[i] = f2bf(P[oW1 + (int64_t)k * kH + o]);
  } else {
    const int64_t j = i - (int64_t)kIn * kH;
    const int o = (int)(j / kH), k = (int)(j - (int64_t)o * kH);
    W[i] = f2bf(P[oW2 + (int64_t)k * kH + o]);
  }
}

constexpr int kFusedRows = 32;
constexpr int kH2Pitch = kH + 1;

__global__ void __launch_bounds__(256)
k_mlp_infer(const float* __restrict__ P, const short* __restrict__ W, const float* __restrict__ X,
            float* __restrict__ f) {
  __shared__ short sx[kFusedRows * kIn];
  __shared__ short sh1[kFusedRows * kH];
  __shared__ float sh2[kFusedRows * kH2Pitch];
  const int64_t row0 = (int64_t)blockIdx.x * kFusedRows;
  for (int i = threadIdx.x; i < kFusedRows * kIn; i += blockDim.x) sx[i] = f2bf(X[row0 * kIn + i]);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 31, kq = (lane >> 5) * 4;
  const short* W1t = W;
  const short* W2t = W + (int64_t)kIn * kH;
  // layer 1: this wave's 64 outputs as two 32 x 32 tiles
  {
    const int nA = 64 * wave + r, nB = nA + 32;
    v16f a0, a1;
    for (int i = 0; i < 16; ++i) a0[i] = a1[i] = 0.f;
    for (int k0 = 0; k0 < kIn; k0 += 8) {
      const v4s x = *reinterpret_cast<const v4s*>(&sx[r * kIn + k0 + kq]);
      const v4s bA = *reinterpret_cast<const v4s*>(&W1t[(int64_t)nA * kIn + k0 + kq]);
      const v4s bB = *reinterpret_cast<const v4s*>(&W1t[(int64_t)nB * kIn + k0 + kq]);
      a0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(x, bA, a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(x, bB, a1, 0, 0, 0);
    }
    for (int rr = 0; rr < 16; ++rr) {
      const int row = 8 * (rr / 4) + 4 * (lane >> 5) + (rr % 4);
      const int cA = 64 * wave + (lane & 31), cB = cA + 32;
      sh1[row * kH + cA] = f2bf(fmaxf(a0[rr] + P[ob1 + cA], 0.f));
      sh1[row * kH + cB] = f2bf(fmaxf(a1[rr] + P[ob1 + cB], 0.f));
    }
  }
  __syncthreads();
  // layer 2
  {
    const int nA = 64 * wave + r, nB = nA + 32;
    v16f a0, a1;
    for (int i = 0; i < 16; ++i) a0[i] = a1[i] = 0.f;
    for (int k0 = 0; k0 < kH; k0 += 8) {
      const v4s h = *reinterpret_cast<const v4s*>(&sh1[r * kH + k0 + kq]);
      const v4s bA = *reinterpret_cast<const v4s*>(&W2t[(int64_t)nA * kH + k0 + kq]);
      const v4s bB = *reinterpret_cast<const v4s*>(&W2t[(int64_t)nB * kH + k0 + kq]);
      a0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(h, bA, a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(h, bB, a1, 0, 0, 0);
    }
    for (int rr = 0; rr < 16; ++rr) {
      const int row = 8 * (rr / 4) + 4 * (lane >> 5) + (rr % 4);
      const int cA = 64 * wave + (lane & 31), cB = cA + 32;
      sh2[row * kH2Pitch + cA] = fmaxf(a0[rr] + P[ob2 + cA], 0.f);
      sh2[row * kH2Pitch + cB] = fmaxf(a1[rr] + P[ob2 + cB], 0.f);
    }
  }
  __syncthreads();
  // head, one thread per row (the order of k_head)
  if (threadIdx.x < kFusedRows) {
    const int row = threadIdx.x;
    float z = 0.f;
    for (int c = 0; c < kH; ++c) z = fmaf(bf(sh2[row * kH2Pitch + c]), bf(P[ow3 + c]), z);
    z += P[ob3];
    const float* x = X + (row0 + row) * kIn;
    float occ = 0.f;
    for (int c = 15; c < 527; ++c) occ += x[c];
    const float sig = 1.f / (1.f + expf(-z));
    f[row0 + row] = (1.f - occ / 512.f) + sig - 0.5f;
  }
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
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)(n / kFusedRows)), dim3(256), 0, s, params, packed, X, out_f);
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

extern "C" int obbv_mlp_forward(const float* params, const float* X, int32_t n, float* out_f, void* stream) {
  clear_error();
  return mlp_forward_impl(params, X, n, out_f, (hipStream_t)stream);
}

extern "C" int obbv_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, const float* X,
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
