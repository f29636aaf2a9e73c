// Ranker input row of one box sampled from an occupancy volume.  Shared by the
// feature kernel (rows written to memory) and the fused rank kernel (rows built
// in LDS), so both produce the same float values.
//
// Row layout (544 floats; 527..543 are zero padding for the MFMA K-steps):
//   [0..2]    (c - frame centre) / frame diagonal
//   [3..11]   the axes, row-major (row k = local axis k)
//   [12..14]  log(h / frame diagonal)
//   [15..526] the volume at the 8 x 8 x 8 sub-cell centres of the box,
//             trilinear, x-major then y then z, 0 outside the volume
// Frame: [0..2] volume origin, [3..5] voxel edge per axis, [6..8] mesh bbox
// centre, [9] bbox diagonal.  Voxel centres sit at origin + (i + 1/2) voxel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace obbv {

constexpr int kFeatIn = 544;       // padded row length
constexpr int kFeatOcc0 = 15;      // first occupancy sample
constexpr int kFeatOccN = 512;     // occupancy samples per row

// Voxel (x, y, z), 0 outside.  Branch-free: the read is clamped into the volume
// and its value dropped outside, so a thread's reads can all be in flight at once.
__device__ inline float occ_volume_at(const float* __restrict__ vol, int N, int x, int y, int z) {
  const bool in = (unsigned)x < (unsigned)N && (unsigned)y < (unsigned)N && (unsigned)z < (unsigned)N;
  const int xc = min(max(x, 0), N - 1), yc = min(max(y, 0), N - 1), zc = min(max(z, 0), N - 1);
  const float v = vol[((int64_t)zc * N + yc) * N + xc];
  return in ? v : 0.f;
}

// Trilinear sample r (0..511) of the box p: the voxel corner (x0, y0, z0) and
// the fractions (fx, fy, fz) of the sub-cell centre.
struct OccSample {
  int x0, y0, z0;
  float fx, fy, fz;
};

__device__ inline OccSample occ_sample_at(int r, const float* p, const float* __restrict__ frame) {
  const int ix = r / 64, iy = (r / 8) % 8, iz = r % 8;
  const float l0 = ((ix + 0.5f) / 4.0f - 1.0f) * p[12];
  const float l1 = ((iy + 0.5f) / 4.0f - 1.0f) * p[13];
  const float l2 = ((iz + 0.5f) / 4.0f - 1.0f) * p[14];
  float g[3];
  for (int d = 0; d < 3; ++d) {
    const float w = p[d] + l0 * p[3 + d] + l1 * p[6 + d] + l2 * p[9 + d];
    g[d] = (w - frame[d]) / frame[3 + d] - 0.5f;  // continuous voxel coordinate
  }
  OccSample s;
  s.x0 = (int)floorf(g[0]);
  s.y0 = (int)floorf(g[1]);
  s.z0 = (int)floorf(g[2]);
  s.fx = g[0] - s.x0;
  s.fy = g[1] - s.y0;
  s.fz = g[2] - s.z0;
  return s;
}

// corner c = dx + 2 dy + 4 dz of the sample's voxel cube
__device__ inline float occ_corner(const float* __restrict__ vol, int N, const OccSample& s, int c) {
  return occ_volume_at(vol, N, s.x0 + (c & 1), s.y0 + ((c >> 1) & 1), s.z0 + (c >> 2));
}

__device__ inline float occ_blend(const OccSample& s, const float* v) {
  float acc = 0.f;
  for (int c = 0; c < 8; ++c) {
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    const float wgt = (dx ? s.fx : 1.f - s.fx) * (dy ? s.fy : 1.f - s.fy) * (dz ? s.fz : 1.f - s.fz);
    acc += wgt * v[c];
  }
  return acc;
}

// Features k < 15 of the box p (no volume reads).
__device__ inline float box_param_feature(int k, const float* p, const float* __restrict__ frame) {
  if (k < 3) return (p[k] - frame[6 + k]) / frame[9];
  if (k < 12) return p[k];
  return logf(fmaxf(p[k], 1e-30f) / frame[9]);
}

// Feature k of the box p (15 floats: centre, axes, half extents).
__device__ inline float box_feature(int k, const float* p, const float* __restrict__ frame,
                                    const float* __restrict__ vol, int N) {
  if (k < kFeatOcc0) return box_param_feature(k, p, frame);
  if (k >= kFeatOcc0 + kFeatOccN) return 0.f;
  const OccSample s = occ_sample_at(k - kFeatOcc0, p, frame);
  float v[8];
  for (int c = 0; c < 8; ++c) v[c] = occ_corner(vol, N, s, c);
  return occ_blend(s, v);
}

// Sum of the 512 occupancy inputs of a row in a fixed order, by one wave: lane j
// adds the inputs k = j (mod 64) in increasing k, then the lanes combine by an
// xor butterfly (32, 16, ..., 1).  Addition commutes, so every lane ends with
// the same bits; `x(k)` returns input k of the row.
template <class Get>
__device__ inline float occ_sum_wave(Get x) {
  const int lane = threadIdx.x & 63;
  float s = 0.f;
  for (int k = lane; k < kFeatIn; k += 64)
    if (k >= kFeatOcc0 && k < kFeatOcc0 + kFeatOccN) s += x(k);
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  return s;
}

}  // namespace obbv
