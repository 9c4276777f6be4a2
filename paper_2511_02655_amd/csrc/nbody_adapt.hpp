// Pre-pass of the adaptive-separation FP32 mode (single systems on symmetric tiles).
//
// Float separations of near pairs carry the rounding of the coordinates themselves,
// u |x| / |d| relative, which no accumulation scheme removes. Double-float separations
// (x = hi + lo) remove it at about 1.4x the cost of a float pair. Only near pairs need
// them, so this mode orders the particles along a Morton (Z-order) curve, which makes
// every 64-particle sub-block spatially compact, and the symmetric force tile takes the
// double-float form only for the (wave, sub-block) iterations whose bounding boxes lie
// within a threshold T of each other. Every other pair has |d| >= T and a float
// separation error below u (|x_i| + |x_j|) <= 2 u X_max, so its relative error is at most
// 2 u X_max / T (X_max: the largest coordinate magnitude of the system); T = X_max / 256
// keeps that below 3.1e-5 per far pair.
//
// Steps (all on the device, no host synchronisation):
//   adapt_bbox_partial / adapt_bbox_final  bounding box of the positions, T^2;
//   adapt_keys                             64-bit keys (Morton code << 32 | index): unique,
//                                          so the sorted order is unique (deterministic);
//   bitonic_local / bitonic_global /       ascending bitonic sort of the keys, padded to a
//   bitonic_merge_local                    power of two with all-ones keys;
//   adapt_stage                            the j-array in sorted order (float hi and the
//                                          low words, as in the double-float mode), the
//                                          permutation and one bounding box per sub-block.
// The per-particle reduction then reads slot planes in sorted order and writes every output
// at the particle's own index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbody {

constexpr int kAdaptBS = 256;          // block size of the pre-pass kernels
constexpr int kBitonicBS = 1024;       // threads of a bitonic block
constexpr int kBitonicLocal = 2 * kBitonicBS;  // keys sorted in LDS by one block
constexpr int kSub = 64;               // particles per sub-block (one wave's lanes)

// Spread the low 10 bits of v to every third bit (bit k -> bit 3k).
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Per-block min and max of the three coordinates (the bounding box), written as
// part[block][6] = (min x, min y, min z, max x, max y, max z).
__global__ __launch_bounds__(kAdaptBS) void adapt_bbox_partial(int64_t n, const double* __restrict__ pos,
                                                               double* __restrict__ part) {
  __shared__ double sh[6][kAdaptBS];
  const double inf = __builtin_inf();
  double v[6] = {inf, inf, inf, -inf, -inf, -inf};
  for (int64_t i = (int64_t)blockIdx.x * kAdaptBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kAdaptBS)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double x = pos[c * n + i];
      v[c] = fmin(v[c], x);
      v[3 + c] = fmax(v[3 + c], x);
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int s = kAdaptBS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + s]);
        sh[3 + c][threadIdx.x] = fmax(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// The bounding box from `blocks` partials (min and max are exact, so any order gives the
// same box), and the threshold: bbox[0..5] = box, bbox[6] = T^2 (as a double) with
// T = X_max / 256, X_max = the largest coordinate magnitude, in staged units (coordinates
// times xs). One block of kAdaptBS threads.
__global__ __launch_bounds__(kAdaptBS) void adapt_bbox_final(int32_t blocks, const double* __restrict__ part,
                                                             double xs, double* __restrict__ bbox) {
  __shared__ double sh[6][kAdaptBS];
  const double inf = __builtin_inf();
  double v[6] = {inf, inf, inf, -inf, -inf, -inf};
  for (int b = threadIdx.x; b < blocks; b += kAdaptBS)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = fmin(v[c], part[b * 6 + c]);
      v[3 + c] = fmax(v[3 + c], part[b * 6 + 3 + c]);
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int s = kAdaptBS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + s]);
        sh[3 + c][threadIdx.x] = fmax(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double xmax = 0.0;
    for (int c = 0; c < 6; ++c) {
      bbox[c] = sh[c][0];
      xmax = fmax(xmax, fabs(sh[c][0]));
    }
    const double t = xmax * xs * (1.0 / 256.0);
    bbox[6] = t * t;
  }
}

// Key of particle i: its Morton code on a 1024^3 grid over the bounding box, shifted left by
// 32, with the index i in the low 32 bits. Slots i in [n, padded) hold all-ones keys.
__global__ __launch_bounds__(kAdaptBS) void adapt_keys(int64_t n, int64_t padded, const double* __restrict__ pos,
                                                       const double* __restrict__ bbox, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kAdaptBS + threadIdx.x;
  if (i >= padded) return;
  if (i >= n) {
    keys[i] = ~0ull;
    return;
  }
  uint32_t code = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double lo = bbox[c], ext = bbox[3 + c] - lo;
    double q = ext > 0.0 ? (pos[c * n + i] - lo) / ext * 1024.0 : 0.0;
    q = fmin(fmax(q, 0.0), 1023.0);
    code |= spread3((uint32_t)q) << c;
  }
  keys[i] = ((uint64_t)code << 32) | (uint64_t)(uint32_t)i;
}

// One compare-exchange of a bitonic network: elements i and i ^ j (i the lower), ascending
// when (i & k) == 0.
__device__ __forceinline__ void bitonic_cx(uint64_t& a, uint64_t& b, bool up) {
  const bool swap = up ? (a > b) : (a < b);
  const uint64_t t = swap ? b : a;
  b = swap ? a : b;
  a = t;
}

// Stages k = 2 .. kBitonicLocal of the network inside each block's chunk of kBitonicLocal
// keys (the direction of stage k depends on the global index, as in the full network).
__global__ __launch_bounds__(kBitonicBS) void bitonic_local(uint64_t* __restrict__ keys) {
  __shared__ uint64_t sh[kBitonicLocal];
  const int64_t base = (int64_t)blockIdx.x * kBitonicLocal;
  const int t = threadIdx.x;
  sh[t] = keys[base + t];
  sh[t + kBitonicBS] = keys[base + t + kBitonicBS];
  __syncthreads();
  for (int k = 2; k <= kBitonicLocal; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int lo = 2 * t - (t & (j - 1));  // t-th lower element of the pairs at distance j
      const bool up = ((base + lo) & k) == 0;
      bitonic_cx(sh[lo], sh[lo + j], up);
      __syncthreads();
    }
  keys[base + t] = sh[t];
  keys[base + t + kBitonicBS] = sh[t + kBitonicBS];
}

// One step (k, j) of the network with j >= kBitonicLocal, on the whole array (padded / 2
// threads, each one compare-exchange).
__global__ __launch_bounds__(kAdaptBS) void bitonic_global(uint64_t* __restrict__ keys, int64_t padded, int64_t k,
                                                           int64_t j) {
  const int64_t t = (int64_t)blockIdx.x * kAdaptBS + threadIdx.x;
  if (t >= padded / 2) return;
  const int64_t lo = 2 * t - (t & (j - 1));
  uint64_t a = keys[lo], b = keys[lo + j];
  bitonic_cx(a, b, (lo & k) == 0);
  keys[lo] = a;
  keys[lo + j] = b;
}

// The steps j = kBitonicLocal / 2 .. 1 of stage k inside each block's chunk.
__global__ __launch_bounds__(kBitonicBS) void bitonic_merge_local(uint64_t* __restrict__ keys, int64_t k) {
  __shared__ uint64_t sh[kBitonicLocal];
  const int64_t base = (int64_t)blockIdx.x * kBitonicLocal;
  const int t = threadIdx.x;
  sh[t] = keys[base + t];
  sh[t + kBitonicBS] = keys[base + t + kBitonicBS];
  __syncthreads();
  const bool up = (base & k) == 0;  // k > kBitonicLocal: one direction for the whole chunk
  for (int j = kBitonicLocal >> 1; j > 0; j >>= 1) {
    const int lo = 2 * t - (t & (j - 1));
    bitonic_cx(sh[lo], sh[lo + j], up);
    __syncthreads();
  }
  keys[base + t] = sh[t];
  keys[base + t + kBitonicBS] = sh[t + kBitonicBS];
}

// Sorted staging: for sorted position p, particle i = the key's index; perm[p] = i; the
// float j-array entry (fl(x s), m) at jhi[p] and the low words (fl(x s - hi), 0) at jlo[p]
// (s: the staging scale), exactly as the double-float mode stages them; and per sub-block
// of kSub consecutive positions (one wave), the bounding box of its float coordinates:
// box[2 q] = (min x, min y, min z, 0), box[2 q + 1] = (max x, max y, max z, 0).
__global__ __launch_bounds__(kAdaptBS) void adapt_stage(int64_t n, const uint64_t* __restrict__ keys,
                                                        const double* __restrict__ pos,
                                                        const double* __restrict__ mass, double xs,
                                                        uint32_t* __restrict__ perm, float4* __restrict__ jhi,
                                                        float4* __restrict__ jlo, float4* __restrict__ box) {
  const int64_t p = (int64_t)blockIdx.x * kAdaptBS + threadIdx.x;
  const int64_t q = p / kSub;
  const int64_t nsub = (n + kSub - 1) / kSub;
  if (q >= nsub) return;  // whole waves past the last sub-block
  const float inf = __builtin_inff();
  float b[6] = {inf, inf, inf, -inf, -inf, -inf};
  if (p < n) {
    const uint32_t i = (uint32_t)keys[p];
    perm[p] = i;
    const double x[3] = {pos[i] * xs, pos[n + i] * xs, pos[2 * (int64_t)n + i] * xs};
    float4 h, l;
    h.x = (float)x[0]; h.y = (float)x[1]; h.z = (float)x[2]; h.w = (float)mass[i];
    l.x = (float)(x[0] - (double)h.x);
    l.y = (float)(x[1] - (double)h.y);
    l.z = (float)(x[2] - (double)h.z);
    l.w = 0.f;
    jhi[p] = h;
    jlo[p] = l;
    b[0] = b[3] = h.x;
    b[1] = b[4] = h.y;
    b[2] = b[5] = h.z;
  }
  // wave-wide min / max (a wave is exactly one sub-block)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      b[c] = fminf(b[c], __shfl_xor(b[c], off, 64));
      b[3 + c] = fmaxf(b[3 + c], __shfl_xor(b[3 + c], off, 64));
    }
  if ((threadIdx.x & 63) == 0) {
    box[2 * q] = make_float4(b[0], b[1], b[2], 0.f);
    box[2 * q + 1] = make_float4(b[3], b[4], b[5], 0.f);
  }
}

}  // namespace nbody
