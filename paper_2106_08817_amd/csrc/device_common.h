// Device helpers shared by the fused and the per-pair kernels.
#pragma once

#include "shoot_internal.h"

namespace shoot {

// Native 4-float vector: LDS loads of it become one aligned ds_read_b128.
typedef float vf4 __attribute__((ext_vector_type(4)));

// Global access at element i of a uniform base: the byte offset is formed in
// 32 bits, so the access uses the scalar-base + 32-bit-offset addressing mode
// (one VALU op per address instead of a 64-bit add). Every array the kernels
// index is below 4 GiB per pair.
__device__ __forceinline__ float gld(const float* __restrict__ base, unsigned i) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (i << 2));
}
__device__ __forceinline__ void gst(float* __restrict__ base, unsigned i, float v) {
  *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (i << 2)) = v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
  return v;
}

// Deterministic block sum (fixed shuffle tree, then the NT/64 wave partials in
// order). The result is valid in thread 0.
__device__ __forceinline__ float block_sum(float v, float* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sh[w];
  }
  return s;
}

__device__ __forceinline__ float block_max(float v, float* sh) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s = fmaxf(s, sh[w]);
  }
  return s;
}

// Clamped central difference helpers: neighbour offsets along an axis of
// length n with stride s at index j.
__device__ __forceinline__ int up(int j, int n, int s) { return j + 1 < n ? s : 0; }
__device__ __forceinline__ int dn(int j, int s) { return j > 0 ? s : 0; }

// One axis of a foot point in local form: the foot is q + d with d = -dt v.
// The integer part comes from floor(d) alone, so no absolute coordinate is
// ever rounded. Clamping follows c = clamp(q + d, 0, n - 1),
// i = min(floor(c), n - 2), f = c - i; live = 1 iff 0 < q + d < n - 1.
struct Axis {
  int i;       // cell index
  float f;     // fraction in [0, 1]
  float live;  // 1 where the coordinate is not clamped
};

__device__ __forceinline__ Axis foot_axis(int q, float d, int n) {
  d = fminf(fmaxf(d, -1.0e7f), 1.0e7f);
  const float kf = floorf(d);
  const float fl = d - kf;            // in [0, 1]; may round to 1 for tiny negative d
  const int yb = q + (int)kf;
  const bool lo = yb < 0, hi = yb >= n - 1;
  const bool edge = (yb == 0 && fl == 0.f) || (yb == n - 2 && fl >= 1.f);
  Axis a;
  a.i = lo ? 0 : (hi ? n - 2 : yb);
  a.f = lo ? 0.f : (hi ? 1.f : fl);
  a.live = (lo || hi || edge) ? 0.f : 1.f;
  return a;
}

}  // namespace shoot
