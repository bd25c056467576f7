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

// Four consecutive floats at element i of a uniform base (one dwordx4 access).
// The aligned form needs i to be a multiple of 4 and the base 16-byte aligned;
// the unaligned form (4-byte alignment) serves shifted stencil neighbours.
typedef float vf4u __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ vf4 gld4(const float* __restrict__ base, unsigned i) {
  return *reinterpret_cast<const vf4*>(reinterpret_cast<const char*>(base) + (i << 2));
}
__device__ __forceinline__ vf4 gld4u(const float* __restrict__ base, unsigned i) {
  const vf4u v = *reinterpret_cast<const vf4u*>(reinterpret_cast<const char*>(base) + (i << 2));
  return vf4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void gst4(float* __restrict__ base, unsigned i, vf4 v) {
  *reinterpret_cast<vf4*>(reinterpret_cast<char*>(base) + (i << 2)) = v;
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
// The clamped offset e = clamp(d, -q, n - 1 - q) = clamp(q + d, 0, n - 1) - q
// is formed without rounding any absolute coordinate; the cell is
// i = min(q + floor(e), n - 2) and the fraction f = q + e - i (1 when the
// foot sits on the last grid line). live = 1 iff 0 < q + d < n - 1 (strict).
struct Axis {
  int i;       // cell index
  float f;     // fraction in [0, 1]
  float live;  // 1 where the coordinate is not clamped
};

__device__ __forceinline__ Axis foot_axis(int q, float d, int n) {
  const float qf = (float)q;
  const float lo = -qf, hi = (float)(n - 1) - qf;
  // clamp with one median-of-three; a NaN d gives 0 (the foot at the arrival
  // point), so that a foot never leaves the neighbourhood a kernel stages
  const float m = __builtin_amdgcn_fmed3f(d, lo, hi);
  const float e = m == m ? m : 0.f;
  const float kf = floorf(e);
  const int yb = q + (int)kf;
  const bool top = yb > n - 2;              // only when the foot is on the last line
  Axis a;
  a.i = top ? n - 2 : yb;
  a.f = top ? 1.f : e - kf;
  a.live = (d > lo && d < hi) ? 1.f : 0.f;
  return a;
}

}  // namespace shoot
