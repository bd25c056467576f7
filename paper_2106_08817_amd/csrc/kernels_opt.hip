// gfx950 vector kernels of the batched L-BFGS driver: every pair's p0 is a
// vector of N_i floats, stored contiguously at offset off_i of batch-wide
// buffers; one launch covers every pair through a list of 1-D tiles.
// Dot products accumulate in double, per tile and then per pair in a fixed
// order (deterministic).
#include "opt.h"

namespace shoot {
namespace opt {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ double block_sum_d(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sh[w];
  }
  return s;
}

// element range of a tile
struct Range {
  long long base;  // batch offset of the pair
  int lo, hi;      // element range within the pair
};

__device__ __forceinline__ Range range_of(const VecPair* vp, const VecTile* vt) {
  const VecTile t = vt[blockIdx.x];
  const VecPair& P = vp[t.pair];
  Range r;
  r.base = P.off;
  r.lo = t.start;
  r.hi = min(t.start + VEC_TILE, (int)P.n);
  return r;
}

__global__ __launch_bounds__(NT) void k_load(const VecPair* __restrict__ vp, const VecTile* __restrict__ vt,
                                             float* __restrict__ dst, int which) {
  const Range r = range_of(vp, vt);
  const VecPair& P = vp[vt[blockIdx.x].pair];
  const float* __restrict__ src = which == 0 ? P.p0 : P.grad;
  for (int i = r.lo + threadIdx.x; i < r.hi; i += NT) dst[r.base + i] = src[i];
}

__global__ __launch_bounds__(NT) void k_set_p0(const VecPair* __restrict__ vp, const VecTile* __restrict__ vt,
                                               const float* __restrict__ X, const float* __restrict__ D,
                                               const double* __restrict__ t) {
  const Range r = range_of(vp, vt);
  const int pair = vt[blockIdx.x].pair;
  float* __restrict__ p0 = vp[pair].p0;
  const float tf = (float)t[pair];
  for (int i = r.lo + threadIdx.x; i < r.hi; i += NT) p0[i] = fmaf(tf, D[r.base + i], X[r.base + i]);
}

// Y = a Y + b X per pair (a == 0 ignores the old Y entirely)
__global__ __launch_bounds__(NT) void k_comb(const VecPair* __restrict__ vp, const VecTile* __restrict__ vt,
                                             float* __restrict__ Y, const float* __restrict__ X,
                                             const double* __restrict__ a, const double* __restrict__ b) {
  const Range r = range_of(vp, vt);
  const int pair = vt[blockIdx.x].pair;
  const float af = (float)a[pair], bf = (float)b[pair];
  const bool keep = af != 0.f;
  for (int i = r.lo + threadIdx.x; i < r.hi; i += NT) {
    const long long j = r.base + i;
    const float x = X ? bf * X[j] : 0.f;
    Y[j] = keep ? fmaf(af, Y[j], x) : x;
  }
}

__global__ __launch_bounds__(NT) void k_sub(const VecPair* __restrict__ vp, const VecTile* __restrict__ vt,
                                            float* __restrict__ out, const float* __restrict__ A,
                                            const float* __restrict__ B) {
  const Range r = range_of(vp, vt);
  for (int i = r.lo + threadIdx.x; i < r.hi; i += NT) out[r.base + i] = A[r.base + i] - B[r.base + i];
}

__global__ __launch_bounds__(NT) void k_dot_tiles(const VecPair* __restrict__ vp, const VecTile* __restrict__ vt,
                                                  const float* __restrict__ A, const float* __restrict__ B,
                                                  double* __restrict__ partial) {
  __shared__ double sh[NT / 64];
  const Range r = range_of(vp, vt);
  double s = 0.0;
  for (int i = r.lo + threadIdx.x; i < r.hi; i += NT) s = fma((double)A[r.base + i], (double)B[r.base + i], s);
  const double tot = block_sum_d(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(NT) void k_dot_pairs(const VecPair* __restrict__ vp, const double* __restrict__ partial,
                                                  double* __restrict__ out) {
  __shared__ double sh[NT / 64];
  const VecPair& P = vp[blockIdx.x];
  double s = 0.0;
  for (int i = threadIdx.x; i < P.tile_count; i += NT) s += partial[P.tile_first + i];
  const double tot = block_sum_d(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

__global__ __launch_bounds__(NT) void k_costs(const VecPair* __restrict__ vp, int npairs, double* __restrict__ out) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < npairs) out[i] = (double)vp[i].cost[0];
}

}  // namespace

hipError_t costs(const VecPair* vp, int npairs, double* out, hipStream_t s) {
  k_costs<<<(npairs + NT - 1) / NT, NT, 0, s>>>(vp, npairs, out);
  return hipGetLastError();
}

hipError_t load(const VecPair* vp, const VecTile* vt, int nt, float* dst, int which, hipStream_t s) {
  k_load<<<nt, NT, 0, s>>>(vp, vt, dst, which);
  return hipGetLastError();
}

hipError_t set_p0(const VecPair* vp, const VecTile* vt, int nt, const float* X, const float* D, const double* t,
                  hipStream_t s) {
  k_set_p0<<<nt, NT, 0, s>>>(vp, vt, X, D, t);
  return hipGetLastError();
}

hipError_t comb(const VecPair* vp, const VecTile* vt, int nt, float* Y, const float* X, const double* a,
                const double* b, hipStream_t s) {
  k_comb<<<nt, NT, 0, s>>>(vp, vt, Y, X, a, b);
  return hipGetLastError();
}

hipError_t sub(const VecPair* vp, const VecTile* vt, int nt, float* out, const float* A, const float* B,
               hipStream_t s) {
  k_sub<<<nt, NT, 0, s>>>(vp, vt, out, A, B);
  return hipGetLastError();
}

hipError_t dot(const VecPair* vp, const VecTile* vt, int nt, int npairs, const float* A, const float* B,
               double* partial, double* out, hipStream_t s) {
  k_dot_tiles<<<nt, NT, 0, s>>>(vp, vt, A, B, partial);
  k_dot_pairs<<<npairs, NT, 0, s>>>(vp, partial, out);
  return hipGetLastError();
}

}  // namespace opt
}  // namespace shoot
