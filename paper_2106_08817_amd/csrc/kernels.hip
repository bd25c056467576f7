// gfx950 kernels of the batched shooting path (one launch covers every pair
// of a plan through its tile lists).
//
// Forward step (Methods, Eq. 3 and the semi-Lagrangian section):
//   k_xpass<GRADMUL>   m_c = z D_c I formed on the fly, Gaussian pass along x
//   k_spass            Gaussian pass along y (and z in 3-D); the last pass
//                      negates (v = -G m)
//   k_advect           foot q - dt v(q), one shared set of multilinear weights
//                      gathers I and z, div v at q, I' = Ih + rho dt zh,
//                      z' = zh (1 - dt div v); cost partials at the first and
//                      last step
// Adjoint step (transpose of the above, in reverse):
//   k_adv_adj_tile     tile-owned transpose of the interpolation (gathered in
//                      LDS), foot-point cotangent and div^T
//   k_xpass<plain>, k_spass  G is symmetric, so the same passes smooth vbar
//   k_epilogue         transpose of m = z D I
//
// Data movement conventions: loads address a uniform base with an unsigned
// 32-bit offset, and are issued unconditionally from coordinates clamped into
// the image (results of out-of-range lanes are discarded), so that the
// compiler can keep many independent loads in flight.
#include "kernels.h"
#include "device_common.h"

// No implicit multiply-add contraction in this file: every fused operation is
// an explicit fmaf, so an output's arithmetic does not depend on how the
// compiler schedules a particular launch-shape variant (the tuning options are
// bit-identical).
#pragma clang fp contract(off)

namespace shoot {

// Geometry of the block tiles shared by the elementwise kernels.
template <int NDIM>
struct Blk {
  static constexpr int X = NDIM == 2 ? BLK2_X : BLK3_X;
  static constexpr int Y = NDIM == 2 ? BLK2_Y : BLK3_Y;
  static constexpr int Z = NDIM == 2 ? 1 : BLK3_Z;
  static constexpr int HS = NDIM == 2 ? BLK2_HS : BLK3_HS;
  static constexpr int NP = X * Y * Z;
  static constexpr int PPT = NP / NT;
  static_assert(NP % NT == 0, "block tile must be a multiple of the block");
  // local coordinates of the k-th voxel of thread t (x fastest)
  __device__ static void local(int t, int k, int& lx, int& ly, int& lz) {
    const int li = t + k * NT;
    lx = li % X;
    ly = (li / X) % Y;
    lz = li / (X * Y);
  }
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }
// quotient of two non-negative ints as unsigned division (no sign handling)
__device__ __forceinline__ unsigned udiv(int a, int b) { return (unsigned)a / (unsigned)b; }

// ----------------------------------------------------------------------------
// small utility kernels
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_fill_u32(unsigned* __restrict__ p, long long n, unsigned v) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    p[i] = v;
}

// Plain streaming copy of n4 16-byte groups (the achievable-bandwidth
// reference of the measurements): block b moves groups [4 NT b, 4 NT (b + 1)),
// each thread four of them NT apart, their loads in flight together.
__global__ __launch_bounds__(NT) void k_stream_copy(const vf4* __restrict__ src, vf4* __restrict__ dst,
                                                    long long n4) {
  const long long i0 = (long long)blockIdx.x * (4 * NT) + threadIdx.x;
  if (i0 + 3 * NT < n4) {
    const vf4 a = src[i0], b = src[i0 + NT], c = src[i0 + 2 * NT], d = src[i0 + 3 * NT];
    dst[i0] = a;
    dst[i0 + NT] = b;
    dst[i0 + 2 * NT] = c;
    dst[i0 + 3 * NT] = d;
  } else {
    for (long long i = i0; i < n4; i += NT) dst[i] = src[i];
  }
}

// State slot <- (S, p0) for every pair.
template <int NDIM>
__global__ __launch_bounds__(NT) void k_init(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                             float* __restrict__ st) {
  using B = Blk<NDIM>;
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  float* __restrict__ I = st + 2 * P.off;
  const float* __restrict__ S = P.S;
  const float* __restrict__ Q = P.p0;
  unsigned idx[B::PPT];
  bool inside[B::PPT];
  float sv[B::PPT], qv[B::PPT];
#pragma unroll
  for (int k = 0; k < B::PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    inside[k] = t.a + lx < nx && t.b + ly < ny && t.c + lz < nz;
    idx[k] = (unsigned)((min(t.c + lz, nz - 1) * ny + min(t.b + ly, ny - 1)) * nx + min(t.a + lx, nx - 1));
    sv[k] = gld(S, idx[k]);
    qv[k] = gld(Q, idx[k]);
  }
#pragma unroll
  for (int k = 0; k < B::PPT; ++k) {
    if (!inside[k]) continue;
    gst(I, idx[k], sv[k]);
    gst(I, N + idx[k], qv[k]);
  }
}

// Count of the non-finite values of every pair's inputs (image, target when
// given, p0) into cnt[pair], for the optional input check; cnt starts at 0.
template <int NDIM>
__global__ __launch_bounds__(NT) void k_count_nonfinite(const PairDev* __restrict__ pd,
                                                        const Tile* __restrict__ tl, unsigned* __restrict__ cnt) {
  using B = Blk<NDIM>;
  __shared__ unsigned bc;
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  if (threadIdx.x == 0) bc = 0u;
  __syncthreads();
  unsigned c = 0u;
#pragma unroll
  for (int k = 0; k < B::PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    if (t.a + lx >= nx || t.b + ly >= ny || t.c + lz >= nz) continue;
    const unsigned idx = (unsigned)(((t.c + lz) * ny + (t.b + ly)) * nx + (t.a + lx));
    // a value is finite when its magnitude compares <= FLT_MAX (false for NaN)
    c += fabsf(gld(P.S, idx)) <= 3.402823466e38f ? 0u : 1u;
    c += fabsf(gld(P.p0, idx)) <= 3.402823466e38f ? 0u : 1u;
    if (P.J) c += fabsf(gld(P.J, idx)) <= 3.402823466e38f ? 0u : 1u;
  }
  if (c) atomicAdd(&bc, c);
  __syncthreads();
  if (threadIdx.x == 0 && bc) atomicAdd(cnt + t.pair, bc);
}

// ----------------------------------------------------------------------------
// Gaussian pass along x (the contiguous axis)
// ----------------------------------------------------------------------------
//
// A tile is a run of rows of one pair. Each row is staged in LDS with r zeros
// in front and zeros behind (zero padding of G), stride L = 4 (G4 + ntap4),
// G4 = ceil(nx / 4). When nx is a multiple of four the fill moves four
// consecutive x per 16-byte access (the central difference's x neighbours by
// the row shifted one element either way); otherwise it loads one element per
// lane. A thread produces four consecutive outputs of one row; the taps run in
// blocks of four (weights zero past 2r), so each block reads one new aligned
// float4 of the row and does 16 FMAs, and the last block applies only its
// nonzero taps.
template <int NDIM, bool GRADMUL>
__global__ __launch_bounds__(NT) void k_xpass(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                              const float* __restrict__ src, float* __restrict__ dst) {
  extern __shared__ vf4 smem4[];
  float* lds = reinterpret_cast<float*>(smem4);
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz, r = P.r, ntap4 = P.ntap4;
  const unsigned N = (unsigned)P.N;
  const int G4 = (nx + 3) >> 2;
  const int L = 4 * (G4 + ntap4);
  const int row0 = t.a, nrows = t.b;
  const int plane = nrows * L;

  const float* __restrict__ I = src + (GRADMUL ? 2 : NDIM) * P.off;
  const float* __restrict__ Z = I + N;
  if ((nx & 3) == 0) {
    // fill by 16-byte accesses (rows are 16-byte aligned): an item is four
    // consecutive x of one row, XV items per thread with their loads in
    // flight together; the x neighbours of the central difference come from
    // the same row shifted by one element (clamped at the row's ends)
    constexpr int XV = 2;
    const int G = nx >> 2;
    const int ni = nrows * G;
    const bool vst = (r & 3) == 0;  // the row's first column is 16-byte aligned in LDS
    for (int i0 = threadIdx.x; i0 < ni; i0 += XV * NT) {
      vf4 m[XV][NDIM];
      int lcol[XV];
      // the wave's first item: a wave whose items all lie past the tile skips
      // the batch slot (the whole wave, so that the lane shuffles below always
      // run on full waves)
      const int wfirst = __builtin_amdgcn_readfirstlane(i0 - (int)(threadIdx.x & 63));
#pragma unroll
      for (int u = 0; u < XV; ++u) {
        if (wfirst + u * NT >= ni) {
          lcol[u] = -1;
          continue;
        }
        const int i = min(i0 + u * NT, ni - 1);
        const int rl = (int)udiv(i, G);
        const int x = 4 * (i - rl * G);
        lcol[u] = i0 + u * NT < ni ? rl * L + r + x : -1;
        const int row = row0 + rl;
        const unsigned idx = (unsigned)(row * nx + x);
        if (GRADMUL) {
          const int y = row - ny * (int)udiv(row, ny);
          const unsigned yu = (unsigned)up(y, ny, nx), yd = (unsigned)dn(y, nx);
          const vf4 zc = gld4(Z, idx);
          const vf4 ic = gld4(I, idx);
          const vf4 iu = gld4(I, idx + yu), id = gld4(I, idx - yd);
          vf4 izu = ic, izd = ic;
          if (NDIM == 3) {
            const int z = (int)udiv(row, ny);
            const unsigned zu = (unsigned)up(z, nz, ny * nx), zd = (unsigned)dn(z, ny * nx);
            izu = gld4(I, idx + zu);
            izd = gld4(I, idx - zd);
          }
          // x neighbours: the adjacent lanes hold the adjacent groups of the
          // row (items are consecutive across lanes); the wave's end lanes
          // load theirs, the row's ends clamp
          const int lane = threadIdx.x & 63;
          float left = __shfl_up(ic.w, 1, 64), right = __shfl_down(ic.x, 1, 64);
          if (lane == 0 && x > 0) left = gld(I, idx - 1u);
          if (lane == 63 && x + 4 < nx) right = gld(I, idx + 4u);
          const vf4 lm = x > 0 ? vf4{left, ic.x, ic.y, ic.z} : vf4{ic.x, ic.x, ic.y, ic.z};
          const vf4 rp = x + 4 < nx ? vf4{ic.y, ic.z, ic.w, right} : vf4{ic.y, ic.z, ic.w, ic.w};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float zq = 0.5f * zc[k];
            m[u][NDIM - 1][k] = zq * (rp[k] - lm[k]);
            m[u][NDIM - 2][k] = zq * (iu[k] - id[k]);
            if (NDIM == 3) m[u][0][k] = zq * (izu[k] - izd[k]);
          }
        } else {
#pragma unroll
          for (int c = 0; c < NDIM; ++c) m[u][c] = gld4(I, c * N + idx);
        }
      }
#pragma unroll
      for (int u = 0; u < XV; ++u) {
        if (lcol[u] < 0) continue;
#pragma unroll
        for (int c = 0; c < NDIM; ++c) {
          float* dstl = lds + c * plane + lcol[u];
          if (vst) {
            *reinterpret_cast<vf4*>(dstl) = m[u][c];
          } else {
            dstl[0] = m[u][c].x; dstl[1] = m[u][c].y; dstl[2] = m[u][c].z; dstl[3] = m[u][c].w;
          }
        }
      }
    }
    // zero padding: r columns in front of each row, the rest of the row behind
    const int pad = L - nx;
    for (int i = threadIdx.x; i < nrows * pad; i += NT) {
      const int rl = (int)udiv(i, pad);
      const int k = i - rl * pad;
      const int col = k < r ? k : nx + k;
#pragma unroll
      for (int c = 0; c < NDIM; ++c) lds[c * plane + rl * L + col] = 0.f;
    }
  } else {
  // fill: the tile is cut into segments of 64 columns of one row; wave w
  // takes segments w, w + 4, ... and issues the loads of XSEG of them at once
  // (clamped loads, zero outside the row)
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nch = (L + 63) >> 6;
  const int nseg = nrows * nch;
  for (int sb = 0; sb < nseg; sb += XSEG * (NT / 64)) {
    float m[XSEG][NDIM];
    int lcol[XSEG];
#pragma unroll
    for (int u = 0; u < XSEG; ++u) {
      const int sg = min(sb + wv + u * (NT / 64), nseg - 1);  // wave-uniform
      const int rl = (int)udiv(sg, nch);
      const int col = (sg - rl * nch) * 64 + lane;
      lcol[u] = (sb + wv + u * (NT / 64) < nseg && col < L) ? rl * L + col : -1;
      const int row = row0 + rl;
      const int x = col - r;
      const int xc = clampi(x, 0, nx - 1);
      const unsigned idx = (unsigned)(row * nx + xc);
      const bool in = x >= 0 && x < nx;
      if (GRADMUL) {
        const int y = row - ny * (int)udiv(row, ny);
        const unsigned yu = (unsigned)up(y, ny, nx), yd = (unsigned)dn(y, nx);
        const float zq = 0.5f * gld(Z, idx);
        const float gx = gld(I, idx + (xc + 1 < nx ? 1u : 0u)) - gld(I, idx - (xc > 0 ? 1u : 0u));
        const float gy = gld(I, idx + yu) - gld(I, idx - yd);
        m[u][NDIM - 1] = in ? zq * gx : 0.f;
        m[u][NDIM - 2] = in ? zq * gy : 0.f;
        if (NDIM == 3) {
          const int z = (int)udiv(row, ny);
          const unsigned zu = (unsigned)up(z, nz, ny * nx), zd = (unsigned)dn(z, ny * nx);
          m[u][0] = in ? zq * (gld(I, idx + zu) - gld(I, idx - zd)) : 0.f;
        }
      } else {
#pragma unroll
        for (int c = 0; c < NDIM; ++c) {
          const float v = gld(I, c * N + idx);
          m[u][c] = in ? v : 0.f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < XSEG; ++u) {
      if (lcol[u] >= 0) {
#pragma unroll
        for (int c = 0; c < NDIM; ++c) lds[c * plane + lcol[u]] = m[u][c];
      }
    }
  }
  }
  __syncthreads();

  const float4* W4 = reinterpret_cast<const float4*>(P.w);
  // 2r + 1 taps: nfull blocks of four, then rem taps (the rest of the padded
  // last block has zero weights, which leave a finite sum unchanged)
  const int nfull = (2 * r + 1) >> 2, rem = (2 * r + 1) & 3;
  float* __restrict__ D = dst + NDIM * P.off;
  const int ngroups = nrows * G4;
  for (int g = threadIdx.x; g < ngroups; g += NT) {
    const int rl = (int)udiv(g, G4);
    const int x = 4 * (g - rl * G4);
    const unsigned obase = (unsigned)((row0 + rl) * nx + x);
#pragma unroll
    for (int c = 0; c < NDIM; ++c) {
      // row offsets are multiples of four floats: index the LDS as vf4 so the
      // reads are aligned ds_read_b128 (consecutive lanes, consecutive 16 B)
      const vf4* R4 = smem4 + ((c * plane + rl * L + x) >> 2);
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      vf4 lo = R4[0];
      for (int b = 0; b < nfull; ++b) {
        const vf4 hi = R4[b + 1];
        const float4 w = W4[b];
        a0 = fmaf(w.x, lo.x, a0); a1 = fmaf(w.x, lo.y, a1); a2 = fmaf(w.x, lo.z, a2); a3 = fmaf(w.x, lo.w, a3);
        a0 = fmaf(w.y, lo.y, a0); a1 = fmaf(w.y, lo.z, a1); a2 = fmaf(w.y, lo.w, a2); a3 = fmaf(w.y, hi.x, a3);
        a0 = fmaf(w.z, lo.z, a0); a1 = fmaf(w.z, lo.w, a1); a2 = fmaf(w.z, hi.x, a2); a3 = fmaf(w.z, hi.y, a3);
        a0 = fmaf(w.w, lo.w, a0); a1 = fmaf(w.w, hi.x, a1); a2 = fmaf(w.w, hi.y, a2); a3 = fmaf(w.w, hi.z, a3);
        lo = hi;
      }
      if (rem > 0) {  // the last block's nonzero taps, in the same order
        const float4 w = W4[nfull];
        a0 = fmaf(w.x, lo.x, a0); a1 = fmaf(w.x, lo.y, a1); a2 = fmaf(w.x, lo.z, a2); a3 = fmaf(w.x, lo.w, a3);
        if (rem > 1) {
          const vf4 hi = R4[nfull + 1];
          a0 = fmaf(w.y, lo.y, a0); a1 = fmaf(w.y, lo.z, a1); a2 = fmaf(w.y, lo.w, a2); a3 = fmaf(w.y, hi.x, a3);
          if (rem > 2) {
            a0 = fmaf(w.z, lo.z, a0); a1 = fmaf(w.z, lo.w, a1); a2 = fmaf(w.z, hi.x, a2); a3 = fmaf(w.z, hi.y, a3);
          }
        }
      }
      float* o = D + c * N + obase;
      if ((nx & 3) == 0) {
        *reinterpret_cast<float4*>(o) = make_float4(a0, a1, a2, a3);
      } else {
        o[0] = a0;
        if (x + 1 < nx) o[1] = a1;
        if (x + 2 < nx) o[2] = a2;
        if (x + 3 < nx) o[3] = a3;
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Gaussian pass along a strided axis (y, or z in 3-D)
// ----------------------------------------------------------------------------
//
// A tile is 64 consecutive x x SEG = 4 RB outputs along the pass axis at one
// index of the third axis, for the channel blockIdx.y. The input is staged in
// LDS as (SEG + 4 ntap4) rows x 64 floats; LDS row j holds the input at
// s = s0 - r + j. The block is 16 column groups (four consecutive x, moved as
// one dwordx4 access) x 16 row groups; a thread produces RB / 4 consecutive
// outputs along the axis for its four columns, reading the LDS window as
// aligned 16-byte vectors. Every output sums its taps in blocks of four in the
// same order whatever RB is (the last block's nonzero taps only).
// MODE 0: plain pass. MODE 1: negated (v = -G m). MODE 2: negated, plus
// -2 lambda * extra (the regulariser's cotangent at t = 0).
template <int NDIM, bool PASSZ, int MODE, int RB>
__global__ __launch_bounds__(NT) void k_spass(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                              const float* __restrict__ src, float* __restrict__ dst,
                                              const float* __restrict__ extra) {
  constexpr int RQ = RB / 4;      // outputs per thread along the axis
  constexpr int SEG = 16 * RQ;    // outputs per tile along the axis
  constexpr int FU = 4;           // fill loads per thread in flight per round
  static_assert(SEG == (NT / 64) * RB, "tile geometry");
  extern __shared__ vf4 smem4[];
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz, r = P.r, ntap4 = P.ntap4;
  const unsigned N = (unsigned)P.N;
  // pass axis: length ns, stride ss; third axis index t.b with stride so
  const int ns = PASSZ ? nz : ny;
  const unsigned ss = (unsigned)(PASSZ ? ny * nx : nx);
  const unsigned so = (unsigned)(PASSZ ? nx : ny * nx);
  const int cg = threadIdx.x & 15, rg = threadIdx.x >> 4;
  const int x = t.a + 4 * cg;
  const bool xin = x < nx;
  const bool vec = (nx & 3) == 0;   // rows are 16-byte aligned: whole dwordx4 accesses
  const int s0 = t.c;
  const int rows = SEG + 4 * ntap4;
  const int c = blockIdx.y;  // one channel per block
  const unsigned base = (unsigned)t.b * so;
  const float* __restrict__ Fc = src + NDIM * P.off + c * N;

  // fill: clamped loads, FU rows per thread in flight per round; rows outside
  // the axis and columns beyond nx are zeroed when stored
  for (int j0 = rg; j0 < rows; j0 += FU * 16) {
    vf4 v[FU];
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int j = j0 + 16 * u;
      const unsigned rowi = base + (unsigned)clampi(s0 - r + j, 0, ns - 1) * ss;
      if (j < rows) {
        if (vec) {
          v[u] = gld4(Fc, rowi + (unsigned)min(x, nx - 4));
        } else {
          v[u] = vf4{gld(Fc, rowi + (unsigned)min(x, nx - 1)), gld(Fc, rowi + (unsigned)min(x + 1, nx - 1)),
                     gld(Fc, rowi + (unsigned)min(x + 2, nx - 1)), gld(Fc, rowi + (unsigned)min(x + 3, nx - 1))};
        }
      }
    }
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int j = j0 + 16 * u;
      const int s = s0 - r + j;
      if (j < rows) {
        const bool in = s >= 0 && s < ns;
        vf4 w = v[u];
        w.x = (in && x < nx) ? w.x : 0.f;
        w.y = (in && x + 1 < nx) ? w.y : 0.f;
        w.z = (in && x + 2 < nx) ? w.z : 0.f;
        w.w = (in && x + 3 < nx) ? w.w : 0.f;
        smem4[j * 16 + cg] = w;
      }
    }
  }
  __syncthreads();

  vf4 acc[RQ];
#pragma unroll
  for (int i = 0; i < RQ; ++i) acc[i] = vf4{0.f, 0.f, 0.f, 0.f};
  const float4* W4 = reinterpret_cast<const float4*>(P.w);
  const vf4* col = smem4 + (rg * RQ) * 16 + cg;
  // 2r + 1 taps: nfull blocks of four, then rem taps (the rest of the padded
  // last block has zero weights, which leave a finite sum unchanged)
  const int nfull = (2 * r + 1) >> 2, rem = (2 * r + 1) & 3;
  for (int b = 0; b < nfull; ++b) {
    const float4 w = W4[b];
    vf4 win[RQ + 3];
#pragma unroll
    for (int j = 0; j < RQ + 3; ++j) win[j] = col[(4 * b + j) * 16];
#pragma unroll
    for (int i = 0; i < RQ; ++i) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float a = acc[i][k];
        a = fmaf(w.x, win[i][k], a);
        a = fmaf(w.y, win[i + 1][k], a);
        a = fmaf(w.z, win[i + 2][k], a);
        a = fmaf(w.w, win[i + 3][k], a);
        acc[i][k] = a;
      }
    }
  }
  if (rem > 0) {
    const float4 w = W4[nfull];
    vf4 win[RQ + 2];
#pragma unroll
    for (int j = 0; j < RQ + 2; ++j) win[j] = col[(4 * nfull + j) * 16];
#pragma unroll
    for (int i = 0; i < RQ; ++i) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float a = acc[i][k];
        a = fmaf(w.x, win[i][k], a);
        if (rem > 1) a = fmaf(w.y, win[i + 1][k], a);
        if (rem > 2) a = fmaf(w.z, win[i + 2][k], a);
        acc[i][k] = a;
      }
    }
  }
  if (xin) {
    float* __restrict__ Dc = dst + NDIM * P.off + c * N;
    const float* __restrict__ Ec = (MODE == 2 && extra != nullptr) ? extra + NDIM * P.off + c * N : nullptr;
    const float escale = -2.f * P.lam;
#pragma unroll
    for (int i = 0; i < RQ; ++i) {
      const int s = s0 + rg * RQ + i;
      if (s < ns) {
        const unsigned idx = base + (unsigned)s * ss + (unsigned)x;
        vf4 o = acc[i];
        if (MODE >= 1) o = -o;
        if (vec) {
          if (MODE == 2 && Ec != nullptr) {
            const vf4 e = gld4(Ec, idx);
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = fmaf(escale, e[k], o[k]);
          }
          gst4(Dc, idx, o);
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (x + k < nx) {
              float ok = o[k];
              if (MODE == 2 && Ec != nullptr) ok = fmaf(escale, gld(Ec, idx + k), ok);
              gst(Dc, idx + k, ok);
            }
          }
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// semi-Lagrangian advection (forward step)
// ----------------------------------------------------------------------------
//
// The voxels of a thread are handled in batches of GS: all loads of a batch
// (velocity at q and its axis neighbours) are issued together, then all feet
// are formed and all corner gathers issued together, so each batch costs two
// memory round trips rather than two per voxel.

// velocity at q (channel order) and its clamped axis neighbours for div v
template <int NDIM>
__device__ __forceinline__ void load_v_div(const float* __restrict__ V, unsigned N, unsigned idx, int qx, int qy,
                                           int qz, int nx, int ny, int nz, float v[NDIM], float vn[2 * NDIM]) {
  const unsigned sxy = (unsigned)(nx * ny);
  const float* Vx = V + (NDIM - 1) * N;
  const float* Vy = V + (NDIM - 2) * N;
#pragma unroll
  for (int c = 0; c < NDIM; ++c) v[c] = gld(V, c * N + idx);
  vn[0] = gld(Vx, idx + (unsigned)up(qx, nx, 1));
  vn[1] = gld(Vx, idx - (unsigned)dn(qx, 1));
  vn[2] = gld(Vy, idx + (unsigned)up(qy, ny, nx));
  vn[3] = gld(Vy, idx - (unsigned)dn(qy, nx));
  if (NDIM == 3) {
    vn[4] = gld(V, idx + (unsigned)up(qz, nz, sxy));
    vn[5] = gld(V, idx - (unsigned)dn(qz, sxy));
  }
}

template <int NDIM>
__device__ __forceinline__ float div_of(const float vn[2 * NDIM]) {
  float d = 0.5f * (vn[0] - vn[1]);
  d = fmaf(0.5f, vn[2] - vn[3], d);
  if (NDIM == 3) d = fmaf(0.5f, vn[4] - vn[5], d);
  return d;
}

// Multilinear combination of the 2^d corner values (corner k: bit 0 = x,
// bit 1 = y, bit 2 = z) with fractions f = (fz, fy, fx).
template <int NDIM>
__device__ __forceinline__ float mlerp(const float* c, const float f[3]) {
  const float wx0 = 1.f - f[2], wx1 = f[2], wy0 = 1.f - f[1], wy1 = f[1];
  const float a = fmaf(wy1, fmaf(wx1, c[3], wx0 * c[2]), wy0 * fmaf(wx1, c[1], wx0 * c[0]));
  if (NDIM == 2) return a;
  const float b = fmaf(wy1, fmaf(wx1, c[7], wx0 * c[6]), wy0 * fmaf(wx1, c[5], wx0 * c[4]));
  return fmaf(f[0], b, (1.f - f[0]) * a);
}

// SCHEME 0: the semi-Lagrangian step. SCHEME 1: the Eulerian step (explicit
// Euler, clamped central differences: I' = I - dt sum_a v_a D_a I + rho dt z,
// z' = z - dt sum_a D_a (z v_a)). SCHEME 2: semi-Lagrangian image, Eulerian
// momentum.
template <int NDIM, int GS, int SCHEME = 0>
__global__ __launch_bounds__(NT) void k_advect(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                               const float* __restrict__ Vg, const float* __restrict__ stg,
                                               float* __restrict__ stog, AdvectArgs A) {
  using B = Blk<NDIM>;
  constexpr int NC = NDIM == 3 ? 8 : 4;
  static_assert(B::PPT % GS == 0, "batch must divide the voxels per thread");
  __shared__ float sh[NT / 64];
  const int tix = xcd_tile(gridDim.x);
  const Tile t = tl[tix];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  const unsigned sxy = (unsigned)(nx * ny);
  const float dt = P.dt, rdt = P.rho * P.dt;
  const float* __restrict__ V = Vg + NDIM * P.off;
  const float* __restrict__ I = stg + 2 * P.off;
  const float* __restrict__ Z = I + N;
  float* __restrict__ Io = stog ? stog + 2 * P.off : nullptr;
  float reg = 0.f, ssd = 0.f, dm = 0.f;
#pragma unroll
  for (int k0 = 0; k0 < B::PPT; k0 += GS) {
    int qx[GS], qy[GS], qz[GS];
    unsigned idx[GS];
    bool inside[GS];
    float v[GS][NDIM], vn[GS][2 * NDIM];
#pragma unroll
    for (int g = 0; g < GS; ++g) {
      int lx, ly, lz;
      B::local(threadIdx.x, k0 + g, lx, ly, lz);
      inside[g] = t.a + lx < nx && t.b + ly < ny && t.c + lz < nz;
      qx[g] = min(t.a + lx, nx - 1); qy[g] = min(t.b + ly, ny - 1); qz[g] = min(t.c + lz, nz - 1);
      idx[g] = (unsigned)((qz[g] * ny + qy[g]) * nx + qx[g]);
      load_v_div<NDIM>(V, N, idx[g], qx[g], qy[g], qz[g], nx, ny, nz, v[g], vn[g]);
    }
    float iv[GS][NC], zv[GS][NC], fr[GS][3], dmq[GS];
#pragma unroll
    for (int g = 0; g < GS; ++g) {
      const float dx = -dt * v[g][NDIM - 1], dy = -dt * v[g][NDIM - 2];
      const Axis ax = foot_axis(qx[g], dx, nx);
      const Axis ay = foot_axis(qy[g], dy, ny);
      dmq[g] = fmaxf(fabsf(dx), fabsf(dy));
      int zi = 0;
      fr[g][0] = 0.f;
      if (NDIM == 3) {
        const float dz = -dt * v[g][0];
        const Axis az = foot_axis(qz[g], dz, nz);
        dmq[g] = fmaxf(dmq[g], fabsf(dz));
        zi = az.i;
        fr[g][0] = az.f;
      }
      fr[g][1] = ay.f;
      fr[g][2] = ax.f;
      const unsigned c0 = (unsigned)(zi * (int)sxy + ay.i * nx + ax.i);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const unsigned gi = c0 + (unsigned)(j >> 2) * sxy + (unsigned)(((j >> 1) & 1) * nx + (j & 1));
        iv[g][j] = SCHEME == 1 ? 0.f : gld(I, gi);
        zv[g][j] = SCHEME == 1 ? 0.f : gld(Z, gi);
      }
    }
    float In[GS], zn[GS];
#pragma unroll
    for (int g = 0; g < GS; ++g) {
      const float Ih = mlerp<NDIM>(iv[g], fr[g]);
      const float zh = mlerp<NDIM>(zv[g], fr[g]);
      In[g] = fmaf(rdt, zh, Ih);
      zn[g] = zh * fmaf(-dt, div_of<NDIM>(vn[g]), 1.f);
    }
    if (SCHEME != 0) {
      // Eulerian momentum (and image for SCHEME 1) at q, axes in array order
#pragma unroll
      for (int g = 0; g < GS; ++g) {
        const unsigned i0 = idx[g];
        const int q3[3] = {qz[g], qy[g], qx[g]};
        const int n3[3] = {nz, ny, nx};
        const unsigned s3[3] = {sxy, (unsigned)nx, 1u};
        const float Iq = gld(I, i0), zq = gld(Z, i0);
        float adv = 0.f, flux = 0.f;
#pragma unroll
        for (int c = 0; c < NDIM; ++c) {
          const int a = 3 - NDIM + c;                 // array axis of channel c
          const int vi = 2 * (2 - a);                 // vn holds (+, -) per axis, x first
          const unsigned sp = (unsigned)up(q3[a], n3[a], (int)s3[a]), sm = (unsigned)dn(q3[a], (int)s3[a]);
          adv = fmaf(v[g][c], 0.5f * (gld(I, i0 + sp) - gld(I, i0 - sm)), adv);
          flux = fmaf(0.5f, gld(Z, i0 + sp) * vn[g][vi] - gld(Z, i0 - sm) * vn[g][vi + 1], flux);
        }
        if (SCHEME == 1) In[g] = fmaf(rdt, zq, fmaf(-dt, adv, Iq));
        zn[g] = fmaf(-dt, flux, zq);
      }
    }
#pragma unroll
    for (int g = 0; g < GS; ++g) {
      if (!inside[g]) continue;
      dm = fmaxf(dm, dmq[g]);
      if (Io) {
        gst(Io, idx[g], In[g]);
        gst(Io, N + idx[g], zn[g]);
      }
    }
    if (A.red_reg) {
      // -<m_0, v_0> + rho |p0|^2 at q, with m_c = z D_c I
#pragma unroll
      for (int g = 0; g < GS; ++g) {
        if (!inside[g]) continue;
        const unsigned i0 = idx[g];
        const float zq0 = gld(Z, i0);
        float gr[NDIM];
        gr[NDIM - 1] = 0.5f * (gld(I, i0 + (unsigned)up(qx[g], nx, 1)) - gld(I, i0 - (unsigned)dn(qx[g], 1)));
        gr[NDIM - 2] = 0.5f * (gld(I, i0 + (unsigned)up(qy[g], ny, nx)) - gld(I, i0 - (unsigned)dn(qy[g], nx)));
        if (NDIM == 3)
          gr[0] = 0.5f * (gld(I, i0 + (unsigned)up(qz[g], nz, sxy)) - gld(I, i0 - (unsigned)dn(qz[g], sxy)));
        float mv = 0.f;
#pragma unroll
        for (int c = 0; c < NDIM; ++c) mv = fmaf(zq0 * gr[c], v[g][c], mv);
        reg += fmaf(P.rho * zq0, zq0, -mv);
      }
    }
    if (A.last) {
#pragma unroll
      for (int g = 0; g < GS; ++g) {
        if (!inside[g]) continue;
        const unsigned i0 = idx[g];
        if (P.outI) P.outI[i0] = In[g];
        if (P.outZ) P.outZ[i0] = zn[g];
        if (P.J) {
          const float R = In[g] - P.J[i0];
          ssd = fmaf(0.5f * R, R, ssd);
          if (A.ab_out) {
            float* AB = A.ab_out + 2 * P.off;
            AB[i0] = R;
            AB[N + i0] = 0.f;
          }
        }
        if (A.sc_zero) {
          float* SC = A.sc_zero + 2 * P.off;
          SC[i0] = 0.f;
          SC[N + i0] = 0.f;
        }
      }
    }
  }
  if (A.red_reg) {
    const float s = block_sum(reg, sh);
    if (threadIdx.x == 0) A.red_reg[tix] = s;
  }
  if (A.red_ssd) {
    const float s = block_sum(ssd, sh);
    if (threadIdx.x == 0) A.red_ssd[tix] = s;
  }
  if (A.dmax) {
    const float m = block_max(dm, sh);
    if (threadIdx.x == 0) atomicMax(A.dmax + (long long)t.pair * A.T + A.t, __float_as_uint(m));
  }
}

// LDS staging of a block tile: two scalar fields on the box P +- 1 and the
// NDIM channels of a vector field, the channel of axis a with a halo of one
// cell along a only. Positions outside the image hold the clamped neighbour,
// which is exactly the clamping of the central difference. All loads of a
// thread are issued before the LDS stores.
template <int NDIM>
struct Stage {
  using B = Blk<NDIM>;
  static constexpr int X = B::X, Y = B::Y, Z = B::Z;
  static constexpr int SX = X + 2, SY = Y + 2, SZ = NDIM == 3 ? Z + 2 : 1;
  static constexpr int NS = SX * SY * SZ;
  static constexpr int NVX = SX * Y * Z, NVY = X * SY * Z, NVZ = NDIM == 3 ? X * Y * (Z + 2) : 1;
  // box index of local (lx, ly, lz) in P
  __device__ static int box(int lx, int ly, int lz) { return ((NDIM == 3 ? lz + 1 : 0) * SY + ly + 1) * SX + lx + 1; }
  __device__ static int vx(int lx, int ly, int lz) { return (lz * Y + ly) * SX + lx + 1; }   // +-1 along x
  __device__ static int vy(int lx, int ly, int lz) { return (lz * SY + ly + 1) * X + lx; }   // +-X along y
  __device__ static int vz(int lx, int ly, int lz) { return ((lz + 1) * Y + ly) * X + lx; }  // +-X*Y along z
};

template <int NDIM>
__device__ __forceinline__ void stage_tile(int x0, int y0, int z0, int nx, int ny, int nz,
                                           const float* __restrict__ F0, const float* __restrict__ F1,
                                           const float* __restrict__ Cx, const float* __restrict__ Cy,
                                           const float* __restrict__ Cz, float* s0, float* s1, float* sx, float* sy,
                                           float* sz) {
  using S = Stage<NDIM>;
  constexpr int X = S::X, Y = S::Y, SX = S::SX, SY = S::SY;
  constexpr int UI = (S::NS + NT - 1) / NT, UX = (S::NVX + NT - 1) / NT, UY = (S::NVY + NT - 1) / NT;
  constexpr int UZ = NDIM == 3 ? (S::NVZ + NT - 1) / NT : 0;
  auto gidx = [&](int bx, int by, int bz, int ox, int oy, int oz) -> unsigned {
    const int gx = clampi(x0 + ox + bx, 0, nx - 1), gy = clampi(y0 + oy + by, 0, ny - 1);
    const int gz = NDIM == 3 ? clampi(z0 + oz + bz, 0, nz - 1) : 0;
    return (unsigned)((gz * ny + gy) * nx + gx);
  };
  // a wave whose slots of a round all lie past the box skips that round (the
  // stores below skip those slots)
  const int wfirst = __builtin_amdgcn_readfirstlane((int)threadIdx.x);  // the wave's first thread
  float a[UI], b[UI], cx[UX], cy[UY], cz[UZ > 0 ? UZ : 1];
#pragma unroll
  for (int u = 0; u < UI; ++u) {
    if (wfirst + u * NT >= S::NS) {
      a[u] = b[u] = 0.f;
      continue;
    }
    const int j = min((int)threadIdx.x + u * NT, S::NS - 1);
    const unsigned g = gidx(j % SX, (j / SX) % SY, j / (SX * SY), -1, -1, -1);
    a[u] = gld(F0, g);
    b[u] = gld(F1, g);
  }
#pragma unroll
  for (int u = 0; u < UX; ++u) {
    if (wfirst + u * NT >= S::NVX) {
      cx[u] = 0.f;
      continue;
    }
    const int j = min((int)threadIdx.x + u * NT, S::NVX - 1);
    cx[u] = gld(Cx, gidx(j % SX, (j / SX) % Y, j / (SX * Y), -1, 0, 0));
  }
#pragma unroll
  for (int u = 0; u < UY; ++u) {
    if (wfirst + u * NT >= S::NVY) {
      cy[u] = 0.f;
      continue;
    }
    const int j = min((int)threadIdx.x + u * NT, S::NVY - 1);
    cy[u] = gld(Cy, gidx(j % X, (j / X) % SY, j / (X * SY), 0, -1, 0));
  }
#pragma unroll
  for (int u = 0; u < UZ; ++u) {
    if (wfirst + u * NT >= S::NVZ) {
      cz[u] = 0.f;
      continue;
    }
    const int j = min((int)threadIdx.x + u * NT, S::NVZ - 1);
    cz[u] = gld(Cz, gidx(j % X, (j / X) % Y, j / (X * Y), 0, 0, -1));
  }
#pragma unroll
  for (int u = 0; u < UI; ++u) {
    const int j = threadIdx.x + u * NT;
    if (j < S::NS) { s0[j] = a[u]; s1[j] = b[u]; }
  }
#pragma unroll
  for (int u = 0; u < UX; ++u) {
    const int j = threadIdx.x + u * NT;
    if (j < S::NVX) sx[j] = cx[u];
  }
#pragma unroll
  for (int u = 0; u < UY; ++u) {
    const int j = threadIdx.x + u * NT;
    if (j < S::NVY) sy[j] = cy[u];
  }
#pragma unroll
  for (int u = 0; u < UZ; ++u) {
    const int j = threadIdx.x + u * NT;
    if (j < S::NVZ) sz[j] = cz[u];
  }
}

// Staged-tile advection. The block stages I and z on P +- 1 and each velocity
// channel with a halo of one cell along its own axis (clamped into the image,
// which is exactly the clamping of the central difference), all with
// coalesced loads. When the block's largest displacement is below one cell,
// every foot's corners lie in P +- 1 and are read from LDS; otherwise they are
// gathered from global memory. Same arithmetic as k_advect.
template <int NDIM>
__global__ __launch_bounds__(NT) void k_advect_lds(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                                   const float* __restrict__ Vg, const float* __restrict__ stg,
                                                   float* __restrict__ stog, AdvectArgs A) {
  using B = Blk<NDIM>;
  using S = Stage<NDIM>;
  constexpr int X = B::X, Y = B::Y, PPT = B::PPT;
  constexpr int NC = NDIM == 3 ? 8 : 4;
  constexpr int SX = S::SX, SY = S::SY;
  __shared__ float sI[S::NS], sZ[S::NS], sVx[S::NVX], sVy[S::NVY], sVz[S::NVZ];
  __shared__ float sh[NT / 64];
  __shared__ float sD;
  const int tix = xcd_tile(gridDim.x);
  const Tile t = tl[tix];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  const unsigned sxy = (unsigned)(nx * ny);
  const float dt = P.dt, rdt = P.rho * P.dt;
  const float* __restrict__ V = Vg + NDIM * P.off;
  const float* __restrict__ Vx = V + (NDIM - 1) * N;
  const float* __restrict__ Vy = V + (NDIM - 2) * N;
  const float* __restrict__ I = stg + 2 * P.off;
  const float* __restrict__ Zs = I + N;
  float* __restrict__ Io = stog ? stog + 2 * P.off : nullptr;
  const int x0 = t.a, y0 = t.b, z0 = t.c;
  stage_tile<NDIM>(x0, y0, z0, nx, ny, nz, I, Zs, Vx, Vy, V, sI, sZ, sVx, sVy, sVz);
  __syncthreads();

  // velocity, divergence and displacement at the thread's voxels
  int lq[PPT][3];
  bool inside[PPT];
  float v[PPT][NDIM], div[PPT];
  float dm = 0.f;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    inside[k] = x0 + lx < nx && y0 + ly < ny && z0 + lz < nz;
    lx = min(lx, nx - 1 - x0); ly = min(ly, ny - 1 - y0); lz = min(lz, nz - 1 - z0);  // clamped into the image
    lq[k][0] = lz; lq[k][1] = ly; lq[k][2] = lx;
    const int ix = (lz * Y + ly) * SX + lx + 1, iy = (lz * SY + ly + 1) * X + lx;
    float vn[2 * NDIM];
    vn[0] = sVx[ix + 1]; vn[1] = sVx[ix - 1];
    vn[2] = sVy[iy + X]; vn[3] = sVy[iy - X];
    v[k][NDIM - 1] = sVx[ix];
    v[k][NDIM - 2] = sVy[iy];
    if (NDIM == 3) {
      const int iz = ((lz + 1) * Y + ly) * X + lx;
      vn[4] = sVz[iz + X * Y]; vn[5] = sVz[iz - X * Y];
      v[k][0] = sVz[iz];
    }
    div[k] = div_of<NDIM>(vn);
    float d = 0.f;
#pragma unroll
    for (int c = 0; c < NDIM; ++c) d = fmaxf(d, fabsf(-dt * v[k][c]));
    if (inside[k]) dm = fmaxf(dm, d);
  }
  {
    const float m = block_max(dm, sh);
    if (threadIdx.x == 0) sD = m;
    __syncthreads();
  }
  const bool staged = sD < 1.f;
  float reg = 0.f, ssd = 0.f;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int lz = lq[k][0], ly = lq[k][1], lx = lq[k][2];
    const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
    const unsigned idx = (unsigned)((qz * ny + qy) * nx + qx);
    const Axis ax = foot_axis(qx, -dt * v[k][NDIM - 1], nx);
    const Axis ay = foot_axis(qy, -dt * v[k][NDIM - 2], ny);
    Axis az;
    if (NDIM == 3) {
      az = foot_axis(qz, -dt * v[k][0], nz);
    } else {
      az.i = 0; az.f = 0.f; az.live = 0.f;
    }
    float iv[NC], zv[NC];
    if (staged) {
      const int s0 = ((NDIM == 3 ? az.i - z0 + 1 : 0) * SY + (ay.i - y0 + 1)) * SX + (ax.i - x0 + 1);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int sj = s0 + (j >> 2) * SX * SY + ((j >> 1) & 1) * SX + (j & 1);
        iv[j] = sI[sj];
        zv[j] = sZ[sj];
      }
    } else {
      const unsigned c0 = (unsigned)(az.i * (int)sxy + ay.i * nx + ax.i);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const unsigned gi = c0 + (unsigned)(j >> 2) * sxy + (unsigned)(((j >> 1) & 1) * nx + (j & 1));
        iv[j] = gld(I, gi);
        zv[j] = gld(Zs, gi);
      }
    }
    const float fr[3] = {az.f, ay.f, ax.f};
    const float Ih = mlerp<NDIM>(iv, fr);
    const float zh = mlerp<NDIM>(zv, fr);
    const float In = fmaf(rdt, zh, Ih);
    const float zn = zh * fmaf(-dt, div[k], 1.f);
    if (!inside[k]) continue;
    if (Io) {
      gst(Io, idx, In);
      gst(Io, N + idx, zn);
    }
    if (A.red_reg) {
      // -<m_0, v_0> + rho |p0|^2 at q, with m_c = z D_c I (neighbours from the staged, clamped box)
      const int sq = ((NDIM == 3 ? lz + 1 : 0) * SY + ly + 1) * SX + lx + 1;
      const float zq0 = sZ[sq];
      float gr[NDIM];
      gr[NDIM - 1] = 0.5f * (sI[sq + 1] - sI[sq - 1]);
      gr[NDIM - 2] = 0.5f * (sI[sq + SX] - sI[sq - SX]);
      if (NDIM == 3) gr[0] = 0.5f * (sI[sq + SX * SY] - sI[sq - SX * SY]);
      float mv = 0.f;
#pragma unroll
      for (int c = 0; c < NDIM; ++c) mv = fmaf(zq0 * gr[c], v[k][c], mv);
      reg += fmaf(P.rho * zq0, zq0, -mv);
    }
    if (A.last) {
      if (P.outI) P.outI[idx] = In;
      if (P.outZ) P.outZ[idx] = zn;
      if (P.J) {
        const float R = In - P.J[idx];
        ssd = fmaf(0.5f * R, R, ssd);
        if (A.ab_out) {
          float* AB = A.ab_out + 2 * P.off;
          AB[idx] = R;
          AB[N + idx] = 0.f;
        }
      }
      if (A.sc_zero) {
        float* SC = A.sc_zero + 2 * P.off;
        SC[idx] = 0.f;
        SC[N + idx] = 0.f;
      }
    }
  }
  if (A.red_reg) {
    const float s2 = block_sum(reg, sh);
    if (threadIdx.x == 0) A.red_reg[tix] = s2;
  }
  if (A.red_ssd) {
    const float s2 = block_sum(ssd, sh);
    if (threadIdx.x == 0) A.red_ssd[tix] = s2;
  }
  if (A.dmax && threadIdx.x == 0) atomicMax(A.dmax + (long long)t.pair * A.T + A.t, __float_as_uint(sD));
}

// ----------------------------------------------------------------------------
// adjoint of the advection, tile-owned, gather form
// ----------------------------------------------------------------------------
//
// For each arrival point q with cotangents (Ib, zb) of (I_{t+1}, z_{t+1}):
//   zh_bar = rho dt Ib + (1 - dt div v) zb,   div_bar = -dt zh zb,
//   Ibar_t += Interp^T(Ib),  zbar_t += Interp^T(zh_bar)
//   vbar_c = -dt (Ib dInterp(I_t)/dy_c + zh_bar dInterp(z_t)/dy_c) + D_c^T div_bar
//
// A block owns a tile P of outputs. With D = max |dt v| of this pair and step
// (recorded by the forward pass) every corner a foot touches lies within
// H = floor(D) + 1 cells of its arrival point, so only the q in P +- H reach
// P. Phase 1 visits those q and leaves one record per q in LDS (the foot's
// clamped offset per axis, Ib and zh_bar), plus div_bar on P +- 1 and the
// foot-point part of vbar of the thread's own outputs. Phase 2 forms
// Interp^T at each p of P as a gather over the (2H+1)^d candidate q around
// it with hat weights, in a fixed order and without branches: no atomics,
// deterministic, each output written once.
// For D >= HS (or when forced) the block instead scatters its own q with
// global atomics into the accumulator, which the previous adjoint step (or
// the last forward step) cleared.
// (D^T g) at index j of an axis of length n (stride s in the LDS array):
// 0.5 (g[j-1] - g[j+1]) inside, -0.5 (g[0] + g[1]) at j = 0 and
// 0.5 (g[n-2] + g[n-1]) at j = n - 1, written with selects (both neighbours
// are always inside the staged P +- 1 array).
__device__ __forceinline__ float diffT_lds(const float* g, int b, int j, int n, int s) {
  const float c = g[b];
  const float lo = j == 0 ? -c : g[b - s];
  const float hi = j == n - 1 ? -c : g[b + s];
  return 0.5f * (lo - hi);
}

// Record of one arrival point q for the gather: the foot's offset from q per
// axis after clamping, e = clamp(q + d, 0, n - 1) - q, and the cotangents
// (Ib, zh_bar). Linear interpolation gives q's corner q + o the weight
// hat(e - o) = max(0, 1 - |e - o|) along each axis; for |e| < 1 that is
// max(-e, 0), 1 - |e|, max(e, 0) at o = -1, 0, 1. 2-D keeps
// (e_x, e_y, Ib, zh_bar) in one vector; 3-D keeps (e_x, e_y, e_z, Ib) and
// zh_bar beside it.
template <int NDIM>
struct Rec {
  vf4* v;
  float* zb;  // 3-D only
  __device__ __forceinline__ void put(int r, float ex, float ey, float ez, float ib, float zhb) const {
    if (NDIM == 2) {
      v[r] = vf4{ex, ey, ib, zhb};
    } else {
      v[r] = vf4{ex, ey, ez, ib};
      zb[r] = zhb;
    }
  }
  __device__ __forceinline__ void clear(int r) const { put(r, 0.f, 0.f, 0.f, 0.f, 0.f); }
};

// weight of a record toward its corner at offset O (|e| < 1)
template <int O>
__device__ __forceinline__ float tap3(float e) {
  return O < 0 ? fmaxf(-e, 0.f) : (O == 0 ? 1.f - fabsf(e) : fmaxf(e, 0.f));
}

__device__ __forceinline__ float hat(float x) { return fmaxf(1.f - fabsf(x), 0.f); }

// The j-th point of the ring P +- W minus P (ring order: the W full planes /
// rows on each side, then the sides of the remaining ones), as local
// coordinates relative to the tile origin; RING_N<NDIM, W>() points in all.
template <int NDIM, int W>
__host__ __device__ constexpr int RING_N() {
  using B = Blk<NDIM>;
  return (B::X + 2 * W) * (B::Y + 2 * W) * (NDIM == 3 ? B::Z + 2 * W : 1) - B::NP;
}

template <int NDIM, int W>
__host__ __device__ __forceinline__ void ring_point(int j, int& lx, int& ly, int& lz) {
  using B = Blk<NDIM>;
  constexpr int QX = B::X + 2 * W, QY = B::Y + 2 * W, QZ = B::Z + 2 * W;
  constexpr int R2 = QX * QY - B::X * B::Y;  // ring of one plane
  int qzl = 0;
  if (NDIM == 3) {
    constexpr int FP = QX * QY;
    if (j < 2 * W * FP) {
      const int pl = j / FP;
      qzl = pl < W ? pl : QZ - 2 * W + pl;
      j -= pl * FP;
      ly = j / QX - W;
      lx = j % QX - W;
      lz = qzl - W;
      return;
    }
    j -= 2 * W * FP;
    qzl = W + j / R2;
    j %= R2;
  }
  constexpr int TOP = W * QX;
  int qyl, qxl;
  if (j < 2 * TOP) {
    const int rw = j / QX;
    qyl = rw < W ? rw : QY - 2 * W + rw;
    qxl = j % QX;
  } else {
    j -= 2 * TOP;
    qyl = W + j / (2 * W);
    const int c = j % (2 * W);
    qxl = c < W ? c : B::X + c;
  }
  lx = qxl - W;
  ly = qyl - W;
  lz = NDIM == 3 ? qzl - W : 0;
}

// Phase-1 work of the adjoint for a batch of G arrival points (local
// coordinates l*, record slots li; act = the point is in the image and
// within reach of P): its record, div_bar on P +- 1, the global scatter
// (fallback mode) and, for OWN points (the thread's outputs), the foot-point
// part of vbar. The loads of the whole batch are issued together in two
// rounds (fields at q, then the corners of the feet).
template <int NDIM, int G, bool OWN>
__device__ __forceinline__ void adj_batch(const int (&lx)[G], const int (&ly)[G], const int (&lz)[G],
                                          const int (&li)[G], const bool (&act)[G], const bool (&slot)[G],
                                          bool gmode, int x0, int y0, int z0, int nx, int ny, int nz, unsigned N,
                                          float dt, float rdt, const float* __restrict__ V,
                                          const float* __restrict__ I, const float* __restrict__ Z,
                                          const float* __restrict__ AB, float* __restrict__ SI,
                                          float* __restrict__ SZ, const Rec<NDIM>& rec, float* dbar,
                                          float (*vq)[NDIM]) {
  using B = Blk<NDIM>;
  constexpr int DX = B::X + 2, DY = B::Y + 2;
  constexpr int ZO = NDIM == 3 ? 1 : 0;
  constexpr int NC = NDIM == 3 ? 8 : 4;
  const unsigned sxy = (unsigned)(nx * ny);
  int qx[G], qy[G], qz[G];
  unsigned idx[G];
  float v[G][NDIM], vn[G][2 * NDIM], ib[G], zb[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    qx[g] = clampi(x0 + lx[g], 0, nx - 1);
    qy[g] = clampi(y0 + ly[g], 0, ny - 1);
    qz[g] = clampi(z0 + lz[g], 0, nz - 1);
    idx[g] = (unsigned)((qz[g] * ny + qy[g]) * nx + qx[g]);
    load_v_div<NDIM>(V, N, idx[g], qx[g], qy[g], qz[g], nx, ny, nz, v[g], vn[g]);
    ib[g] = gld(AB, idx[g]);
    zb[g] = gld(AB, N + idx[g]);
  }
  Axis ax[G], ay[G], az[G];
  float zv[G][NC], iv[G][NC];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    ax[g] = foot_axis(qx[g], -dt * v[g][NDIM - 1], nx);
    ay[g] = foot_axis(qy[g], -dt * v[g][NDIM - 2], ny);
    if (NDIM == 3) {
      az[g] = foot_axis(qz[g], -dt * v[g][0], nz);
    } else {
      az[g].i = 0; az[g].f = 0.f; az[g].live = 0.f;
    }
    const unsigned c0 = (unsigned)(az[g].i * (int)sxy + ay[g].i * nx + ax[g].i);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const unsigned gi = c0 + (unsigned)(k >> 2) * sxy + (unsigned)(((k >> 1) & 1) * nx + (k & 1));
      zv[g][k] = gld(Z, gi);
      if (OWN) iv[g][k] = gld(I, gi);
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const float fr[3] = {az[g].f, ay[g].f, ax[g].f};
    const float zh = mlerp<NDIM>(zv[g], fr);
    const float zhb = fmaf(rdt, ib[g], fmaf(-dt, div_of<NDIM>(vn[g]), 1.f) * zb[g]);
    const bool inP1 = lx[g] >= -1 && lx[g] <= B::X && ly[g] >= -1 && ly[g] <= B::Y &&
                      (NDIM == 2 || (lz[g] >= -1 && lz[g] <= B::Z));
    if (act[g] && inP1) dbar[((lz[g] + ZO) * DY + (ly[g] + 1)) * DX + (lx[g] + 1)] = -dt * zh * zb[g];
    if (gmode) {
      if (act[g])
        rec.put(li[g], (float)(ax[g].i - qx[g]) + ax[g].f, (float)(ay[g].i - qy[g]) + ay[g].f,
                NDIM == 3 ? (float)(az[g].i - qz[g]) + az[g].f : 0.f, ib[g], zhb);
      else if (slot[g])
        rec.clear(li[g]);
    } else if (OWN && act[g]) {
      const float wz[2] = {1.f - az[g].f, az[g].f}, wy[2] = {1.f - ay[g].f, ay[g].f};
      const float wx[2] = {1.f - ax[g].f, ax[g].f};
      const unsigned c0 = (unsigned)(az[g].i * (int)sxy + ay[g].i * nx + ax[g].i);
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
        const float w = (NDIM == 3 ? wz[bz] : 1.f) * wy[by] * wx[bx];
        const unsigned gi = c0 + (unsigned)bz * sxy + (unsigned)(by * nx + bx);
        unsafeAtomicAdd(SI + gi, w * ib[g]);
        unsafeAtomicAdd(SZ + gi, w * zhb);
      }
    }
    if (OWN) {
      const float wz[2] = {1.f - az[g].f, az[g].f}, wy[2] = {1.f - ay[g].f, ay[g].f};
      const float wx[2] = {1.f - ax[g].f, ax[g].f};
      float gI[3] = {0.f, 0.f, 0.f}, gZ[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
        const float wzz = NDIM == 3 ? wz[bz] : 1.f;
        const float ddz = (bz ? 1.f : -1.f) * wy[by] * wx[bx];
        const float ddy = (by ? 1.f : -1.f) * wzz * wx[bx];
        const float ddx = (bx ? 1.f : -1.f) * wzz * wy[by];
        gI[0] = fmaf(ddz, iv[g][k], gI[0]); gZ[0] = fmaf(ddz, zv[g][k], gZ[0]);
        gI[1] = fmaf(ddy, iv[g][k], gI[1]); gZ[1] = fmaf(ddy, zv[g][k], gZ[1]);
        gI[2] = fmaf(ddx, iv[g][k], gI[2]); gZ[2] = fmaf(ddx, zv[g][k], gZ[2]);
      }
      vq[g][NDIM - 1] = -dt * ax[g].live * fmaf(ib[g], gI[2], zhb * gZ[2]);
      vq[g][NDIM - 2] = -dt * ay[g].live * fmaf(ib[g], gI[1], zhb * gZ[1]);
      if (NDIM == 3) vq[g][0] = -dt * az[g].live * fmaf(ib[g], gI[0], zhb * gZ[0]);
    }
  }
}

// One gather candidate: the record at slot r, which reaches p at offset
// (oz, oy, ox) from its arrival point.
template <int NDIM>
__device__ __forceinline__ void cand_acc(const Rec<NDIM>& rec, int r, const vf4& a, float wx, float wy, float wz,
                                         float& accI, float& accZ) {
  (void)wz;
  if (NDIM == 2) {
    const float w = wx * wy;
    accI = fmaf(w, a[2], accI);
    accZ = fmaf(w, a[3], accZ);
  } else {
    const float w = wx * wy * wz;
    accI = fmaf(w, a[3], accI);
    accZ = fmaf(w, rec.zb[r], accZ);
  }
}

template <int NDIM, int OZ, int OY, int OX>
__device__ __forceinline__ void cand3(const Rec<NDIM>& rec, int rp, float& accI, float& accZ) {
  constexpr int QX = Blk<NDIM>::X + 2 * Blk<NDIM>::HS, QY = Blk<NDIM>::Y + 2 * Blk<NDIM>::HS;
  const int r = rp - (OZ * QY + OY) * QX - OX;  // q = p - o
  const vf4 a = rec.v[r];
  cand_acc<NDIM>(rec, r, a, tap3<OX>(a[0]), tap3<OY>(a[1]), NDIM == 3 ? tap3<OZ>(a[2]) : 1.f, accI, accZ);
}

// Phase 1 over the ring P +- W minus P in batches of G points per thread.
template <int NDIM, int W, int G>
__device__ __forceinline__ void adj_ring(int hq, bool gmode, int x0, int y0, int z0, int nx, int ny, int nz,
                                         unsigned N, float dt, float rdt, const float* __restrict__ V,
                                         const float* __restrict__ I, const float* __restrict__ Z,
                                         const float* __restrict__ AB, float* __restrict__ SI,
                                         float* __restrict__ SZ, const Rec<NDIM>& rec, float* dbar) {
  using B = Blk<NDIM>;
  constexpr int HS = B::HS, QX = B::X + 2 * HS, QY = B::Y + 2 * HS;
  constexpr int ZH = NDIM == 3 ? HS : 0;
  constexpr int NR = RING_N<NDIM, W>();
  constexpr int NRB = (NR + G * NT - 1) / (G * NT);
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    int lx[G], ly[G], lz[G], li[G];
    bool act[G], slot[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = threadIdx.x + (rb * G + g) * NT;
      slot[g] = j < NR;
      ring_point<NDIM, W>(slot[g] ? j : 0, lx[g], ly[g], lz[g]);
      li[g] = ((lz[g] + ZH) * QY + (ly[g] + HS)) * QX + (lx[g] + HS);
      const int qx = x0 + lx[g], qy = y0 + ly[g], qz = z0 + lz[g];
      act[g] = slot[g] && lx[g] >= -hq && lx[g] < B::X + hq && ly[g] >= -hq && ly[g] < B::Y + hq &&
               (NDIM == 2 || (lz[g] >= -hq && lz[g] < B::Z + hq)) && qx >= 0 && qx < nx && qy >= 0 &&
               qy < ny && qz >= 0 && qz < nz;
    }
    adj_batch<NDIM, G, false>(lx, ly, lz, li, act, slot, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB,
                              SI, SZ, rec, dbar, nullptr);
  }
}

template <int NDIM, int GS>
__global__ __launch_bounds__(NT) void k_adv_adj_tile(const PairDev* __restrict__ pd, const Tile* __restrict__ tla,
                                                     const float* __restrict__ Vg, const float* __restrict__ stg,
                                                     const float* __restrict__ abg, float* __restrict__ scg,
                                                     float* __restrict__ vbg, AdjArgs A) {
  using B = Blk<NDIM>;
  constexpr int PX = B::X, PY = B::Y, PZ = B::Z, HS = B::HS, PPT = B::PPT;
  // P +- 1 (div_bar) and P +- HS (arrival points that may reach P)
  constexpr int DX = PX + 2, DY = PY + 2, DZ = NDIM == 3 ? PZ + 2 : 1;
  constexpr int QX = PX + 2 * HS, QY = PY + 2 * HS;
  constexpr int NQ = ADJ_NQ<NDIM>();
  constexpr int ZO = NDIM == 3 ? 1 : 0;
  constexpr int ZH = NDIM == 3 ? HS : 0;
  constexpr int GR = NDIM == 2 ? ADJ_RING_BATCH2 : ADJ_RING_BATCH3;  // ring points per batch
  static_assert(PPT % GS == 0, "batch must divide the voxels per thread");
  __shared__ vf4 rvec[NQ];
  __shared__ float rzb[NDIM == 3 ? NQ : 1];
  __shared__ float dbar[DX * DY * DZ];
  const Rec<NDIM> rec{rvec, rzb};
  const Tile tl = tla[xcd_tile(gridDim.x)];
  const PairDev& P = pd[tl.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  const float dt = P.dt, rdt = P.rho * P.dt;
  const int x0 = tl.a, y0 = tl.b, z0 = tl.c;
  const float D = __uint_as_float(A.dmax[(long long)tl.pair * A.T + A.t]);
  const bool gmode = !A.force_global && (D < (float)HS);
  const int H = gmode ? (int)floorf(D) + 1 : 1;
  const float* __restrict__ V = Vg + NDIM * P.off;
  const float* __restrict__ I = stg + 2 * P.off;
  const float* __restrict__ Z = I + N;
  const float* __restrict__ AB = abg + 2 * P.off;
  float* __restrict__ SI = scg + 2 * P.off;
  float* __restrict__ SZ = SI + N;
  float* __restrict__ VB = vbg + NDIM * P.off;

  // phase 1a: the outputs of this thread (same mapping as phase 2)
  float vq[PPT][NDIM];
#pragma unroll
  for (int k0 = 0; k0 < PPT; k0 += GS) {
    int lx[GS], ly[GS], lz[GS], li[GS];
    bool act[GS], slot[GS];
#pragma unroll
    for (int g = 0; g < GS; ++g) {
      B::local(threadIdx.x, k0 + g, lx[g], ly[g], lz[g]);
      li[g] = ((lz[g] + ZH) * QY + (ly[g] + HS)) * QX + (lx[g] + HS);
      act[g] = x0 + lx[g] < nx && y0 + ly[g] < ny && z0 + lz[g] < nz;
      slot[g] = true;
    }
    adj_batch<NDIM, GS, true>(lx, ly, lz, li, act, slot, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB,
                              SI, SZ, rec, dbar, vq + k0);
  }
  // Materialise the foot-point parts of vbar here: otherwise the compiler
  // sinks their arithmetic past the barrier and keeps every corner value live
  // across it (far more registers than the NDIM results).
#pragma unroll
  for (int k = 0; k < PPT; ++k)
#pragma unroll
    for (int c = 0; c < NDIM; ++c) asm volatile("" : "+v"(vq[k][c]));
  // phase 1b: the ring around P (records and div_bar only); slots of points
  // outside the image or beyond P +- H hold zero cotangents
  const int hq = gmode ? H : 1;
  if (hq == HS) {
    adj_ring<NDIM, HS, GR>(hq, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB, SI, SZ, rec, dbar);
  } else {
    // H = 1 below a wider staged bound (2-D): visit the width-1 ring, then
    // clear the record slots of the outer ring
    adj_ring<NDIM, 1, 1>(hq, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB, SI, SZ, rec, dbar);
    if (gmode) {
      for (int j = threadIdx.x; j < RING_N<NDIM, HS>(); j += NT) {
        int lx, ly, lz;
        ring_point<NDIM, HS>(j, lx, ly, lz);
        const bool outer = lx < -1 || lx > PX || ly < -1 || ly > PY || (NDIM == 3 && (lz < -1 || lz > PZ));
        if (outer) rec.clear(((lz + ZH) * QY + (ly + HS)) * QX + (lx + HS));
      }
    }
  }
  __syncthreads();

  // phase 2: vbar and the gathered transpose of the interpolation, for every
  // output of the thread (outputs beyond the image are computed on clamped
  // indices and not stored)
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
    const bool inside = qx < nx && qy < ny && qz < nz;
    const unsigned idx = (unsigned)((min(qz, nz - 1) * ny + min(qy, ny - 1)) * nx + min(qx, nx - 1));
    const int b = ((lz + ZO) * DY + (ly + 1)) * DX + (lx + 1);
    float vb[NDIM];
    vb[NDIM - 1] = vq[k][NDIM - 1] + diffT_lds(dbar, b, qx, nx, 1);
    vb[NDIM - 2] = vq[k][NDIM - 2] + diffT_lds(dbar, b, qy, ny, DX);
    if (NDIM == 3) vb[0] = vq[k][0] + diffT_lds(dbar, b, qz, nz, DX * DY);
    // Interp^T at p: sum over the arrival points q = p - o, |o| <= H per axis
    float accI = 0.f, accZ = 0.f;
    if (gmode) {
      const int rp = ((lz + ZH) * QY + (ly + HS)) * QX + (lx + HS);
      if (H == 1) {
        // fixed 3^d stencil, fixed order
        if (NDIM == 3) {
          cand3<NDIM, -1, -1, -1>(rec, rp, accI, accZ); cand3<NDIM, -1, -1, 0>(rec, rp, accI, accZ);
          cand3<NDIM, -1, -1, 1>(rec, rp, accI, accZ); cand3<NDIM, -1, 0, -1>(rec, rp, accI, accZ);
          cand3<NDIM, -1, 0, 0>(rec, rp, accI, accZ);  cand3<NDIM, -1, 0, 1>(rec, rp, accI, accZ);
          cand3<NDIM, -1, 1, -1>(rec, rp, accI, accZ); cand3<NDIM, -1, 1, 0>(rec, rp, accI, accZ);
          cand3<NDIM, -1, 1, 1>(rec, rp, accI, accZ);
          cand3<NDIM, 1, -1, -1>(rec, rp, accI, accZ); cand3<NDIM, 1, -1, 0>(rec, rp, accI, accZ);
          cand3<NDIM, 1, -1, 1>(rec, rp, accI, accZ);  cand3<NDIM, 1, 0, -1>(rec, rp, accI, accZ);
          cand3<NDIM, 1, 0, 0>(rec, rp, accI, accZ);   cand3<NDIM, 1, 0, 1>(rec, rp, accI, accZ);
          cand3<NDIM, 1, 1, -1>(rec, rp, accI, accZ);  cand3<NDIM, 1, 1, 0>(rec, rp, accI, accZ);
          cand3<NDIM, 1, 1, 1>(rec, rp, accI, accZ);
        }
        cand3<NDIM, 0, -1, -1>(rec, rp, accI, accZ); cand3<NDIM, 0, -1, 0>(rec, rp, accI, accZ);
        cand3<NDIM, 0, -1, 1>(rec, rp, accI, accZ);  cand3<NDIM, 0, 0, -1>(rec, rp, accI, accZ);
        cand3<NDIM, 0, 0, 0>(rec, rp, accI, accZ);   cand3<NDIM, 0, 0, 1>(rec, rp, accI, accZ);
        cand3<NDIM, 0, 1, -1>(rec, rp, accI, accZ);  cand3<NDIM, 0, 1, 0>(rec, rp, accI, accZ);
        cand3<NDIM, 0, 1, 1>(rec, rp, accI, accZ);
      } else {
        // general bound (2-D, 1 <= D < HS): hat weights over (2H + 1)^d offsets
        const int hz = NDIM == 3 ? H : 0;
        for (int oz = -hz; oz <= hz; ++oz)
          for (int oy = -H; oy <= H; ++oy)
            for (int ox = -H; ox <= H; ++ox) {
              const int r = rp - (oz * QY + oy) * QX - ox;
              const vf4 a = rec.v[r];
              cand_acc<NDIM>(rec, r, a, hat(a[0] - (float)ox), hat(a[1] - (float)oy),
                             NDIM == 3 ? hat(a[2] - (float)oz) : 1.f, accI, accZ);
            }
      }
    }
    if (inside) {
#pragma unroll
      for (int c = 0; c < NDIM; ++c) gst(VB, c * N + idx, vb[c]);
      if (gmode) {
        gst(SI, idx, accI);
        gst(SZ, idx, accZ);
      }
    }
  }
}

// Staged-tile variant of the adjoint epilogue (below): I and z on P +- 1 and
// the channel of mbar of axis a with a halo along a, staged in LDS with
// coalesced loads; same arithmetic as k_epilogue.
template <int NDIM>
__global__ __launch_bounds__(NT) void k_epilogue_lds(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                                     const float* __restrict__ mbg, const float* __restrict__ stg,
                                                     float* __restrict__ scg, float* __restrict__ abg, EpiArgs A) {
  using B = Blk<NDIM>;
  using S = Stage<NDIM>;
  constexpr int PPT = B::PPT, SX = S::SX, SY = S::SY, X = S::X, Y = S::Y;
  __shared__ float sI[S::NS], sZ[S::NS], sMx[S::NVX], sMy[S::NVY], sMz[S::NVZ];
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  const float* __restrict__ MB = mbg + NDIM * P.off;
  const float* __restrict__ I = stg + 2 * P.off;
  const float* __restrict__ Z = I + N;
  float* __restrict__ SI = scg + 2 * P.off;
  float* __restrict__ SZ = SI + N;
  const int x0 = t.a, y0 = t.b, z0 = t.c;
  bool clear = false;
  if (!A.first) {
    const float Dn = __uint_as_float(A.dmax[(long long)t.pair * A.T + A.t - 1]);
    clear = A.force_global || !(Dn < (float)B::HS);
  }
  int lq[PPT][3];
  bool inside[PPT];
  unsigned idx[PPT];
  float si[PPT], sz[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    inside[k] = x0 + lx < nx && y0 + ly < ny && z0 + lz < nz;
    lx = min(lx, nx - 1 - x0); ly = min(ly, ny - 1 - y0); lz = min(lz, nz - 1 - z0);
    lq[k][0] = lz; lq[k][1] = ly; lq[k][2] = lx;
    idx[k] = (unsigned)(((z0 + lz) * ny + y0 + ly) * nx + x0 + lx);
    sz[k] = gld(SZ, idx[k]);
    si[k] = gld(SI, idx[k]);
  }
  stage_tile<NDIM>(x0, y0, z0, nx, ny, nz, I, Z, MB + (NDIM - 1) * N, MB + (NDIM - 2) * N, MB, sI, sZ, sMx, sMy,
                   sMz);
  __syncthreads();
  const int n[3] = {nz, ny, nx};
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int lz = lq[k][0], ly = lq[k][1], lx = lq[k][2];
    const int q[3] = {z0 + lz, y0 + ly, x0 + lx};
    const int sq = S::box(lx, ly, lz);
    const float zc = sZ[sq];
    float zbar = sz[k], Ibar = si[k];
#pragma unroll
    for (int c = 0; c < NDIM; ++c) {
      const int a = 3 - NDIM + c;  // geometric axis of channel c
      const int so = a == 2 ? 1 : (a == 1 ? SX : SX * SY);   // box stride along a
      const float* sm = a == 2 ? sMx : (a == 1 ? sMy : sMz);
      const int mi = a == 2 ? S::vx(lx, ly, lz) : (a == 1 ? S::vy(lx, ly, lz) : S::vz(lx, ly, lz));
      const int mo = a == 2 ? 1 : (a == 1 ? X : X * Y);      // stride along a in the channel's array
      const float m0 = sm[mi];
      zbar = fmaf(m0, 0.5f * (sI[sq + so] - sI[sq - so]), zbar);
      const float zmu = sZ[sq + so] * sm[mi + mo], zmd = sZ[sq - so] * sm[mi - mo], zm = zc * m0;
      const bool lo = q[a] == 0, hi = q[a] == n[a] - 1;
      Ibar += lo ? -0.5f * (zm + zmu) : (hi ? 0.5f * (zmd + zm) : 0.5f * (zmd - zmu));
    }
    if (!inside[k]) continue;
    if (A.first) {
      if (P.outG) gst(P.outG, idx[k], fmaf(2.f * P.lam * P.rho, zc, zbar));
    } else {
      float* __restrict__ ABo = abg + 2 * P.off;
      gst(ABo, idx[k], Ibar);
      gst(ABo, N + idx[k], zbar);
    }
    if (clear) {
      gst(SI, idx[k], 0.f);
      gst(SZ, idx[k], 0.f);
    }
  }
}

// Transpose of m_c = z D_c I given mbar (already -G vbar, plus the
// regulariser's term at t = 0):
//   zbar_t = scatter part + sum_c mbar_c D_c I_t
//   Ibar_t = scatter part + sum_c D_c^T (z_t mbar_c)
// At t = 0 only dH/dp0 = zbar_0 + 2 lambda rho p0 is written. The scatter
// accumulator is cleared when the next (earlier) step scatters with global
// atomics. Voxels are handled in batches whose loads are issued together.
template <int NDIM, int GS>
__global__ __launch_bounds__(NT) void k_epilogue(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                                 const float* __restrict__ mbg, const float* __restrict__ stg,
                                                 float* __restrict__ scg, float* __restrict__ abg, EpiArgs A) {
  using B = Blk<NDIM>;
  static_assert(B::PPT % GS == 0, "batch must divide the voxels per thread");
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  const int sxy = nx * ny;
  const float* __restrict__ MB = mbg + NDIM * P.off;
  const float* __restrict__ I = stg + 2 * P.off;
  const float* __restrict__ Z = I + N;
  float* __restrict__ SI = scg + 2 * P.off;
  float* __restrict__ SZ = SI + N;
  bool clear = false;
  if (!A.first) {
    const float Dn = __uint_as_float(A.dmax[(long long)t.pair * A.T + A.t - 1]);
    clear = A.force_global || !(Dn < (float)B::HS);
  }
  const int n[3] = {nz, ny, nx};
  const int s[3] = {sxy, nx, 1};
#pragma unroll
  for (int k0 = 0; k0 < B::PPT; k0 += GS) {
    int q[GS][3];
    unsigned idx[GS];
    bool inside[GS];
    float si[GS], sz[GS], zc[GS];
    float m0[GS][NDIM], ip[GS][NDIM], im[GS][NDIM], zu[GS][NDIM], zd[GS][NDIM], mu[GS][NDIM], md[GS][NDIM];
#pragma unroll
    for (int g = 0; g < GS; ++g) {
      int lx, ly, lz;
      B::local(threadIdx.x, k0 + g, lx, ly, lz);
      inside[g] = t.a + lx < nx && t.b + ly < ny && t.c + lz < nz;
      q[g][0] = min(t.c + lz, nz - 1); q[g][1] = min(t.b + ly, ny - 1); q[g][2] = min(t.a + lx, nx - 1);
      idx[g] = (unsigned)((q[g][0] * ny + q[g][1]) * nx + q[g][2]);
      sz[g] = gld(SZ, idx[g]);
      si[g] = gld(SI, idx[g]);
      zc[g] = gld(Z, idx[g]);
#pragma unroll
      for (int c = 0; c < NDIM; ++c) {
        const int a = 3 - NDIM + c;  // geometric axis of channel c
        const float* M = MB + c * N;
        const unsigned sp = (unsigned)up(q[g][a], n[a], s[a]), sm = (unsigned)dn(q[g][a], s[a]);
        m0[g][c] = gld(M, idx[g]);
        ip[g][c] = gld(I, idx[g] + sp);
        im[g][c] = gld(I, idx[g] - sm);
        zu[g][c] = gld(Z, idx[g] + sp);   // clamped neighbours
        zd[g][c] = gld(Z, idx[g] - sm);
        mu[g][c] = gld(M, idx[g] + sp);
        md[g][c] = gld(M, idx[g] - sm);
      }
    }
#pragma unroll
    for (int g = 0; g < GS; ++g) {
      float zbar = sz[g], Ibar = si[g];
#pragma unroll
      for (int c = 0; c < NDIM; ++c) {
        const int a = 3 - NDIM + c;
        zbar = fmaf(m0[g][c], 0.5f * (ip[g][c] - im[g][c]), zbar);
        // D^T (z m) at q along axis a
        const float zmu = zu[g][c] * mu[g][c], zmd = zd[g][c] * md[g][c], zm = zc[g] * m0[g][c];
        const bool lo = q[g][a] == 0, hi = q[g][a] == n[a] - 1;
        Ibar += lo ? -0.5f * (zm + zmu) : (hi ? 0.5f * (zmd + zm) : 0.5f * (zmd - zmu));
      }
      if (!inside[g]) continue;
      if (A.first) {
        if (P.outG) gst(P.outG, idx[g], fmaf(2.f * P.lam * P.rho, zc[g], zbar));
      } else {
        float* __restrict__ ABo = abg + 2 * P.off;
        gst(ABo, idx[g], Ibar);
        gst(ABo, N + idx[g], zbar);
      }
      if (clear) {
        gst(SI, idx[g], 0.f);
        gst(SZ, idx[g], 0.f);
      }
    }
  }
}

// Cost of every pair from the per-tile partials, summed in a fixed order:
// out_cost = (data + lambda reg, data, lambda reg).
__global__ __launch_bounds__(NT) void k_finalize(const PairDev* __restrict__ pd, const float* __restrict__ red_reg,
                                                 const float* __restrict__ red_ssd) {
  __shared__ float sh[NT / 64];
  const PairDev& P = pd[blockIdx.x];
  if (!P.active) return;
  float a = 0.f, b = 0.f;
  for (int i = threadIdx.x; i < P.elem_count; i += NT) {
    a += red_ssd ? red_ssd[P.elem_first + i] : 0.f;
    b += red_reg[P.elem_first + i];
  }
  const float data = block_sum(a, sh);
  const float reg = block_sum(b, sh);
  if (threadIdx.x == 0 && P.outCost) {
    const float lr = P.lam * reg;
    P.outCost[0] = data + lr;
    P.outCost[1] = data;
    P.outCost[2] = lr;
  }
}

// One step of the deformation map psi_{t+1} = psi_t o (Id - dt v_t): every
// component is re-interpolated at the step's feet with the weights that move
// I and z (psi_0 = Id: the corner values are the corners' coordinates). The
// result goes to psi_out, or at the last step to each pair's outD.
template <int NDIM>
__global__ __launch_bounds__(NT) void k_deform(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                               const float* __restrict__ Vg, const float* __restrict__ psi_in,
                                               float* __restrict__ psi_out) {
  using B = Blk<NDIM>;
  constexpr int NC = NDIM == 3 ? 8 : 4;
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  const unsigned sxy = (unsigned)(nx * ny);
  const float dt = P.dt;
  const float* __restrict__ V = Vg + NDIM * P.off;
  const float* __restrict__ Pin = psi_in ? psi_in + NDIM * P.off : nullptr;
  float* __restrict__ Pout = psi_out ? psi_out + NDIM * P.off : P.outD;
  if (!Pout) return;  // this pair wants no deformation map
#pragma unroll
  for (int k = 0; k < B::PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const bool inside = t.a + lx < nx && t.b + ly < ny && t.c + lz < nz;
    const int qx = min(t.a + lx, nx - 1), qy = min(t.b + ly, ny - 1), qz = min(t.c + lz, nz - 1);
    const unsigned idx = (unsigned)((qz * ny + qy) * nx + qx);
    Axis ax[3];
    ax[2] = foot_axis(qx, -dt * gld(V, (NDIM - 1) * N + idx), nx);
    ax[1] = foot_axis(qy, -dt * gld(V, (NDIM - 2) * N + idx), ny);
    if (NDIM == 3) {
      ax[0] = foot_axis(qz, -dt * gld(V, idx), nz);
    } else {
      ax[0].i = 0; ax[0].f = 0.f; ax[0].live = 0.f;
    }
    const unsigned c0 = (unsigned)(ax[0].i * (int)sxy + ax[1].i * nx + ax[2].i);
    const float fr[3] = {ax[0].f, ax[1].f, ax[2].f};
    float out[NDIM];
#pragma unroll
    for (int c = 0; c < NDIM; ++c) {
      const int a = 3 - NDIM + c;  // geometric axis of component c
      float cv[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const int b[3] = {j >> 2, (j >> 1) & 1, j & 1};
        if (Pin) {
          cv[j] = gld(Pin, c * N + c0 + (unsigned)b[0] * sxy + (unsigned)(b[1] * nx + b[2]));
        } else {
          cv[j] = (float)(ax[a].i + b[a]);
        }
      }
      out[c] = mlerp<NDIM>(cv, fr);
    }
    if (inside) {
#pragma unroll
      for (int c = 0; c < NDIM; ++c) gst(Pout, c * N + idx, out[c]);
    }
  }
}

// Fixed-step gradient descent on p0 (the optional update after the
// gradient): the step of a pair is halved when its cost rose since the
// previous iteration (on reset the step is eta0 and no cost precedes).
__global__ __launch_bounds__(NT) void k_descend_eta(const PairDev* __restrict__ pd, int npairs,
                                                    float* __restrict__ eta, float* __restrict__ prev, int reset,
                                                    float eta0) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= npairs || !pd[i].active) return;
  const float H = pd[i].outCost[0];
  float e = reset ? eta0 : eta[i];
  if (!reset && H > prev[i]) e *= 0.5f;
  eta[i] = e;
  prev[i] = H;
}

// p0 <- p0 - eta dH/dp0, in the caller's p0 buffer (the next evaluation copies
// it into the state afresh).
template <int NDIM>
__global__ __launch_bounds__(NT) void k_descend(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                                const float* __restrict__ eta) {
  using B = Blk<NDIM>;
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  float* __restrict__ p0 = const_cast<float*>(P.p0);
  const float* __restrict__ G = P.outG;
  const float e = eta[t.pair];
#pragma unroll
  for (int k = 0; k < B::PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const int x = t.a + lx, y = t.b + ly, z = t.c + lz;
    if (x < P.nx && y < P.ny && z < P.nz) {
      const unsigned idx = (unsigned)((z * P.ny + y) * P.nx + x);
      gst(p0, idx, fmaf(-e, gld(G, idx), gld(p0, idx)));
    }
  }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

static inline hipError_t post() { return hipGetLastError(); }

hipError_t launch_fill_u32(unsigned* p, long long n, unsigned v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long nb = (n + NT - 1) / NT;
  k_fill_u32<<<(unsigned)(nb < 4096 ? nb : 4096), NT, 0, s>>>(p, n, v);
  return post();
}

hipError_t launch_stream_copy(const void* src, void* dst, long long n4, hipStream_t s) {
  if (n4 <= 0) return hipSuccess;
  const long long nb = (n4 + 4 * NT - 1) / (4 * NT);
  if (nb > 0x7fffffffll) return hipErrorInvalidValue;
  k_stream_copy<<<(unsigned)nb, NT, 0, s>>>(reinterpret_cast<const vf4*>(src), reinterpret_cast<vf4*>(dst), n4);
  return post();
}

hipError_t launch_count_nonfinite(int ndim, const PairDev* pd, const Tile* tl, int nt, unsigned* cnt, hipStream_t s) {
  if (ndim == 2) k_count_nonfinite<2><<<nt, NT, 0, s>>>(pd, tl, cnt);
  else k_count_nonfinite<3><<<nt, NT, 0, s>>>(pd, tl, cnt);
  return post();
}

hipError_t launch_init(int ndim, const PairDev* pd, const Tile* tl, int nt, float* st, hipStream_t s) {
  if (ndim == 2) k_init<2><<<nt, NT, 0, s>>>(pd, tl, st);
  else k_init<3><<<nt, NT, 0, s>>>(pd, tl, st);
  return post();
}

hipError_t launch_xpass(int ndim, bool gradmul, const PairDev* pd, const Tile* tl, int nt, size_t lds,
                        const float* src, float* dst, hipStream_t s) {
  if (ndim == 2) {
    if (gradmul) k_xpass<2, true><<<nt, NT, lds, s>>>(pd, tl, src, dst);
    else k_xpass<2, false><<<nt, NT, lds, s>>>(pd, tl, src, dst);
  } else {
    if (gradmul) k_xpass<3, true><<<nt, NT, lds, s>>>(pd, tl, src, dst);
    else k_xpass<3, false><<<nt, NT, lds, s>>>(pd, tl, src, dst);
  }
  return post();
}

template <int NDIM, bool PASSZ, int MODE>
static void spass_rb(int rb, dim3 grid, size_t lds, const PairDev* pd, const Tile* tl, const float* src, float* dst,
                     const float* extra, hipStream_t s) {
  if (rb == 8) k_spass<NDIM, PASSZ, MODE, 8><<<grid, NT, lds, s>>>(pd, tl, src, dst, extra);
  else k_spass<NDIM, PASSZ, MODE, 16><<<grid, NT, lds, s>>>(pd, tl, src, dst, extra);
}

template <int NDIM, bool PASSZ>
static void spass_dispatch(int mode, int rb, const PairDev* pd, const Tile* tl, int nt, size_t lds, const float* src,
                           float* dst, const float* extra, hipStream_t s) {
  const dim3 grid(nt, NDIM);
  if (mode == 0) spass_rb<NDIM, PASSZ, 0>(rb, grid, lds, pd, tl, src, dst, extra, s);
  else if (mode == 1) spass_rb<NDIM, PASSZ, 1>(rb, grid, lds, pd, tl, src, dst, extra, s);
  else spass_rb<NDIM, PASSZ, 2>(rb, grid, lds, pd, tl, src, dst, extra, s);
}

hipError_t launch_spass(int ndim, bool passz, int mode, int rb, const PairDev* pd, const Tile* tl, int nt,
                        size_t lds, const float* src, float* dst, const float* extra, hipStream_t s) {
  if (rb != 8 && rb != 16) return hipErrorInvalidValue;
  if (ndim == 2) spass_dispatch<2, false>(mode, rb, pd, tl, nt, lds, src, dst, extra, s);
  else if (passz) spass_dispatch<3, true>(mode, rb, pd, tl, nt, lds, src, dst, extra, s);
  else spass_dispatch<3, false>(mode, rb, pd, tl, nt, lds, src, dst, extra, s);
  return post();
}

hipError_t launch_advect(int ndim, int opt, int nt, const AdvectArgs& a, hipStream_t s) {
  if (a.scheme == 1 || a.scheme == 2) {
    if (ndim == 2) {
      if (a.scheme == 1) k_advect<2, ADV_BATCH[0], 1><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
      else k_advect<2, ADV_BATCH[0], 2><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
    } else {
      if (a.scheme == 1) k_advect<3, ADV_BATCH[1], 1><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
      else k_advect<3, ADV_BATCH[1], 2><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
    }
    return post();
  }
  if (ndim == 2) {
    if (opt == 0) k_advect_lds<2><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
    else k_advect<2, ADV_BATCH[0]><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
  } else {
    if (opt == 0) k_advect_lds<3><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
    else k_advect<3, ADV_BATCH[1]><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
  }
  return post();
}

// 2-D only: the 3-D adjoint is k_adv_adj3 (launch_adv_adj3).
hipError_t launch_adv_adj(int ndim, int opt, int nt, const AdjArgs& a, hipStream_t s) {
  if (ndim != 2) return hipErrorInvalidValue;
  if (opt == 0) k_adv_adj_tile<2, ADJ_BATCH[0][0]><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.ab_in, a.sc, a.vb, a);
  else k_adv_adj_tile<2, ADJ_BATCH[0][1]><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.ab_in, a.sc, a.vb, a);
  return post();
}

hipError_t launch_epilogue(int ndim, int opt, int nt, const EpiArgs& a, hipStream_t s) {
  if (ndim == 2) {
    if (opt == 0) k_epilogue_lds<2><<<nt, NT, 0, s>>>(a.pd, a.tl, a.mb, a.st, a.sc, a.ab_out, a);
    else k_epilogue<2, EPI_BATCH[0]><<<nt, NT, 0, s>>>(a.pd, a.tl, a.mb, a.st, a.sc, a.ab_out, a);
  } else {
    if (opt == 0) k_epilogue_lds<3><<<nt, NT, 0, s>>>(a.pd, a.tl, a.mb, a.st, a.sc, a.ab_out, a);
    else k_epilogue<3, EPI_BATCH[1]><<<nt, NT, 0, s>>>(a.pd, a.tl, a.mb, a.st, a.sc, a.ab_out, a);
  }
  return post();
}

hipError_t launch_deform(int ndim, const PairDev* pd, const Tile* tl, int nt, const float* V, const float* psi_in,
                         float* psi_out, hipStream_t s) {
  if (ndim == 2) k_deform<2><<<nt, NT, 0, s>>>(pd, tl, V, psi_in, psi_out);
  else k_deform<3><<<nt, NT, 0, s>>>(pd, tl, V, psi_in, psi_out);
  return post();
}

hipError_t launch_descend(int ndim, int npairs, const PairDev* pd, const Tile* tl, int nt, float* eta, float* prev,
                          int reset, float eta0, hipStream_t s) {
  k_descend_eta<<<(npairs + NT - 1) / NT, NT, 0, s>>>(pd, npairs, eta, prev, reset, eta0);
  if (ndim == 2) k_descend<2><<<nt, NT, 0, s>>>(pd, tl, eta);
  else k_descend<3><<<nt, NT, 0, s>>>(pd, tl, eta);
  return post();
}

hipError_t launch_finalize(int npairs, const PairDev* pd, const float* red_reg, const float* red_ssd,
                           hipStream_t s) {
  k_finalize<<<npairs, NT, 0, s>>>(pd, red_reg, red_ssd);
  return post();
}

}  // namespace shoot
