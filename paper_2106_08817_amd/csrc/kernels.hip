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

// ----------------------------------------------------------------------------
// small utility kernels
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_fill_u32(unsigned* __restrict__ p, long long n, unsigned v) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    p[i] = v;
}

// State slot <- (S, p0) for every pair.
template <int NDIM>
__global__ __launch_bounds__(NT) void k_init(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                             float* __restrict__ st) {
  using B = Blk<NDIM>;
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const unsigned N = (unsigned)P.N;
  float* __restrict__ I = st + 2 * P.off;
  const float* __restrict__ S = P.S;
  const float* __restrict__ Q = P.p0;
#pragma unroll
  for (int k = 0; k < B::PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const int x = t.a + lx, y = t.b + ly, z = t.c + lz;
    if (x < nx && y < ny && z < nz) {
      const unsigned idx = (unsigned)((z * ny + y) * nx + x);
      gst(I, idx, gld(S, idx));
      gst(I, N + idx, gld(Q, idx));
    }
  }
}

// ----------------------------------------------------------------------------
// Gaussian pass along x (the contiguous axis)
// ----------------------------------------------------------------------------
//
// A tile is a run of rows of one pair. Each row is staged in LDS with r zeros
// in front and zeros behind (zero padding of G), stride L = 4 (G4 + ntap4),
// G4 = ceil(nx / 4). A thread produces four consecutive outputs of one row; the
// taps run in blocks of four (weights zero past 2r), so each block reads one
// new aligned float4 of the row and does 16 FMAs.
template <int NDIM, bool GRADMUL>
__global__ __launch_bounds__(NT) void k_xpass(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                              const float* __restrict__ src, float* __restrict__ dst) {
  extern __shared__ vf4 smem4[];
  float* lds = reinterpret_cast<float*>(smem4);
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz, r = P.r, ntap4 = P.ntap4;
  const unsigned N = (unsigned)P.N;
  const int G4 = (nx + 3) >> 2;
  const int L = 4 * (G4 + ntap4);
  const int row0 = t.a, nrows = t.b;
  const int plane = nrows * L;

  // fill: one wave per row, lanes along the row, four columns per lane in
  // flight (clamped loads, zero outside the row)
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  if (GRADMUL) {
    const float* __restrict__ I = src + 2 * P.off;
    const float* __restrict__ Z = I + N;
    for (int rl = wv; rl < nrows; rl += NT / 64) {
      const int row = row0 + rl;
      const int y = row % ny;
      const unsigned rbase = (unsigned)(row * nx);
      const unsigned yu = (unsigned)up(y, ny, nx), yd = (unsigned)dn(y, nx);
      unsigned zu = 0, zd = 0;
      if (NDIM == 3) {
        const int z = row / ny;
        zu = (unsigned)up(z, nz, ny * nx);
        zd = (unsigned)dn(z, ny * nx);
      }
      float* Lrow = lds + rl * L;
      for (int c0 = 0; c0 < L; c0 += 4 * 64) {
        float m[4][NDIM];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int x = c0 + u * 64 + lane - r;
          const int xc = clampi(x, 0, nx - 1);
          const unsigned idx = rbase + (unsigned)xc;
          const float zq = 0.5f * gld(Z, idx);
          const float gx = gld(I, idx + (xc + 1 < nx ? 1u : 0u)) - gld(I, idx - (xc > 0 ? 1u : 0u));
          const float gy = gld(I, idx + yu) - gld(I, idx - yd);
          const bool in = x >= 0 && x < nx;
          m[u][NDIM - 1] = in ? zq * gx : 0.f;
          m[u][NDIM - 2] = in ? zq * gy : 0.f;
          if (NDIM == 3) m[u][0] = in ? zq * (gld(I, idx + zu) - gld(I, idx - zd)) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int col = c0 + u * 64 + lane;
          if (col < L) {
#pragma unroll
            for (int c = 0; c < NDIM; ++c) Lrow[c * plane + col] = m[u][c];
          }
        }
      }
    }
  } else {
    const float* __restrict__ F = src + NDIM * P.off;
    for (int rl = wv; rl < nrows; rl += NT / 64) {
      const unsigned rbase = (unsigned)((row0 + rl) * nx);
      float* Lrow = lds + rl * L;
      for (int c0 = 0; c0 < L; c0 += 4 * 64) {
        float m[4][NDIM];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int x = c0 + u * 64 + lane - r;
          const unsigned idx = rbase + (unsigned)clampi(x, 0, nx - 1);
          const bool in = x >= 0 && x < nx;
#pragma unroll
          for (int c = 0; c < NDIM; ++c) {
            const float v = gld(F, c * N + idx);
            m[u][c] = in ? v : 0.f;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int col = c0 + u * 64 + lane;
          if (col < L) {
#pragma unroll
            for (int c = 0; c < NDIM; ++c) Lrow[c * plane + col] = m[u][c];
          }
        }
      }
    }
  }
  __syncthreads();

  const float4* W4 = reinterpret_cast<const float4*>(P.w);
  float* __restrict__ D = dst + NDIM * P.off;
  const int ngroups = nrows * G4;
  for (int g = threadIdx.x; g < ngroups; g += NT) {
    const int rl = g / G4;
    const int x = 4 * (g - rl * G4);
    const unsigned obase = (unsigned)((row0 + rl) * nx + x);
#pragma unroll
    for (int c = 0; c < NDIM; ++c) {
      // row offsets are multiples of four floats: index the LDS as vf4 so the
      // reads are aligned ds_read_b128 (consecutive lanes, consecutive 16 B)
      const vf4* R4 = smem4 + ((c * plane + rl * L + x) >> 2);
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      vf4 lo = R4[0];
      for (int b = 0; b < ntap4; ++b) {
        const vf4 hi = R4[b + 1];
        const float4 w = W4[b];
        a0 = fmaf(w.x, lo.x, a0); a1 = fmaf(w.x, lo.y, a1); a2 = fmaf(w.x, lo.z, a2); a3 = fmaf(w.x, lo.w, a3);
        a0 = fmaf(w.y, lo.y, a0); a1 = fmaf(w.y, lo.z, a1); a2 = fmaf(w.y, lo.w, a2); a3 = fmaf(w.y, hi.x, a3);
        a0 = fmaf(w.z, lo.z, a0); a1 = fmaf(w.z, lo.w, a1); a2 = fmaf(w.z, hi.x, a2); a3 = fmaf(w.z, hi.y, a3);
        a0 = fmaf(w.w, lo.w, a0); a1 = fmaf(w.w, hi.x, a1); a2 = fmaf(w.w, hi.y, a2); a3 = fmaf(w.w, hi.z, a3);
        lo = hi;
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
// A tile is 64 consecutive x (one per lane) x SSEG outputs along the pass axis
// at one index of the third axis, for the channel blockIdx.y. The input is
// staged in LDS as (SSEG + 4 ntap4) rows x 64 floats; LDS row j holds the
// input at s = s0 - r + j. Each thread produces SRB consecutive outputs.
// MODE 0: plain pass. MODE 1: negated (v = -G m). MODE 2: negated, plus
// -2 lambda * extra (the regulariser's cotangent at t = 0).
template <int NDIM, bool PASSZ, int MODE>
__global__ __launch_bounds__(NT) void k_spass(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                              const float* __restrict__ src, float* __restrict__ dst,
                                              const float* __restrict__ extra) {
  extern __shared__ vf4 smem4[];
  float* lds = reinterpret_cast<float*>(smem4);
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz, r = P.r, ntap4 = P.ntap4;
  const unsigned N = (unsigned)P.N;
  // pass axis: length ns, stride ss; third axis index t.b with stride so
  const int ns = PASSZ ? nz : ny;
  const unsigned ss = (unsigned)(PASSZ ? ny * nx : nx);
  const unsigned so = (unsigned)(PASSZ ? nx : ny * nx);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int x = t.a + lane;
  const bool xin = x < nx;
  const int s0 = t.c;
  const int rows = SSEG + 4 * ntap4;
  const int c = blockIdx.y;  // one channel per block
  const unsigned base = (unsigned)t.b * so + (unsigned)min(x, nx - 1);
  const float* __restrict__ Fc = src + NDIM * P.off + c * N;

  // fill: clamped loads, eight rows per thread in flight
  for (int j0 = wv; j0 < rows; j0 += 8 * (NT / 64)) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int s = s0 - r + j0 + u * (NT / 64);
      const float f = gld(Fc, base + (unsigned)clampi(s, 0, ns - 1) * ss);
      v[u] = (xin && s >= 0 && s < ns) ? f : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * (NT / 64);
      if (j < rows) lds[j * 64 + lane] = v[u];
    }
  }
  __syncthreads();

  float acc[SRB];
#pragma unroll
  for (int i = 0; i < SRB; ++i) acc[i] = 0.f;
  const float4* W4 = reinterpret_cast<const float4*>(P.w);
  const float* col = lds + (wv * SRB) * 64 + lane;
  for (int b = 0; b < ntap4; ++b) {
    const float4 w = W4[b];
    float win[SRB + 3];
#pragma unroll
    for (int j = 0; j < SRB + 3; ++j) win[j] = col[(4 * b + j) * 64];
#pragma unroll
    for (int i = 0; i < SRB; ++i) {
      acc[i] = fmaf(w.x, win[i], acc[i]);
      acc[i] = fmaf(w.y, win[i + 1], acc[i]);
      acc[i] = fmaf(w.z, win[i + 2], acc[i]);
      acc[i] = fmaf(w.w, win[i + 3], acc[i]);
    }
  }
  if (xin) {
    float* __restrict__ Dc = dst + NDIM * P.off + c * N;
    const float* __restrict__ Ec = (MODE == 2 && extra != nullptr) ? extra + NDIM * P.off + c * N : nullptr;
    const float escale = -2.f * P.lam;
#pragma unroll
    for (int i = 0; i < SRB; ++i) {
      const int s = s0 + wv * SRB + i;
      if (s < ns) {
        const unsigned idx = base + (unsigned)s * ss;
        float o = acc[i];
        if (MODE >= 1) o = -o;
        if (MODE == 2 && Ec != nullptr) o = fmaf(escale, gld(Ec, idx), o);
        gst(Dc, idx, o);
      }
    }
  }
}

// ----------------------------------------------------------------------------
// semi-Lagrangian advection (forward step)
// ----------------------------------------------------------------------------

template <int NDIM>
__global__ __launch_bounds__(NT) void k_advect(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                               const float* __restrict__ Vg, const float* __restrict__ stg,
                                               float* __restrict__ stog, AdvectArgs A) {
  using B = Blk<NDIM>;
  __shared__ float sh[NT / 64];
  const int tix = xcd_tile(gridDim.x);
  const Tile t = tl[tix];
  const PairDev& P = pd[t.pair];
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
  for (int k = 0; k < B::PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const bool inside = t.a + lx < nx && t.b + ly < ny && t.c + lz < nz;
    const int xq = min(t.a + lx, nx - 1), yq = min(t.b + ly, ny - 1), zq = min(t.c + lz, nz - 1);
    const unsigned idx = (unsigned)((zq * ny + yq) * nx + xq);
    float v[NDIM];
#pragma unroll
    for (int c = 0; c < NDIM; ++c) v[c] = gld(V, c * N + idx);
    // div v at q (clamped central differences)
    const float* Vx = V + (NDIM - 1) * N;
    const float* Vy = V + (NDIM - 2) * N;
    float div = 0.5f * (gld(Vx, idx + (unsigned)up(xq, nx, 1)) - gld(Vx, idx - (unsigned)dn(xq, 1)));
    div += 0.5f * (gld(Vy, idx + (unsigned)up(yq, ny, nx)) - gld(Vy, idx - (unsigned)dn(yq, nx)));
    if (NDIM == 3) div += 0.5f * (gld(V, idx + (unsigned)up(zq, nz, sxy)) - gld(V, idx - (unsigned)dn(zq, sxy)));
    const float dx = -dt * v[NDIM - 1], dy = -dt * v[NDIM - 2];
    const Axis ax = foot_axis(xq, dx, nx);
    const Axis ay = foot_axis(yq, dy, ny);
    float dmq = fmaxf(fabsf(dx), fabsf(dy));
    float Ih, zh;
    if (NDIM == 2) {
      const unsigned c00 = (unsigned)(ay.i * nx + ax.i);
      const float wy0 = 1.f - ay.f, wy1 = ay.f, wx0 = 1.f - ax.f, wx1 = ax.f;
      const unsigned c10 = c00 + (unsigned)nx;
      Ih = wy0 * (wx0 * gld(I, c00) + wx1 * gld(I, c00 + 1)) + wy1 * (wx0 * gld(I, c10) + wx1 * gld(I, c10 + 1));
      zh = wy0 * (wx0 * gld(Z, c00) + wx1 * gld(Z, c00 + 1)) + wy1 * (wx0 * gld(Z, c10) + wx1 * gld(Z, c10 + 1));
    } else {
      const float dz = -dt * v[0];
      dmq = fmaxf(dmq, fabsf(dz));
      const Axis az = foot_axis(zq, dz, nz);
      const unsigned c000 = (unsigned)(az.i * (int)sxy + ay.i * nx + ax.i);
      const float wz0 = 1.f - az.f, wz1 = az.f, wy0 = 1.f - ay.f, wy1 = ay.f, wx0 = 1.f - ax.f, wx1 = ax.f;
      const unsigned c010 = c000 + nx, c100 = c000 + sxy, c110 = c100 + nx;
      Ih = wz0 * (wy0 * (wx0 * gld(I, c000) + wx1 * gld(I, c000 + 1)) + wy1 * (wx0 * gld(I, c010) + wx1 * gld(I, c010 + 1))) +
           wz1 * (wy0 * (wx0 * gld(I, c100) + wx1 * gld(I, c100 + 1)) + wy1 * (wx0 * gld(I, c110) + wx1 * gld(I, c110 + 1)));
      zh = wz0 * (wy0 * (wx0 * gld(Z, c000) + wx1 * gld(Z, c000 + 1)) + wy1 * (wx0 * gld(Z, c010) + wx1 * gld(Z, c010 + 1))) +
           wz1 * (wy0 * (wx0 * gld(Z, c100) + wx1 * gld(Z, c100 + 1)) + wy1 * (wx0 * gld(Z, c110) + wx1 * gld(Z, c110 + 1)));
    }
    const float In = fmaf(rdt, zh, Ih);
    const float zn = zh * (1.f - dt * div);
    if (!inside) continue;
    dm = fmaxf(dm, dmq);
    if (Io) {
      gst(Io, idx, In);
      gst(Io, N + idx, zn);
    }
    if (A.red_reg) {
      // -<m_0, v_0> + rho |p0|^2 at q, with m_c = z D_c I
      const float zq0 = gld(Z, idx);
      float g[NDIM];
      g[NDIM - 1] = 0.5f * (gld(I, idx + (unsigned)up(xq, nx, 1)) - gld(I, idx - (unsigned)dn(xq, 1)));
      g[NDIM - 2] = 0.5f * (gld(I, idx + (unsigned)up(yq, ny, nx)) - gld(I, idx - (unsigned)dn(yq, nx)));
      if (NDIM == 3) g[0] = 0.5f * (gld(I, idx + (unsigned)up(zq, nz, sxy)) - gld(I, idx - (unsigned)dn(zq, sxy)));
      float mv = 0.f;
#pragma unroll
      for (int c = 0; c < NDIM; ++c) mv = fmaf(zq0 * g[c], v[c], mv);
      reg += P.rho * zq0 * zq0 - mv;
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
__device__ __forceinline__ float diffT_lds(const float* g, int b, int j, int n, int s) {
  if (j == 0) return -0.5f * (g[b] + g[b + s]);
  if (j == n - 1) return 0.5f * (g[b - s] + g[b]);
  return 0.5f * (g[b - s] - g[b + s]);
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

// Phase-1 work for one arrival point (local coordinates l* relative to P,
// record slot li): its record, div_bar (on P +- 1), the global scatter
// (fallback mode) and, for q in P, the foot-point part of vbar (into vq).
template <int NDIM>
__device__ __forceinline__ void adj_point(int lx, int ly, int lz, int li, bool inP, bool gmode, int x0, int y0,
                                          int z0, int nx, int ny, int nz, unsigned N, float dt, float rdt,
                                          const float* __restrict__ V, const float* __restrict__ I,
                                          const float* __restrict__ Z, const float* __restrict__ AB,
                                          float* __restrict__ SI, float* __restrict__ SZ, const Rec<NDIM>& rec,
                                          float* dbar, float vq[NDIM]) {
  using B = Blk<NDIM>;
  constexpr int DX = B::X + 2, DY = B::Y + 2;
  constexpr int ZO = NDIM == 3 ? 1 : 0;
  constexpr int NC = NDIM == 3 ? 8 : 4;
  const unsigned sxy = (unsigned)(nx * ny);
  const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
  const bool inP1 = lx >= -1 && lx <= B::X && ly >= -1 && ly <= B::Y && (NDIM == 2 || (lz >= -1 && lz <= B::Z));
  const unsigned idx = (unsigned)((qz * ny + qy) * nx + qx);
  const float* Vx = V + (NDIM - 1) * N;
  const float* Vy = V + (NDIM - 2) * N;
  float div = 0.5f * (gld(Vx, idx + (unsigned)up(qx, nx, 1)) - gld(Vx, idx - (unsigned)dn(qx, 1)));
  div += 0.5f * (gld(Vy, idx + (unsigned)up(qy, ny, nx)) - gld(Vy, idx - (unsigned)dn(qy, nx)));
  if (NDIM == 3) div += 0.5f * (gld(V, idx + (unsigned)up(qz, nz, sxy)) - gld(V, idx - (unsigned)dn(qz, sxy)));
  const float Ib = gld(AB, idx);
  const float zb = gld(AB, N + idx);
  const Axis ax = foot_axis(qx, -dt * gld(Vx, idx), nx);
  const Axis ay = foot_axis(qy, -dt * gld(Vy, idx), ny);
  Axis az;
  if (NDIM == 3) {
    az = foot_axis(qz, -dt * gld(V, idx), nz);
  } else {
    az.i = 0; az.f = 0.f; az.live = 0.f;
  }
  const float wz[2] = {1.f - az.f, az.f}, wy[2] = {1.f - ay.f, ay.f}, wx[2] = {1.f - ax.f, ax.f};
  const unsigned c0 = (unsigned)(az.i * (int)sxy + ay.i * nx + ax.i);
  float zv[NC], iv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
    const unsigned g = c0 + (unsigned)bz * sxy + (unsigned)(by * nx + bx);
    zv[k] = gld(Z, g);
    if (inP) iv[k] = gld(I, g);
  }
  float zh = 0.f;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
    zh = fmaf((NDIM == 3 ? wz[bz] : 1.f) * wy[by] * wx[bx], zv[k], zh);
  }
  const float zhb = fmaf(rdt, Ib, (1.f - dt * div) * zb);
  if (inP1) dbar[((lz + ZO) * DY + (ly + 1)) * DX + (lx + 1)] = -dt * zh * zb;
  if (gmode) {
    rec.put(li, (float)(ax.i - qx) + ax.f, (float)(ay.i - qy) + ay.f, NDIM == 3 ? (float)(az.i - qz) + az.f : 0.f,
            Ib, zhb);
  } else if (inP) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
      const float w = (NDIM == 3 ? wz[bz] : 1.f) * wy[by] * wx[bx];
      const unsigned g = c0 + (unsigned)bz * sxy + (unsigned)(by * nx + bx);
      unsafeAtomicAdd(SI + g, w * Ib);
      unsafeAtomicAdd(SZ + g, w * zhb);
    }
  }
  if (inP) {
    float gI[3] = {0.f, 0.f, 0.f}, gZ[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
      const float wzz = NDIM == 3 ? wz[bz] : 1.f;
      const float ddz = (bz ? 1.f : -1.f) * wy[by] * wx[bx];
      const float ddy = (by ? 1.f : -1.f) * wzz * wx[bx];
      const float ddx = (bx ? 1.f : -1.f) * wzz * wy[by];
      gI[0] = fmaf(ddz, iv[k], gI[0]); gZ[0] = fmaf(ddz, zv[k], gZ[0]);
      gI[1] = fmaf(ddy, iv[k], gI[1]); gZ[1] = fmaf(ddy, zv[k], gZ[1]);
      gI[2] = fmaf(ddx, iv[k], gI[2]); gZ[2] = fmaf(ddx, zv[k], gZ[2]);
    }
    vq[NDIM - 1] = -dt * ax.live * fmaf(Ib, gI[2], zhb * gZ[2]);
    vq[NDIM - 2] = -dt * ay.live * fmaf(Ib, gI[1], zhb * gZ[1]);
    if (NDIM == 3) vq[0] = -dt * az.live * fmaf(Ib, gI[0], zhb * gZ[0]);
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

template <int NDIM>
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
  __shared__ vf4 rvec[NQ];
  __shared__ float rzb[NDIM == 3 ? NQ : 1];
  __shared__ float dbar[DX * DY * DZ];
  const Rec<NDIM> rec{rvec, rzb};
  const Tile tl = tla[xcd_tile(gridDim.x)];
  const PairDev& P = pd[tl.pair];
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
  for (int k = 0; k < PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const int r = ((lz + ZH) * QY + (ly + HS)) * QX + (lx + HS);
#pragma unroll
    for (int c = 0; c < NDIM; ++c) vq[k][c] = 0.f;
    if (x0 + lx < nx && y0 + ly < ny && z0 + lz < nz)
      adj_point<NDIM>(lx, ly, lz, r, true, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB, SI, SZ, rec,
                      dbar, vq[k]);
    else
      rec.clear(r);
  }
  // phase 1b: the halo points around P (records and div_bar only); slots of
  // points outside the image or beyond P +- H hold zero cotangents
  const int hq = gmode ? H : 1;
  for (int li = threadIdx.x; li < NQ; li += NT) {
    const int lx = li % QX - HS, ly = (li / QX) % QY - HS, lz = NDIM == 3 ? li / (QX * QY) - HS : 0;
    const bool inP = lx >= 0 && lx < PX && ly >= 0 && ly < PY && lz >= 0 && lz < PZ;
    if (inP) continue;
    const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
    const bool visit = lx >= -hq && lx < PX + hq && ly >= -hq && ly < PY + hq &&
                       (NDIM == 2 || (lz >= -hq && lz < PZ + hq)) && qx >= 0 && qx < nx && qy >= 0 &&
                       qy < ny && qz >= 0 && qz < nz;
    if (!visit) {
      rec.clear(li);
      continue;
    }
    float dummy[NDIM];
    adj_point<NDIM>(lx, ly, lz, li, false, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB, SI, SZ, rec,
                    dbar, dummy);
  }
  __syncthreads();

  // phase 2: vbar and the gathered transpose of the interpolation
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
    if (qx >= nx || qy >= ny || qz >= nz) continue;
    const unsigned idx = (unsigned)((qz * ny + qy) * nx + qx);
    const int b = ((lz + ZO) * DY + (ly + 1)) * DX + (lx + 1);
    gst(VB, (NDIM - 1) * N + idx, vq[k][NDIM - 1] + diffT_lds(dbar, b, qx, nx, 1));
    gst(VB, (NDIM - 2) * N + idx, vq[k][NDIM - 2] + diffT_lds(dbar, b, qy, ny, DX));
    if (NDIM == 3) gst(VB, idx, vq[k][0] + diffT_lds(dbar, b, qz, nz, DX * DY));
    if (!gmode) continue;
    // Interp^T at p: sum over the arrival points q = p - o, |o| <= H per axis
    const int rp = ((lz + ZH) * QY + (ly + HS)) * QX + (lx + HS);
    float accI = 0.f, accZ = 0.f;
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
    gst(SI, idx, accI);
    gst(SZ, idx, accZ);
  }
}

// Transpose of m_c = z D_c I given mbar (already -G vbar, plus the
// regulariser's term at t = 0):
//   zbar_t = scatter part + sum_c mbar_c D_c I_t
//   Ibar_t = scatter part + sum_c D_c^T (z_t mbar_c)
// At t = 0 only dH/dp0 = zbar_0 + 2 lambda rho p0 is written. The scatter
// accumulator is cleared when the next (earlier) step scatters with global
// atomics.
template <int NDIM>
__global__ __launch_bounds__(NT) void k_epilogue(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                                 const float* __restrict__ mbg, const float* __restrict__ stg,
                                                 float* __restrict__ scg, float* __restrict__ abg, EpiArgs A) {
  using B = Blk<NDIM>;
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
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
#pragma unroll
  for (int k = 0; k < B::PPT; ++k) {
    int lx, ly, lz;
    B::local(threadIdx.x, k, lx, ly, lz);
    const bool inside = t.a + lx < nx && t.b + ly < ny && t.c + lz < nz;
    const int q[3] = {min(t.c + lz, nz - 1), min(t.b + ly, ny - 1), min(t.a + lx, nx - 1)};
    const int n[3] = {nz, ny, nx};
    const int s[3] = {sxy, nx, 1};
    const unsigned idx = (unsigned)((q[0] * ny + q[1]) * nx + q[2]);
    float zbar = gld(SZ, idx);
    float Ibar = gld(SI, idx);
#pragma unroll
    for (int c = 0; c < NDIM; ++c) {
      const int a = 3 - NDIM + c;  // geometric axis of channel c
      const float* M = MB + c * N;
      const unsigned sp = (unsigned)up(q[a], n[a], s[a]), sm = (unsigned)dn(q[a], s[a]);
      const float m0 = gld(M, idx);
      zbar = fmaf(m0, 0.5f * (gld(I, idx + sp) - gld(I, idx - sm)), zbar);
      if (!A.first) {
        // D^T (z m) at q along axis a
        float dT;
        const float zc = gld(Z, idx);
        const float zmu = gld(Z, idx + sp) * gld(M, idx + sp);   // clamped neighbours
        const float zmd = gld(Z, idx - sm) * gld(M, idx - sm);
        if (q[a] == 0)
          dT = -0.5f * (zc * m0 + zmu);
        else if (q[a] == n[a] - 1)
          dT = 0.5f * (zmd + zc * m0);
        else
          dT = 0.5f * (zmd - zmu);
        Ibar += dT;
      }
    }
    if (!inside) continue;
    if (A.first) {
      if (P.outG) gst(P.outG, idx, fmaf(2.f * P.lam * P.rho, gld(Z, idx), zbar));
    } else {
      float* __restrict__ AB = abg + 2 * P.off;
      gst(AB, idx, Ibar);
      gst(AB, N + idx, zbar);
    }
    if (clear) {
      gst(SI, idx, 0.f);
      gst(SZ, idx, 0.f);
    }
  }
}

// Cost of every pair from the per-tile partials, summed in a fixed order:
// out_cost = (data + lambda reg, data, lambda reg).
__global__ __launch_bounds__(NT) void k_finalize(const PairDev* __restrict__ pd, const float* __restrict__ red_reg,
                                                 const float* __restrict__ red_ssd) {
  __shared__ float sh[NT / 64];
  const PairDev& P = pd[blockIdx.x];
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

template <int NDIM, bool PASSZ>
static void spass_dispatch(int mode, const PairDev* pd, const Tile* tl, int nt, size_t lds, const float* src,
                           float* dst, const float* extra, hipStream_t s) {
  const dim3 grid(nt, NDIM);
  if (mode == 0) k_spass<NDIM, PASSZ, 0><<<grid, NT, lds, s>>>(pd, tl, src, dst, extra);
  else if (mode == 1) k_spass<NDIM, PASSZ, 1><<<grid, NT, lds, s>>>(pd, tl, src, dst, extra);
  else k_spass<NDIM, PASSZ, 2><<<grid, NT, lds, s>>>(pd, tl, src, dst, extra);
}

hipError_t launch_spass(int ndim, bool passz, int mode, const PairDev* pd, const Tile* tl, int nt, size_t lds,
                        const float* src, float* dst, const float* extra, hipStream_t s) {
  if (ndim == 2) spass_dispatch<2, false>(mode, pd, tl, nt, lds, src, dst, extra, s);
  else if (passz) spass_dispatch<3, true>(mode, pd, tl, nt, lds, src, dst, extra, s);
  else spass_dispatch<3, false>(mode, pd, tl, nt, lds, src, dst, extra, s);
  return post();
}

hipError_t launch_advect(int ndim, int nt, const AdvectArgs& a, hipStream_t s) {
  if (ndim == 2) k_advect<2><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
  else k_advect<3><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.st_out, a);
  return post();
}

hipError_t launch_adv_adj(int ndim, int nt, const AdjArgs& a, hipStream_t s) {
  if (ndim == 2) k_adv_adj_tile<2><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.ab_in, a.sc, a.vb, a);
  else k_adv_adj_tile<3><<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.ab_in, a.sc, a.vb, a);
  return post();
}

hipError_t launch_epilogue(int ndim, int nt, const EpiArgs& a, hipStream_t s) {
  if (ndim == 2) k_epilogue<2><<<nt, NT, 0, s>>>(a.pd, a.tl, a.mb, a.st, a.sc, a.ab_out, a);
  else k_epilogue<3><<<nt, NT, 0, s>>>(a.pd, a.tl, a.mb, a.st, a.sc, a.ab_out, a);
  return post();
}

hipError_t launch_finalize(int npairs, const PairDev* pd, const float* red_reg, const float* red_ssd,
                           hipStream_t s) {
  k_finalize<<<npairs, NT, 0, s>>>(pd, red_reg, red_ssd);
  return post();
}

}  // namespace shoot
