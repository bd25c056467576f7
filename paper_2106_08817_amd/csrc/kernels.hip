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
//   k_adv_adj_tile        tile-owned transpose of the interpolation (LDS
//                         accumulation), foot-point cotangent and div^T
//   k_xpass<plain>, k_spass  G is symmetric, so the same passes smooth vbar
//   k_epilogue            transpose of m = z D I
#include "kernels.h"
#include "device_common.h"

namespace shoot {

// ----------------------------------------------------------------------------
// small utility kernels
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(NT) void k_fill_u32(unsigned* __restrict__ p, long long n, unsigned v) {
  for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    p[i] = v;
}

// State slot <- (S, p0) for every pair.
__global__ __launch_bounds__(NT) void k_init(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                             float* __restrict__ st) {
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  float* I = st + 2 * P.off;
  float* Z = I + P.N;
  for (int j = threadIdx.x; j < t.b; j += NT) {
    const int i = t.a + j;
    I[i] = P.S[i];
    Z[i] = P.p0[i];
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
  const int N = (int)P.N;
  const int G4 = (nx + 3) >> 2;
  const int L = 4 * (G4 + ntap4);
  const int row0 = t.a, nrows = t.b;
  const int plane = nrows * L;

  // fill: one wave per row, lanes along the row (every load of a row is
  // independent, so the unrolled column loop keeps several in flight)
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  if (GRADMUL) {
    const float* __restrict__ I = src + 2 * P.off;
    const float* __restrict__ Z = I + N;
    for (int rl = wv; rl < nrows; rl += NT / 64) {
      const int row = row0 + rl;
      const int y = row % ny;
      const int rbase = row * nx;
      const int yu = up(y, ny, nx), yd = dn(y, nx);
      int zu = 0, zd = 0;
      if (NDIM == 3) {
        const int z = row / ny;
        zu = up(z, nz, ny * nx);
        zd = dn(z, ny * nx);
      }
      float* Lrow = lds + rl * L;
#pragma unroll 4
      for (int col = lane; col < L; col += 64) {
        const int x = col - r;
        float m[NDIM];
#pragma unroll
        for (int c = 0; c < NDIM; ++c) m[c] = 0.f;
        if (x >= 0 && x < nx) {
          const int idx = rbase + x;
          const float zq = 0.5f * Z[idx];
          m[NDIM - 1] = zq * (I[idx + up(x, nx, 1)] - I[idx - dn(x, 1)]);
          m[NDIM - 2] = zq * (I[idx + yu] - I[idx - yd]);
          if (NDIM == 3) m[0] = zq * (I[idx + zu] - I[idx - zd]);
        }
#pragma unroll
        for (int c = 0; c < NDIM; ++c) Lrow[c * plane + col] = m[c];
      }
    }
  } else {
    const float* __restrict__ F = src + NDIM * P.off;
    for (int rl = wv; rl < nrows; rl += NT / 64) {
      const int rbase = (row0 + rl) * nx;
      float* Lrow = lds + rl * L;
#pragma unroll 4
      for (int col = lane; col < L; col += 64) {
        const int x = col - r;
        const bool in = (x >= 0 && x < nx);
#pragma unroll
        for (int c = 0; c < NDIM; ++c) Lrow[c * plane + col] = in ? F[c * N + rbase + x] : 0.f;
      }
    }
  }
  __syncthreads();

  const float4* W4 = reinterpret_cast<const float4*>(P.w);
  float* D = dst + NDIM * P.off;
  const int ngroups = nrows * G4;
  for (int g = threadIdx.x; g < ngroups; g += NT) {
    const int rl = g / G4;
    const int x = 4 * (g - rl * G4);
    const int obase = (row0 + rl) * nx + x;
#pragma unroll
    for (int c = 0; c < NDIM; ++c) {
      // row offsets are multiples of four floats: index the LDS as float4 so
      // the reads are aligned ds_read_b128 (consecutive lanes, consecutive 16 B)
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
// extra_scale * extra (the regulariser's cotangent at t = 0).
template <int NDIM, bool PASSZ, int MODE>
__global__ __launch_bounds__(NT) void k_spass(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                              const float* __restrict__ src, float* __restrict__ dst,
                                              const float* __restrict__ extra) {
  extern __shared__ vf4 smem4[];
  float* lds = reinterpret_cast<float*>(smem4);
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz, r = P.r, ntap4 = P.ntap4;
  const int N = (int)P.N;
  // pass axis: length ns, stride ss; third axis index t.b with stride so
  const int ns = PASSZ ? nz : ny;
  const int ss = PASSZ ? ny * nx : nx;
  const int so = PASSZ ? nx : ny * nx;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int x = t.a + lane;
  const int s0 = t.c;
  const int rows = SSEG + 4 * ntap4;
  const int base = t.b * so + x;           // offset of (s = 0, x) in the pair
  const float* F = src + NDIM * P.off;
  float* D = dst + NDIM * P.off;
  const float* E = (MODE == 2 && extra != nullptr) ? extra + NDIM * P.off : nullptr;
  const float escale = -2.f * P.lam;
  const float4* W4 = reinterpret_cast<const float4*>(P.w);
  const bool xin = x < nx;

  {
    const int c = blockIdx.y;  // one channel per block
    const float* Fc = F + c * N;
#pragma unroll 8
    for (int j = wv; j < rows; j += NT / 64) {
      const int s = s0 - r + j;
      lds[j * 64 + lane] = (xin && s >= 0 && s < ns) ? Fc[base + s * ss] : 0.f;
    }
    __syncthreads();
    float acc[SRB];
#pragma unroll
    for (int i = 0; i < SRB; ++i) acc[i] = 0.f;
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
#pragma unroll
      for (int i = 0; i < SRB; ++i) {
        const int s = s0 + wv * SRB + i;
        if (s < ns) {
          const int idx = base + s * ss;
          float o = acc[i];
          if (MODE >= 1) o = -o;
          if (MODE == 2 && E != nullptr) o = fmaf(escale, E[c * N + idx], o);
          D[c * N + idx] = o;
        }
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
  __shared__ float sh[NT / 64];
  const int tix = xcd_tile(gridDim.x);
  const Tile t = tl[tix];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int N = (int)P.N;
  const int sxy = nx * ny;
  const float dt = P.dt, rdt = P.rho * P.dt;
  const float* __restrict__ V = Vg + NDIM * P.off;
  const float* __restrict__ I = stg + 2 * P.off;
  const float* __restrict__ Z = I + N;
  float* __restrict__ Io = stog ? stog + 2 * P.off : nullptr;
  float reg = 0.f, ssd = 0.f, dm = 0.f;
#pragma unroll
  for (int k = 0; k < ELEM / NT; ++k) {
    const int j = threadIdx.x + k * NT;
    if (j >= t.b) continue;
    const int idx = t.a + j;
    const int xq = idx % nx;
    const int yq = (idx / nx) % ny;
    const int zq = idx / sxy;
    float v[NDIM];
#pragma unroll
    for (int c = 0; c < NDIM; ++c) v[c] = V[c * N + idx];
    // div v at q (clamped central differences)
    float div = 0.5f * (V[(NDIM - 1) * N + idx + up(xq, nx, 1)] - V[(NDIM - 1) * N + idx - dn(xq, 1)]);
    div += 0.5f * (V[(NDIM - 2) * N + idx + up(yq, ny, nx)] - V[(NDIM - 2) * N + idx - dn(yq, nx)]);
    if (NDIM == 3) div += 0.5f * (V[idx + up(zq, nz, sxy)] - V[idx - dn(zq, sxy)]);
    float dx = -dt * v[NDIM - 1], dy = -dt * v[NDIM - 2];
    dm = fmaxf(dm, fmaxf(fabsf(dx), fabsf(dy)));
    const Axis ax = foot_axis(xq, dx, nx);
    const Axis ay = foot_axis(yq, dy, ny);
    float Ih, zh;
    if (NDIM == 2) {
      const int c00 = ay.i * nx + ax.i;
      const float wy0 = 1.f - ay.f, wy1 = ay.f, wx0 = 1.f - ax.f, wx1 = ax.f;
      Ih = wy0 * (wx0 * I[c00] + wx1 * I[c00 + 1]) + wy1 * (wx0 * I[c00 + nx] + wx1 * I[c00 + nx + 1]);
      zh = wy0 * (wx0 * Z[c00] + wx1 * Z[c00 + 1]) + wy1 * (wx0 * Z[c00 + nx] + wx1 * Z[c00 + nx + 1]);
    } else {
      const float dz = -dt * v[0];
      dm = fmaxf(dm, fabsf(dz));
      const Axis az = foot_axis(zq, dz, nz);
      const int c000 = az.i * sxy + ay.i * nx + ax.i;
      const float wz0 = 1.f - az.f, wz1 = az.f, wy0 = 1.f - ay.f, wy1 = ay.f, wx0 = 1.f - ax.f, wx1 = ax.f;
      const int c010 = c000 + nx, c100 = c000 + sxy, c110 = c100 + nx;
      Ih = wz0 * (wy0 * (wx0 * I[c000] + wx1 * I[c000 + 1]) + wy1 * (wx0 * I[c010] + wx1 * I[c010 + 1])) +
           wz1 * (wy0 * (wx0 * I[c100] + wx1 * I[c100 + 1]) + wy1 * (wx0 * I[c110] + wx1 * I[c110 + 1]));
      zh = wz0 * (wy0 * (wx0 * Z[c000] + wx1 * Z[c000 + 1]) + wy1 * (wx0 * Z[c010] + wx1 * Z[c010 + 1])) +
           wz1 * (wy0 * (wx0 * Z[c100] + wx1 * Z[c100 + 1]) + wy1 * (wx0 * Z[c110] + wx1 * Z[c110 + 1]));
    }
    const float In = fmaf(rdt, zh, Ih);
    const float zn = zh * (1.f - dt * div);
    if (Io) {
      Io[idx] = In;
      Io[N + idx] = zn;
    }
    if (A.red_reg) {
      // -<m_0, v_0> + rho |p0|^2 at q, with m_c = z D_c I
      const float zq0 = Z[idx];
      float g[NDIM];
      g[NDIM - 1] = 0.5f * (I[idx + up(xq, nx, 1)] - I[idx - dn(xq, 1)]);
      g[NDIM - 2] = 0.5f * (I[idx + up(yq, ny, nx)] - I[idx - dn(yq, nx)]);
      if (NDIM == 3) g[0] = 0.5f * (I[idx + up(zq, nz, sxy)] - I[idx - dn(zq, sxy)]);
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
// P. Phase 1 visits those q and leaves one record per q in LDS (cell of the
// foot, its fractions, Ib and zh_bar), plus div_bar on P +- 1 and the
// foot-point part of vbar on P. Phase 2 forms Interp^T at each p of P as a
// gather over the (2H+1)^d candidate q around it, in a fixed order: no
// atomics, deterministic, each output written once. For D >= HS (or when
// forced) the block instead scatters its own q with global atomics into the
// accumulator, which the previous adjoint step (or the last forward step)
// cleared.
__device__ __forceinline__ float diffT_lds(const float* g, int b, int j, int n, int s) {
  if (j == 0) return -0.5f * (g[b] + g[b + s]);
  if (j == n - 1) return 0.5f * (g[b - s] + g[b]);
  return 0.5f * (g[b - s] - g[b + s]);
}

// Phase-1 work for one arrival point q (local coordinates l* relative to P):
// its record, div_bar (on P +- 1), the global scatter (fallback mode) and,
// for q in P, the foot-point part of vbar (returned in vq).
template <int NDIM>
__device__ __forceinline__ void adj_point(int lx, int ly, int lz, int li, bool inP, bool gmode, int x0, int y0,
                                          int z0, int nx, int ny, int nz, int N, float dt, float rdt,
                                          const float* __restrict__ V, const float* __restrict__ I,
                                          const float* __restrict__ Z, const float* __restrict__ AB,
                                          float* __restrict__ SI, float* __restrict__ SZ, int* rcell,
                                          float (*rf)[ADJ_NQ<NDIM>()], float* rib, float* rzb, float* dbar,
                                          float vq[NDIM]) {
  constexpr int PX = NDIM == 2 ? ADJ2_X : ADJ3_X;
  constexpr int PY = NDIM == 2 ? ADJ2_Y : ADJ3_Y;
  constexpr int PZ = NDIM == 2 ? 1 : ADJ3_Z;
  constexpr int HS = NDIM == 2 ? ADJ2_HS : ADJ3_HS;
  constexpr int DX = PX + 2, DY = PY + 2;
  constexpr int ZO = NDIM == 3 ? 1 : 0;
  constexpr int NC = NDIM == 3 ? 8 : 4;
  constexpr int COFF = 2 * HS;
  const int sxy = nx * ny;
  const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
  const bool inP1 = lx >= -1 && lx <= PX && ly >= -1 && ly <= PY && (NDIM == 2 || (lz >= -1 && lz <= PZ));
  const int idx = (qz * ny + qy) * nx + qx;
  float div = 0.5f * (V[(NDIM - 1) * N + idx + up(qx, nx, 1)] - V[(NDIM - 1) * N + idx - dn(qx, 1)]);
  div += 0.5f * (V[(NDIM - 2) * N + idx + up(qy, ny, nx)] - V[(NDIM - 2) * N + idx - dn(qy, nx)]);
  if (NDIM == 3) div += 0.5f * (V[idx + up(qz, nz, sxy)] - V[idx - dn(qz, sxy)]);
  const float Ib = AB[idx];
  const float zb = AB[N + idx];
  const Axis ax = foot_axis(qx, -dt * V[(NDIM - 1) * N + idx], nx);
  const Axis ay = foot_axis(qy, -dt * V[(NDIM - 2) * N + idx], ny);
  Axis az;
  if (NDIM == 3) {
    az = foot_axis(qz, -dt * V[idx], nz);
  } else {
    az.i = 0; az.f = 0.f; az.live = 0.f;
  }
  const float wz[2] = {1.f - az.f, az.f}, wy[2] = {1.f - ay.f, ay.f}, wx[2] = {1.f - ax.f, ax.f};
  const int c0 = az.i * sxy + ay.i * nx + ax.i;
  float zv[NC], iv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
    const int g = c0 + bz * sxy + by * nx + bx;
    zv[k] = Z[g];
    iv[k] = inP ? I[g] : 0.f;
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
    rcell[li] = (ax.i - x0 + COFF) | ((ay.i - y0 + COFF) << 8) | ((NDIM == 3 ? az.i - z0 + COFF : 0) << 16);
    rf[NDIM - 1][li] = ax.f;
    rf[NDIM - 2][li] = ay.f;
    if (NDIM == 3) rf[0][li] = az.f;
    rib[li] = Ib;
    rzb[li] = zhb;
  } else {
    rcell[li] = -1;
    if (inP) {
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
        const float w = (NDIM == 3 ? wz[bz] : 1.f) * wy[by] * wx[bx];
        const int g = c0 + bz * sxy + by * nx + bx;
        unsafeAtomicAdd(SI + g, w * Ib);
        unsafeAtomicAdd(SZ + g, w * zhb);
      }
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

template <int NDIM>
__global__ __launch_bounds__(NT) void k_adv_adj_tile(const PairDev* __restrict__ pd, const Tile* __restrict__ tla,
                                                     const float* __restrict__ Vg, const float* __restrict__ stg,
                                                     const float* __restrict__ abg, float* __restrict__ scg,
                                                     float* __restrict__ vbg, AdjArgs A) {
  constexpr int PX = NDIM == 2 ? ADJ2_X : ADJ3_X;
  constexpr int PY = NDIM == 2 ? ADJ2_Y : ADJ3_Y;
  constexpr int PZ = NDIM == 2 ? 1 : ADJ3_Z;
  constexpr int HS = NDIM == 2 ? ADJ2_HS : ADJ3_HS;   // gather mode handles D < HS
  constexpr int NP = PX * PY * PZ;
  constexpr int PPT = NP / NT;                        // outputs per thread
  static_assert(NP % NT == 0, "tile must be a multiple of the block");
  // P +- 1 (div_bar) and P +- HS (arrival points that may reach P)
  constexpr int DX = PX + 2, DY = PY + 2, DZ = NDIM == 3 ? PZ + 2 : 1;
  constexpr int QX = PX + 2 * HS, QY = PY + 2 * HS;
  constexpr int NQ = ADJ_NQ<NDIM>();
  constexpr int ZO = NDIM == 3 ? 1 : 0;
  constexpr int ZH = NDIM == 3 ? HS : 0;
  constexpr int COFF = 2 * HS;  // cell coordinates relative to P, shifted to be >= 0
  __shared__ int rcell[NQ];
  __shared__ float rf[NDIM][NQ];
  __shared__ float rib[NQ], rzb[NQ];
  __shared__ float dbar[DX * DY * DZ];
  const Tile tl = tla[xcd_tile(gridDim.x)];
  const PairDev& P = pd[tl.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int N = (int)P.N;
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
    const int li = threadIdx.x + k * NT;
    const int lx = li % PX, ly = (li / PX) % PY, lz = li / (PX * PY);
    const int r = ((lz + ZH) * QY + (ly + HS)) * QX + (lx + HS);
#pragma unroll
    for (int c = 0; c < NDIM; ++c) vq[k][c] = 0.f;
    if (x0 + lx < nx && y0 + ly < ny && z0 + lz < nz)
      adj_point<NDIM>(lx, ly, lz, r, true, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB, SI, SZ,
                      rcell, rf, rib, rzb, dbar, vq[k]);
    else
      rcell[r] = -1;
  }
  // phase 1b: the halo points P +- H around P (records and div_bar only)
  const int hq = gmode ? H : 1;
#pragma unroll 2
  for (int li = threadIdx.x; li < NQ; li += NT) {
    const int lx = li % QX - HS, ly = (li / QX) % QY - HS, lz = NDIM == 3 ? li / (QX * QY) - HS : 0;
    const bool inP = lx >= 0 && lx < PX && ly >= 0 && ly < PY && lz >= 0 && lz < PZ;
    if (inP) continue;
    const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
    const bool visit = lx >= -hq && lx < PX + hq && ly >= -hq && ly < PY + hq &&
                       (NDIM == 2 || (lz >= -hq && lz < PZ + hq)) && qx >= 0 && qx < nx && qy >= 0 &&
                       qy < ny && qz >= 0 && qz < nz;
    if (!visit) {
      rcell[li] = -1;
      continue;
    }
    float dummy[NDIM];
    adj_point<NDIM>(lx, ly, lz, li, false, gmode, x0, y0, z0, nx, ny, nz, N, dt, rdt, V, I, Z, AB, SI, SZ,
                    rcell, rf, rib, rzb, dbar, dummy);
  }
  __syncthreads();

  // phase 2: vbar and the gathered transpose of the interpolation
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = threadIdx.x + k * NT;
    const int lx = li % PX, ly = (li / PX) % PY, lz = li / (PX * PY);
    const int qx = x0 + lx, qy = y0 + ly, qz = z0 + lz;
    if (qx >= nx || qy >= ny || (NDIM == 3 && qz >= nz)) continue;
    const int idx = (qz * ny + qy) * nx + qx;
    const int b = ((lz + ZO) * DY + (ly + 1)) * DX + (lx + 1);
    VB[(NDIM - 1) * N + idx] = vq[k][NDIM - 1] + diffT_lds(dbar, b, qx, nx, 1);
    VB[(NDIM - 2) * N + idx] = vq[k][NDIM - 2] + diffT_lds(dbar, b, qy, ny, DX);
    if (NDIM == 3) VB[idx] = vq[k][0] + diffT_lds(dbar, b, qz, nz, DX * DY);
    if (gmode) {
      // Interp^T at p: sum over candidate arrival points q = p + (oz, oy, ox)
      float accI = 0.f, accZ = 0.f;
      const int hz = NDIM == 3 ? H : 0;
      for (int oz = -hz; oz <= hz; ++oz)
        for (int oy = -H; oy <= H; ++oy)
          for (int ox = -H; ox <= H; ++ox) {
            const int r = ((lz + oz + ZH) * QY + (ly + oy + HS)) * QX + (lx + ox + HS);
            const int code = rcell[r];
            if (code < 0) continue;
            const int bx = lx + COFF - (code & 0xff);
            const int by = ly + COFF - ((code >> 8) & 0xff);
            const int bz = NDIM == 3 ? lz + COFF - ((code >> 16) & 0xff) : 0;
            if ((unsigned)bx > 1u || (unsigned)by > 1u || (unsigned)bz > 1u) continue;
            float w = (bx ? rf[NDIM - 1][r] : 1.f - rf[NDIM - 1][r]) * (by ? rf[NDIM - 2][r] : 1.f - rf[NDIM - 2][r]);
            if (NDIM == 3) w *= bz ? rf[0][r] : 1.f - rf[0][r];
            accI = fmaf(w, rib[r], accI);
            accZ = fmaf(w, rzb[r], accZ);
          }
      SI[idx] = accI;
      SZ[idx] = accZ;
    }
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
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int N = (int)P.N;
  const int sxy = nx * ny;
  const float* __restrict__ MB = mbg + NDIM * P.off;
  const float* __restrict__ I = stg + 2 * P.off;
  const float* __restrict__ Z = I + N;
  float* __restrict__ SI = scg + 2 * P.off;
  float* __restrict__ SZ = SI + N;
  bool clear = false;
  if (!A.first) {
    const float Dn = __uint_as_float(A.dmax[(long long)t.pair * A.T + A.t - 1]);
    clear = A.force_global || !(Dn < (float)(NDIM == 2 ? ADJ2_HS : ADJ3_HS));
  }
#pragma unroll
  for (int k = 0; k < ELEM / NT; ++k) {
    const int j = threadIdx.x + k * NT;
    if (j >= t.b) continue;
    const int idx = t.a + j;
    const int xq = idx % nx;
    const int yq = (idx / nx) % ny;
    const int zq = idx / sxy;
    const int n[3] = {nz, ny, nx};
    const int q[3] = {zq, yq, xq};
    const int s[3] = {sxy, nx, 1};
    float zbar = SZ[idx];
    float Ibar = SI[idx];
#pragma unroll
    for (int c = 0; c < NDIM; ++c) {
      const int a = 3 - NDIM + c;  // geometric axis of channel c
      const float* M = MB + c * N;
      const int sp = up(q[a], n[a], s[a]), sm = dn(q[a], s[a]);
      zbar = fmaf(M[idx], 0.5f * (I[idx + sp] - I[idx - sm]), zbar);
      if (!A.first) {
        // D^T (z m) at q along axis a
        float dT;
        if (q[a] == 0)
          dT = -0.5f * (Z[idx] * M[idx] + Z[idx + s[a]] * M[idx + s[a]]);
        else if (q[a] == n[a] - 1)
          dT = 0.5f * (Z[idx - s[a]] * M[idx - s[a]] + Z[idx] * M[idx]);
        else
          dT = 0.5f * (Z[idx - s[a]] * M[idx - s[a]] - Z[idx + s[a]] * M[idx + s[a]]);
        Ibar += dT;
      }
    }
    if (A.first) {
      if (P.outG) P.outG[idx] = fmaf(2.f * P.lam * P.rho, Z[idx], zbar);
    } else {
      float* __restrict__ AB = abg + 2 * P.off;
      AB[idx] = Ibar;
      AB[N + idx] = zbar;
    }
    if (clear) {
      SI[idx] = 0.f;
      SZ[idx] = 0.f;
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

hipError_t launch_init(const PairDev* pd, const Tile* tl, int nt, float* st, hipStream_t s) {
  k_init<<<nt, NT, 0, s>>>(pd, tl, st);
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
