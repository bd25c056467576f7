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
//   k_adv_adj + k_divT    scatter-add of the interpolation transpose, the
//                         foot-point cotangent and div^T
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
  extern __shared__ float4 smem4[];
  float* lds = reinterpret_cast<float*>(smem4);
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz, r = P.r, ntap4 = P.ntap4;
  const int N = (int)P.N;
  const int G4 = (nx + 3) >> 2;
  const int L = 4 * (G4 + ntap4);
  const int row0 = t.a, nrows = t.b;
  const int plane = nrows * L;

  if (GRADMUL) {
    const float* I = src + 2 * P.off;
    const float* Z = I + N;
    for (int li = threadIdx.x; li < plane; li += NT) {
      const int rl = li / L;
      const int x = li - rl * L - r;
      float m[NDIM];
#pragma unroll
      for (int c = 0; c < NDIM; ++c) m[c] = 0.f;
      if (x >= 0 && x < nx) {
        const int row = row0 + rl;
        const int y = row % ny;
        const int idx = row * nx + x;
        const float zq = Z[idx];
        m[NDIM - 1] = zq * 0.5f * (I[idx + up(x, nx, 1)] - I[idx - dn(x, 1)]);
        m[NDIM - 2] = zq * 0.5f * (I[idx + up(y, ny, nx)] - I[idx - dn(y, nx)]);
        if (NDIM == 3) {
          const int z = row / ny;
          const int s = ny * nx;
          m[0] = zq * 0.5f * (I[idx + up(z, nz, s)] - I[idx - dn(z, s)]);
        }
      }
#pragma unroll
      for (int c = 0; c < NDIM; ++c) lds[c * plane + li] = m[c];
    }
  } else {
    const float* F = src + NDIM * P.off;
    for (int li = threadIdx.x; li < plane; li += NT) {
      const int rl = li / L;
      const int x = li - rl * L - r;
      const bool in = (x >= 0 && x < nx);
      const int idx = (row0 + rl) * nx + x;
#pragma unroll
      for (int c = 0; c < NDIM; ++c) lds[c * plane + li] = in ? F[c * N + idx] : 0.f;
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
      const float4* R4 = reinterpret_cast<const float4*>(lds + c * plane + rl * L + x);
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      float4 lo = R4[0];
      for (int b = 0; b < ntap4; ++b) {
        const float4 hi = R4[b + 1];
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
// at one index of the third axis. Channels are processed one after another
// through one LDS buffer of (SSEG + 4 ntap4) rows x 64 floats; LDS row j holds
// the input at s = s0 - r + j. Each thread produces SRB consecutive outputs.
// MODE 0: plain pass. MODE 1: negated (v = -G m). MODE 2: negated, plus
// extra_scale * extra (the regulariser's cotangent at t = 0).
template <int NDIM, bool PASSZ, int MODE>
__global__ __launch_bounds__(NT) void k_spass(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                              const float* __restrict__ src, float* __restrict__ dst,
                                              const float* __restrict__ extra) {
  extern __shared__ float4 smem4[];
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

  for (int c = 0; c < NDIM; ++c) {
    const float* Fc = F + c * N;
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
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// semi-Lagrangian advection (forward step)
// ----------------------------------------------------------------------------


template <int NDIM>
__global__ __launch_bounds__(NT) void k_advect(AdvectArgs A) {
  __shared__ float sh[NT / 64];
  const int tix = xcd_tile(gridDim.x);
  const Tile t = A.tl[tix];
  const PairDev& P = A.pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int N = (int)P.N;
  const int sxy = nx * ny;
  const float dt = P.dt, rdt = P.rho * P.dt;
  const float* V = A.V + NDIM * P.off;
  const float* I = A.st + 2 * P.off;
  const float* Z = I + N;
  float* Io = A.st_out ? A.st_out + 2 * P.off : nullptr;
  float reg = 0.f, ssd = 0.f, dm = 0.f;
  for (int j = threadIdx.x; j < t.b; j += NT) {
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
// adjoint of the advection (global-atomic scatter)
// ----------------------------------------------------------------------------
//
// For each arrival point q with cotangents (Ib, zb) of (I_{t+1}, z_{t+1}):
//   zh_bar = rho dt Ib + (1 - dt div v) zb,   div_bar = -dt zh zb,
//   Ibar_t += Interp^T(Ib),  zbar_t += Interp^T(zh_bar)       (scatter-add)
//   vbar_c = -dt (Ib dInterp(I_t)/dy_c + zh_bar dInterp(z_t)/dy_c)
// div_bar is stored; k_divT then adds D_c^T div_bar to vbar_c.

template <int NDIM>
__global__ __launch_bounds__(NT) void k_adv_adj(AdjArgs A) {
  const Tile t = A.tl[xcd_tile(gridDim.x)];
  const PairDev& P = A.pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int N = (int)P.N;
  const int sxy = nx * ny;
  const float dt = P.dt, rdt = P.rho * P.dt;
  const float* V = A.V + NDIM * P.off;
  const float* I = A.st + 2 * P.off;
  const float* Z = I + N;
  const float* AB = A.ab_in + 2 * P.off;
  float* SI = A.sc + 2 * P.off;
  float* SZ = SI + N;
  float* DB = A.db + P.off;
  float* VB = A.vb + NDIM * P.off;
  for (int j = threadIdx.x; j < t.b; j += NT) {
    const int idx = t.a + j;
    const int xq = idx % nx;
    const int yq = (idx / nx) % ny;
    const int zq = idx / sxy;
    float div = 0.5f * (V[(NDIM - 1) * N + idx + up(xq, nx, 1)] - V[(NDIM - 1) * N + idx - dn(xq, 1)]);
    div += 0.5f * (V[(NDIM - 2) * N + idx + up(yq, ny, nx)] - V[(NDIM - 2) * N + idx - dn(yq, nx)]);
    if (NDIM == 3) div += 0.5f * (V[idx + up(zq, nz, sxy)] - V[idx - dn(zq, sxy)]);
    const Axis ax = foot_axis(xq, -dt * V[(NDIM - 1) * N + idx], nx);
    const Axis ay = foot_axis(yq, -dt * V[(NDIM - 2) * N + idx], ny);
    const float Ib = AB[idx];
    const float zb = AB[N + idx];
    const float wx0 = 1.f - ax.f, wx1 = ax.f, wy0 = 1.f - ay.f, wy1 = ay.f;
    if (NDIM == 2) {
      const int c00 = ay.i * nx + ax.i, c10 = c00 + nx;
      const float i00 = I[c00], i01 = I[c00 + 1], i10 = I[c10], i11 = I[c10 + 1];
      const float z00 = Z[c00], z01 = Z[c00 + 1], z10 = Z[c10], z11 = Z[c10 + 1];
      const float zh = wy0 * (wx0 * z00 + wx1 * z01) + wy1 * (wx0 * z10 + wx1 * z11);
      const float zhb = fmaf(rdt, Ib, (1.f - dt * div) * zb);
      DB[idx] = -dt * zh * zb;
      const float w00 = wy0 * wx0, w01 = wy0 * wx1, w10 = wy1 * wx0, w11 = wy1 * wx1;
      unsafeAtomicAdd(SI + c00, w00 * Ib);
      unsafeAtomicAdd(SI + c00 + 1, w01 * Ib);
      unsafeAtomicAdd(SI + c10, w10 * Ib);
      unsafeAtomicAdd(SI + c10 + 1, w11 * Ib);
      unsafeAtomicAdd(SZ + c00, w00 * zhb);
      unsafeAtomicAdd(SZ + c00 + 1, w01 * zhb);
      unsafeAtomicAdd(SZ + c10, w10 * zhb);
      unsafeAtomicAdd(SZ + c10 + 1, w11 * zhb);
      const float gIy = ay.live * (wx0 * (i10 - i00) + wx1 * (i11 - i01));
      const float gIx = ax.live * (wy0 * (i01 - i00) + wy1 * (i11 - i10));
      const float gzy = ay.live * (wx0 * (z10 - z00) + wx1 * (z11 - z01));
      const float gzx = ax.live * (wy0 * (z01 - z00) + wy1 * (z11 - z10));
      VB[idx] = -dt * fmaf(Ib, gIy, zhb * gzy);
      VB[N + idx] = -dt * fmaf(Ib, gIx, zhb * gzx);
    } else {
      const Axis az = foot_axis(zq, -dt * V[idx], nz);
      const float wz0 = 1.f - az.f, wz1 = az.f;
      const int c000 = az.i * sxy + ay.i * nx + ax.i;
      const int cc[8] = {c000, c000 + 1, c000 + nx, c000 + nx + 1,
                         c000 + sxy, c000 + sxy + 1, c000 + sxy + nx, c000 + sxy + nx + 1};
      float iv[8], zv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) { iv[k] = I[cc[k]]; zv[k] = Z[cc[k]]; }
      // corner k = 4 bz + 2 by + bx
      const float wz[2] = {wz0, wz1}, wy[2] = {wy0, wy1}, wx[2] = {wx0, wx1};
      float zh = 0.f;
      float w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        w[k] = wz[k >> 2] * wy[(k >> 1) & 1] * wx[k & 1];
        zh = fmaf(w[k], zv[k], zh);
      }
      const float zhb = fmaf(rdt, Ib, (1.f - dt * div) * zb);
      DB[idx] = -dt * zh * zb;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        unsafeAtomicAdd(SI + cc[k], w[k] * Ib);
        unsafeAtomicAdd(SZ + cc[k], w[k] * zhb);
      }
      // derivatives of the trilinear weights along each axis
      float gI[3] = {0.f, 0.f, 0.f}, gZ[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
        const float dz = (bz ? 1.f : -1.f) * wy[by] * wx[bx];
        const float dy = (by ? 1.f : -1.f) * wz[bz] * wx[bx];
        const float dxw = (bx ? 1.f : -1.f) * wz[bz] * wy[by];
        gI[0] = fmaf(dz, iv[k], gI[0]); gZ[0] = fmaf(dz, zv[k], gZ[0]);
        gI[1] = fmaf(dy, iv[k], gI[1]); gZ[1] = fmaf(dy, zv[k], gZ[1]);
        gI[2] = fmaf(dxw, iv[k], gI[2]); gZ[2] = fmaf(dxw, zv[k], gZ[2]);
      }
      const float live[3] = {az.live, ay.live, ax.live};
#pragma unroll
      for (int c = 0; c < 3; ++c)
        VB[c * N + idx] = -dt * live[c] * fmaf(Ib, gI[c], zhb * gZ[c]);
    }
  }
}

// vbar_c += D_c^T div_bar (transpose of the clamped central difference:
// interior (g[j-1] - g[j+1]) / 2, first -(g[0] + g[1]) / 2, last
// (g[n-2] + g[n-1]) / 2).
__device__ __forceinline__ float diffT(const float* g, int idx, int j, int n, int s) {
  if (j == 0) return -0.5f * (g[idx] + g[idx + s]);
  if (j == n - 1) return 0.5f * (g[idx - s] + g[idx]);
  return 0.5f * (g[idx - s] - g[idx + s]);
}

template <int NDIM>
__global__ __launch_bounds__(NT) void k_divT(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                             const float* __restrict__ db, float* __restrict__ vb) {
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int N = (int)P.N;
  const int sxy = nx * ny;
  const float* DB = db + P.off;
  float* VB = vb + NDIM * P.off;
  for (int j = threadIdx.x; j < t.b; j += NT) {
    const int idx = t.a + j;
    const int xq = idx % nx;
    const int yq = (idx / nx) % ny;
    VB[(NDIM - 1) * N + idx] += diffT(DB, idx, xq, nx, 1);
    VB[(NDIM - 2) * N + idx] += diffT(DB, idx, yq, ny, nx);
    if (NDIM == 3) VB[idx] += diffT(DB, idx, idx / sxy, nz, sxy);
  }
}

// Transpose of m_c = z D_c I given mbar (already -G vbar, plus the
// regulariser's term at t = 0):
//   zbar_t = scatter part + sum_c mbar_c D_c I_t
//   Ibar_t = scatter part + sum_c D_c^T (z_t mbar_c)
// At t = 0 only dH/dp0 = zbar_0 + 2 lambda rho p0 is written. The scatter
// accumulator is cleared for the next (earlier) step.

template <int NDIM>
__global__ __launch_bounds__(NT) void k_epilogue(EpiArgs A) {
  const Tile t = A.tl[xcd_tile(gridDim.x)];
  const PairDev& P = A.pd[t.pair];
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int N = (int)P.N;
  const int sxy = nx * ny;
  const float* MB = A.mb + NDIM * P.off;
  const float* I = A.st + 2 * P.off;
  const float* Z = I + N;
  float* SI = A.sc + 2 * P.off;
  float* SZ = SI + N;
  for (int j = threadIdx.x; j < t.b; j += NT) {
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
      float* AB = A.ab_out + 2 * P.off;
      AB[idx] = Ibar;
      AB[N + idx] = zbar;
    }
    SI[idx] = 0.f;
    SZ[idx] = 0.f;
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
  if (mode == 0) k_spass<NDIM, PASSZ, 0><<<nt, NT, lds, s>>>(pd, tl, src, dst, extra);
  else if (mode == 1) k_spass<NDIM, PASSZ, 1><<<nt, NT, lds, s>>>(pd, tl, src, dst, extra);
  else k_spass<NDIM, PASSZ, 2><<<nt, NT, lds, s>>>(pd, tl, src, dst, extra);
}

hipError_t launch_spass(int ndim, bool passz, int mode, const PairDev* pd, const Tile* tl, int nt, size_t lds,
                        const float* src, float* dst, const float* extra, hipStream_t s) {
  if (ndim == 2) spass_dispatch<2, false>(mode, pd, tl, nt, lds, src, dst, extra, s);
  else if (passz) spass_dispatch<3, true>(mode, pd, tl, nt, lds, src, dst, extra, s);
  else spass_dispatch<3, false>(mode, pd, tl, nt, lds, src, dst, extra, s);
  return post();
}

hipError_t launch_advect(int ndim, int nt, const AdvectArgs& a, hipStream_t s) {
  if (ndim == 2) k_advect<2><<<nt, NT, 0, s>>>(a);
  else k_advect<3><<<nt, NT, 0, s>>>(a);
  return post();
}

hipError_t launch_adv_adj(int ndim, int nt, const AdjArgs& a, hipStream_t s) {
  if (ndim == 2) k_adv_adj<2><<<nt, NT, 0, s>>>(a);
  else k_adv_adj<3><<<nt, NT, 0, s>>>(a);
  return post();
}

hipError_t launch_divT(int ndim, const PairDev* pd, const Tile* tl, int nt, const float* db, float* vb,
                       hipStream_t s) {
  if (ndim == 2) k_divT<2><<<nt, NT, 0, s>>>(pd, tl, db, vb);
  else k_divT<3><<<nt, NT, 0, s>>>(pd, tl, db, vb);
  return post();
}

hipError_t launch_epilogue(int ndim, int nt, const EpiArgs& a, hipStream_t s) {
  if (ndim == 2) k_epilogue<2><<<nt, NT, 0, s>>>(a);
  else k_epilogue<3><<<nt, NT, 0, s>>>(a);
  return post();
}

hipError_t launch_finalize(int npairs, const PairDev* pd, const float* red_reg, const float* red_ssd,
                           hipStream_t s) {
  k_finalize<<<npairs, NT, 0, s>>>(pd, red_reg, red_ssd);
  return post();
}

}  // namespace shoot
