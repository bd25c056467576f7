// gfx950 Gaussian pass along x (first pass of v = -G m and of mbar = -G vbar)
// on the fp32 matrix cores, as a banded Toeplitz product.
//
// Along a row, out[x] = sum_t w[t] row[x + t] (t = 0..2r; the row staged with
// r zeros in front, zero padding of G). For 16 outputs x0 + m, m < 16, and
// K = 4 KB >= 16 + 2r staged inputs x0 + k, this is D = A B with the band
// A[m][k] = w[k - m] (zero outside 0 <= k - m <= 2r) and B[k][n] = row_n[x0 + k]
// for 16 rows n (rows of every channel of the tile, stacked). One
// v_mfma_f32_16x16x4f32 consumes four k; A is the same for every tile of a
// pair and stays in registers. Lane l holds A[l % 16][l / 16], B[l / 16][l % 16]
// and D[4 (l / 16) + j][l % 16], j < 4: four consecutive outputs of one row.
#include "kernels.h"
#include "device_common.h"

namespace shoot {

namespace {

typedef float f4m __attribute__((ext_vector_type(4)));

constexpr int KB_MAX = (16 + 2 * RMAX + 3) / 4;

__device__ __forceinline__ int mfma_kb(int r) { return (16 + 2 * r + 3) / 4; }
// staged row stride: every k of every column tile, rounded up to 4 mod 8
// floats so that the 16 rows a B read spans fall in distinct banks
__device__ __forceinline__ int mfma_row(int nx, int r) {
  const int need = 16 * ((nx + 15) / 16) + 4 * mfma_kb(r);
  return need + ((12 - (need & 7)) & 7);
}

}  // namespace

template <int NDIM, bool GRADMUL>
__global__ __launch_bounds__(NT) void k_xpass_mfma(const PairDev* __restrict__ pd, const Tile* __restrict__ tl,
                                                   const float* __restrict__ src, float* __restrict__ dst) {
  extern __shared__ vf4 smem4[];
  float* lds = reinterpret_cast<float*>(smem4);
  const Tile t = tl[xcd_tile(gridDim.x)];
  const PairDev& P = pd[t.pair];
  if (!P.active) return;
  const int nx = P.nx, ny = P.ny, nz = P.nz, r = P.r;
  const unsigned N = (unsigned)P.N;
  const int row0 = t.a, nrows = t.b;
  const int LM = mfma_row(nx, r), KB = mfma_kb(r);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // the band of the pair's taps, A[m][k] for m = lane % 16, k = 4 kb + lane / 16
  float a[KB_MAX];
#pragma unroll
  for (int kb = 0; kb < KB_MAX; ++kb) {
    const int tt = 4 * kb + (lane >> 4) - (lane & 15);
    a[kb] = (kb < KB && tt >= 0 && tt < WPAD) ? P.w[tt] : 0.f;
  }

  // fill: four consecutive x per 16-byte access, the central difference's x
  // neighbours by the row shifted one element (clamped at the row's ends);
  // staged row (c, rl) at (c nrows + rl) LM, x at column r + x
  const float* __restrict__ I = src + (GRADMUL ? 2 : NDIM) * P.off;
  const float* __restrict__ Z = I + N;
  const int G = nx >> 2;
  const int ni = nrows * G;
  for (int i0 = threadIdx.x; i0 < ni; i0 += 2 * NT) {
    vf4 m[2][NDIM];
    int lrow[2];
    // a wave whose items all lie past the tile skips the batch slot
    const int wfirst = __builtin_amdgcn_readfirstlane(i0 - (int)(threadIdx.x & 63));
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (wfirst + u * NT >= ni) {
        lrow[u] = -1;
        continue;
      }
      const int i = min(i0 + u * NT, ni - 1);
      const int rl = i / G;
      const int x = 4 * (i - rl * G);
      lrow[u] = i0 + u * NT < ni ? rl * LM + r + x : -1;
      const int row = row0 + rl;
      const unsigned idx = (unsigned)(row * nx + x);
      if (GRADMUL) {
        const int y = row % ny;
        const unsigned yu = (unsigned)up(y, ny, nx), yd = (unsigned)dn(y, nx);
        const vf4 zc = gld4(Z, idx);
        const vf4 ic = gld4(I, idx);
        const vf4 il = gld4u(I, x > 0 ? idx - 1u : idx);
        const vf4 ir = gld4u(I, x + 4 < nx ? idx + 1u : idx);
        const vf4 iu = gld4(I, idx + yu), id = gld4(I, idx - yd);
        vf4 izu = ic, izd = ic;
        if (NDIM == 3) {
          const int z = row / ny;
          const unsigned zu = (unsigned)up(z, nz, ny * nx), zd = (unsigned)dn(z, ny * nx);
          izu = gld4(I, idx + zu);
          izd = gld4(I, idx - zd);
        }
        const vf4 lm = x > 0 ? il : vf4{ic.x, ic.x, ic.y, ic.z};
        const vf4 rp = x + 4 < nx ? ir : vf4{ic.y, ic.z, ic.w, ic.w};
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
    for (int u = 0; u < 2; ++u) {
      if (lrow[u] < 0) continue;
#pragma unroll
      for (int c = 0; c < NDIM; ++c) {
        float* d = lds + c * nrows * LM + lrow[u];
        d[0] = m[u][c].x; d[1] = m[u][c].y; d[2] = m[u][c].z; d[3] = m[u][c].w;
      }
    }
  }
  // zeros: r columns in front of each staged row, everything behind the row
  const int pad = LM - nx;
  for (int i = threadIdx.x; i < NDIM * nrows * pad; i += NT) {
    const int rr = i / pad;
    const int k = i - rr * pad;
    lds[rr * LM + (k < r ? k : nx + k)] = 0.f;
  }
  __syncthreads();

  // output tiles: 16 columns x 16 stacked rows, two per wave in flight
  const int RC = NDIM * nrows;
  const int CT = (nx + 15) >> 4, NTI = (RC + 15) >> 4;
  const int nout = CT * NTI;
  float* __restrict__ D = dst + NDIM * P.off;
  for (int o0 = wv; o0 < nout; o0 += 2 * (NT / 64)) {
    f4m acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    int base[2], x0[2], nrc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int o = min(o0 + h * (NT / 64), nout - 1);
      const int ct = o % CT, nt = o / CT;
      x0[h] = 16 * ct;
      nrc[h] = 16 * nt + (lane & 15);
      base[h] = min(nrc[h], RC - 1) * LM + x0[h] + (lane >> 4);
    }
#pragma unroll
    for (int kb = 0; kb < KB_MAX; ++kb) {
      if (kb < KB) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kb], lds[base[h] + 4 * kb], acc[h], 0, 0, 0);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (o0 + h * (NT / 64) >= nout || nrc[h] >= RC) continue;
      const int c = nrc[h] / nrows, rl = nrc[h] - c * nrows;
      const int x = x0[h] + 4 * (lane >> 4);
      if (x < nx) {
        const unsigned idx = (unsigned)((row0 + rl) * nx + x);
        gst4(D, c * N + idx, vf4{acc[h][0], acc[h][1], acc[h][2], acc[h][3]});
      }
    }
  }
}

size_t xpass_mfma_lds(int ndim, int nx, int r, int nrows) {
  const int need = 16 * ((nx + 15) / 16) + 4 * ((16 + 2 * r + 3) / 4);
  const int LM = need + ((12 - (need & 7)) & 7);
  return (size_t)ndim * nrows * LM * sizeof(float);
}

hipError_t launch_xpass_mfma(int ndim, bool gradmul, const PairDev* pd, const Tile* tl, int nt, size_t lds,
                             const float* src, float* dst, hipStream_t s) {
  if (ndim == 2) {
    if (gradmul) k_xpass_mfma<2, true><<<nt, NT, lds, s>>>(pd, tl, src, dst);
    else k_xpass_mfma<2, false><<<nt, NT, lds, s>>>(pd, tl, src, dst);
  } else {
    if (gradmul) k_xpass_mfma<3, true><<<nt, NT, lds, s>>>(pd, tl, src, dst);
    else k_xpass_mfma<3, false><<<nt, NT, lds, s>>>(pd, tl, src, dst);
  }
  return hipGetLastError();
}

}  // namespace shoot
