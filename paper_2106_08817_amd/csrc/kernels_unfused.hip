// Per-pair unfused path: one launch per primitive, one voxel per thread, all
// intermediates through global memory, full trajectory stored. Same
// arithmetic as the batched path (same foot-point rule, same taps), none of
// its fusion, batching, LDS tiling or graph capture.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device_common.h"
#include "unfused.h"

namespace shoot {
namespace unfused {

struct Geo {
  int nz, ny, nx, N;
};

struct Taps {
  int r;
  float w[2 * RMAX + 1];
};

__device__ __forceinline__ void coords(const Geo& g, int idx, int q[3]) {
  q[2] = idx % g.nx;
  q[1] = (idx / g.nx) % g.ny;
  q[0] = idx / (g.nx * g.ny);
}

__device__ __forceinline__ void geo_axes(const Geo& g, int n[3], int s[3]) {
  n[0] = g.nz; n[1] = g.ny; n[2] = g.nx;
  s[0] = g.nx * g.ny; s[1] = g.nx; s[2] = 1;
}

#define UF_INDEX                                      \
  const int idx = blockIdx.x * NT + threadIdx.x;      \
  if (idx >= g.N) return;

// G_c = D_c F
template <int NDIM>
__global__ __launch_bounds__(NT) void u_grad(Geo g, const float* __restrict__ F, float* __restrict__ G) {
  UF_INDEX
  int q[3], n[3], s[3];
  coords(g, idx, q);
  geo_axes(g, n, s);
#pragma unroll
  for (int c = 0; c < NDIM; ++c) {
    const int a = 3 - NDIM + c;
    G[c * g.N + idx] = 0.5f * (F[idx + up(q[a], n[a], s[a])] - F[idx - dn(q[a], s[a])]);
  }
}

// M_c = z G_c
template <int NDIM>
__global__ __launch_bounds__(NT) void u_mul(Geo g, const float* __restrict__ z, const float* __restrict__ G,
                                            float* __restrict__ M) {
  UF_INDEX
  const float zq = z[idx];
#pragma unroll
  for (int c = 0; c < NDIM; ++c) M[c * g.N + idx] = zq * G[c * g.N + idx];
}

// one zero-padded Gaussian pass along geometric axis `a`, every channel
template <int NDIM>
__global__ __launch_bounds__(NT) void u_conv(Geo g, int a, Taps tp, const float* __restrict__ in,
                                             float* __restrict__ out) {
  UF_INDEX
  int q[3], n[3], s[3];
  coords(g, idx, q);
  geo_axes(g, n, s);
  for (int c = 0; c < NDIM; ++c) {
    const float* F = in + c * g.N;
    float acc = 0.f;
    for (int k = -tp.r; k <= tp.r; ++k) {
      const int j = q[a] + k;
      if (j >= 0 && j < n[a]) acc = fmaf(tp.w[k + tp.r], F[idx + k * s[a]], acc);
    }
    out[c * g.N + idx] = acc;
  }
}

// out = -in (+ escale * extra)
template <int NDIM>
__global__ __launch_bounds__(NT) void u_neg(Geo g, const float* __restrict__ in, float* __restrict__ out,
                                            const float* __restrict__ extra, float escale) {
  UF_INDEX
#pragma unroll
  for (int c = 0; c < NDIM; ++c) {
    float o = -in[c * g.N + idx];
    if (extra) o = fmaf(escale, extra[c * g.N + idx], o);
    out[c * g.N + idx] = o;
  }
}

// DIV = sum_c D_c V_c
template <int NDIM>
__global__ __launch_bounds__(NT) void u_div(Geo g, const float* __restrict__ V, float* __restrict__ D) {
  UF_INDEX
  int q[3], n[3], s[3];
  coords(g, idx, q);
  geo_axes(g, n, s);
  float d = 0.f;
#pragma unroll
  for (int c = 0; c < NDIM; ++c) {
    const int a = 3 - NDIM + c;
    const float* Vc = V + c * g.N;
    d += 0.5f * (Vc[idx + up(q[a], n[a], s[a])] - Vc[idx - dn(q[a], s[a])]);
  }
  D[idx] = d;
}

template <int NDIM>
__device__ __forceinline__ void feet(const Geo& g, float dt, const float* V, int idx, Axis ax[3]) {
  int q[3], n[3], s[3];
  coords(g, idx, q);
  geo_axes(g, n, s);
#pragma unroll
  for (int c = 0; c < NDIM; ++c) {
    const int a = 3 - NDIM + c;
    ax[a] = foot_axis(q[a], -dt * V[c * g.N + idx], n[a]);
  }
  if (NDIM == 2) { ax[0].i = 0; ax[0].f = 0.f; ax[0].live = 0.f; }
}

// out = Interp(F; q - dt V(q))
template <int NDIM>
__global__ __launch_bounds__(NT) void u_gather(Geo g, float dt, const float* __restrict__ V,
                                               const float* __restrict__ F, float* __restrict__ out) {
  UF_INDEX
  Axis ax[3];
  feet<NDIM>(g, dt, V, idx, ax);
  const int sxy = g.nx * g.ny;
  const int c0 = ax[0].i * sxy + ax[1].i * g.nx + ax[2].i;
  const float wy0 = 1.f - ax[1].f, wy1 = ax[1].f, wx0 = 1.f - ax[2].f, wx1 = ax[2].f;
  float v = wy0 * (wx0 * F[c0] + wx1 * F[c0 + 1]) + wy1 * (wx0 * F[c0 + g.nx] + wx1 * F[c0 + g.nx + 1]);
  if (NDIM == 3) {
    const int c1 = c0 + sxy;
    const float v1 =
        wy0 * (wx0 * F[c1] + wx1 * F[c1 + 1]) + wy1 * (wx0 * F[c1 + g.nx] + wx1 * F[c1 + g.nx + 1]);
    v = (1.f - ax[0].f) * v + ax[0].f * v1;
  }
  out[idx] = v;
}

__global__ __launch_bounds__(NT) void u_update(Geo g, float rdt, float dt, const float* __restrict__ Ih,
                                               const float* __restrict__ zh, const float* __restrict__ D,
                                               float* __restrict__ I1, float* __restrict__ z1) {
  UF_INDEX
  I1[idx] = fmaf(rdt, zh[idx], Ih[idx]);
  z1[idx] = zh[idx] * (1.f - dt * D[idx]);
}

// per-block partials of -<M, V> + rho |p0|^2
template <int NDIM>
__global__ __launch_bounds__(NT) void u_reg(Geo g, const float* __restrict__ M, const float* __restrict__ V,
                                            const float* __restrict__ p0, float rho, float* __restrict__ part) {
  __shared__ float sh[NT / 64];
  const int idx = blockIdx.x * NT + threadIdx.x;
  float v = 0.f;
  if (idx < g.N) {
    float mv = 0.f;
#pragma unroll
    for (int c = 0; c < NDIM; ++c) mv = fmaf(M[c * g.N + idx], V[c * g.N + idx], mv);
    v = rho * p0[idx] * p0[idx] - mv;
  }
  const float s = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// R = I - J, per-block partials of R^2 / 2
__global__ __launch_bounds__(NT) void u_resid(Geo g, const float* __restrict__ I, const float* __restrict__ J,
                                              float* __restrict__ R, float* __restrict__ part) {
  __shared__ float sh[NT / 64];
  const int idx = blockIdx.x * NT + threadIdx.x;
  float v = 0.f;
  if (idx < g.N) {
    const float r = I[idx] - J[idx];
    if (R) R[idx] = r;
    v = 0.5f * r * r;
  }
  const float s = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(NT) void u_cost(const float* __restrict__ pssd, const float* __restrict__ preg, int nb,
                                             float lam, float* __restrict__ out) {
  __shared__ float sh[NT / 64];
  float a = 0.f, b = 0.f;
  for (int i = threadIdx.x; i < nb; i += NT) {
    a += pssd ? pssd[i] : 0.f;
    b += preg[i];
  }
  const float data = block_sum(a, sh);
  const float reg = block_sum(b, sh);
  if (threadIdx.x == 0) {
    out[0] = data + lam * reg;
    out[1] = data;
    out[2] = lam * reg;
  }
}

__global__ __launch_bounds__(NT) void u_fill(float* __restrict__ p, int n, float v) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(NT) void u_copy(float* __restrict__ d, const float* __restrict__ s, int n) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// zh_bar = rho dt Ib + (1 - dt DIV) zb ; div_bar = -dt zh zb
__global__ __launch_bounds__(NT) void u_zhbar(Geo g, float rdt, float dt, const float* __restrict__ Ib,
                                              const float* __restrict__ zb, const float* __restrict__ D,
                                              const float* __restrict__ zh, float* __restrict__ zhb,
                                              float* __restrict__ db) {
  UF_INDEX
  zhb[idx] = fmaf(rdt, Ib[idx], (1.f - dt * D[idx]) * zb[idx]);
  db[idx] = -dt * zh[idx] * zb[idx];
}

// out += Interp^T(a) (global atomics)
template <int NDIM>
__global__ __launch_bounds__(NT) void u_scatter(Geo g, float dt, const float* __restrict__ V,
                                                const float* __restrict__ a, float* __restrict__ out) {
  UF_INDEX
  Axis ax[3];
  feet<NDIM>(g, dt, V, idx, ax);
  const int sxy = g.nx * g.ny;
  const float val = a[idx];
  for (int bz = 0; bz < (NDIM == 3 ? 2 : 1); ++bz)
    for (int by = 0; by < 2; ++by)
      for (int bx = 0; bx < 2; ++bx) {
        const float w = (NDIM == 3 ? (bz ? ax[0].f : 1.f - ax[0].f) : 1.f) * (by ? ax[1].f : 1.f - ax[1].f) *
                        (bx ? ax[2].f : 1.f - ax[2].f);
        const int c = (ax[0].i + bz) * sxy + (ax[1].i + by) * g.nx + ax[2].i + bx;
        unsafeAtomicAdd(out + c, w * val);
      }
}

// vbar_c = -dt (Ib dInterp(I)/dy_c + zhb dInterp(z)/dy_c)
template <int NDIM>
__global__ __launch_bounds__(NT) void u_ygrad(Geo g, float dt, const float* __restrict__ V,
                                              const float* __restrict__ I, const float* __restrict__ Z,
                                              const float* __restrict__ Ib, const float* __restrict__ zhb,
                                              float* __restrict__ vb) {
  UF_INDEX
  Axis ax[3];
  feet<NDIM>(g, dt, V, idx, ax);
  const int sxy = g.nx * g.ny;
  float gI[3] = {0.f, 0.f, 0.f}, gZ[3] = {0.f, 0.f, 0.f};
  for (int bz = 0; bz < (NDIM == 3 ? 2 : 1); ++bz)
    for (int by = 0; by < 2; ++by)
      for (int bx = 0; bx < 2; ++bx) {
        const int c = (ax[0].i + bz) * sxy + (ax[1].i + by) * g.nx + ax[2].i + bx;
        const float wz = NDIM == 3 ? (bz ? ax[0].f : 1.f - ax[0].f) : 1.f;
        const float wy = by ? ax[1].f : 1.f - ax[1].f;
        const float wx = bx ? ax[2].f : 1.f - ax[2].f;
        const float dz = (bz ? 1.f : -1.f) * wy * wx;
        const float dy = (by ? 1.f : -1.f) * wz * wx;
        const float dxw = (bx ? 1.f : -1.f) * wz * wy;
        gI[0] = fmaf(dz, I[c], gI[0]); gZ[0] = fmaf(dz, Z[c], gZ[0]);
        gI[1] = fmaf(dy, I[c], gI[1]); gZ[1] = fmaf(dy, Z[c], gZ[1]);
        gI[2] = fmaf(dxw, I[c], gI[2]); gZ[2] = fmaf(dxw, Z[c], gZ[2]);
      }
  const float ib = Ib[idx], zb = zhb[idx];
#pragma unroll
  for (int c = 0; c < NDIM; ++c) {
    const int a = 3 - NDIM + c;
    vb[c * g.N + idx] = -dt * ax[a].live * fmaf(ib, gI[a], zb * gZ[a]);
  }
}

__device__ __forceinline__ float dT1(const float* g, int idx, int j, int n, int s) {
  if (j == 0) return -0.5f * (g[idx] + g[idx + s]);
  if (j == n - 1) return 0.5f * (g[idx - s] + g[idx]);
  return 0.5f * (g[idx - s] - g[idx + s]);
}

// vbar_c += D_c^T db
template <int NDIM>
__global__ __launch_bounds__(NT) void u_divT(Geo g, const float* __restrict__ db, float* __restrict__ vb) {
  UF_INDEX
  int q[3], n[3], s[3];
  coords(g, idx, q);
  geo_axes(g, n, s);
#pragma unroll
  for (int c = 0; c < NDIM; ++c) {
    const int a = 3 - NDIM + c;
    vb[c * g.N + idx] += dT1(db, idx, q[a], n[a], s[a]);
  }
}

// zbar = sz + sum_c mb_c G_c
template <int NDIM>
__global__ __launch_bounds__(NT) void u_adj_z(Geo g, const float* __restrict__ sz, const float* __restrict__ mb,
                                              const float* __restrict__ G, float* __restrict__ zbar) {
  UF_INDEX
  float v = sz[idx];
#pragma unroll
  for (int c = 0; c < NDIM; ++c) v = fmaf(mb[c * g.N + idx], G[c * g.N + idx], v);
  zbar[idx] = v;
}

// Ibar = si + sum_c D_c^T zm_c
template <int NDIM>
__global__ __launch_bounds__(NT) void u_adj_I(Geo g, const float* __restrict__ si, const float* __restrict__ zm,
                                              float* __restrict__ Ibar) {
  UF_INDEX
  int q[3], n[3], s[3];
  coords(g, idx, q);
  geo_axes(g, n, s);
  float v = si[idx];
#pragma unroll
  for (int c = 0; c < NDIM; ++c) {
    const int a = 3 - NDIM + c;
    v += dT1(zm + c * g.N, idx, q[a], n[a], s[a]);
  }
  Ibar[idx] = v;
}

// grad = zbar + c2 p0
__global__ __launch_bounds__(NT) void u_gradout(Geo g, const float* __restrict__ zbar, const float* __restrict__ p0,
                                                float c2, float* __restrict__ out) {
  UF_INDEX
  out[idx] = fmaf(c2, p0[idx], zbar[idx]);
}

// ---------------------------------------------------------------------------- host

struct Plan {
  std::vector<shoot_pair> pairs;
  int T = 1, ndim = 2;
  long long nmax = 0;
  size_t bytes = 0;
  char* ws = nullptr;
  // byte offsets
  size_t o_st, o_vs, o_g, o_m, o_u1, o_u2, o_div, o_ih, o_zh, o_ab, o_sc, o_vb, o_db, o_zhb, o_zm, o_pssd, o_preg;
};

static size_t al(size_t v) { return (v + 255) / 256 * 256; }

Plan* create(const shoot_pair* pairs, int n, int T) {
  Plan* p = new (std::nothrow) Plan();
  if (!p) return nullptr;
  p->pairs.assign(pairs, pairs + n);
  p->T = T;
  p->ndim = pairs[0].ndim;
  for (int i = 0; i < n; ++i) {
    long long N = 1;
    for (int a = 0; a < pairs[i].ndim; ++a) N *= pairs[i].shape[a];
    p->nmax = std::max(p->nmax, N);
  }
  const size_t f = sizeof(float) * (size_t)p->nmax;
  const size_t d = (size_t)p->ndim;
  const size_t nb = (size_t)((p->nmax + NT - 1) / NT);
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = al(o + b); return r; };
  p->o_st = take((size_t)(T + 1) * 2 * f);
  p->o_vs = take((size_t)T * d * f);
  p->o_g = take(d * f);
  p->o_m = take(d * f);
  p->o_u1 = take(d * f);
  p->o_u2 = take(d * f);
  p->o_div = take(f);
  p->o_ih = take(f);
  p->o_zh = take(f);
  p->o_ab = take(2 * 2 * f);
  p->o_sc = take(2 * f);
  p->o_vb = take(d * f);
  p->o_db = take(f);
  p->o_zhb = take(f);
  p->o_zm = take(d * f);
  p->o_pssd = take(nb * sizeof(float));
  p->o_preg = take(nb * sizeof(float));
  p->bytes = o;
  return p;
}

size_t workspace_bytes(const Plan* p) { return p->bytes; }

hipError_t bind(Plan* p, char* ws, hipStream_t) {
  p->ws = ws;
  return hipSuccess;
}

void destroy(Plan* p) { delete p; }

#define UFCHK()                                  \
  do {                                           \
    hipError_t e_ = hipGetLastError();           \
    if (e_ != hipSuccess) return e_;             \
  } while (0)

template <int NDIM>
static hipError_t run_pair(Plan* p, const shoot_pair& q, int op, hipStream_t s) {
  Geo g;
  g.nz = NDIM == 3 ? q.shape[0] : 1;
  g.ny = q.shape[NDIM - 2];
  g.nx = q.shape[NDIM - 1];
  g.N = g.nz * g.ny * g.nx;
  const int T = p->T;
  const float dt = (float)(1.0 / (double)T);
  const float rdt = q.rho * dt;
  Taps tp;
  tp.r = (int)std::floor(3.0 * (double)q.sigma);
  {
    double w[2 * RMAX + 1], sum = 0.0;
    for (int k = -tp.r; k <= tp.r; ++k) {
      w[k + tp.r] = std::exp(-(double)k * k / (2.0 * (double)q.sigma * (double)q.sigma));
      sum += w[k + tp.r];
    }
    for (int k = 0; k <= 2 * tp.r; ++k) tp.w[k] = (float)(w[k] / sum);
  }
  const int nb = (g.N + NT - 1) / NT;
  const size_t N = (size_t)g.N;
  char* b = p->ws;
  float* st = (float*)(b + p->o_st);
  float* vs = (float*)(b + p->o_vs);
  float* G = (float*)(b + p->o_g);
  float* M = (float*)(b + p->o_m);
  float* U1 = (float*)(b + p->o_u1);
  float* U2 = (float*)(b + p->o_u2);
  float* DIV = (float*)(b + p->o_div);
  float* IH = (float*)(b + p->o_ih);
  float* ZH = (float*)(b + p->o_zh);
  float* AB = (float*)(b + p->o_ab);
  float* SC = (float*)(b + p->o_sc);
  float* VB = (float*)(b + p->o_vb);
  float* DB = (float*)(b + p->o_db);
  float* ZHB = (float*)(b + p->o_zhb);
  float* ZM = (float*)(b + p->o_zm);
  float* pssd = (float*)(b + p->o_pssd);
  float* preg = (float*)(b + p->o_preg);
  auto I_at = [&](int t) { return st + (size_t)t * 2 * N; };
  auto Z_at = [&](int t) { return st + (size_t)t * 2 * N + N; };
  auto V_at = [&](int t) { return vs + (size_t)t * NDIM * N; };

  // -G applied to the d channels of `in` -> out (extra: out += escale * extra)
  auto smooth_neg = [&](const float* in, float* out, const float* extra, float escale) -> hipError_t {
    const float* src = in;
    float* bufs[2] = {U1, U2};
    for (int a = 3 - NDIM, k = 0; a < 3; ++a, ++k) {
      u_conv<NDIM><<<nb, NT, 0, s>>>(g, a, tp, src, bufs[k & 1]);
      UFCHK();
      src = bufs[k & 1];
    }
    u_neg<NDIM><<<nb, NT, 0, s>>>(g, src, out, extra, escale);
    UFCHK();
    return hipSuccess;
  };

  u_copy<<<nb, NT, 0, s>>>(I_at(0), q.image, g.N); UFCHK();
  u_copy<<<nb, NT, 0, s>>>(Z_at(0), q.p0, g.N); UFCHK();
  for (int t = 0; t < T; ++t) {
    u_grad<NDIM><<<nb, NT, 0, s>>>(g, I_at(t), G); UFCHK();
    u_mul<NDIM><<<nb, NT, 0, s>>>(g, Z_at(t), G, M); UFCHK();
    hipError_t e = smooth_neg(M, V_at(t), nullptr, 0.f);
    if (e != hipSuccess) return e;
    if (t == 0) { u_reg<NDIM><<<nb, NT, 0, s>>>(g, M, V_at(0), Z_at(0), q.rho, preg); UFCHK(); }
    u_div<NDIM><<<nb, NT, 0, s>>>(g, V_at(t), DIV); UFCHK();
    u_gather<NDIM><<<nb, NT, 0, s>>>(g, dt, V_at(t), I_at(t), IH); UFCHK();
    u_gather<NDIM><<<nb, NT, 0, s>>>(g, dt, V_at(t), Z_at(t), ZH); UFCHK();
    u_update<<<nb, NT, 0, s>>>(g, rdt, dt, IH, ZH, DIV, I_at(t + 1), Z_at(t + 1)); UFCHK();
  }
  if (q.out_image) { u_copy<<<nb, NT, 0, s>>>(q.out_image, I_at(T), g.N); UFCHK(); }
  if (q.out_momentum) { u_copy<<<nb, NT, 0, s>>>(q.out_momentum, Z_at(T), g.N); UFCHK(); }
  float* R = AB + (size_t)(T & 1) * 2 * N;  // Ibar_T
  if (q.target) {
    u_resid<<<nb, NT, 0, s>>>(g, I_at(T), q.target, op == 2 ? R : nullptr, pssd); UFCHK();
  }
  if (q.out_cost && (q.target || op != 0)) {
    u_cost<<<1, NT, 0, s>>>(q.target ? pssd : nullptr, preg, nb, q.lambda, q.out_cost); UFCHK();
  }
  if (op != 2) return hipSuccess;
  u_fill<<<nb, NT, 0, s>>>(R + N, g.N, 0.f); UFCHK();  // zbar_T = 0
  for (int t = T - 1; t >= 0; --t) {
    const float* Ib = AB + (size_t)((t + 1) & 1) * 2 * N;
    const float* zb = Ib + N;
    float* Io = AB + (size_t)(t & 1) * 2 * N;
    float* zo = Io + N;
    u_div<NDIM><<<nb, NT, 0, s>>>(g, V_at(t), DIV); UFCHK();
    u_gather<NDIM><<<nb, NT, 0, s>>>(g, dt, V_at(t), Z_at(t), ZH); UFCHK();
    u_zhbar<<<nb, NT, 0, s>>>(g, rdt, dt, Ib, zb, DIV, ZH, ZHB, DB); UFCHK();
    u_fill<<<(2 * g.N + NT - 1) / NT, NT, 0, s>>>(SC, 2 * g.N, 0.f); UFCHK();
    u_scatter<NDIM><<<nb, NT, 0, s>>>(g, dt, V_at(t), Ib, SC); UFCHK();
    u_scatter<NDIM><<<nb, NT, 0, s>>>(g, dt, V_at(t), ZHB, SC + N); UFCHK();
    u_ygrad<NDIM><<<nb, NT, 0, s>>>(g, dt, V_at(t), I_at(t), Z_at(t), Ib, ZHB, VB); UFCHK();
    u_divT<NDIM><<<nb, NT, 0, s>>>(g, DB, VB); UFCHK();
    hipError_t e = smooth_neg(VB, VB, t == 0 ? V_at(0) : nullptr, -2.f * q.lambda);
    if (e != hipSuccess) return e;
    u_grad<NDIM><<<nb, NT, 0, s>>>(g, I_at(t), G); UFCHK();
    u_adj_z<NDIM><<<nb, NT, 0, s>>>(g, SC + N, VB, G, zo); UFCHK();
    if (t > 0) {
      u_mul<NDIM><<<nb, NT, 0, s>>>(g, Z_at(t), VB, ZM); UFCHK();
      u_adj_I<NDIM><<<nb, NT, 0, s>>>(g, SC, ZM, Io); UFCHK();
    } else {
      u_gradout<<<nb, NT, 0, s>>>(g, zo, q.p0, 2.f * q.lambda * q.rho, q.out_grad); UFCHK();
    }
  }
  return hipSuccess;
}

hipError_t run(Plan* p, int op, hipStream_t s) {
  for (const shoot_pair& q : p->pairs) {
    hipError_t e = p->ndim == 2 ? run_pair<2>(p, q, op, s) : run_pair<3>(p, q, op, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace unfused
}  // namespace shoot
