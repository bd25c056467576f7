// gfx950 kernel of the 3-D adjoint of the semi-Lagrangian step, LDS-staged.
//
// For each arrival point q with cotangents (Ib, zb) of (I_{t+1}, z_{t+1})
// (transpose of the forward step of the semi-Lagrangian section):
//   zh_bar = rho dt Ib + (1 - dt div v) zb,   div_bar = -dt zh zb,
//   Ibar_t += Interp^T(Ib),  zbar_t += Interp^T(zh_bar)
//   vbar_c = -dt chi_c (Ib dInterp(I_t)/dy_c + zh_bar dInterp(z_t)/dy_c) + D_c^T div_bar
//
// A block owns a 16 x 8 x 8 tile P of outputs. With D = max |dt v| of the
// pair and step below one voxel, every corner a foot touches lies within one
// voxel of its arrival point, so the block needs the arrival points of P +- 1
// and the fields z_t, I_t and v_t on P +- 2. Those five fields are staged in
// LDS on the tile grown by 2 along y and z and by 4 along x (whole 16-byte
// groups), with 16-byte loads; positions outside the image hold the clamped
// neighbour (replicate border), which is exactly the clamping of the central
// difference.
//
// Phase 1 visits the tile's own points (a thread takes four x four apart,
// which spreads a wave's LDS reads over all banks) and the ring P +- 1 minus
// P, reading velocity, divergence and foot corners from LDS; it keeps per
// point the record (the foot's clamped offset e per axis, Ib, zh_bar) in
// registers, writes div_bar on P +- 1 into LDS, and forms the foot-point part
// of vbar of the own points. After a barrier the records and those vbar parts
// replace the staged fields in LDS. Phase 2 gives a thread four consecutive x
// of one row and forms Interp^T at each as a gather over the 27 arrival points
// q = p - o, |o_a| <= 1, with the weights prod_a hat(e_a(q) - o_a) of linear
// interpolation (each hat scaled by 2 so that it is one operation, the
// records' cotangents by 1/8: exact powers of two); it reads each record of
// its outputs' 3 x 3 x 6 candidates once and applies it to the outputs it
// reaches, in a fixed order, without atomics: deterministic, each output
// written once.
//
// When 1 <= D < 3 voxels every corner of an own point's foot lies in P +- M,
// M = 2 below two voxels and 3 above: the block adds its own points'
// Interp^T with LDS atomics into a box over P +- M (in the records' space)
// and then adds each touched cell of the box with one global float atomic
// into the accumulator that the previous adjoint step (or the last forward
// step) cleared, a fraction of the global atomics of a per-corner scatter.
// Below two voxels the own points' foot corners come from the staged fields,
// above from global memory. When D >= 3 (or a forced global scatter) the own
// points scatter per corner with global float atomics. In all these modes the
// ring points' foot corners come from global memory; velocity and divergence
// still come from LDS. Sums through atomics depend on their order.
#include "kernels.h"
#include "device_common.h"

// Every fused operation is an explicit fmaf (see kernels.hip).
#pragma clang fp contract(off)

namespace shoot {

namespace {

// clamp into [0, n - 1]
__device__ __forceinline__ int clampi3(int v, int n) { return min(max(v, 0), n - 1); }

// (D^T g) at index j of an axis of length n, stride s in the record box:
// 0.5 (g[j-1] - g[j+1]) inside, -0.5 (g[0] + g[1]) at j = 0 and
// 0.5 (g[n-2] + g[n-1]) at j = n - 1 (both neighbours of an output lie in
// the box, so the selects never read outside it).
__device__ __forceinline__ float diffT_box(const float* g, int b, int j, int n, int s) {
  const float c = g[b];
  const float lo = j == 0 ? -c : g[b - s];
  const float hi = j == n - 1 ? -c : g[b + s];
  return 0.5f * (lo - hi);
}

constexpr int AX = ADJ3_X, AY = ADJ3_Y, AZ = ADJ3_Z;
// staged fields: x in [x0 - 4, x0 + AX + 4), y in [y0 - 2, y0 + AY + 2),
// z in [z0 - 2, z0 + AZ + 2); rows of SXW floats, planes padded by four
// floats so that the phase-1 reads of a wave fall in distinct banks
constexpr int SXW = AX + 8, SYW = AY + 4, SZW = AZ + 4;
constexpr int SPL = SXW * SYW + 4;
constexpr int BOXP = SZW * SPL;             // floats per staged field
constexpr int G4 = SXW / 4;                 // 16-byte groups per staged row
constexpr int SROWS = SYW * SZW;            // staged rows per field
constexpr int NF = 5;                       // I, z, v_z, v_y, v_x
constexpr int FI = 0, FZ = 1, FVZ = 2, FVY = 3, FVX = 4;
constexpr int FILL_T = NT / G4 * G4;        // threads of the fill (whole rows)
constexpr int FILL_R = FILL_T / G4;         // rows per fill round
constexpr int FILL_U = (SROWS + FILL_R - 1) / FILL_R;
// records and div_bar on P +- 1 (rows padded to RXP: conflict-free vector reads)
constexpr int RX = AX + 2, RY = AY + 2, RZ = AZ + 2;
constexpr int RXP = AX + 3;
constexpr int NRP = RXP * RY * RZ;
constexpr int NOWN = AX * AY * AZ;
// LDS scatter box over P +- M (M = 2 for 1 <= D < 2, 3 for 2 <= D < 3):
// rows of XW floats, N floats per cotangent field
template <int M>
struct LBox {
  static constexpr int XW = AX + 2 * M, PL = XW * (AY + 2 * M), N = PL * (AZ + 2 * M);
  // box index of the cell (cx, cy, cz) relative to the tile origin
  __device__ static int idx(int cx, int cy, int cz) { return ((cz + M) * (AY + 2 * M) + cy + M) * XW + cx + M; }
};
constexpr int NRING = RX * RY * RZ - NOWN;
constexpr int RING_B = (NRING + NT - 1) / NT;  // ring points per thread (rounds)
// the own points' foot-point parts of vbar, handed from phase 1 to phase 2
constexpr int VQR = 20, VQP = 160, VQN = VQP * AZ;
constexpr int O_ZHB = 4 * NRP, O_VQ = O_ZHB + NRP;
static_assert(AX * AY * AZ == 4 * NT && AX == 16 && AY == 8, "a thread owns four outputs");
static_assert(SXW % 4 == 0 && SPL % 4 == 0 && BOXP % 4 == 0, "16-byte groups");
static_assert(O_VQ % 4 == 0 && VQR % 4 == 0 && VQP % 4 == 0, "16-byte vbar rows");
static_assert(O_VQ + 3 * VQN <= NF * BOXP, "records and vbar parts fit in the staged fields' space");
static_assert(FILL_U % 2 == 0, "fill rounds in pairs");
static_assert(2 * LBox<2>::N % 4 == 0 && 2 * LBox<3>::N % 4 == 0 && 2 * LBox<2>::N <= O_VQ &&
                  2 * LBox<3>::N <= O_VQ,
              "the LDS scatter boxes fit below the vbar parts");

constexpr int SBY = SXW, SBZ = SPL;
__device__ __forceinline__ int bidx(int lx, int ly, int lz) { return (lz + 2) * SPL + (ly + 2) * SXW + lx + 4; }
constexpr int RBY = RXP, RBZ = RXP * RY;
__device__ __forceinline__ int ridx(int lx, int ly, int lz) { return ((lz + 1) * RY + ly + 1) * RXP + lx + 1; }
__device__ __forceinline__ int vqi(int lx, int ly, int lz) { return lz * VQP + ly * VQR + lx; }

// The ring P +- 1 minus P as packed local coordinates (lx + 1) | (ly + 1) << 8
// | (lz + 1) << 16, in raster order.
struct RingTab {
  unsigned c[NRING];
};
constexpr RingTab make_ring() {
  RingTab r{};
  int j = 0;
  for (int lz = -1; lz <= AZ; ++lz)
    for (int ly = -1; ly <= AY; ++ly)
      for (int lx = -1; lx <= AX; ++lx) {
        const bool own = lx >= 0 && lx < AX && ly >= 0 && ly < AY && lz >= 0 && lz < AZ;
        if (!own) r.c[j++] = (unsigned)(lx + 1) | ((unsigned)(ly + 1) << 8) | ((unsigned)(lz + 1) << 16);
      }
  return r;
}
__constant__ const RingTab kRing = make_ring();

// Scaled weight 2 hat(e - O) of a record toward its corner at offset O along
// one axis (|e| < 1): |e| - e, 2 - 2 |e|, |e| + e for O = -1, 0, 1.
template <int O>
__device__ __forceinline__ float tap2(float e) {
  return O < 0 ? fabsf(e) - e : (O == 0 ? fmaf(-2.f, fabsf(e), 2.f) : fabsf(e) + e);
}

// One axis of a foot (the forward step's local form): clamped offset
// e = clamp(d, -q, n - 1 - q) (a NaN d gives 0), cell i = min(q + floor(e),
// n - 2), fraction f = e - floor(e) (1 on the last grid line), live = 1 where
// the coordinate is not clamped.
struct Foot {
  int i;
  float e, f, live;
};
__device__ __forceinline__ Foot foot3(int q, float d, int n) {
  const float qf = (float)q;
  const float lo = -qf, hi = (float)(n - 1) - qf;
  const float m = __builtin_amdgcn_fmed3f(d, lo, hi);
  const float e = m == m ? m : 0.f;
  const float kf = floorf(e);
  const int yb = q + (int)kf;
  const bool top = yb > n - 2;
  Foot F;
  F.i = top ? n - 2 : yb;
  F.f = top ? 1.f : e - kf;
  F.e = e;
  F.live = (d > lo && d < hi) ? 1.f : 0.f;
  return F;
}

struct Rec5 {
  float ex, ey, ez, ib, zhb;
};

// Trilinear value and gradient of the corner values c[bz * 4 + by * 2 + bx]
// at fractions (fz, fy, fx): differences along x interpolated in (y, z),
// values along x interpolated, then along y, then along z.
__device__ __forceinline__ void trilin_grad(const float c[8], float fz, float fy, float fx, float& val, float g[3]) {
  float dx[4], ax[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    dx[k] = c[2 * k + 1] - c[2 * k];
    ax[k] = fmaf(fx, dx[k], c[2 * k]);
  }
  const float gx0 = fmaf(fy, dx[1] - dx[0], dx[0]);
  const float gx1 = fmaf(fy, dx[3] - dx[2], dx[2]);
  g[2] = fmaf(fz, gx1 - gx0, gx0);
  const float dy0 = ax[1] - ax[0], dy1 = ax[3] - ax[2];
  const float ay0 = fmaf(fy, dy0, ax[0]), ay1 = fmaf(fy, dy1, ax[2]);
  g[1] = fmaf(fz, dy1 - dy0, dy0);
  g[0] = ay1 - ay0;
  val = fmaf(fz, g[0], ay0);
}

__device__ __forceinline__ float trilin(const float c[8], float fz, float fy, float fx) {
  float ax[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) ax[k] = fmaf(fx, c[2 * k + 1] - c[2 * k], c[2 * k]);
  const float ay0 = fmaf(fy, ax[1] - ax[0], ax[0]), ay1 = fmaf(fy, ax[3] - ax[2], ax[2]);
  return fmaf(fz, ay1 - ay0, ay0);
}

struct Adj3Ctx {
  int x0, y0, z0, nx, ny, nz;
  unsigned N;
  float dt, rdt;
  const float* __restrict__ I;   // I_t
  const float* __restrict__ Z;   // z_t
  float* __restrict__ SI;        // scatter accumulators (fallback)
  float* __restrict__ SZ;
  const float* st;               // staged fields (LDS)
  float* dbar;                   // div_bar on P +- 1 (LDS)
};

// How a block forms Interp^T (chosen per pair and step from D = max |dt v|):
// a gather over the records in LDS (D < 1), atomics into an LDS box over
// P +- 2 (1 <= D < 2) or P +- 3 (2 <= D < 3) flushed with one global atomic
// per cell, or global atomics per corner (D >= 3, or a forced global
// scatter).
constexpr int M_GATHER = 0, M_LDS2 = 1, M_LDS3 = 2, M_GLOBAL = 3;

// A foot's cell (relative to the tile origin), fractions and cotangents, for
// the LDS scatter.
struct Scat {
  int cx, cy, cz;
  float fx, fy, fz, ib, zhb;
};

// Phase 1 at one arrival point, local coordinates (lx, ly, lz) in P +- 1.
// The point's computations use its coordinates clamped into the image; act
// marks a point inside the image (only those contribute). The foot corners
// come from LDS in M_GATHER, and for own points in M_LDS2 (|e| < 2 keeps them
// within P +- 2); otherwise from global memory. M_GATHER keeps the record,
// M_LDS2 and M_LDS3 the foot's cell and weights, M_GLOBAL scatters an own
// point's Interp^T with global atomics.
template <bool OWN, int MODE>
__device__ __forceinline__ void adj3_point(const Adj3Ctx& C, int lx, int ly, int lz, bool act, float ib, float zb,
                                           Rec5& rec, Scat& sc, float vq[3]) {
  constexpr bool STAGED = MODE == M_GATHER || (MODE == M_LDS2 && OWN);
  const int qx = clampi3(C.x0 + lx, C.nx), qy = clampi3(C.y0 + ly, C.ny), qz = clampi3(C.z0 + lz, C.nz);
  const int b = bidx(qx - C.x0, qy - C.y0, qz - C.z0);
  const float* S = C.st;
  const float vz = S[FVZ * BOXP + b], vy = S[FVY * BOXP + b], vx = S[FVX * BOXP + b];
  float div = 0.5f * (S[FVX * BOXP + b + 1] - S[FVX * BOXP + b - 1]);
  div = fmaf(0.5f, S[FVY * BOXP + b + SBY] - S[FVY * BOXP + b - SBY], div);
  div = fmaf(0.5f, S[FVZ * BOXP + b + SBZ] - S[FVZ * BOXP + b - SBZ], div);
  const Foot ax = foot3(qx, -C.dt * vx, C.nx);
  const Foot ay = foot3(qy, -C.dt * vy, C.ny);
  const Foot az = foot3(qz, -C.dt * vz, C.nz);
  float zc[8], ic[8];
  if (STAGED) {
    const int c0 = bidx(ax.i - C.x0, ay.i - C.y0, az.i - C.z0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int o = c0 + (k >> 2) * SBZ + ((k >> 1) & 1) * SBY + (k & 1);
      zc[k] = S[FZ * BOXP + o];
      if (OWN) ic[k] = S[FI * BOXP + o];
    }
  } else {
    const unsigned sxy = (unsigned)(C.nx * C.ny);
    const unsigned c0 = (unsigned)((az.i * C.ny + ay.i) * C.nx + ax.i);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const unsigned o = c0 + (unsigned)(k >> 2) * sxy + (unsigned)(((k >> 1) & 1) * C.nx + (k & 1));
      zc[k] = gld(C.Z, o);
      if (OWN) ic[k] = gld(C.I, o);
    }
  }
  const float zhb = fmaf(C.rdt, ib, fmaf(-C.dt, div, 1.f) * zb);
  float zh;
  if (OWN) {
    float gZ[3], gI[3], ih;
    trilin_grad(zc, az.f, ay.f, ax.f, zh, gZ);
    trilin_grad(ic, az.f, ay.f, ax.f, ih, gI);
    (void)ih;
    vq[2] = -C.dt * ax.live * fmaf(ib, gI[2], zhb * gZ[2]);
    vq[1] = -C.dt * ay.live * fmaf(ib, gI[1], zhb * gZ[1]);
    vq[0] = -C.dt * az.live * fmaf(ib, gI[0], zhb * gZ[0]);
  } else {
    zh = trilin(zc, az.f, ay.f, ax.f);
  }
  if (act) C.dbar[ridx(lx, ly, lz)] = -C.dt * zh * zb;
  if (MODE == M_GATHER) {
    // cotangents scaled by 1/8 for the scaled hats of the gather
    rec.ex = act ? ax.e : 0.f;
    rec.ey = act ? ay.e : 0.f;
    rec.ez = act ? az.e : 0.f;
    rec.ib = act ? 0.125f * ib : 0.f;
    rec.zhb = act ? 0.125f * zhb : 0.f;
  } else if ((MODE == M_LDS2 || MODE == M_LDS3) && OWN) {
    sc.cx = ax.i - C.x0; sc.cy = ay.i - C.y0; sc.cz = az.i - C.z0;
    sc.fx = ax.f; sc.fy = ay.f; sc.fz = az.f;
    sc.ib = act ? ib : 0.f;
    sc.zhb = act ? zhb : 0.f;
  } else if (MODE == M_GLOBAL && OWN && act) {
    const float wz[2] = {1.f - az.f, az.f}, wy[2] = {1.f - ay.f, ay.f}, wx[2] = {1.f - ax.f, ax.f};
    const unsigned sxy = (unsigned)(C.nx * C.ny);
    const unsigned c0 = (unsigned)((az.i * C.ny + ay.i) * C.nx + ax.i);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int bz = k >> 2, by = (k >> 1) & 1, bx = k & 1;
      const float w = wz[bz] * wy[by] * wx[bx];
      const unsigned o = c0 + (unsigned)bz * sxy + (unsigned)(by * C.nx + bx);
      unsafeAtomicAdd(C.SI + o, w * ib);
      unsafeAtomicAdd(C.SZ + o, w * zhb);
    }
  }
}

// Interp^T of the own points (cells and weights in osc) into an LDS box over
// P +- M, both cotangent fields side by side in the records' space, then one
// global atomic per touched cell of the box into the accumulator the previous
// step cleared. Called by the whole block.
template <int M>
__device__ __forceinline__ void lds_scatter(const Adj3Ctx& C, vf4* stage4, const Scat osc[4]) {
  using Bx = LBox<M>;
  float* acc = reinterpret_cast<float*>(stage4);
  for (int i = threadIdx.x; i < 2 * Bx::N / 4; i += NT) stage4[i] = vf4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const Scat& q = osc[k];
    if (q.ib == 0.f && q.zhb == 0.f) continue;
    const float wz[2] = {1.f - q.fz, q.fz}, wy[2] = {1.f - q.fy, q.fy}, wx[2] = {1.f - q.fx, q.fx};
    const int c0 = Bx::idx(q.cx, q.cy, q.cz);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int bz = c >> 2, by = (c >> 1) & 1, bx = c & 1;
      const float w = wz[bz] * wy[by] * wx[bx];
      const int o = c0 + bz * Bx::PL + by * Bx::XW + bx;
      atomicAdd(acc + o, w * q.ib);
      atomicAdd(acc + Bx::N + o, w * q.zhb);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < Bx::N; i += NT) {
    const int lz = i / Bx::PL, rem = i - Bx::PL * (i / Bx::PL), ly = rem / Bx::XW, lx = rem - Bx::XW * (rem / Bx::XW);
    const int x = C.x0 - M + lx, y = C.y0 - M + ly, z = C.z0 - M + lz;
    if (x < 0 || x >= C.nx || y < 0 || y >= C.ny || z < 0 || z >= C.nz) continue;
    const unsigned o = (unsigned)((z * C.ny + y) * C.nx + x);
    const float a = acc[i], b = acc[Bx::N + i];
    if (a != 0.f) unsafeAtomicAdd(C.SI + o, a);
    if (b != 0.f) unsafeAtomicAdd(C.SZ + o, b);
  }
}

}  // namespace

__global__ __launch_bounds__(NT, 2) void k_adv_adj3(const PairDev* __restrict__ pd, const Tile* __restrict__ tla,
                                                    const float* __restrict__ Vg, const float* __restrict__ stg,
                                                    const float* __restrict__ abg, float* __restrict__ scg,
                                                    float* __restrict__ vbg, AdjArgs A) {
  __shared__ vf4 stage4[NF * BOXP / 4];
  __shared__ float dbar[NRP];
  float* stage = reinterpret_cast<float*>(stage4);
  const Tile tl = tla[xcd_tile(gridDim.x)];
  const PairDev& P = pd[tl.pair];
  if (!P.active) return;
  Adj3Ctx C;
  C.x0 = tl.a; C.y0 = tl.b; C.z0 = tl.c;
  C.nx = P.nx; C.ny = P.ny; C.nz = P.nz;
  C.N = (unsigned)P.N;
  C.dt = P.dt; C.rdt = P.rho * P.dt;
  const float* __restrict__ V = Vg + 3 * P.off;
  C.I = stg + 2 * P.off;
  C.Z = C.I + C.N;
  const float* __restrict__ AB = abg + 2 * P.off;
  C.SI = scg + 2 * P.off;
  C.SZ = C.SI + C.N;
  C.st = stage;
  C.dbar = dbar;
  float* __restrict__ VB = vbg + 3 * P.off;
  const int nx = C.nx, ny = C.ny, nz = C.nz;
  const unsigned N = C.N;
  const float D = __uint_as_float(A.dmax[(long long)tl.pair * A.T + A.t]);
  const bool gmode = !A.force_global && D < 1.f;
  const bool lmode2 = !A.force_global && !gmode && D < 2.f;
  const bool lmode3 = !A.force_global && !gmode && !lmode2 && D < 3.f;
  const bool vec = (nx & 3) == 0;

  const int gx = threadIdx.x & 3, oly = (threadIdx.x >> 2) & (AY - 1), olz = threadIdx.x >> 5;
  const int oqy = C.y0 + oly, oqz = C.z0 + olz;
  const bool orow = oqy < ny && oqz < nz;
  const unsigned orowi = (unsigned)((min(oqz, nz - 1) * ny + min(oqy, ny - 1)) * nx);

  // phase-1 own points: x = gx + 4k; their cotangents
  float ib[4], zb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned o = orowi + (unsigned)min(C.x0 + gx + 4 * k, nx - 1);
    ib[k] = gld(AB, o);
    zb[k] = gld(AB, N + o);
  }
  // the ring points' cotangents (slots past the ring load the last point's
  // and are never used: skipping them per wave measured slower, the branch
  // splitting the batch of loads)
  float rib[RING_B], rzb[RING_B];
  unsigned rc[RING_B];
#pragma unroll
  for (int u = 0; u < RING_B; ++u) {
    rc[u] = kRing.c[min((int)threadIdx.x + u * NT, NRING - 1)];
    const int lx = (int)(rc[u] & 255u) - 1, ly = (int)((rc[u] >> 8) & 255u) - 1, lz = (int)(rc[u] >> 16) - 1;
    const unsigned o =
        (unsigned)((clampi3(C.z0 + lz, nz) * ny + clampi3(C.y0 + ly, ny)) * nx + clampi3(C.x0 + lx, nx));
    rib[u] = gld(AB, o);
    rzb[u] = gld(AB, N + o);
  }

  // staging: a fill thread takes one 16-byte group g of a staged row and the
  // same group of rows FILL_R apart; the row's global offset serves all five
  // fields (rows clamped into the image; groups left or right of the image
  // hold the row's first or last value); a wave whose rows of a round all lie
  // past the box skips that round
  {
    const float* F[NF] = {C.I, C.Z, V, V + N, V + 2 * N};
    const int t = threadIdx.x;
    const int row0 = t / G4, g = t - G4 * (t / G4);
    const int wrow0 = __builtin_amdgcn_readfirstlane(row0);  // the wave's first row
    const int xs = C.x0 - 4 + 4 * g;
    const bool xedge = C.x0 < 4 || C.x0 + AX + 4 > nx;  // block-uniform
#pragma unroll
    for (int m0 = 0; m0 < FILL_U; m0 += 2) {
      vf4 v[2][NF];
      int ld[2];
#pragma unroll
      for (int mm = 0; mm < 2; ++mm) {
        const int row = row0 + FILL_R * (m0 + mm);
        if (wrow0 + FILL_R * (m0 + mm) >= SROWS) {  // every row of the wave is past the box
          ld[mm] = -1;
#pragma unroll
          for (int f = 0; f < NF; ++f) v[mm][f] = vf4{0.f, 0.f, 0.f, 0.f};
          continue;
        }
        const int rr = min(row, SROWS - 1);
        const int rz = rr / SYW, ry = rr - SYW * (rr / SYW);
        ld[mm] = (t < FILL_T && row < SROWS) ? rz * SPL + ry * SXW + 4 * g : -1;
        const int y = clampi3(C.y0 - 2 + ry, ny), z = clampi3(C.z0 - 2 + rz, nz);
        const unsigned rowi = (unsigned)((z * ny + y) * nx);
        if (vec) {
          const unsigned o = rowi + (unsigned)min(max(xs, 0), nx - 4);
#pragma unroll
          for (int f = 0; f < NF; ++f) v[mm][f] = gld4(F[f], o);
        } else {
#pragma unroll
          for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int k = 0; k < 4; ++k) v[mm][f][k] = gld(F[f], rowi + (unsigned)clampi3(xs + k, nx));
        }
      }
      if (vec && xedge) {
#pragma unroll
        for (int mm = 0; mm < 2; ++mm)
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const vf4 a = v[mm][f];
            v[mm][f] = xs < 0 ? vf4{a.x, a.x, a.x, a.x} : (xs >= nx ? vf4{a.w, a.w, a.w, a.w} : a);
          }
      }
#pragma unroll
      for (int mm = 0; mm < 2; ++mm)
        if (ld[mm] >= 0) {
#pragma unroll
          for (int f = 0; f < NF; ++f) stage4[(f * BOXP + ld[mm]) >> 2] = v[mm][f];
        }
    }
  }
  __syncthreads();

  // phase 1: own points and the ring
  Rec5 orec[4], rrec[RING_B];
  Scat osc[4], dsc;
  float vq[4][3];
  // one loop per mode (block-uniform), so that each mode's code is contiguous
  if (gmode) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool act = orow && C.x0 + gx + 4 * k < nx;
      adj3_point<true, M_GATHER>(C, gx + 4 * k, oly, olz, act, ib[k], zb[k], orec[k], osc[k], vq[k]);
    }
  } else if (lmode2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool act = orow && C.x0 + gx + 4 * k < nx;
      adj3_point<true, M_LDS2>(C, gx + 4 * k, oly, olz, act, ib[k], zb[k], orec[k], osc[k], vq[k]);
    }
  } else if (lmode3) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool act = orow && C.x0 + gx + 4 * k < nx;
      adj3_point<true, M_LDS3>(C, gx + 4 * k, oly, olz, act, ib[k], zb[k], orec[k], osc[k], vq[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool act = orow && C.x0 + gx + 4 * k < nx;
      adj3_point<true, M_GLOBAL>(C, gx + 4 * k, oly, olz, act, ib[k], zb[k], orec[k], osc[k], vq[k]);
    }
  }
  if (gmode) {
#pragma unroll
    for (int u = 0; u < RING_B; ++u) {
      if ((int)threadIdx.x + u * NT < NRING) {
        const int lx = (int)(rc[u] & 255u) - 1, ly = (int)((rc[u] >> 8) & 255u) - 1, lz = (int)(rc[u] >> 16) - 1;
        const int qx = C.x0 + lx, qy = C.y0 + ly, qz = C.z0 + lz;
        const bool act = qx >= 0 && qx < nx && qy >= 0 && qy < ny && qz >= 0 && qz < nz;
        float dummy[3];
        adj3_point<false, M_GATHER>(C, lx, ly, lz, act, rib[u], rzb[u], rrec[u], dsc, dummy);
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < RING_B; ++u) {
      if ((int)threadIdx.x + u * NT < NRING) {
        const int lx = (int)(rc[u] & 255u) - 1, ly = (int)((rc[u] >> 8) & 255u) - 1, lz = (int)(rc[u] >> 16) - 1;
        const int qx = C.x0 + lx, qy = C.y0 + ly, qz = C.z0 + lz;
        const bool act = qx >= 0 && qx < nx && qy >= 0 && qy < ny && qz >= 0 && qz < nz;
        float dummy[3];
        adj3_point<false, M_GLOBAL>(C, lx, ly, lz, act, rib[u], rzb[u], rrec[u], dsc, dummy);
      }
    }
  }
  __syncthreads();  // every staged field has been read

  // the records ((e_x, e_y, e_z, Ib / 8) as one vector, zh_bar / 8 beside
  // them) and the own points' vbar parts replace the staged fields
  vf4* rv = stage4;
  float* rz = stage + O_ZHB;
  float* vqs = stage + O_VQ;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int lx = gx + 4 * k;
#pragma unroll
    for (int c = 0; c < 3; ++c) vqs[c * VQN + vqi(lx, oly, olz)] = vq[k][c];
    if (gmode) {
      const int r = ridx(lx, oly, olz);
      rv[r] = vf4{orec[k].ex, orec[k].ey, orec[k].ez, orec[k].ib};
      rz[r] = orec[k].zhb;
    }
  }
  if (gmode) {
#pragma unroll
    for (int u = 0; u < RING_B; ++u) {
      if ((int)threadIdx.x + u * NT < NRING) {
        const int lx = (int)(rc[u] & 255u) - 1, ly = (int)((rc[u] >> 8) & 255u) - 1, lz = (int)(rc[u] >> 16) - 1;
        const int r = ridx(lx, ly, lz);
        rv[r] = vf4{rrec[u].ex, rrec[u].ey, rrec[u].ez, rrec[u].ib};
        rz[r] = rrec[u].zhb;
      }
    }
  }
  __syncthreads();

  if (lmode2) lds_scatter<2>(C, stage4, osc);
  else if (lmode3) lds_scatter<3>(C, stage4, osc);

  // phase 2: the thread's outputs are x = 4 gx + k of its row
  const int plx = 4 * gx;
  const int pqx = C.x0 + plx;
  float accI[4] = {0.f, 0.f, 0.f, 0.f}, accZ[4] = {0.f, 0.f, 0.f, 0.f};
  if (gmode) {
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz) {
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy) {
        // candidates q = (plx - 1 + j, oly - oy, olz - oz), j = 0..5
        const int r0 = ridx(plx - 1, oly - oy, olz - oz);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          const vf4 a = rv[r0 + j];
          const float zhb = rz[r0 + j];
          const float ty = oy < 0 ? tap2<-1>(a[1]) : (oy == 0 ? tap2<0>(a[1]) : tap2<1>(a[1]));
          const float tz = oz < 0 ? tap2<-1>(a[2]) : (oz == 0 ? tap2<0>(a[2]) : tap2<1>(a[2]));
          const float tyz = ty * tz;
          const float wi = tyz * a[3], wz = tyz * zhb;
          // output k = j - 1 + ox is reached at offset ox = k - j + 1
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int ox = k - j + 1;
            if (ox < -1 || ox > 1) continue;
            const float tx = ox < 0 ? tap2<-1>(a[0]) : (ox == 0 ? tap2<0>(a[0]) : tap2<1>(a[0]));
            accI[k] = fmaf(tx, wi, accI[k]);
            accZ[k] = fmaf(tx, wz, accZ[k]);
          }
        }
      }
    }
  }
  vf4 vb4[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) vb4[c] = *reinterpret_cast<const vf4*>(vqs + c * VQN + vqi(plx, oly, olz));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int qx = min(pqx + k, nx - 1), qy = min(oqy, ny - 1), qz = min(oqz, nz - 1);
    const int r = ridx(plx + k, oly, olz);
    vb4[2][k] += diffT_box(dbar, r, qx, nx, 1);
    vb4[1][k] += diffT_box(dbar, r, qy, ny, RBY);
    vb4[0][k] += diffT_box(dbar, r, qz, nz, RBZ);
  }
  if (orow && pqx < nx) {
    const unsigned o = orowi + (unsigned)pqx;
    if (vec) {
#pragma unroll
      for (int c = 0; c < 3; ++c) gst4(VB, c * N + o, vb4[c]);
      if (gmode) {
        gst4(C.SI, o, vf4{accI[0], accI[1], accI[2], accI[3]});
        gst4(C.SZ, o, vf4{accZ[0], accZ[1], accZ[2], accZ[3]});
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (pqx + k >= nx) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) gst(VB, c * N + o + k, vb4[c][k]);
        if (gmode) {
          gst(C.SI, o + k, accI[k]);
          gst(C.SZ, o + k, accZ[k]);
        }
      }
    }
  }
}

hipError_t launch_adv_adj3(int nt, const AdjArgs& a, hipStream_t s) {
  k_adv_adj3<<<nt, NT, 0, s>>>(a.pd, a.tl, a.V, a.st, a.ab_in, a.sc, a.vb, a);
  return hipGetLastError();
}

}  // namespace shoot
