// Host runtime behind include/shoot.h: validation, plans (ragged batch
// descriptors, tile lists, workspace layout, admission waves), the step and
// checkpoint schedule, and HIP-graph capture.
#include "shoot.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan_access.h"
#include "unfused.h"

using namespace shoot;

namespace {

thread_local std::string g_err;

shoot_status fail(shoot_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(SHOOT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

constexpr size_t ALIGN = 256;
constexpr long long VOX_ALIGN = 64;             // per-pair voxel offsets are multiples of this
constexpr long long MAX_VOXELS = 1ll << 28;     // per pair (32-bit index arithmetic in the kernels)
constexpr size_t XPASS_LDS_CAP = 40 * 1024;     // bytes of LDS per x-pass block (soft)
constexpr size_t LDS_HARD = 64 * 1024;
// Without a fixed lane count, a group of at least this many voxels runs as one
// lane: each of its launches covers thousands of tiles, and a second lane
// gained under 1 % on a 37 M-voxel 3-D batch while splitting every launch.
constexpr long long ONE_LANE_VOXELS = 1LL << 23;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

enum Op { OP_FORWARD = 0, OP_COST = 1, OP_GRAD = 2, OP_DESCEND = 3, OP_DESCEND_RESET = 4, OP_N = 5 };
bool is_grad(int op) { return op == OP_GRAD || op == OP_DESCEND || op == OP_DESCEND_RESET; }

// One admission wave: a subset of the pairs run together.
struct Wave {
  std::vector<int> ids;
  std::vector<PairDev> pdev;
  std::vector<Tile> tb;
  std::vector<Tile> ta;                   // 3-D adjoint tiles (ADJ3)
  std::vector<Tile> tm;                   // x-pass tiles on the matrix cores (empty: not used)
  size_t lds_m = 0;
  std::vector<Tile> tx[2], ty[2], tz[2];  // per tuning option of the x-pass / strided passes
  long long ntot = 0;                     // padded voxel total
  size_t lds_x[2] = {0, 0}, lds_y[2] = {0, 0}, lds_z[2] = {0, 0};
  // header offsets (bytes from the workspace base)
  size_t o_pd = 0, o_tb = 0, o_ta = 0, o_tm = 0, o_tx[2] = {0, 0}, o_ty[2] = {0, 0}, o_tz[2] = {0, 0};
  size_t o_dmax = 0, o_rreg = 0, o_rssd = 0, o_eta = 0, o_prev = 0, o_nf = 0;
  size_t header_bytes = 0;
  size_t field_bytes = 0;
  size_t field_off = 0;  // of this lane's fields inside the field region
};

struct Fields {  // byte offsets of the field arrays inside the field region
  size_t st, vs, u, u2, ab, sc, vb, psi, end;
};

// Kernel families, for the profiling statistics.
enum KId {
  KI_FILL, KI_INIT, KI_XPASS_M, KI_XPASS_V, KI_SPASS_MID, KI_SPASS_V, KI_SPASS_MBAR,
  KI_ADVECT, KI_ADV_ADJ, KI_EPILOGUE, KI_FINALIZE, KI_DESCEND, KI_DEFORM, KI_COUNT
};
const char* const KNAMES[KI_COUNT] = {
    "fill", "init", "xpass_gradmul", "xpass_plain", "spass_mid", "spass_v", "spass_mbar",
    "advect", "advect_adjoint", "epilogue", "finalize", "descend", "deform"};

// Event pairs around launches; resolved after the stream is synchronised.
struct Prof {
  struct Rec { int kid; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  long long launches[KI_COUNT] = {};
  double ms[KI_COUNT] = {};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipError_t resolve() {
    hipError_t err = hipSuccess;
    for (Rec& r : pending) {
      float t = 0.f;
      if (r.a && r.b) {
        hipError_t e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) err = e;
        launches[r.kid] += 1;
        ms[r.kid] += t;
      }
      if (r.a) pool.push_back(r.a);
      if (r.b) pool.push_back(r.b);
    }
    pending.clear();
    return err;
  }
  void release() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

}  // namespace

struct shoot_plan_s {
  int npairs = 0, T = 0, ndim = 0, k = 1, nck = 1, nst = 1, nv = 1;
  uint32_t flags = 0;
  size_t budget = 0;
  std::vector<shoot_pair> pairs;
  // Waves (lanes) in execution order; groups[g] = (first wave, lane count):
  // the lanes of a group run concurrently, groups one after another.
  std::vector<Wave> waves;
  std::vector<std::pair<int, int>> groups;
  int lanes = 1;                      // most lanes of a group
  size_t header_total = 0, field_max = 0, ws_bytes = 0;
  std::vector<unsigned char> blob;  // header image uploaded at bind
  char* ws = nullptr;
  int device = -1;
  hipStream_t cap = nullptr;           // the device's capture stream (shared, not owned)
  std::vector<hipStream_t> side;      // streams of lanes 0 .. lanes-2 (the device's shared pool)
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  std::vector<hipGraphExec_t> graph[OP_N];  // per wave
  float eta0 = 1.f;           // step of the descent after a reset
  bool descend_ready = false; // the descent's per-pair step state is initialised
  bool scratch_bound = false; // bound to the library's static scratch (shoot_plan_bind_scratch)
  unfused::Plan* uf = nullptr;      // SHOOT_UNFUSED state
  bool profiling = false;
  Prof prof;
  int tune[TUNE_N] = {0, 0, 0, 0, 0, 0};
  bool has_def = false;        // some pair asks for its deformation map
};

namespace {

bool fullstore(const shoot_plan_s* p) { return (p->flags & SHOOT_FULL_STORE) != 0; }

Fields field_layout(const shoot_plan_s* p, long long ntot) {
  const size_t f = sizeof(float);
  const size_t d = (size_t)p->ndim;
  Fields F{};
  size_t o = 0;
  F.st = o; o = align_up(o + (size_t)p->nst * 2 * ntot * f, ALIGN);
  F.vs = o; o = align_up(o + (size_t)p->nv * d * ntot * f, ALIGN);
  F.u = o; o = align_up(o + d * ntot * f, ALIGN);
  F.u2 = o; o = align_up(o + (p->ndim == 3 ? d * ntot * f : 0), ALIGN);
  F.ab = o; o = align_up(o + 2 * 2 * ntot * f, ALIGN);
  F.sc = o; o = align_up(o + 2 * ntot * f, ALIGN);
  F.vb = o; o = align_up(o + d * ntot * f, ALIGN);
  F.psi = o; o = align_up(o + (p->has_def ? 2 * d * ntot * f : 0), ALIGN);
  F.end = o;
  return F;
}

long long pair_voxels(const shoot_pair& q) {
  long long n = 1;
  for (int a = 0; a < q.ndim; ++a) n *= q.shape[a];
  return n;
}

int radius_of(float sigma) { return (int)std::floor(3.0 * (double)sigma); }

void fill_taps(PairDev& P, float sigma) {
  const int r = P.r;
  double w[2 * RMAX + 1];
  double sum = 0.0;
  for (int k = -r; k <= r; ++k) {
    w[k + r] = std::exp(-(double)k * k / (2.0 * (double)sigma * (double)sigma));
    sum += w[k + r];
  }
  for (int t = 0; t < WPAD; ++t) P.w[t] = t <= 2 * r ? (float)(w[t] / sum) : 0.f;
}

size_t xpass_row_bytes(int ndim, int nx, int ntap4) {
  const int G4 = (nx + 3) / 4;
  return (size_t)ndim * 4 * (G4 + ntap4) * sizeof(float);
}

shoot_status validate(const shoot_pair* pairs, int32_t n, int32_t T) {
  if (!pairs) return fail(SHOOT_E_ARG, "pairs is NULL");
  if (n < 1) return fail(SHOOT_E_ARG, "n_pairs must be >= 1");
  if (T < 1) return fail(SHOOT_E_ARG, "T must be >= 1");
  const int nd = pairs[0].ndim;
  for (int i = 0; i < n; ++i) {
    const shoot_pair& q = pairs[i];
    const std::string at = " (pair " + std::to_string(i) + ")";
    if (q.ndim != 2 && q.ndim != 3) return fail(SHOOT_E_SHAPE, "ndim must be 2 or 3" + at);
    if (q.ndim != nd) return fail(SHOOT_E_SHAPE, "all pairs of a plan must share ndim" + at);
    for (int a = 0; a < q.ndim; ++a)
      if (q.shape[a] < 2) return fail(SHOOT_E_SHAPE, "every extent must be >= 2" + at);
    if (pair_voxels(q) > MAX_VOXELS) return fail(SHOOT_E_SHAPE, "pair too large" + at);
    if (!(q.sigma > 0.f) || !std::isfinite(q.sigma)) return fail(SHOOT_E_ARG, "sigma must be finite and > 0" + at);
    if (radius_of(q.sigma) > RMAX) return fail(SHOOT_E_ARG, "sigma too large: floor(3 sigma) > 31" + at);
    if (!(q.rho >= 0.f) || !std::isfinite(q.rho)) return fail(SHOOT_E_ARG, "rho must be finite and >= 0" + at);
    if (!(q.lambda >= 0.f) || !std::isfinite(q.lambda))
      return fail(SHOOT_E_ARG, "lambda must be finite and >= 0" + at);
    if (!q.image) return fail(SHOOT_E_ARG, "image is NULL" + at);
    if (!q.p0) return fail(SHOOT_E_ARG, "p0 is NULL" + at);
    const int nx = q.shape[q.ndim - 1];
    const int ntap4 = (2 * radius_of(q.sigma) + 1 + 3) / 4;
    if (xpass_row_bytes(q.ndim, nx, ntap4) > LDS_HARD) return fail(SHOOT_E_SHAPE, "last extent too large" + at);
  }
  return SHOOT_OK;
}

// Builds descriptors and tile lists of one wave (header offsets are set later).
void build_wave(shoot_plan_s* p, Wave& w) {
  w.pdev.clear(); w.tb.clear(); w.ta.clear(); w.tm.clear();
  w.lds_m = 0;
  // the matrix-core x-pass needs every last extent a multiple of 4 and one
  // staged row of every channel within the LDS limit
  bool mfma = true;
  for (int id : w.ids) {
    const shoot_pair& q = p->pairs[id];
    const int nx = q.shape[p->ndim - 1];
    mfma = mfma && nx % 4 == 0 && xpass_mfma_lds(p->ndim, nx, radius_of(q.sigma), 1) <= LDS_HARD;
  }
  for (int o = 0; o < 2; ++o) {
    w.tx[o].clear(); w.ty[o].clear(); w.tz[o].clear();
    w.lds_x[o] = w.lds_y[o] = w.lds_z[o] = 0;
  }
  long long off = 0;
  for (size_t li = 0; li < w.ids.size(); ++li) {
    const shoot_pair& q = p->pairs[w.ids[li]];
    PairDev P;
    std::memset(&P, 0, sizeof(P));
    P.nz = q.ndim == 3 ? q.shape[0] : 1;
    P.ny = q.shape[q.ndim - 2];
    P.nx = q.shape[q.ndim - 1];
    P.r = radius_of(q.sigma);
    P.ntap4 = (2 * P.r + 1 + 3) / 4;
    P.N = pair_voxels(q);
    P.off = off;
    off += (P.N + VOX_ALIGN - 1) / VOX_ALIGN * VOX_ALIGN;
    P.rho = q.rho;
    P.lam = q.lambda;
    P.dt = (float)(1.0 / (double)p->T);
    P.active = 1;
    P.S = q.image; P.J = q.target; P.p0 = q.p0;
    P.outI = q.out_image; P.outZ = q.out_momentum; P.outG = q.out_grad; P.outCost = q.out_cost;
    P.outD = q.out_deformation;
    fill_taps(P, q.sigma);
    const int pi = (int)li;
    // block tiles (init, advect, adjoint, epilogue); cost partials are per block tile
    P.elem_first = (int)w.tb.size();
    {
      const int BX = p->ndim == 2 ? BLK2_X : BLK3_X, BY = p->ndim == 2 ? BLK2_Y : BLK3_Y;
      const int BZ = p->ndim == 2 ? 1 : BLK3_Z;
      for (int z0 = 0; z0 < P.nz; z0 += BZ)
        for (int y0 = 0; y0 < P.ny; y0 += BY)
          for (int x0 = 0; x0 < P.nx; x0 += BX) w.tb.push_back(Tile{pi, x0, y0, z0});
    }
    P.elem_count = (int)w.tb.size() - P.elem_first;
    if (p->ndim == 3) {
      for (int z0 = 0; z0 < P.nz; z0 += ADJ3_Z)
        for (int y0 = 0; y0 < P.ny; y0 += ADJ3_Y)
          for (int x0 = 0; x0 < P.nx; x0 += ADJ3_X) w.ta.push_back(Tile{pi, x0, y0, z0});
    }
    // x-pass tiles: rows of the pair, at most as many as one batch of the fill
    // covers (XSEG 64-column segments per wave). Option 0: also at most one
    // group of four outputs per thread (nr * G4 <= NT), so the tap loop runs
    // in a single round; option 1: the full fill batch. Both within the LDS
    // budget.
    const size_t rb = xpass_row_bytes(p->ndim, P.nx, P.ntap4);
    const int G4 = (P.nx + 3) / 4;
    const int L = 4 * (G4 + P.ntap4);
    const int nch = (L + 63) / 64;
    const int rows = P.nz * P.ny;
    for (int opt = 0; opt < 2; ++opt) {
      int nr = std::max(1, XSEG * (NT / 64) / nch);
      if (opt == 0) nr = std::max(1, std::min(nr, NT / G4));
      nr = std::min(nr, std::max(1, (int)(XPASS_LDS_CAP / rb)));
      if (opt == 0) P.xrows = nr;
      for (int r0 = 0; r0 < rows; r0 += nr) {
        const int cnt = std::min(nr, rows - r0);
        w.tx[opt].push_back(Tile{pi, r0, cnt, 0});
        w.lds_x[opt] = std::max(w.lds_x[opt], rb * (size_t)cnt);
      }
    }
    if (mfma) {
      int nr = XPASS_MFMA_ROWS[p->ndim - 2];
      while (nr > 1 && xpass_mfma_lds(p->ndim, P.nx, P.r, nr) > LDS_HARD) --nr;
      for (int r0 = 0; r0 < rows; r0 += nr) {
        const int cnt = std::min(nr, rows - r0);
        w.tm.push_back(Tile{pi, r0, cnt, 0});
        w.lds_m = std::max(w.lds_m, xpass_mfma_lds(p->ndim, P.nx, P.r, cnt));
      }
    }
    // strided passes: tiles of 4 RB outputs along the pass axis
    for (int opt = 0; opt < 2; ++opt) {
      const int seg = (NT / 64) * SPASS_RB[opt];
      const size_t sb = (size_t)(seg + 4 * P.ntap4) * 64 * sizeof(float);
      for (int o = 0; o < P.nz; ++o)
        for (int x0 = 0; x0 < P.nx; x0 += 64)
          for (int s0 = 0; s0 < P.ny; s0 += seg) w.ty[opt].push_back(Tile{pi, x0, o, s0});
      w.lds_y[opt] = std::max(w.lds_y[opt], sb);
      if (p->ndim == 3) {
        for (int o = 0; o < P.ny; ++o)
          for (int x0 = 0; x0 < P.nx; x0 += 64)
            for (int s0 = 0; s0 < P.nz; s0 += seg) w.tz[opt].push_back(Tile{pi, x0, o, s0});
        w.lds_z[opt] = std::max(w.lds_z[opt], sb);
      }
    }
    w.pdev.push_back(P);
  }
  w.ntot = off;
  w.field_bytes = field_layout(p, w.ntot).end;
}

// Splits the pairs `ids` into at most L lanes of balanced voxel count (each
// keeping the pairs' order; one lane for a large group unless the caller
// fixed the count) and builds them with consecutive field regions; returns
// the bytes of the group's field region.
size_t build_group(shoot_plan_s* p, const std::vector<int>& ids, int L, bool fixed, std::vector<Wave>& out) {
  int n = std::max(1, std::min(L, (int)ids.size()));
  long long total = 0;
  for (int i : ids) total += pair_voxels(p->pairs[i]);
  if (!fixed && total >= ONE_LANE_VOXELS) n = 1;  // its launches fill the GPU by themselves
  std::vector<int> order = ids;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return pair_voxels(p->pairs[a]) > pair_voxels(p->pairs[b]); });
  std::vector<long long> load(n, 0);
  out.assign(n, Wave());
  for (int i : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    out[l].ids.push_back(i);
    load[l] += pair_voxels(p->pairs[i]);
  }
  size_t off = 0;
  for (Wave& w : out) {
    std::sort(w.ids.begin(), w.ids.end());
    build_wave(p, w);
    w.field_off = off;
    off += align_up(w.field_bytes, ALIGN);
  }
  return off;
}

size_t header_size(shoot_plan_s* p, Wave& w, size_t base) {
  size_t o = base;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, ALIGN); return r; };
  w.o_pd = take(w.pdev.size() * sizeof(PairDev));
  w.o_tb = take(w.tb.size() * sizeof(Tile));
  w.o_ta = take(w.ta.size() * sizeof(Tile));
  w.o_tm = take(w.tm.size() * sizeof(Tile));
  for (int o = 0; o < 2; ++o) {
    w.o_tx[o] = take(w.tx[o].size() * sizeof(Tile));
    w.o_ty[o] = take(w.ty[o].size() * sizeof(Tile));
    w.o_tz[o] = take(w.tz[o].size() * sizeof(Tile));
  }
  w.o_dmax = take(w.pdev.size() * (size_t)p->T * sizeof(unsigned));
  w.o_rreg = take(w.tb.size() * sizeof(float));
  w.o_rssd = take(w.tb.size() * sizeof(float));
  w.o_eta = take(w.pdev.size() * sizeof(float));
  w.o_prev = take(w.pdev.size() * sizeof(float));
  w.o_nf = take(w.pdev.size() * sizeof(unsigned));
  w.header_bytes = o - base;
  return o;
}

// -------------------------------------------------------------------- schedule

// One recorded kernel launch of a wave's schedule.
struct Launch {
  int kid;
  std::function<hipError_t()> fn;
};

struct Ctx {
  shoot_plan_s* p;
  Wave* w;
  hipStream_t s;
  const PairDev* pd;
  const Tile *tb, *ta, *tm, *tx, *ty, *tz;
  int ntb, nta, ntm, ntx, nty, ntz;
  size_t lds_m;
  size_t lds_x, lds_y, lds_z;
  int rb;                 // strided-pass outputs per thread
  int o_adv, o_adj, o_epi;  // load-batch options
  unsigned* dmax;
  float *rreg, *rssd, *eta, *prev;
  float *st, *vs, *u, *u2, *ab, *sc, *vb, *psi;
  long long ntot;
  std::vector<Launch>* rec;  // when set, launches are recorded here instead of issued
};

Ctx make_ctx(shoot_plan_s* p, Wave& w, hipStream_t s) {
  Ctx c{};
  c.p = p; c.w = &w; c.s = s;
  char* b = p->ws;
  c.pd = (const PairDev*)(b + w.o_pd);
  c.tb = (const Tile*)(b + w.o_tb); c.ntb = (int)w.tb.size();
  c.ta = (const Tile*)(b + w.o_ta); c.nta = (int)w.ta.size();
  c.tm = (const Tile*)(b + w.o_tm); c.ntm = p->tune[TUNE_XMFMA] ? (int)w.tm.size() : 0; c.lds_m = w.lds_m;
  const int ox = p->tune[TUNE_XPASS], os = p->tune[TUNE_SPASS];
  c.tx = (const Tile*)(b + w.o_tx[ox]); c.ntx = (int)w.tx[ox].size(); c.lds_x = w.lds_x[ox];
  c.ty = (const Tile*)(b + w.o_ty[os]); c.nty = (int)w.ty[os].size(); c.lds_y = w.lds_y[os];
  c.tz = (const Tile*)(b + w.o_tz[os]); c.ntz = (int)w.tz[os].size(); c.lds_z = w.lds_z[os];
  c.rb = SPASS_RB[os];
  c.o_adv = p->tune[TUNE_ADVECT]; c.o_adj = p->tune[TUNE_ADJ]; c.o_epi = p->tune[TUNE_EPI];
  c.dmax = (unsigned*)(b + w.o_dmax);
  c.rreg = (float*)(b + w.o_rreg);
  c.rssd = (float*)(b + w.o_rssd);
  c.eta = (float*)(b + w.o_eta);
  c.prev = (float*)(b + w.o_prev);
  char* f = b + p->header_total + w.field_off;
  const Fields F = field_layout(p, w.ntot);
  c.st = (float*)(f + F.st); c.vs = (float*)(f + F.vs); c.u = (float*)(f + F.u); c.u2 = (float*)(f + F.u2);
  c.ab = (float*)(f + F.ab); c.sc = (float*)(f + F.sc); c.vb = (float*)(f + F.vb);
  c.psi = (float*)(f + F.psi);
  c.ntot = w.ntot;
  return c;
}

int st_slot(const shoot_plan_s* p, int t) {
  if (fullstore(p)) return t;
  return (t % p->k == 0) ? t / p->k : p->nck + (t % p->k) - 1;
}
// Velocity slots: with checkpoints, k - 1 slots for the steps inside a
// segment, then one per checkpoint (a checkpoint keeps its state and its
// velocity, so a recomputed segment starts with the advection).
int v_slot(const shoot_plan_s* p, int t) {
  if (fullstore(p)) return t;
  return (t % p->k == 0) ? p->k - 1 + t / p->k : (t % p->k) - 1;
}
float* ST(const Ctx& c, int t) { return c.st + (size_t)st_slot(c.p, t) * 2 * c.ntot; }
float* VS(const Ctx& c, int t) { return c.vs + (size_t)v_slot(c.p, t) * c.p->ndim * c.ntot; }
float* AB(const Ctx& c, int t) { return c.ab + (size_t)(t & 1) * 2 * c.ntot; }

#define LAUNCH(kid, expr)                                      \
  do {                                                         \
    if (c.rec) {                                               \
      c.rec->push_back(Launch{kid, [=]() { return (expr); }}); \
    } else {                                                   \
      hipError_t e_ = (expr);                                  \
      if (e_ != hipSuccess) return e_;                         \
    }                                                          \
  } while (0)

// v_t = -G (z_t grad I_t) into the v slot of t.
hipError_t velocity(const Ctx& c, int t) {
  const int nd = c.p->ndim;
  if (c.ntm) LAUNCH(KI_XPASS_M, launch_xpass_mfma(nd, true, c.pd, c.tm, c.ntm, c.lds_m, ST(c, t), c.u, c.s));
  else LAUNCH(KI_XPASS_M, launch_xpass(nd, true, c.pd, c.tx, c.ntx, c.lds_x, ST(c, t), c.u, c.s));
  if (nd == 2) {
    LAUNCH(KI_SPASS_V, launch_spass(2, false, 1, c.rb, c.pd, c.ty, c.nty, c.lds_y, c.u, VS(c, t), nullptr, c.s));
    return hipSuccess;
  }
  LAUNCH(KI_SPASS_MID, launch_spass(3, false, 0, c.rb, c.pd, c.ty, c.nty, c.lds_y, c.u, c.u2, nullptr, c.s));
  LAUNCH(KI_SPASS_V, launch_spass(3, true, 1, c.rb, c.pd, c.tz, c.ntz, c.lds_z, c.u2, VS(c, t), nullptr, c.s));
  return hipSuccess;
}

// One forward step t -> t + 1. `store` writes state t + 1 to its slot;
// `have_v`: the velocity of step t is already in its slot.
hipError_t fwd_step(const Ctx& c, int t, bool store, int op, bool first_pass, bool have_v = false) {
  if (!have_v) {
    hipError_t e = velocity(c, t);
    if (e != hipSuccess) return e;
  }
  const int T = c.p->T;
  AdvectArgs a{};
  a.pd = c.pd; a.tl = c.tb; a.V = VS(c, t); a.st = ST(c, t);
  a.st_out = (store && t + 1 < T) ? ST(c, t + 1) : nullptr;
  a.T = T; a.t = t;
  a.dmax = first_pass ? c.dmax : nullptr;
  a.last = (first_pass && t == T - 1) ? 1 : 0;
  a.red_reg = (first_pass && t == 0) ? c.rreg : nullptr;
  a.red_ssd = (first_pass && t == T - 1) ? c.rssd : nullptr;
  a.scheme = (c.p->flags & SHOOT_SCHEME_EULERIAN) ? 1 : ((c.p->flags & SHOOT_SCHEME_MIXED) ? 2 : 0);
  if (a.last && is_grad(op)) { a.ab_out = AB(c, T); a.sc_zero = c.sc; }
  LAUNCH(KI_ADVECT, launch_advect(c.p->ndim, c.o_adv, c.ntb, a, c.s));
  return hipSuccess;
}

hipError_t run_forward(const Ctx& c, int op) {
  const int T = c.p->T;
  LAUNCH(KI_FILL, launch_fill_u32(c.dmax, (long long)c.w->pdev.size() * T, 0u, c.s));
  LAUNCH(KI_INIT, launch_init(c.p->ndim, c.pd, c.tb, c.ntb, ST(c, 0), c.s));
  const bool def = op == OP_FORWARD && c.p->has_def;
  const size_t psz = (size_t)c.p->ndim * c.ntot;
  for (int t = 0; t < T; ++t) {
    hipError_t e = fwd_step(c, t, true, op, true);
    if (e != hipSuccess) return e;
    if (def) {
      // psi_{t+1} = psi_t o (Id - dt v_t); psi_0 = Id, psi_T to the outputs
      const float* pin = t == 0 ? nullptr : c.psi + (size_t)(t & 1) * psz;
      float* pout = t == T - 1 ? nullptr : c.psi + (size_t)((t + 1) & 1) * psz;
      LAUNCH(KI_DEFORM, launch_deform(c.p->ndim, c.pd, c.tb, c.ntb, VS(c, t), pin, pout, c.s));
    }
  }
  LAUNCH(KI_FINALIZE, launch_finalize((int)c.w->pdev.size(), c.pd, c.rreg, c.rssd, c.s));
  return hipSuccess;
}

// Adjoint of step t: (Ibar_{t+1}, zbar_{t+1}) in AB(t+1) -> AB(t) (or dH/dp0 at t = 0).
hipError_t bwd_step(const Ctx& c, int t) {
  const int nd = c.p->ndim;
  const int force = (c.p->flags & SHOOT_FORCE_GLOBAL_SCATTER) ? 1 : 0;
  AdjArgs a{};
  a.pd = c.pd; a.tl = c.tb; a.V = VS(c, t); a.st = ST(c, t); a.ab_in = AB(c, t + 1);
  a.sc = c.sc; a.vb = c.vb;
  a.dmax = c.dmax; a.T = c.p->T; a.t = t; a.force_global = force;
  if (nd == 3) {
    a.tl = c.ta;
    LAUNCH(KI_ADV_ADJ, launch_adv_adj3(c.nta, a, c.s));
  } else {
    LAUNCH(KI_ADV_ADJ, launch_adv_adj(nd, c.o_adj, c.ntb, a, c.s));
  }
  // mbar = -G vbar (+ -2 lambda v_0 at t = 0), written back into vb
  if (c.ntm) LAUNCH(KI_XPASS_V, launch_xpass_mfma(nd, false, c.pd, c.tm, c.ntm, c.lds_m, c.vb, c.u, c.s));
  else LAUNCH(KI_XPASS_V, launch_xpass(nd, false, c.pd, c.tx, c.ntx, c.lds_x, c.vb, c.u, c.s));
  const float* extra = t == 0 ? VS(c, 0) : nullptr;
  if (nd == 2) {
    LAUNCH(KI_SPASS_MBAR, launch_spass(2, false, 2, c.rb, c.pd, c.ty, c.nty, c.lds_y, c.u, c.vb, extra, c.s));
  } else {
    LAUNCH(KI_SPASS_MID, launch_spass(3, false, 0, c.rb, c.pd, c.ty, c.nty, c.lds_y, c.u, c.u2, nullptr, c.s));
    LAUNCH(KI_SPASS_MBAR, launch_spass(3, true, 2, c.rb, c.pd, c.tz, c.ntz, c.lds_z, c.u2, c.vb, extra, c.s));
  }
  EpiArgs ep{};
  ep.pd = c.pd; ep.tl = c.tb; ep.mb = c.vb; ep.st = ST(c, t); ep.sc = c.sc;
  ep.ab_out = t > 0 ? AB(c, t) : nullptr;
  ep.dmax = c.dmax; ep.T = c.p->T; ep.t = t; ep.force_global = force;
  ep.first = t == 0 ? 1 : 0;
  LAUNCH(KI_EPILOGUE, launch_epilogue(nd, c.o_epi, c.ntb, ep, c.s));
  return hipSuccess;
}

hipError_t run_grad(const Ctx& c) {
  hipError_t e = run_forward(c, OP_GRAD);
  if (e != hipSuccess) return e;
  const shoot_plan_s* p = c.p;
  const int T = p->T;
  const int k = fullstore(p) ? T : p->k;
  const int nseg = (T + k - 1) / k;
  for (int s = nseg - 1; s >= 0; --s) {
    const int t0 = s * k, t1 = std::min(T, t0 + k);
    if (s != nseg - 1) {
      // restore states t0+1 .. t1-1 and velocities t0+1 .. t1-1 from
      // checkpoint t0, whose velocity the forward pass kept (the last step
      // needs only its velocity: state t1 is a checkpoint)
      for (int t = t0; t < t1; ++t) {
        if (t + 1 < t1) e = fwd_step(c, t, true, OP_GRAD, false, t == t0);
        else e = t == t0 ? hipSuccess : velocity(c, t);
        if (e != hipSuccess) return e;
      }
    }
    for (int t = t1 - 1; t >= t0; --t) {
      e = bwd_step(c, t);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// The whole schedule of one wave for `op` on stream s (recorded into `rec`
// instead when given).
hipError_t enqueue_wave(shoot_plan_s* p, Wave& w, int op, hipStream_t s, std::vector<Launch>* rec = nullptr) {
  Ctx c = make_ctx(p, w, s);
  c.rec = rec;
  hipError_t e = is_grad(op) ? run_grad(c) : run_forward(c, op);
  if (e != hipSuccess) return e;
  if (op == OP_DESCEND || op == OP_DESCEND_RESET) {
    const int reset = op == OP_DESCEND_RESET ? 1 : 0;
    LAUNCH(KI_DESCEND, launch_descend(p->ndim, (int)w.pdev.size(), c.pd, c.tb, c.ntb, c.eta, c.prev, reset,
                                      p->eta0, c.s));
  }
  return hipSuccess;
}

// Stream of lane i of a group of n lanes called on stream s: the last lane
// runs on s itself, lanes 0 .. n-2 on the device's lane pool; with n = 1
// (one lane, or lanes run one after another) every lane runs on s.
hipStream_t lane_stream(const shoot_plan_s* p, hipStream_t s, int n, int i) {
  return (n < 2 || i == n - 1) ? s : p->side[i];
}

// Fork: the pool lanes wait for the work already on s. Join: s waits for them.
hipError_t fork_lanes(shoot_plan_s* p, hipStream_t s, int n) {
  if (n < 2) return hipSuccess;
  hipError_t e = hipEventRecord(p->ev_fork, s);
  for (int i = 0; i < n - 1 && e == hipSuccess; ++i) e = hipStreamWaitEvent(p->side[i], p->ev_fork, 0);
  return e;
}
hipError_t join_lanes(shoot_plan_s* p, hipStream_t s, int n) {
  if (n < 2) return hipSuccess;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n - 1 && e == hipSuccess; ++i) {
    e = hipEventRecord(p->ev_join[i], p->side[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_join[i], 0);
  }
  return e;
}

// Eager launches: every group's lanes concurrently (one after another on s
// when `serial`, e.g. inside the caller's stream capture).
hipError_t enqueue(shoot_plan_s* p, int op, hipStream_t s, bool serial) {
  for (const auto& g : p->groups) {
    const int n = serial ? 1 : g.second;
    hipError_t e = fork_lanes(p, s, n);
    if (e != hipSuccess) return e;
    for (int i = 0; i < g.second; ++i) {
      e = enqueue_wave(p, p->waves[g.first + i], op, lane_stream(p, s, n, i));
      if (e != hipSuccess) return e;
    }
    e = join_lanes(p, s, n);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Profiling: the lanes of a group run one after another on s, the k-th
// launches of all lanes together between one event pair, so a timed launch
// covers every pair of the group (as one launch over all of them would,
// plus the extra launches' ramp and drain).
hipError_t enqueue_profiled(shoot_plan_s* p, int op, hipStream_t s) {
  for (const auto& g : p->groups) {
    const int n = g.second;
    std::vector<std::vector<Launch>> rec(n);
    for (int i = 0; i < n; ++i) {
      hipError_t e = enqueue_wave(p, p->waves[g.first + i], op, s, &rec[i]);
      if (e != hipSuccess) return e;
    }
    for (int i = 1; i < n; ++i) {
      if (rec[i].size() != rec[0].size()) return hipErrorInvalidValue;
      for (size_t k = 0; k < rec[0].size(); ++k)
        if (rec[i][k].kid != rec[0][k].kid) return hipErrorInvalidValue;
    }
    for (size_t k = 0; k < rec[0].size(); ++k) {
      Prof::Rec r{rec[0][k].kid, p->prof.get(), p->prof.get()};
      if (r.a) (void)hipEventRecord(r.a, s);
      hipError_t e = hipSuccess;
      for (int i = 0; i < n && e == hipSuccess; ++i) e = rec[i][k].fn();
      if (r.b) (void)hipEventRecord(r.b, s);
      p->prof.pending.push_back(r);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// Streams of a device, shared by every plan of the process and kept until the
// process ends: the lane pool and one capture stream. Each stream takes one of
// the device's few hardware queues (handed out as streams are created, shared
// once they run out), and lanes whose queues were shared with each other or
// with the caller's stream would run one after the other; so the lane pool is
// created first, at the first bind on the device, with DEFAULT_POOL streams
// (the last lane of a group runs on the caller's stream).
constexpr int DEFAULT_POOL = 3;
struct DevStreams {
  std::vector<hipStream_t> pool;
  hipStream_t cap = nullptr;
};
std::mutex g_streams_mu;                 // guards g_streams
std::mutex g_capture_mu;                 // one graph capture at a time on the shared capture stream

// Static device scratch for plans bound without a caller workspace
// (shoot_plan_bind_scratch): one array per device, held until the process
// ends. Host code uses only the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in). The plan whose
// header the array holds is its owner; an execution call of another
// scratch-bound plan uploads that plan's header first.
constexpr size_t SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
struct ScratchDev {
  void* ptr = nullptr;
  const shoot_plan_s* owner = nullptr;
};
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;                         // guards g_scratch
ScratchDev g_scratch[SCRATCH_DEVICES];           // [device]

// The current device's scratch address (looked up once per device, with that
// device current).
hipError_t scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
  ScratchDev& d = g_scratch[dev];
  if (!d.ptr) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr || ((uintptr_t)ptr) % ALIGN) return hipErrorInvalidSymbol;
    d.ptr = ptr;
  }
  *out = d.ptr;
  return hipSuccess;
}

// Before an execution call of a scratch-bound plan: upload its header if
// another plan used the scratch since (the previous contents stay otherwise).
shoot_status scratch_claim(shoot_plan_s* p, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  ScratchDev& d = g_scratch[p->device];
  if (d.owner != p) {
    if (p->header_total) HIPCHK(hipMemcpyAsync(p->ws, p->blob.data(), p->header_total, hipMemcpyHostToDevice, s));
    d.owner = p;
    p->descend_ready = false;
  }
  return SHOOT_OK;
}
std::vector<DevStreams> g_streams;       // [device]

hipError_t device_streams(shoot_plan_s* p, int dev) {
  std::lock_guard<std::mutex> lock(g_streams_mu);
  if ((int)g_streams.size() <= dev) g_streams.resize(dev + 1);
  DevStreams& d = g_streams[dev];
  const int want = std::max(d.cap ? 0 : DEFAULT_POOL, p->lanes - 1);
  while ((int)d.pool.size() < want) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    d.pool.push_back(st);
  }
  if (!d.cap) {
    hipError_t e = hipStreamCreateWithFlags(&d.cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  p->cap = d.cap;
  p->side.assign(d.pool.begin(), d.pool.begin() + (p->lanes - 1));
  return hipSuccess;
}

void release_streams(shoot_plan_s* p) {
  p->cap = nullptr;
  p->side.clear();
  for (hipEvent_t ev : p->ev_join) (void)hipEventDestroy(ev);
  p->ev_join.clear();
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  p->ev_fork = nullptr;
}

void drop_graphs(shoot_plan_s* p, int only_op = -1) {
  for (int op = 0; op < OP_N; ++op) {
    if (only_op >= 0 && op != only_op) continue;
    for (hipGraphExec_t g : p->graph[op])
      if (g) (void)hipGraphExecDestroy(g);
    p->graph[op].clear();
  }
}

// SHOOT_CHECK_FINITE: counts the non-finite values of every pair's inputs on
// the device, reads the counts back (synchronising s) and fails on the first
// pair that has any, before any other work is enqueued.
shoot_status check_finite(shoot_plan_s* p, hipStream_t s) {
  std::vector<unsigned> cnt(p->npairs, 0u);
  for (Wave& w : p->waves) {
    unsigned* nf = (unsigned*)(p->ws + w.o_nf);
    const PairDev* pd = (const PairDev*)(p->ws + w.o_pd);
    const Tile* tb = (const Tile*)(p->ws + w.o_tb);
    HIPCHK(launch_fill_u32(nf, (long long)w.pdev.size(), 0u, s));
    HIPCHK(launch_count_nonfinite(p->ndim, pd, tb, (int)w.tb.size(), nf, s));
    std::vector<unsigned> h(w.pdev.size());
    HIPCHK(hipMemcpyAsync(h.data(), nf, h.size() * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t li = 0; li < w.ids.size(); ++li) cnt[w.ids[li]] = h[li];
  }
  for (int i = 0; i < p->npairs; ++i)
    if (cnt[i])
      return fail(SHOOT_E_ARG, "pair " + std::to_string(i) + ": " + std::to_string(cnt[i]) +
                                   " non-finite values in its image, target or p0");
  return SHOOT_OK;
}

shoot_status execute(shoot_plan_s* p, int op, void* stream) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (!p->ws) return fail(SHOOT_E_STATE, "plan is not bound to a workspace");
  for (int i = 0; i < p->npairs; ++i) {
    const shoot_pair& q = p->pairs[i];
    if (op != OP_FORWARD && !q.target) return fail(SHOOT_E_ARG, "target is NULL (pair " + std::to_string(i) + ")");
    if (op == OP_COST && !q.out_cost) return fail(SHOOT_E_ARG, "out_cost is NULL (pair " + std::to_string(i) + ")");
    if (is_grad(op) && !q.out_grad) return fail(SHOOT_E_ARG, "out_grad is NULL (pair " + std::to_string(i) + ")");
    if (is_grad(op) && (p->flags & (SHOOT_SCHEME_EULERIAN | SHOOT_SCHEME_MIXED)))
      return fail(SHOOT_E_ARG, "the gradient is available for the semi-Lagrangian scheme only");
    if (op >= OP_DESCEND && !q.out_cost) return fail(SHOOT_E_ARG, "out_cost is NULL (pair " + std::to_string(i) + ")");
  }
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != p->device) return fail(SHOOT_E_STATE, "current device differs from the device the plan was bound on");
  hipStream_t s = (hipStream_t)stream;
  if (p->scratch_bound) {
    shoot_status st = scratch_claim(p, s);
    if (st != SHOOT_OK) return st;
  }
  if (p->uf) {
    hipError_t e = unfused::run(p->uf, op, s);
    if (e != hipSuccess) return fail(SHOOT_E_HIP, std::string("unfused path: ") + hipGetErrorString(e));
    return SHOOT_OK;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s) HIPCHK(hipStreamIsCapturing(s, &cs));
  if (p->profiling) {
    if (cs != hipStreamCaptureStatusNone) return fail(SHOOT_E_STATE, "profiling cannot run under stream capture");
    hipError_t e = enqueue_profiled(p, op, s);
    hipError_t e2 = hipStreamSynchronize(s);
    hipError_t e3 = p->prof.resolve();
    if (e != hipSuccess) return fail(SHOOT_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(SHOOT_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e2));
    if (e3 != hipSuccess) return fail(SHOOT_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e3));
    return SHOOT_OK;
  }
  if (p->flags & SHOOT_CHECK_FINITE) {
    if (cs != hipStreamCaptureStatusNone)
      return fail(SHOOT_E_STATE, "SHOOT_CHECK_FINITE synchronises the stream: not allowed under stream capture");
    shoot_status st = check_finite(p, s);
    if (st != SHOOT_OK) return st;
  }
  if ((p->flags & SHOOT_NO_GRAPH) || cs != hipStreamCaptureStatusNone) {
    // inside the caller's capture the lanes stay on its stream
    hipError_t e = enqueue(p, op, s, cs != hipStreamCaptureStatusNone);
    if (e != hipSuccess) return fail(SHOOT_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SHOOT_OK;
  }
  // one graph per wave, captured on the device's capture stream at the first call
  if (p->graph[op].empty()) {
    std::lock_guard<std::mutex> lock(g_capture_mu);
    std::vector<hipGraphExec_t> gs;
    for (Wave& w : p->waves) {
      hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) {
        for (hipGraphExec_t y : gs) (void)hipGraphExecDestroy(y);
        return fail(SHOOT_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
      }
      e = enqueue_wave(p, w, op, p->cap);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(p->cap, &g);
      hipGraphExec_t x = nullptr;
      if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess || e2 != hipSuccess) {
        for (hipGraphExec_t y : gs) (void)hipGraphExecDestroy(y);
        if (e2 != hipSuccess) return fail(SHOOT_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
        return fail(SHOOT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      }
      gs.push_back(x);
    }
    p->graph[op] = gs;
  }
  for (const auto& g : p->groups) {
    HIPCHK(fork_lanes(p, s, g.second));
    for (int i = 0; i < g.second; ++i)
      HIPCHK(hipGraphLaunch(p->graph[op][g.first + i], lane_stream(p, s, g.second, i)));
    HIPCHK(join_lanes(p, s, g.second));
  }
  return SHOOT_OK;
}

}  // namespace

namespace {

// The operation the autotuner times: the gradient when every pair can take
// it, else the forward shot.
int autotune_op(const shoot_plan_s* p) {
  int op = OP_GRAD;
  for (const shoot_pair& q : p->pairs)
    if (!q.target || !q.out_grad) op = OP_FORWARD;
  if (p->flags & (SHOOT_SCHEME_EULERIAN | SHOOT_SCHEME_MIXED)) op = OP_FORWARD;
  return op;
}

int ceil_log2(long long v) {
  int k = 0;
  while ((1LL << k) < v) ++k;
  return k;
}

}  // namespace

std::string shoot_internal_tune_class(shoot_plan p) {
  if (!p) return "";
  long long vmax = 0;
  for (const Wave& w : p->waves) vmax = std::max(vmax, (long long)w.ntot);
  int xlo = 1 << 30, xhi = 0, rmax = 0;
  for (const shoot_pair& q : p->pairs) {
    const int lx = ceil_log2(q.shape[q.ndim - 1]);
    xlo = std::min(xlo, lx);
    xhi = std::max(xhi, lx);
    rmax = std::max(rmax, radius_of(q.sigma));
  }
  int rb = 1;
  while (rb < rmax) rb *= 2;
  int vlog = 0;
  while ((2LL << vlog) <= vmax) ++vlog;
  const uint32_t kf = p->flags & (SHOOT_FORCE_GLOBAL_SCATTER | SHOOT_SCHEME_EULERIAN | SHOOT_SCHEME_MIXED);
  char buf[128];
  std::snprintf(buf, sizeof(buf), "d%d-%s-v%d-x%d_%d-r%d-l%d-f%x", p->ndim, autotune_op(p) == OP_GRAD ? "grad" : "fwd",
                vlog, xlo, xhi, rb, p->lanes, (unsigned)kf);
  return buf;
}

int shoot_internal_device(shoot_plan p, int* unfused) {
  if (unfused) *unfused = p && p->uf ? 1 : 0;
  return p && (p->ws || p->uf) ? p->device : -1;
}

void shoot_internal_set_error(const char* msg) { g_err = msg ? msg : ""; }

int shoot_internal_pairs(shoot_plan p, const shoot_pair** pairs, int* bound) {
  if (!p) return -1;
  if (pairs) *pairs = p->pairs.data();
  if (bound) *bound = (p->ws != nullptr || p->uf != nullptr) ? 1 : 0;
  return p->npairs;
}

// ====================================================================== C ABI
// The library is built with hidden visibility; only this block is exported.
#pragma GCC visibility push(default)
extern "C" {

const char* shoot_version(void) { return "shoot 1.0 (gfx950)"; }

const char* shoot_last_error(void) { return g_err.c_str(); }

shoot_status shoot_plan_create(const shoot_pair* pairs, int32_t n_pairs, int32_t T, uint32_t flags,
                               size_t budget_bytes, shoot_plan* out) {
  if (!out) return fail(SHOOT_E_ARG, "out is NULL");
  *out = nullptr;
  const uint32_t known = SHOOT_FULL_STORE | SHOOT_UNFUSED | SHOOT_NO_GRAPH | SHOOT_FORCE_GLOBAL_SCATTER |
                         SHOOT_SCHEME_EULERIAN | SHOOT_SCHEME_MIXED | SHOOT_LANES_MASK | SHOOT_CHECK_FINITE;
  if (flags & ~known) return fail(SHOOT_E_ARG, "unknown flag bits");
  if (((flags & SHOOT_LANES_MASK) >> 8) > SHOOT_MAX_LANES) return fail(SHOOT_E_ARG, "SHOOT_LANES(n) needs n <= 8");
  const uint32_t schemes = flags & (SHOOT_SCHEME_EULERIAN | SHOOT_SCHEME_MIXED);
  if (schemes == (SHOOT_SCHEME_EULERIAN | SHOOT_SCHEME_MIXED))
    return fail(SHOOT_E_ARG, "SHOOT_SCHEME_EULERIAN and SHOOT_SCHEME_MIXED exclude each other");
  if (schemes && (flags & SHOOT_UNFUSED)) return fail(SHOOT_E_ARG, "the unfused path integrates semi-Lagrangianly only");
  if ((flags & SHOOT_CHECK_FINITE) && (flags & SHOOT_UNFUSED))
    return fail(SHOOT_E_ARG, "SHOOT_CHECK_FINITE is not available with SHOOT_UNFUSED");
  if (flags & SHOOT_UNFUSED)
    for (int i = 0; i < n_pairs && pairs; ++i)
      if (pairs[i].out_deformation)
        return fail(SHOOT_E_ARG, "the unfused path has no deformation output (pair " + std::to_string(i) + ")");
  shoot_status st = validate(pairs, n_pairs, T);
  if (st != SHOOT_OK) return st;
  shoot_plan_s* p = new (std::nothrow) shoot_plan_s();
  if (!p) return fail(SHOOT_E_ARG, "out of host memory");
  p->npairs = n_pairs;
  p->T = T;
  p->ndim = pairs[0].ndim;
  p->flags = flags;
  p->budget = budget_bytes;
  p->pairs.assign(pairs, pairs + n_pairs);
  for (int i = 0; i < n_pairs; ++i)
    if (pairs[i].out_deformation) p->has_def = true;
  // Checkpoint interval k (the sqrt(T) schedule): the k that needs the fewest
  // state slots, ceil(T / k) checkpoints + k - 1 inside a segment, which is
  // k = ceil(sqrt(T)) or a neighbour of it; among those the one with the fewest
  // recomputed steps, (ceil(T / k) - 1)(k - 1); on a tie the larger k. (T = 15:
  // k = 3, 4 and 5 all need 7 slots, 4 recomputes 9 steps, 3 and 5 recompute 8.)
  {
    long long best_m = -1, best_r = 0;
    for (int k = 1; k <= T; ++k) {
      const long long nck = (T + k - 1) / k, m = nck + k - 1, r = (nck - 1) * (k - 1);
      if (best_m < 0 || m < best_m || (m == best_m && r <= best_r)) {
        best_m = m;
        best_r = r;
        p->k = k;
      }
    }
  }
  p->nck = (T + p->k - 1) / p->k;
  if (fullstore(p)) {
    p->nst = T;
    p->nv = T;
  } else {
    p->nst = p->nck + p->k - 1;
    p->nv = p->k - 1 + p->nck;
  }
  if (flags & SHOOT_UNFUSED) {
    p->uf = unfused::create(p->pairs.data(), n_pairs, T);
    if (!p->uf) { delete p; return fail(SHOOT_E_ARG, "out of host memory"); }
    p->ws_bytes = unfused::workspace_bytes(p->uf);
    *out = p;
    g_err.clear();
    return SHOOT_OK;
  }
  // admission: first-fit in order into groups such that the whole workspace
  // (every wave's header, then the largest group's field region) fits the
  // budget; each group is split into concurrent lanes
  const int want = (int)((flags & SHOOT_LANES_MASK) >> 8);
  const int lanes = want ? want : (p->ndim == 2 ? 3 : 2);
  std::vector<int> cur;
  std::vector<Wave> lw;
  size_t fb = 0;
  size_t hdr_done = 0;  // header bytes of the committed groups' waves
  auto headers = [&](std::vector<Wave>& ws) {
    size_t h = 0;
    for (Wave& w : ws) h = header_size(p, w, h);
    return h;
  };
  auto commit = [&]() {
    p->groups.emplace_back((int)p->waves.size(), (int)lw.size());
    p->lanes = std::max(p->lanes, (int)lw.size());
    p->field_max = std::max(p->field_max, fb);
    hdr_done += headers(lw);
    for (Wave& w : lw) p->waves.push_back(w);
  };
  // workspace bytes if the group `ws` (field region `fbytes`) were committed next
  auto total_with = [&](std::vector<Wave>& ws, size_t fbytes) {
    return align_up(hdr_done + headers(ws), ALIGN) + std::max(p->field_max, fbytes);
  };
  if (!budget_bytes) {
    for (int i = 0; i < n_pairs; ++i) cur.push_back(i);
    fb = build_group(p, cur, lanes, want != 0, lw);
  } else {
    for (int i = 0; i < n_pairs; ++i) {
      std::vector<int> trial = cur;
      trial.push_back(i);
      std::vector<Wave> tw;
      const size_t tb = build_group(p, trial, lanes, want != 0, tw);
      if (!cur.empty() && total_with(tw, tb) > budget_bytes) {
        commit();
        cur.assign(1, i);
        fb = build_group(p, cur, lanes, want != 0, lw);
      } else {
        cur = trial;
        lw = tw;
        fb = tb;
      }
      if (cur.size() == 1 && total_with(lw, fb) > budget_bytes) {
        delete p;
        return fail(SHOOT_E_BUDGET, "pair " + std::to_string(i) + " alone needs " +
                                        std::to_string(total_with(lw, fb)) + " bytes with the plan's headers, over "
                                        "the budget");
      }
    }
  }
  commit();
  size_t o = 0;
  for (Wave& w : p->waves) o = header_size(p, w, o);
  p->header_total = align_up(o, ALIGN);
  p->ws_bytes = p->header_total + p->field_max;
  // host image of the header
  p->blob.assign(p->header_total, 0);
  for (Wave& w : p->waves) {
    auto put = [&](size_t off, const void* src, size_t bytes) {
      if (bytes) std::memcpy(p->blob.data() + off, src, bytes);
    };
    put(w.o_pd, w.pdev.data(), w.pdev.size() * sizeof(PairDev));
    put(w.o_tb, w.tb.data(), w.tb.size() * sizeof(Tile));
    put(w.o_ta, w.ta.data(), w.ta.size() * sizeof(Tile));
    put(w.o_tm, w.tm.data(), w.tm.size() * sizeof(Tile));
    for (int o = 0; o < 2; ++o) {
      put(w.o_tx[o], w.tx[o].data(), w.tx[o].size() * sizeof(Tile));
      put(w.o_ty[o], w.ty[o].data(), w.ty[o].size() * sizeof(Tile));
      put(w.o_tz[o], w.tz[o].data(), w.tz[o].size() * sizeof(Tile));
    }
  }
  *out = p;
  g_err.clear();
  return SHOOT_OK;
}

shoot_status shoot_plan_workspace_bytes(shoot_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(SHOOT_E_ARG, "NULL argument");
  *bytes = p->ws_bytes;
  return SHOOT_OK;
}

shoot_status shoot_plan_waves(shoot_plan p, int32_t* waves) {
  if (!p || !waves) return fail(SHOOT_E_ARG, "NULL argument");
  *waves = p->uf ? p->npairs : (int32_t)p->groups.size();
  return SHOOT_OK;
}

shoot_status shoot_plan_lanes(shoot_plan p, int32_t* lanes) {
  if (!p || !lanes) return fail(SHOOT_E_ARG, "NULL argument");
  *lanes = p->uf ? 1 : p->lanes;
  return SHOOT_OK;
}

shoot_status shoot_plan_bind(shoot_plan p, void* workspace, size_t bytes, void* stream) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (!workspace && p->ws_bytes) return fail(SHOOT_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace) % ALIGN) return fail(SHOOT_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < p->ws_bytes)
    return fail(SHOOT_E_WORKSPACE, "workspace too small: need " + std::to_string(p->ws_bytes) + " bytes");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  drop_graphs(p);
  if (dev != p->device) release_streams(p);
  HIPCHK(device_streams(p, dev));
  while ((int)p->ev_join.size() < p->lanes - 1) {
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    p->ev_join.push_back(ev);
  }
  if (p->lanes > 1 && !p->ev_fork) HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  p->device = dev;
  p->ws = (char*)workspace;
  p->descend_ready = false;
  if (p->scratch_bound) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    for (ScratchDev& d : g_scratch)
      if (d.owner == p) d.owner = nullptr;
    p->scratch_bound = false;
  }
  hipStream_t s = (hipStream_t)stream;
  if (p->uf) {
    hipError_t e = unfused::bind(p->uf, p->ws, s);
    if (e != hipSuccess) return fail(SHOOT_E_HIP, std::string("unfused bind: ") + hipGetErrorString(e));
    return SHOOT_OK;
  }
  if (p->header_total) HIPCHK(hipMemcpyAsync(p->ws, p->blob.data(), p->header_total, hipMemcpyHostToDevice, s));
  return SHOOT_OK;
}

shoot_status shoot_plan_bind_scratch(shoot_plan p, void* stream) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (p->uf) return fail(SHOOT_E_ARG, "the unfused path needs a caller workspace");
  if (!(p->flags & SHOOT_NO_GRAPH) || p->lanes != 1)
    return fail(SHOOT_E_ARG, "a scratch-bound plan runs eagerly in one lane: create it with SHOOT_NO_GRAPH | "
                             "SHOOT_LANES(1)");
  if (p->ws_bytes > SCRATCH_BYTES)
    return fail(SHOOT_E_WORKSPACE, "plan needs " + std::to_string(p->ws_bytes) + " bytes of workspace; the static "
                                   "scratch holds " + std::to_string(SCRATCH_BYTES) + " bytes");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  void* ptr = nullptr;
  HIPCHK(scratch_ptr(dev, &ptr));
  drop_graphs(p);
  if (p->scratch_bound)
    for (ScratchDev& d : g_scratch)
      if (d.owner == p) d.owner = nullptr;
  p->device = dev;
  p->ws = (char*)ptr;
  p->scratch_bound = true;
  p->descend_ready = false;
  if (p->header_total) HIPCHK(hipMemcpyAsync(p->ws, p->blob.data(), p->header_total, hipMemcpyHostToDevice, s));
  g_scratch[dev].owner = p;
  return SHOOT_OK;
}

shoot_status shoot_autotune(shoot_plan p, void* stream) {
  static_assert(SHOOT_TUNE_COUNT == TUNE_N, "tuning choices of the header and the runtime differ");
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (!p->ws) return fail(SHOOT_E_STATE, "plan is not bound to a workspace");
  if (p->uf) return SHOOT_OK;
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s) HIPCHK(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(SHOOT_E_STATE, "autotune cannot run under stream capture");
  const int op = autotune_op(p);
  // kernel families timed for each choice
  static const int fam[TUNE_N][3] = {
      {KI_XPASS_M, KI_XPASS_V, -1},
      {KI_SPASS_MID, KI_SPASS_V, KI_SPASS_MBAR},
      {KI_ADVECT, -1, -1},
      {KI_ADV_ADJ, -1, -1},
      {KI_EPILOGUE, -1, -1},
      {KI_XPASS_M, KI_XPASS_V, -1}};
  const bool was_profiling = p->profiling;
  long long saved_n[KI_COUNT];
  double saved_ms[KI_COUNT];
  for (int i = 0; i < KI_COUNT; ++i) { saved_n[i] = p->prof.launches[i]; saved_ms[i] = p->prof.ms[i]; }
  int saved_tune[TUNE_N];
  for (int k = 0; k < TUNE_N; ++k) saved_tune[k] = p->tune[k];
  auto restore = [&](bool keep_tune) {
    p->profiling = was_profiling;
    for (int i = 0; i < KI_COUNT; ++i) { p->prof.launches[i] = saved_n[i]; p->prof.ms[i] = saved_ms[i]; }
    if (!keep_tune)
      for (int k = 0; k < TUNE_N; ++k) p->tune[k] = saved_tune[k];
    drop_graphs(p);
  };
  // pass 0: every choice 0; pass 1: every choice 1 but the matrix-core x-pass;
  // pass 2: the matrix-core x-pass alone (it replaces the x-pass of both)
  double t[3][TUNE_N] = {};
  p->profiling = true;
  for (int pass = 0; pass < 3; ++pass) {
    for (int k = 0; k < TUNE_N; ++k) p->tune[k] = pass == 1 ? 1 : 0;
    p->tune[TUNE_XMFMA] = pass == 2 ? 1 : 0;
    for (int rep = 0; rep < 4; ++rep) {  // the first evaluation warms up and is not counted
      for (int i = 0; i < KI_COUNT; ++i) { p->prof.launches[i] = 0; p->prof.ms[i] = 0.0; }
      shoot_status st = execute(p, op, stream);
      if (st != SHOOT_OK) {
        restore(false);
        return st;
      }
      if (rep == 0) continue;
      for (int k = 0; k < TUNE_N; ++k)
        for (int j = 0; j < 3; ++j)
          if (fam[k][j] >= 0) t[pass][k] += p->prof.ms[fam[k][j]];
    }
  }
  for (int k = 0; k < TUNE_N; ++k)
    if (k != TUNE_XMFMA) p->tune[k] = (t[0][k] > 0.0 && t[1][k] < 0.97 * t[0][k]) ? 1 : 0;
  const double vec_x = p->tune[TUNE_XPASS] ? t[1][TUNE_XPASS] : t[0][TUNE_XPASS];
  p->tune[TUNE_XMFMA] = (vec_x > 0.0 && t[2][TUNE_XMFMA] < 0.97 * vec_x) ? 1 : 0;
  restore(true);
  return SHOOT_OK;
}

shoot_status shoot_plan_tune_class(shoot_plan p, char* buf, size_t len) {
  if (!p || !buf) return fail(SHOOT_E_ARG, "NULL argument");
  const std::string c = shoot_internal_tune_class(p);
  if (c.size() + 1 > len) return fail(SHOOT_E_ARG, "buffer too small: need " + std::to_string(c.size() + 1) + " bytes");
  std::memcpy(buf, c.c_str(), c.size() + 1);
  return SHOOT_OK;
}

shoot_status shoot_plan_get_tuning(shoot_plan p, int32_t* choices) {
  if (!p || !choices) return fail(SHOOT_E_ARG, "NULL argument");
  for (int k = 0; k < TUNE_N; ++k) choices[k] = p->tune[k];
  return SHOOT_OK;
}

shoot_status shoot_plan_set_tuning(shoot_plan p, const int32_t* choices) {
  if (!p || !choices) return fail(SHOOT_E_ARG, "NULL argument");
  for (int k = 0; k < TUNE_N; ++k)
    if (choices[k] != 0 && choices[k] != 1)
      return fail(SHOOT_E_ARG, "tuning choice " + std::to_string(k) + " must be 0 or 1");
  for (int k = 0; k < TUNE_N; ++k) p->tune[k] = choices[k];
  drop_graphs(p);
  return SHOOT_OK;
}

shoot_status shoot_plan_set_active(shoot_plan p, const int32_t* active, void* stream) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (p->uf) return fail(SHOOT_E_ARG, "pair selection is not available on the unfused path");
  if (active)
    for (int i = 0; i < p->npairs; ++i)
      if (active[i] != 0 && active[i] != 1)
        return fail(SHOOT_E_ARG, "active[" + std::to_string(i) + "] must be 0 or 1");
  hipStream_t s = (hipStream_t)stream;
  if (p->ws) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != p->device) return fail(SHOOT_E_STATE, "current device differs from the device the plan was bound on");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s) HIPCHK(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return fail(SHOOT_E_STATE, "pair selection cannot run under stream capture");
  }
  for (Wave& w : p->waves)
    for (size_t li = 0; li < w.ids.size(); ++li) {
      const int32_t a = active ? active[w.ids[li]] : 1;
      w.pdev[li].active = a;
      std::memcpy(p->blob.data() + w.o_pd + li * sizeof(PairDev) + offsetof(PairDev, active), &a, sizeof(a));
    }
  if (!p->ws) return SHOOT_OK;  // the header goes up with the bind
  if (p->scratch_bound) {
    // the scratch holds another plan's header: this one is uploaded whole at its next call
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[p->device].owner != p) return SHOOT_OK;
  }
  for (Wave& w : p->waves)
    HIPCHK(hipMemcpyAsync(p->ws + w.o_pd, p->blob.data() + w.o_pd, w.pdev.size() * sizeof(PairDev),
                          hipMemcpyHostToDevice, s));
  return SHOOT_OK;
}

shoot_status shoot_forward(shoot_plan p, void* stream) { return execute(p, OP_FORWARD, stream); }
shoot_status shoot_cost(shoot_plan p, void* stream) { return execute(p, OP_COST, stream); }
shoot_status shoot_grad_p0(shoot_plan p, void* stream) { return execute(p, OP_GRAD, stream); }

shoot_status shoot_descend(shoot_plan p, float eta0, int32_t reset, void* stream) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (p->uf) return fail(SHOOT_E_ARG, "descent is not available on the unfused path");
  if (reset) {
    if (!(eta0 > 0.f) || !std::isfinite(eta0)) return fail(SHOOT_E_ARG, "eta0 must be finite and > 0");
    if (eta0 != p->eta0) drop_graphs(p, OP_DESCEND_RESET);
    p->eta0 = eta0;
  } else if (!p->descend_ready) {
    return fail(SHOOT_E_STATE, "the first shoot_descend call after a bind must reset");
  } else if (p->scratch_bound) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[p->device].owner != p)
      return fail(SHOOT_E_STATE, "another plan used the static scratch since the last call: the descent must reset");
  }
  shoot_status st = execute(p, reset ? OP_DESCEND_RESET : OP_DESCEND, stream);
  if (st == SHOOT_OK) p->descend_ready = true;
  return st;
}

shoot_status shoot_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst) return fail(SHOOT_E_ARG, "NULL argument");
  if (((uintptr_t)src | (uintptr_t)dst | bytes) % 16)
    return fail(SHOOT_E_ARG, "pointers and size must be multiples of 16 bytes");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes && bytes) return fail(SHOOT_E_ARG, "src and dst overlap");
  HIPCHK(launch_stream_copy(src, dst, (long long)(bytes / 16), (hipStream_t)stream));
  return SHOOT_OK;
}

shoot_status shoot_plan_displacements(shoot_plan p, float* out, void* stream) {
  if (!p || !out) return fail(SHOOT_E_ARG, "NULL argument");
  if (p->uf) return fail(SHOOT_E_ARG, "displacements are not recorded on the unfused path");
  if (!p->ws) return fail(SHOOT_E_STATE, "plan is not bound to a workspace");
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s) HIPCHK(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(SHOOT_E_STATE, "reading displacements synchronises the stream");
  for (Wave& w : p->waves) {
    std::vector<unsigned> h(w.pdev.size() * (size_t)p->T);
    HIPCHK(hipMemcpyAsync(h.data(), p->ws + w.o_dmax, h.size() * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t li = 0; li < w.ids.size(); ++li)
      for (int t = 0; t < p->T; ++t) {
        float v;
        std::memcpy(&v, &h[li * p->T + t], sizeof(float));
        out[(size_t)w.ids[li] * p->T + t] = v;
      }
  }
  return SHOOT_OK;
}

shoot_status shoot_plan_set_profiling(shoot_plan p, int32_t enable) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (p->uf && enable) return fail(SHOOT_E_ARG, "profiling is not available on the unfused path");
  p->profiling = enable != 0;
  return SHOOT_OK;
}

shoot_status shoot_plan_reset_stats(shoot_plan p) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  for (int i = 0; i < KI_COUNT; ++i) { p->prof.launches[i] = 0; p->prof.ms[i] = 0.0; }
  return SHOOT_OK;
}

shoot_status shoot_plan_kernel_stats(shoot_plan p, int32_t index, const char** name, int64_t* launches,
                                     double* total_ms) {
  if (!p) return fail(SHOOT_E_ARG, "plan is NULL");
  if (index < 0 || index >= KI_COUNT) return fail(SHOOT_E_ARG, "kernel index out of range");
  if (name) *name = KNAMES[index];
  if (launches) *launches = p->prof.launches[index];
  if (total_ms) *total_ms = p->prof.ms[index];
  return SHOOT_OK;
}

shoot_status shoot_plan_destroy(shoot_plan p) {
  if (!p) return SHOOT_OK;
  if (p->scratch_bound) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    for (ScratchDev& d : g_scratch)
      if (d.owner == p) d.owner = nullptr;
  }
  drop_graphs(p);
  p->prof.release();
  release_streams(p);
  if (p->uf) unfused::destroy(p->uf);
  delete p;
  return SHOOT_OK;
}

}  // extern "C"
#pragma GCC visibility pop
