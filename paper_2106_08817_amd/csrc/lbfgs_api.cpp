// Batched L-BFGS on p0 (the paper's alternative optimiser to gradient
// descent, Results) on top of a bound plan: limited-memory BFGS two-loop
// recursion and Armijo backtracking per pair. Vector work (copies,
// combinations, dot products over N_i voxels) runs in the kernels of
// kernels_opt.hip over every pair at once; the per-pair scalars (step
// lengths, curvature, acceptance) are kept on the host, and every cost and
// gradient comes from shoot_grad_p0 on the plan.
//
// Conventions (same as the reference optimiser in the tests):
// * at most m stored pairs (s, y); a new pair is stored after every accepted
//   step with rho = 1 / s.y if s.y > 0, else rho = 0 (a no-op in the
//   recursion); a failed line search stores a zero pair and clears the
//   pair's history (all its rho = 0);
// * initial inverse Hessian gamma Id: gamma = s.y / y.y of the newest pair if
//   s.y > 0 and y.y > 0, else unchanged; 1 / ||g|| at the start and after a
//   failure;
// * d = -H g, replaced by -g / ||g|| when g.d >= 0;
// * t = 1, 1/2, ... for at most `trials` evaluations, accepting
//   H(x + t d) <= H(x) + c1 t g.d; a trial evaluates only the pairs still
//   searching (shoot_plan_set_active).
#include "shoot.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "opt.h"
#include "plan_access.h"

using namespace shoot::opt;

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct shoot_lbfgs_s {
  shoot_plan plan = nullptr;
  int n = 0, m = 0, trials = 0;
  float c1 = 1e-4f;
  std::vector<VecPair> vp;
  std::vector<VecTile> vt;
  long long ntot = 0;
  // workspace layout
  size_t o_vp = 0, o_vt = 0, o_part = 0, o_sc = 0, o_f = 0, ws_bytes = 0;
  char* ws = nullptr;
  // host state
  bool init = false;
  int head = 0;                       // ring slot of the next stored pair
  std::vector<double> f, gamma;       // cost at x, initial scaling
  std::vector<std::vector<double>> rho;  // [m][n]
  std::vector<double> f_start;        // cost at the start of the last step
  int evals = 0;                      // evaluations of the last step
  std::string err;
};

namespace {

shoot_status lfail(shoot_status st, const std::string& msg) {
  shoot_internal_set_error(msg.c_str());
  return st;
}

#define LCHK(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return lfail(SHOOT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Dev {
  const VecPair* vp;
  const VecTile* vt;
  int nt;
  double* part;
  double* sc_a;  // per-pair scalars uploaded from the host
  double* sc_b;
  double* sc_out;
  float* field(const shoot_lbfgs_s* L, int k) const {
    return reinterpret_cast<float*>(L->ws + L->o_f) + (size_t)k * (size_t)L->ntot;
  }
};

// field indices: X, G, Q, D, GN, then S[0..m), Y[0..m)
enum { F_X = 0, F_G, F_Q, F_D, F_GN, F_S };

Dev dev_of(const shoot_lbfgs_s* L) {
  Dev d;
  d.vp = reinterpret_cast<const VecPair*>(L->ws + L->o_vp);
  d.vt = reinterpret_cast<const VecTile*>(L->ws + L->o_vt);
  d.nt = (int)L->vt.size();
  d.part = reinterpret_cast<double*>(L->ws + L->o_part);
  d.sc_a = reinterpret_cast<double*>(L->ws + L->o_sc);
  d.sc_b = d.sc_a + L->n;
  d.sc_out = d.sc_b + L->n;
  return d;
}

hipError_t upload(double* dst, const std::vector<double>& h, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);  // the host vector may change right after
}

hipError_t download(std::vector<double>& h, const double* src, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(h.data(), src, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace

#pragma GCC visibility push(default)
extern "C" {

shoot_status shoot_lbfgs_create(shoot_plan plan, int32_t m, float c1, int32_t trials, shoot_lbfgs* out) {
  if (!out) return lfail(SHOOT_E_ARG, "out is NULL");
  *out = nullptr;
  const shoot_pair* pairs = nullptr;
  int bound = 0;
  const int n = shoot_internal_pairs(plan, &pairs, &bound);
  if (n < 1) return lfail(SHOOT_E_ARG, "plan is NULL");
  if (m < 1 || m > 64) return lfail(SHOOT_E_ARG, "m must be in [1, 64]");
  if (!(c1 > 0.f && c1 < 1.f)) return lfail(SHOOT_E_ARG, "c1 must be in (0, 1)");
  if (trials < 1 || trials > 64) return lfail(SHOOT_E_ARG, "trials must be in [1, 64]");
  for (int i = 0; i < n; ++i) {
    if (!pairs[i].target || !pairs[i].out_grad || !pairs[i].out_cost)
      return lfail(SHOOT_E_ARG, "every pair needs target, out_grad and out_cost (pair " + std::to_string(i) + ")");
  }
  shoot_lbfgs_s* L = new (std::nothrow) shoot_lbfgs_s();
  if (!L) return lfail(SHOOT_E_ARG, "out of host memory");
  L->plan = plan;
  L->n = n;
  L->m = m;
  L->c1 = c1;
  L->trials = trials;
  long long off = 0;
  for (int i = 0; i < n; ++i) {
    long long N = 1;
    for (int a = 0; a < pairs[i].ndim; ++a) N *= pairs[i].shape[a];
    VecPair P;
    P.off = off;
    P.n = N;
    P.p0 = const_cast<float*>(pairs[i].p0);
    P.grad = pairs[i].out_grad;
    P.cost = pairs[i].out_cost;
    P.tile_first = (int)L->vt.size();
    for (long long s0 = 0; s0 < N; s0 += VEC_TILE) L->vt.push_back(VecTile{i, (int)s0});
    P.tile_count = (int)L->vt.size() - P.tile_first;
    L->vp.push_back(P);
    off += (N + 63) / 64 * 64;
  }
  L->ntot = off;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, ALIGN); return r; };
  L->o_vp = take(L->vp.size() * sizeof(VecPair));
  L->o_vt = take(L->vt.size() * sizeof(VecTile));
  L->o_part = take(L->vt.size() * sizeof(double));
  L->o_sc = take(3 * (size_t)n * sizeof(double));
  L->o_f = take((size_t)(F_S + 2 * m) * (size_t)L->ntot * sizeof(float));
  L->ws_bytes = o;
  L->f.assign(n, 0.0);
  L->gamma.assign(n, 1.0);
  L->rho.assign(m, std::vector<double>(n, 0.0));
  L->f_start.assign(n, 0.0);
  *out = L;
  shoot_internal_set_error("");
  return SHOOT_OK;
}

shoot_status shoot_lbfgs_workspace_bytes(shoot_lbfgs L, size_t* bytes) {
  if (!L || !bytes) return lfail(SHOOT_E_ARG, "NULL argument");
  *bytes = L->ws_bytes;
  return SHOOT_OK;
}

shoot_status shoot_lbfgs_bind(shoot_lbfgs L, void* workspace, size_t bytes, void* stream) {
  if (!L) return lfail(SHOOT_E_ARG, "optimiser is NULL");
  if (!workspace) return lfail(SHOOT_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace) % ALIGN) return lfail(SHOOT_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < L->ws_bytes)
    return lfail(SHOOT_E_WORKSPACE, "workspace too small: need " + std::to_string(L->ws_bytes) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  L->ws = (char*)workspace;
  LCHK(hipMemcpyAsync(L->ws + L->o_vp, L->vp.data(), L->vp.size() * sizeof(VecPair), hipMemcpyHostToDevice, s));
  LCHK(hipMemcpyAsync(L->ws + L->o_vt, L->vt.data(), L->vt.size() * sizeof(VecTile), hipMemcpyHostToDevice, s));
  // history fields start at zero: unused ring slots are exact no-ops
  LCHK(hipMemsetAsync(L->ws + L->o_f, 0, L->ws_bytes - L->o_f, s));
  LCHK(hipStreamSynchronize(s));
  L->init = false;
  return SHOOT_OK;
}

shoot_status shoot_lbfgs_step(shoot_lbfgs L, void* stream) {
  if (!L) return lfail(SHOOT_E_ARG, "optimiser is NULL");
  if (!L->ws) return lfail(SHOOT_E_STATE, "optimiser is not bound to a workspace");
  int bound = 0;
  if (shoot_internal_pairs(L->plan, nullptr, &bound) < 1 || !bound)
    return lfail(SHOOT_E_STATE, "plan is not bound to a workspace");
  hipStream_t s = (hipStream_t)stream;
  const int n = L->n, m = L->m;
  const Dev d = dev_of(L);
  float* X = d.field(L, F_X);
  float* G = d.field(L, F_G);
  float* Q = d.field(L, F_Q);
  float* D = d.field(L, F_D);
  float* GN = d.field(L, F_GN);
  auto S = [&](int k) { return d.field(L, F_S + k); };
  auto Y = [&](int k) { return d.field(L, F_S + m + k); };
  std::vector<double> a(n), b(n), r(n);
  auto eval = [&]() -> shoot_status {
    shoot_status st = shoot_grad_p0(L->plan, stream);
    if (st != SHOOT_OK) return lfail(st, std::string("gradient evaluation: ") + shoot_last_error());
    LCHK(costs(d.vp, n, d.sc_out, s));
    LCHK(download(r, d.sc_out, s));
    ++L->evals;
    return SHOOT_OK;
  };
  auto dotp = [&](const float* A, const float* B, std::vector<double>& res) -> hipError_t {
    hipError_t e = dot(d.vp, d.vt, d.nt, n, A, B, d.part, d.sc_out, s);
    if (e != hipSuccess) return e;
    return download(res, d.sc_out, s);
  };
  auto combine = [&](float* Yf, const float* Xf, const std::vector<double>& ca,
                     const std::vector<double>& cb) -> hipError_t {
    hipError_t e = upload(d.sc_a, ca, s);
    if (e != hipSuccess) return e;
    e = upload(d.sc_b, cb, s);
    if (e != hipSuccess) return e;
    return comb(d.vp, d.vt, d.nt, Yf, Xf, d.sc_a, d.sc_b, s);
  };
  L->evals = 0;
  if (!L->init) {
    shoot_status st = eval();
    if (st != SHOOT_OK) return st;
    L->f = r;
    LCHK(load(d.vp, d.vt, d.nt, X, 0, s));
    LCHK(load(d.vp, d.vt, d.nt, G, 1, s));
    LCHK(dotp(G, G, a));
    for (int i = 0; i < n; ++i) L->gamma[i] = 1.0 / std::max(std::sqrt(a[i]), 1e-300);
    for (auto& rr : L->rho) std::fill(rr.begin(), rr.end(), 0.0);
    L->head = 0;
    L->init = true;
  }
  L->f_start = L->f;
  // two-loop recursion: Q = H G (newest to oldest, then back)
  const std::vector<double> zero(n, 0.0), one(n, 1.0);
  LCHK(combine(Q, G, zero, one));
  std::vector<std::vector<double>> alpha(m, std::vector<double>(n, 0.0));
  auto used = [&](int k) {
    for (int i = 0; i < n; ++i)
      if (L->rho[k][i] != 0.0) return true;
    return false;
  };
  for (int j = 0; j < m; ++j) {
    const int k = (L->head - 1 - j + 2 * m) % m;
    if (!used(k)) continue;
    LCHK(dotp(S(k), Q, a));
    for (int i = 0; i < n; ++i) {
      alpha[k][i] = L->rho[k][i] != 0.0 ? L->rho[k][i] * a[i] : 0.0;
      b[i] = -alpha[k][i];
    }
    LCHK(combine(Q, Y(k), one, b));
  }
  LCHK(combine(Q, nullptr, L->gamma, zero));
  for (int j = m - 1; j >= 0; --j) {
    const int k = (L->head - 1 - j + 2 * m) % m;
    if (!used(k)) continue;
    LCHK(dotp(Y(k), Q, a));
    for (int i = 0; i < n; ++i) b[i] = L->rho[k][i] != 0.0 ? alpha[k][i] - L->rho[k][i] * a[i] : 0.0;
    LCHK(combine(Q, S(k), one, b));
  }
  // D = -Q, or -G / ||G|| where that is not a descent direction
  std::vector<double> minus(n, -1.0);
  LCHK(combine(D, Q, zero, minus));
  std::vector<double> gd(n), gg(n);
  LCHK(dotp(G, D, gd));
  LCHK(dotp(G, G, gg));
  {
    std::vector<double> ca(n), cb(n);
    bool any = false;
    for (int i = 0; i < n; ++i) {
      if (!(gd[i] < 0.0)) {
        const double gn = std::max(std::sqrt(gg[i]), 1e-300);
        ca[i] = 0.0; cb[i] = -1.0 / gn; gd[i] = -gn; any = true;
      } else {
        ca[i] = 1.0; cb[i] = 0.0;
      }
    }
    if (any) LCHK(combine(D, G, ca, cb));
  }
  // Armijo backtracking, every pair at once; after the first trial only the
  // pairs still searching are evaluated (the others keep the cost and
  // gradient of their accepted point)
  std::vector<double> t(n, 1.0), tfin(n, 0.0), fnew(L->f);
  std::vector<char> done(n, 0);
  int left = n;
  std::vector<int32_t> searching(n, 1);
  struct AllActive {  // every pair active again when the step ends, however it ends
    shoot_plan plan;
    void* stream;
    bool set = false;
    ~AllActive() {
      if (set) (void)shoot_plan_set_active(plan, nullptr, stream);
    }
  } all_active{L->plan, stream};
  auto select = [&]() -> shoot_status {
    for (int i = 0; i < n; ++i) searching[i] = done[i] ? 0 : 1;
    all_active.set = true;
    shoot_status st = shoot_plan_set_active(L->plan, searching.data(), stream);
    if (st != SHOOT_OK) return lfail(st, std::string("pair selection: ") + shoot_last_error());
    return SHOOT_OK;
  };
  for (int trial = 0; trial < L->trials && left > 0; ++trial) {
    std::vector<double> tt(n);
    for (int i = 0; i < n; ++i) tt[i] = done[i] ? tfin[i] : t[i];
    LCHK(upload(d.sc_a, tt, s));
    LCHK(set_p0(d.vp, d.vt, d.nt, X, D, d.sc_a, s));
    if (left < n) {
      shoot_status st = select();
      if (st != SHOOT_OK) return st;
    }
    shoot_status st = eval();
    if (st != SHOOT_OK) return st;
    for (int i = 0; i < n; ++i) {
      if (done[i]) continue;
      if (r[i] <= L->f[i] + (double)L->c1 * t[i] * gd[i]) {
        done[i] = 1; tfin[i] = t[i]; fnew[i] = r[i]; --left;
      } else {
        t[i] *= 0.5;
      }
    }
  }
  if (left > 0) {
    // failed pairs stay at x: evaluate them once more so that every pair's
    // gradient output is the gradient at its new point
    LCHK(upload(d.sc_a, tfin, s));
    LCHK(set_p0(d.vp, d.vt, d.nt, X, D, d.sc_a, s));
    if (left < n) {
      shoot_status st = select();
      if (st != SHOOT_OK) return st;
    }
    shoot_status st = eval();
    if (st != SHOOT_OK) return st;
  }
  if (all_active.set) {
    all_active.set = false;
    shoot_status st = shoot_plan_set_active(L->plan, nullptr, stream);
    if (st != SHOOT_OK) return lfail(st, std::string("pair selection: ") + shoot_last_error());
  }
  // store (s, y) = (t d, g_new - g) in the ring; x, g <- new point
  const int k = L->head;
  LCHK(combine(S(k), D, zero, tfin));
  LCHK(load(d.vp, d.vt, d.nt, GN, 1, s));
  LCHK(sub(d.vp, d.vt, d.nt, Y(k), GN, G, s));
  std::vector<double> sy(n), yy(n);
  LCHK(dotp(S(k), Y(k), sy));
  LCHK(dotp(Y(k), Y(k), yy));
  for (int i = 0; i < n; ++i) {
    if (!done[i]) {
      for (int j = 0; j < m; ++j) L->rho[j][i] = 0.0;
      L->gamma[i] = 1.0 / std::max(std::sqrt(gg[i]), 1e-300);
      continue;
    }
    L->rho[k][i] = sy[i] > 0.0 ? 1.0 / sy[i] : 0.0;
    if (sy[i] > 0.0 && yy[i] > 0.0) L->gamma[i] = sy[i] / yy[i];
    L->f[i] = fnew[i];
  }
  L->head = (L->head + 1) % m;
  LCHK(load(d.vp, d.vt, d.nt, X, 0, s));
  LCHK(combine(G, GN, zero, one));
  LCHK(hipStreamSynchronize(s));
  return SHOOT_OK;
}

shoot_status shoot_lbfgs_last_step(shoot_lbfgs L, double* cost_at_start, int32_t* evaluations) {
  if (!L) return lfail(SHOOT_E_ARG, "optimiser is NULL");
  if (cost_at_start)
    for (int i = 0; i < L->n; ++i) cost_at_start[i] = L->f_start[i];
  if (evaluations) *evaluations = L->evals;
  return SHOOT_OK;
}

shoot_status shoot_lbfgs_destroy(shoot_lbfgs L) {
  delete L;
  return SHOOT_OK;
}

}  // extern "C"
#pragma GCC visibility pop
