// Launchers of the gfx950 kernels (host side of kernels.hip / kernels_unfused.hip).
#pragma once

#include "shoot_internal.h"

namespace shoot {

struct AdvectArgs {
  const PairDev* pd;
  const Tile* tl;
  const float* V;       // v_t slot [NDIM][N] per pair
  const float* st;      // (I_t, z_t) slot
  float* st_out;        // (I_{t+1}, z_{t+1}) slot or null
  float* ab_out;        // last step: (I_T - J, 0) for the adjoint, or null
  float* sc_zero;       // last step: scatter accumulator to clear, or null
  unsigned* dmax;       // per pair and step: max |dt v| (float bits), or null
  int T, t;
  float* red_reg;       // first step: per-tile regulariser partials, or null
  float* red_ssd;       // last step: per-tile data-term partials, or null
  int last;             // 1 at t = T - 1 (write the outputs)
  int scheme;           // 0 semi-Lagrangian, 1 Eulerian, 2 semi-Lagrangian image + Eulerian momentum
};

struct AdjArgs {
  const PairDev* pd;
  const Tile* tl;        // adjoint tiles (x0, y0, z0)
  const float* V;        // v_t
  const float* st;       // (I_t, z_t)
  const float* ab_in;    // (Ibar_{t+1}, zbar_{t+1})
  float* sc;             // scatter parts of (Ibar_t, zbar_t)
  float* vb;             // vbar [NDIM][N]
  const unsigned* dmax;  // per pair and step: max |dt v| (float bits)
  int T, t;
  int force_global;      // scatter through global atomics regardless of D
};

struct EpiArgs {
  const PairDev* pd;
  const Tile* tl;
  const float* mb;       // mbar [NDIM][N]
  const float* st;       // (I_t, z_t)
  float* sc;             // scatter parts (read; cleared when step t - 1 scatters globally)
  float* ab_out;         // (Ibar_t, zbar_t) or null at t = 0
  const unsigned* dmax;  // per pair and step: max |dt v| (float bits)
  int T, t;
  int force_global;
  int first;             // t == 0: write the gradient
};

hipError_t launch_fill_u32(unsigned* p, long long n, unsigned v, hipStream_t s);
// dst <- src, n4 16-byte groups.
hipError_t launch_stream_copy(const void* src, void* dst, long long n4, hipStream_t s);
hipError_t launch_init(int ndim, const PairDev* pd, const Tile* tl, int nt, float* st, hipStream_t s);
// cnt[pair] += number of non-finite values in the pair's image, target, p0.
hipError_t launch_count_nonfinite(int ndim, const PairDev* pd, const Tile* tl, int nt, unsigned* cnt, hipStream_t s);
hipError_t launch_xpass(int ndim, bool gradmul, const PairDev* pd, const Tile* tl, int nt, size_t lds,
                        const float* src, float* dst, hipStream_t s);
// The x-pass on the matrix cores (kernels_mfma.hip); lds from xpass_mfma_lds.
hipError_t launch_xpass_mfma(int ndim, bool gradmul, const PairDev* pd, const Tile* tl, int nt, size_t lds,
                             const float* src, float* dst, hipStream_t s);
size_t xpass_mfma_lds(int ndim, int nx, int r, int nrows);
// rb: strided-pass outputs per thread (one of SPASS_RB); opt: tuning option
// (0 or 1) selecting the load batch of the elementwise kernels.
hipError_t launch_spass(int ndim, bool passz, int mode, int rb, const PairDev* pd, const Tile* tl, int nt,
                        size_t lds, const float* src, float* dst, const float* extra, hipStream_t s);
hipError_t launch_advect(int ndim, int opt, int nt, const AdvectArgs& a, hipStream_t s);
hipError_t launch_adv_adj(int ndim, int opt, int nt, const AdjArgs& a, hipStream_t s);
// 3-D adjoint of the advection over ADJ3 tiles (a.tl is the adjoint tile list).
hipError_t launch_adv_adj3(int nt, const AdjArgs& a, hipStream_t s);
hipError_t launch_epilogue(int ndim, int opt, int nt, const EpiArgs& a, hipStream_t s);
hipError_t launch_finalize(int npairs, const PairDev* pd, const float* red_reg, const float* red_ssd,
                           hipStream_t s);
// Deformation map, one step: psi_out = psi_in o (Id - dt v) (psi_in null: the
// identity; psi_out null: the pairs' outD).
hipError_t launch_deform(int ndim, const PairDev* pd, const Tile* tl, int nt, const float* V, const float* psi_in,
                         float* psi_out, hipStream_t s);
// Descent step after a gradient: per-pair step control, then p0 -= eta dH/dp0.
hipError_t launch_descend(int ndim, int npairs, const PairDev* pd, const Tile* tl, int nt, float* eta, float* prev,
                          int reset, float eta0, hipStream_t s);

}  // namespace shoot
