// Batched per-pair vector operations of the L-BFGS driver (kernels_opt.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace shoot {
namespace opt {

constexpr int VEC_TILE = 4096;  // elements per 1-D tile

struct VecPair {
  long long off;      // offset of the pair in the batch buffers
  long long n;        // elements
  float* p0;          // the pair's p0 buffer (written by set_p0)
  const float* grad;  // the pair's dH/dp0 output of the plan
  const float* cost;  // the pair's (H, data, reg) output of the plan
  int tile_first, tile_count;
};

struct VecTile {
  int pair, start;
};

// dst = p0 (which = 0) or dH/dp0 (which = 1) of every pair
hipError_t load(const VecPair* vp, const VecTile* vt, int nt, float* dst, int which, hipStream_t s);
// p0 = X + t_pair D
hipError_t set_p0(const VecPair* vp, const VecTile* vt, int nt, const float* X, const float* D, const double* t,
                  hipStream_t s);
// Y = a_pair Y + b_pair X (X may be null: Y = a Y; a_pair = 0: Y = b X)
hipError_t comb(const VecPair* vp, const VecTile* vt, int nt, float* Y, const float* X, const double* a,
                const double* b, hipStream_t s);
// out = A - B
hipError_t sub(const VecPair* vp, const VecTile* vt, int nt, float* out, const float* A, const float* B,
               hipStream_t s);
// out_pair = H of the pair (from the plan's cost output)
hipError_t costs(const VecPair* vp, int npairs, double* out, hipStream_t s);
// out_pair = sum A B over the pair (double; partial holds one value per tile)
hipError_t dot(const VecPair* vp, const VecTile* vt, int nt, int npairs, const float* A, const float* B,
               double* partial, double* out, hipStream_t s);

}  // namespace opt
}  // namespace shoot
