// Internal layout shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shoot {

// Largest Gaussian radius supported: floor(3 sigma) <= RMAX.
constexpr int RMAX = 31;
// Padded tap table: taps t = 0..2r hold w(t - r), the rest are zero, padded to
// a multiple of 4 so the tap loops run in blocks of four.
constexpr int WPAD = 4 * ((2 * RMAX + 1 + 3) / 4);   // 64

// Rows per tile of the x-pass on the matrix cores (tuning choice TUNE_XMFMA;
// all channels of the tile's rows are stacked 16 at a time).
constexpr int XPASS_MFMA_ROWS[2] = {8, 16};  // [ndim - 2]

// Threads per block for every kernel.
constexpr int NT = 256;
// Strided-pass tile: 64 columns along x x (NT/64) RB outputs along the pass
// axis (RB is a tuning option); a thread produces RB/4 outputs along the axis
// for four consecutive columns.
constexpr int SPASS_RB[2] = {16, 8};
// x-pass: 64-column segments per wave whose loads are in flight at once; the
// host sizes x-pass tiles so one batch fills a tile where the row allows.
constexpr int XSEG = 6;
// Block tiles of the elementwise kernels (init, advect, adjoint, epilogue):
// 1024 voxels, four per thread, x fastest. The adjoint gathers in LDS while
// the per-step displacement bound is below BLK*_HS pixels.
constexpr int BLK2_X = 32, BLK2_Y = 32, BLK2_HS = 2;
constexpr int BLK3_X = 32, BLK3_Y = 8, BLK3_Z = 4, BLK3_HS = 1;
// Tile of the 3-D adjoint of the advection (its own tile list): 16 x 8 x 8
// outputs, a thread owns four consecutive x; fields are staged on the tile
// grown by 2 along y and z and by 4 along x (whole 16-byte groups).
constexpr int ADJ3_X = 16, ADJ3_Y = 8, ADJ3_Z = 8;
// Voxels per load batch of the elementwise kernels (a batch's loads are in
// flight together; larger batches trade registers, hence occupancy, for
// memory-level parallelism per wave), per tuning option: [ndim - 2][option].
constexpr int ADV_BATCH[2] = {2, 1};  // [ndim - 2], global-gather advection
constexpr int ADJ_BATCH[1][2] = {{2, 4}};  // 2-D block-tile adjoint only
constexpr int ADJ_RING_BATCH2 = 2, ADJ_RING_BATCH3 = 1;
constexpr int EPI_BATCH[2] = {4, 2};  // [ndim - 2], epilogue without staging
// Tuning choices of a plan (each 0 or 1; 0 is the default): x-pass rows per
// tile (one output group per thread / the full fill batch), strided-pass
// outputs per thread (SPASS_RB), advection from an LDS-staged tile or by
// global gathers, the adjoint's load batch, and the epilogue from an
// LDS-staged tile or direct loads, and the x-pass on the vector units or on
// the fp32 matrix cores.
enum TuneKnob { TUNE_XPASS = 0, TUNE_SPASS, TUNE_ADVECT, TUNE_ADJ, TUNE_EPI, TUNE_XMFMA, TUNE_N };
// arrival points staged per adjoint tile: the tile grown by the bound on each side
template <int NDIM>
constexpr int ADJ_NQ() {
  return NDIM == 2 ? (BLK2_X + 2 * BLK2_HS) * (BLK2_Y + 2 * BLK2_HS)
                   : (BLK3_X + 2 * BLK3_HS) * (BLK3_Y + 2 * BLK3_HS) * (BLK3_Z + 2 * BLK3_HS);
}

// Per-pair descriptor, resident in the workspace. Geometry is stored as
// (nz, ny, nx) with nz = 1 in 2-D; channel / axis c of a vector field follows
// the array's own axis order (2-D: c0 = y, c1 = x; 3-D: c0 = z, c1 = y, c2 = x).
struct alignas(16) PairDev {
  int nz, ny, nx;
  int r;          // Gaussian radius floor(3 sigma)
  int ntap4;      // ceil((2r + 1) / 4)
  int xrows;      // rows per x-pass tile for this pair
  int elem_first; // index of this pair's first block tile
  int elem_count; // number of block tiles of this pair
  long long off;  // voxel offset of the pair in the batch
  long long N;    // voxels
  float rho, lam, dt;
  int active;     // 0: every kernel skips this pair (its outputs stay as they are)
  const float* S;
  const float* J;
  const float* p0;
  float* outI;
  float* outZ;
  float* outG;
  float* outCost;
  float* outD;    // deformation map psi_T [NDIM][N], or null
  float w[WPAD];  // padded taps (see WPAD)
};
static_assert(sizeof(long long) == 8 && sizeof(void*) == 8, "LP64 expected");
static_assert(__builtin_offsetof(PairDev, w) % 16 == 0, "taps must be 16-byte aligned");

// Tile entry of a launch list. Meaning of a/b/c per kernel family:
//   block tile : a = x0, b = y0, c = z0 (origin of a BLK tile)
//   x-pass     : a = first row (rows are (z, y) flattened), b = row count
//   y/z-pass   : a = first x, b = index along the third axis, c = first output
struct alignas(16) Tile {
  int pair, a, b, c;
};

// Maps blockIdx.x to a tile index so that each XCD (blocks are dealt to the 8
// XCDs round-robin) receives one contiguous run of the tile list: neighbouring
// tiles share halos and then share an L2.
__device__ __forceinline__ int xcd_tile(int nb) {
  const int b = blockIdx.x;
  const int q = nb >> 3, rem = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

}  // namespace shoot
