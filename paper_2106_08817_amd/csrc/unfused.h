// Per-pair, one-kernel-per-primitive path (SHOOT_UNFUSED): the baseline the
// batched path is measured against. Pairs run one after another; every
// primitive of a step (gradient, product, each Gaussian pass, negation,
// divergence, each gather, update; and each transpose in the adjoint) is its
// own launch through global memory, and the whole trajectory is stored.
#pragma once

#include <hip/hip_runtime.h>

#include "shoot.h"

namespace shoot {
namespace unfused {

struct Plan;

Plan* create(const shoot_pair* pairs, int n, int T);
size_t workspace_bytes(const Plan* p);
hipError_t bind(Plan* p, char* ws, hipStream_t s);
// op: 0 forward, 1 cost, 2 grad (same numbering as the fused runtime)
hipError_t run(Plan* p, int op, hipStream_t s);
void destroy(Plan* p);

}  // namespace unfused
}  // namespace shoot
