/*
 * shoot.h - C ABI of the MI355X (gfx950) library for semi-Lagrangian geodesic
 * shooting in Metamorphosis / LDDMM image registration
 * (François, Gori, Glaunès, "Metamorphic image registration using a
 * semi-Lagrangian scheme", arXiv:2106.08817).
 *
 * What the library computes, for each image pair (S, J) and initial momentum
 * p0 (Methods, Eqs. 1-9 and the semi-Lagrangian section), with T steps of
 * dt = 1/T on a unit-spaced grid, from (I_0, z_0) = (S, p0):
 *
 *   m_a  = z_t * D_a I_t                      (D_a: clamped central difference)
 *   v_a  = -G m_a                             (Eq. 3; G: separable Gaussian,
 *                                              taps exp(-k^2/2 sigma^2) normalised
 *                                              to sum 1, |k| <= floor(3 sigma),
 *                                              zero padding)
 *   y    = q - dt v(q)                        (foot points, semi-Lagrangian step)
 *   Ih   = Interp(I_t; y), zh = Interp(z_t; y) (clamped bilinear / trilinear)
 *   I_{t+1} = Ih + rho dt zh                  (image characteristic, Eqs. 5-6)
 *   z_{t+1} = zh (1 - dt sum_a D_a v_a)       (momentum characteristic, Eqs. 7-9)
 *
 * and the inexact-matching cost (Eq. 4), with norms taken as plain sums:
 *
 *   H = 1/2 ||I_T - J||^2 + lambda ( <m_0, G m_0> + rho ||p0||^2 ).
 *
 * The paper's mu is taken equal to rho (the LDDMM limit is rho = mu -> 0), so
 * rho = 0 is pure LDDMM. shoot_grad_p0 returns dH/dp0, the exact derivative
 * of this discrete H (a hand-written discrete adjoint of the whole loop; on a
 * grid line the interpolation derivative is one-sided, cell floor(c), and it
 * is zero where a foot coordinate is clamped at or beyond a border).
 *
 * Arithmetic is float32 throughout.
 *
 * Memory and streams
 *   Every buffer the kernels touch is owned by the caller: inputs, outputs and
 *   one workspace. The library allocates no device memory. A plan owns host
 *   memory, HIP events and (unless SHOOT_NO_GRAPH) captured HIP graphs, one
 *   per lane; the library keeps, per device, a few streams shared by all plans
 *   (lanes, graph capture; see SHOOT_LANES) until the process ends. Device
 *   pointers must stay valid and unchanged from shoot_plan_bind to
 *   shoot_plan_destroy (graphs replay them). Streams are hipStream_t passed as
 *   void*; NULL means the null stream. Execution calls are asynchronous on the
 *   stream and never synchronise it (except with SHOOT_CHECK_FINITE, or with
 *   profiling enabled).
 *
 * Errors
 *   Every entry point returns a shoot_status. Arguments are validated on the
 *   host before anything is enqueued; a failed call enqueues nothing.
 *   shoot_last_error() returns a thread-local message describing the last
 *   failure of the calling thread. NaN / Inf in the inputs propagate
 *   (unless SHOOT_CHECK_FINITE).
 *
 * Threads
 *   A plan must not be used by two threads at once. Different plans may be
 *   used from different threads; the library's shared state (the per-device
 *   streams, graph capture on the shared capture stream) is guarded by locks.
 */
#ifndef SHOOT_H
#define SHOOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum shoot_status {
  SHOOT_OK = 0,
  SHOOT_E_ARG = -1,       /* bad argument: null pointer, T < 1, sigma <= 0, ... */
  SHOOT_E_SHAPE = -2,     /* ndim not in {2,3}, an extent < 2, mixed ndim, too large */
  SHOOT_E_WORKSPACE = -3, /* workspace missing, misaligned or too small */
  SHOOT_E_BUDGET = -4,    /* one pair alone exceeds the memory budget */
  SHOOT_E_HIP = -5,       /* a HIP runtime call failed (message has the HIP error) */
  SHOOT_E_STATE = -6,     /* call out of order (e.g. execute before bind) */
  SHOOT_E_IO = -7         /* a file could not be written (message names it) */
} shoot_status;

/*
 * One image pair. Layout: C-contiguous float32, last axis contiguous ("x");
 * shape = (n0, n1) in 2-D or (n0, n1, n2) in 3-D, each extent >= 2.
 * All pointers are device pointers, at least 4-byte aligned (16-byte
 * recommended). image (S) and p0 are required. target (J) is required by
 * shoot_cost and shoot_grad_p0 and optional for shoot_forward. Any out_*
 * pointer may be NULL when that output is not wanted, except out_grad for
 * shoot_grad_p0.
 *   out_image    [N]  I_T              (shoot_forward)
 *   out_momentum [N]  z_T              (shoot_forward)
 *   out_grad     [N]  dH/dp0           (shoot_grad_p0)
 *   out_cost     [3]  (H, 1/2||I_T-J||^2, lambda(<m0,Gm0> + rho||p0||^2))
 *                     (shoot_cost, shoot_grad_p0, and shoot_forward when
 *                     target is given)
 *   out_deformation [ndim][N]  psi_T, the deformation map of the shot
 *                     (shoot_forward): psi_0 = Id, psi_{t+1} = psi_t o
 *                     (Id - dt v_t) with the scheme's clamped multilinear
 *                     weights, so that S o psi_T ~ I_T for rho = 0 (the
 *                     deformation grids of the Results section; the flow of
 *                     Methods integrated semi-Lagrangianly). Component a is
 *                     the grid coordinate along array axis a. Not available
 *                     with SHOOT_UNFUSED (SHOOT_E_ARG at plan creation).
 * rho >= 0 weighs the intensity residual; sigma > 0 is the kernel width in
 * pixels (sigma < 32/3, i.e. radius floor(3 sigma) <= 31); lambda >= 0 weighs
 * the regulariser.
 */
typedef struct shoot_pair {
  int32_t ndim;
  int32_t shape[3];
  float rho;
  float sigma;
  float lambda;
  const float* image;
  const float* target;
  const float* p0;
  float* out_image;
  float* out_momentum;
  float* out_grad;
  float* out_cost;
  float* out_deformation;
} shoot_pair;

typedef struct shoot_plan_s* shoot_plan;

/* Plan flags. */
#define SHOOT_FULL_STORE 1u            /* keep all T states instead of sqrt(T) checkpoints */
#define SHOOT_UNFUSED 2u               /* per-pair, one kernel per primitive (baseline) */
#define SHOOT_NO_GRAPH 4u              /* launch kernels eagerly, no internal HIP graph */
#define SHOOT_FORCE_GLOBAL_SCATTER 8u  /* adjoint scatter through per-corner global atomics only */
/* Integration options the paper compares with the full semi-Lagrangian scheme
 * (semi-Lagrangian section; forward and cost only, SHOOT_E_ARG for the
 * gradient): Eulerian: explicit Euler with clamped central differences,
 * I' = I - dt sum_a v_a D_a I + rho dt z, z' = z - dt sum_a D_a (z v_a);
 * mixed: semi-Lagrangian image, Eulerian momentum. */
#define SHOOT_SCHEME_EULERIAN 16u
#define SHOOT_SCHEME_MIXED 32u
/* Concurrent lanes: the pairs of an admission wave are split into up to n
 * lanes of balanced voxel count (each keeping the pairs' order); every lane
 * runs the whole schedule on its own stream, forked from and joined back into
 * the caller's stream, so that the kernels of different lanes overlap (a
 * lane's pairs fill the GPU while another lane's launch drains). Results are
 * identical whatever the lane count: pairs are independent and every pair's
 * arithmetic is the same. SHOOT_LANES(n), 1 <= n <= SHOOT_MAX_LANES, fixes the
 * count; without it a plan takes 3 lanes in 2-D and 2 in 3-D (at most one
 * lane per pair), and one lane for a wave of at least 2^23 voxels, whose
 * launches fill the GPU by themselves. The last lane runs on the caller's stream, the others on a
 * pool of streams that the library creates at the first bind on a device (3
 * lane streams, more when a plan asks for more lanes, then one graph-capture
 * stream), shared by all plans and kept until the process ends; lanes gain
 * only while the device has a hardware queue for each of their streams. Plans share the pool, so the lanes of two plans called on
 * different streams are ordered with each other. Inside the caller's stream
 * capture the lanes run one after another on the caller's stream. */
/* Input check: every execution call first counts, on the device, the
 * non-finite values (NaN, Inf) of each pair's image, target and p0, reads the
 * counts back (synchronising the stream; SHOOT_E_STATE under stream capture)
 * and fails with SHOOT_E_ARG, naming the first such pair, before enqueueing
 * anything else. Without it, non-finite inputs propagate into the outputs.
 * Not available with SHOOT_UNFUSED. */
#define SHOOT_CHECK_FINITE 64u
#define SHOOT_MAX_LANES 8
#define SHOOT_LANES(n) ((((uint32_t)(n)) & 15u) << 8)
#define SHOOT_LANES_MASK (15u << 8)

/* Library version string. Never NULL. */
const char* shoot_version(void);

/* Thread-local message of the calling thread's last failure ("" if none). */
const char* shoot_last_error(void);

/*
 * Create a plan for n_pairs >= 1 pairs sharing the step count T >= 1
 * (dt = 1/T). All pairs must have the same ndim. The descriptors are copied;
 * their device pointers are used from shoot_plan_bind on. Host-only: no HIP
 * call is made. budget_bytes caps the workspace (0 = no cap): pairs are
 * grouped into waves that each fit (with their lanes), run one after another
 * in the same workspace; SHOOT_E_BUDGET if a single pair does not fit.
 * On success *out receives the plan; on failure *out is set to NULL.
 */
shoot_status shoot_plan_create(const shoot_pair* pairs, int32_t n_pairs, int32_t T,
                               uint32_t flags, size_t budget_bytes, shoot_plan* out);

/* Workspace size in bytes (host-only). The workspace must be 256-byte aligned. */
shoot_status shoot_plan_workspace_bytes(shoot_plan plan, size_t* bytes);

/* Number of admission waves the plan runs (1 unless a budget forced more). */
shoot_status shoot_plan_waves(shoot_plan plan, int32_t* waves);

/* Largest number of concurrent lanes of an admission wave (1 for
 * SHOOT_UNFUSED plans). */
shoot_status shoot_plan_lanes(shoot_plan plan, int32_t* lanes);

/*
 * Attach the caller-owned device workspace and upload the plan's descriptors
 * and tile lists into it, asynchronously on `stream`. May be called again to
 * rebind (captured graphs are then discarded).
 */
shoot_status shoot_plan_bind(shoot_plan plan, void* workspace, size_t bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): attaches
 * the plan to the library's static scratch instead of a caller workspace and
 * uploads its descriptors there, asynchronously on `stream`; execution calls
 * then run as with shoot_plan_bind. Allocates nothing: the scratch is a
 * file-scope device array of 64 MiB per GPU, held from the library's first use
 * on that GPU until the process ends. SHOOT_E_WORKSPACE if the plan's
 * workspace (shoot_plan_workspace_bytes) exceeds 64 MiB (e.g. a 240x240 pair
 * at T = 20 needs about 10 MB, a 64^3 volume at T = 15 about 55 MB);
 * SHOOT_E_ARG unless the plan was created with SHOOT_NO_GRAPH | SHOOT_LANES(1)
 * (it runs eagerly on the caller's stream) or for SHOOT_UNFUSED plans.
 * Every scratch-bound plan on a GPU shares that GPU's array, which keeps the
 * last call's contents: an execution call of a plan other than the last one
 * bound or run there uploads its descriptors again first (a shoot_descend
 * without reset then fails with SHOOT_E_STATE, its step state being gone).
 * Calls of scratch-bound plans that overlap on one GPU (other streams, other
 * threads, or enqueued before the previous one completed on another stream)
 * race for the array. shoot_plan_bind returns the plan to a caller workspace.
 */
shoot_status shoot_plan_bind_scratch(shoot_plan plan, void* stream);

/*
 * Launch-shape tuning. A plan carries SHOOT_TUNE_COUNT choices, each 0 or 1
 * (0 = default), in this order:
 *   [0] x-pass rows per tile (at most one output group per thread / one
 *       full fill batch)
 *   [1] strided (y/z) pass outputs per thread (16 / 8)
 *   [2] advection: from an LDS-staged tile / by global gathers
 *   [3] adjoint load batch in 2-D (voxels per thread whose loads are in
 *       flight together: 2 / 4; the 3-D adjoint has one form)
 *   [4] adjoint epilogue: from an LDS-staged tile / by direct loads
 *   [5] Gaussian pass along x on the vector units / on the fp32 matrix cores
 *       (banded Toeplitz products, v_mfma_f32_16x16x4f32; for waves whose
 *       every last extent is a multiple of 4, else the vector units)
 * Every choice computes each output with the same operations in the same
 * order, so results are bit-identical whatever is chosen.
 */
#define SHOOT_TUNE_COUNT 6

/*
 * Pick the faster option of every tuning choice for this plan on the current
 * device: runs the plan's evaluation (the gradient when every pair has a
 * target and out_grad, else the forward shot; outputs are written as by that
 * call) with each option, timing every kernel with HIP events on `stream`,
 * and keeps an option other than the default only when it is at least 3 %
 * faster. Synchronising; not allowed while `stream` is being captured; a
 * no-op for SHOOT_UNFUSED plans. Optional.
 */
shoot_status shoot_autotune(shoot_plan plan, void* stream);

/*
 * The plan's shape class, the part of a tuning-cache key that describes the
 * plan: dimension, the operation the autotuner times (gradient or forward),
 * log2 of the largest wave's voxel count, the range of ceil(log2) of the
 * last extents, the largest Gaussian radius rounded up to a power of two,
 * the lane count and the flags that change kernels (hexadecimal), e.g.
 * "d3-grad-v25-x7_8-r16-l2-f0". Written NUL-terminated into buf (len bytes;
 * SHOOT_E_ARG if it does not fit). Host-only.
 */
shoot_status shoot_plan_tune_class(shoot_plan plan, char* buf, size_t len);

/*
 * shoot_autotune with a persistent cache: the JSON file `path` maps
 * "<gcnArchName>/<shape class>" (gcnArchName of the plan's device as HIP
 * reports it) to the tuning choices,
 *   {"format": "shoot-tune-1", "entries": {"<key>": [c0, c1, ...], ...}}.
 * When the plan's key is present with SHOOT_TUNE_COUNT values, each 0 or 1,
 * those choices are set and nothing runs (*hit = 1); otherwise the plan is
 * autotuned as by shoot_autotune (its outputs written as by that call) and
 * the file is rewritten with the new entry (*hit = 0); hit may be NULL. A
 * missing or unreadable file counts as empty; one that is not in this format
 * is replaced. The file is replaced whole (a temporary file renamed over
 * it): of concurrent writers the last one's entries remain. SHOOT_E_IO when
 * it cannot be written (the new choices are still set on the plan). A no-op
 * for SHOOT_UNFUSED plans (*hit = 0).
 */
shoot_status shoot_autotune_cached(shoot_plan plan, const char* path, int32_t* hit, void* stream);

/* Read / set the plan's tuning choices (arrays of SHOOT_TUNE_COUNT values;
 * each must be 0 or 1). Setting discards the plan's captured graphs. */
shoot_status shoot_plan_get_tuning(shoot_plan plan, int32_t* choices);
shoot_status shoot_plan_set_tuning(shoot_plan plan, const int32_t* choices);

/*
 * Shoot every pair: writes out_image (I_T) and out_momentum (z_T) when not
 * NULL, out_cost when both target and out_cost are given, and
 * out_deformation (psi_T) when not NULL.
 */
shoot_status shoot_forward(shoot_plan plan, void* stream);

/* Shoot every pair and write its cost (H, data, reg) to out_cost. */
shoot_status shoot_cost(shoot_plan plan, void* stream);

/*
 * Shoot every pair, then run the discrete adjoint backwards through the loop
 * (states restored from sqrt(T) checkpoints by recomputation, unless
 * SHOOT_FULL_STORE: a checkpoint every k steps, k the interval that needs the
 * fewest state slots, ceil(T / k) + k - 1, and of those recomputes the fewest
 * steps) and write dH/dp0 to out_grad, and the cost to out_cost when given.
 */
shoot_status shoot_grad_p0(shoot_plan plan, void* stream);

/*
 * Select the pairs that the execution calls (forward, cost, gradient,
 * descent) work on: active[i] = 1 evaluates pair i, 0 skips it, so that its
 * outputs (image, momentum, gradient, cost, deformation, descent step and p0)
 * keep what the last call that evaluated it wrote, and its displacement
 * record is stale; an optimiser whose pairs converge at different iterations
 * evaluates only those still searching. `active` holds n_pairs values, each 0
 * or 1 (SHOOT_E_ARG otherwise); NULL makes every pair active (the default).
 * On a bound plan the selection is uploaded on `stream` (ordered before the
 * calls enqueued after it there); not allowed while `stream` is being
 * captured (SHOOT_E_STATE). Captured graphs stay valid: the kernels read the
 * selection when they run. Not available on SHOOT_UNFUSED plans (SHOOT_E_ARG).
 */
shoot_status shoot_plan_set_active(shoot_plan plan, const int32_t* active, void* stream);

/*
 * One fixed-step gradient-descent iteration on every pair (the optional
 * update p0 <- p0 - eta dH/dp0 after the gradient; the paper optimises its
 * costs by gradient descent, Results). Evaluates cost and dH/dp0 exactly as
 * shoot_grad_p0 (out_grad and out_cost are required and hold the values at
 * the p0 of this call), then on the device halves a pair's step eta_i when
 * its cost rose since the previous call, and writes p0 - eta_i dH/dp0 into
 * the pair's p0 buffer, which must therefore be writable. With reset != 0
 * every eta_i starts at eta0 (finite, > 0) and no previous cost is compared;
 * the first call after shoot_plan_bind must reset (else SHOOT_E_STATE).
 * Asynchronous and graph-capturable like the other calls; not available on
 * SHOOT_UNFUSED plans (SHOOT_E_ARG).
 */
shoot_status shoot_descend(shoot_plan plan, float eta0, int32_t reset, void* stream);

/* ------------------------------------------------------------------ L-BFGS
 * Batched L-BFGS on every pair's p0 over a bound plan (the paper's
 * alternative to gradient descent for minimising H, Results): the
 * limited-memory BFGS two-loop recursion and Armijo backtracking, per pair,
 * with these conventions: at most m stored pairs (s, y), a new one after
 * every accepted step with rho = 1/(s.y) if s.y > 0 else 0; initial inverse
 * Hessian gamma Id with gamma = s.y / y.y of the newest pair (1/||g|| at the
 * start and after a failed search); d = -H g, or -g/||g|| when g.d >= 0;
 * steps t = 1, 1/2, ... for at most `trials` evaluations, accepting
 * H(x + t d) <= H(x) + c1 t g.d; a pair whose search fails stays at x and
 * forgets its history. Vector work runs on the device; every cost and
 * gradient comes from shoot_grad_p0 on the plan, and after a step's first
 * trial only the pairs still searching are evaluated (shoot_plan_set_active;
 * every pair is active again when the step returns).
 *
 * The plan must be created with target, out_grad and out_cost for every pair
 * (SHOOT_E_ARG otherwise), stay bound and outlive the optimiser; p0 buffers
 * are overwritten with the iterates. The optimiser owns host memory only; its
 * device workspace (shoot_lbfgs_workspace_bytes, 256-byte aligned) belongs to
 * the caller, holds (5 + 2m) floats per voxel, and must stay in place from
 * bind to destroy. Errors are reported through shoot_last_error.
 */
typedef struct shoot_lbfgs_s* shoot_lbfgs;

/* m in [1, 64], c1 in (0, 1), trials in [1, 64]. Host-only. */
shoot_status shoot_lbfgs_create(shoot_plan plan, int32_t m, float c1, int32_t trials, shoot_lbfgs* out);
shoot_status shoot_lbfgs_workspace_bytes(shoot_lbfgs opt, size_t* bytes);
/* Attaches the workspace and (re)starts the iteration at the current p0
 * (synchronises `stream`). */
shoot_status shoot_lbfgs_bind(shoot_lbfgs opt, void* workspace, size_t bytes, void* stream);
/* One iteration for every pair (synchronises `stream`); on return p0 holds the
 * new iterate and the plan's out_grad / out_cost its gradient and cost. */
shoot_status shoot_lbfgs_step(shoot_lbfgs opt, void* stream);
/* The cost of every pair at the start of the last step (host array of n
 * doubles, may be NULL) and the number of gradient evaluations it used. */
shoot_status shoot_lbfgs_last_step(shoot_lbfgs opt, double* cost_at_start, int32_t* evaluations);
shoot_status shoot_lbfgs_destroy(shoot_lbfgs opt);

/*
 * Diagnostics. With profiling enabled, execution calls run eagerly (no graph)
 * and synchronise the stream before returning. The lanes of a wave run one
 * after another on the caller's stream, the k-th launches of all lanes
 * together between one HIP event pair, so one timed launch covers all the
 * pairs of the wave. Per-kernel launch counts and total milliseconds
 * accumulate until reset. shoot_plan_kernel_stats returns
 * SHOOT_E_ARG for an index past the last kernel; *name stays owned by the
 * library.
 */
shoot_status shoot_plan_set_profiling(shoot_plan plan, int32_t enable);
shoot_status shoot_plan_reset_stats(shoot_plan plan);
shoot_status shoot_plan_kernel_stats(shoot_plan plan, int32_t index, const char** name, int64_t* launches,
                                     double* total_ms);

/*
 * Measurement reference: copies `bytes` (a multiple of 16) from src to dst
 * (device pointers, 16-byte aligned, not overlapping: SHOOT_E_ARG otherwise)
 * with a plain streaming kernel (one block of 256 threads per 16 KiB, each
 * thread moving four 16-byte groups), asynchronously on `stream`. Its rate is
 * the bandwidth a kernel that reads and writes every byte once can reach.
 */
shoot_status shoot_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/*
 * Largest foot displacement max_a |dt v_a| of every pair and step recorded by
 * the last execution call (its forward pass): out[i * T + t] for pair i and
 * step t, host memory of n_pairs * T floats. The adjoint of a step takes the
 * LDS gather when this is below 2 px (2-D) or 1 voxel (3-D), in 3-D the
 * scatter into an LDS box below 3 voxels, else the global atomic scatter.
 * Synchronises `stream` (SHOOT_E_STATE under capture);
 * SHOOT_E_ARG for SHOOT_UNFUSED plans. Values before the first execution call
 * are unspecified.
 */
shoot_status shoot_plan_displacements(shoot_plan plan, float* out, void* stream);

/* Release the plan's host memory, events and graphs (the shared streams
 * stay). NULL is a no-op. */
shoot_status shoot_plan_destroy(shoot_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* SHOOT_H */
