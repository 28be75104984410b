/* mpe.h -- C ABI of libmpe, the MI355X (gfx950) implementation of the
 * any-order imaginary-time propagation eigensolver of Chin, Janecek and
 * Krotscheck (arXiv:0809.3739).
 *
 * Problem (Introduction, Eqs. Ham, evol, propstep, ortho): find the lowest
 * n states of H = -(hbar^2/2m) Lap + V on a periodic 3-D grid by repeatedly
 * applying an approximation of exp(-dt H) (dt = -epsilon > 0) to a block of
 * states and orthonormalising the block after every step.
 *
 * Conventions shared by every call:
 *  - A state block is a device array [m][nz][ny][nx] (x fastest, C order),
 *    m = n_states + n_guard, contiguous, of the plan's data type: double for
 *    MPE_FP64, float for MPE_FP32.  States are normalised discretely
 *    (sum over grid points of psi^2 = 1; no volume element).
 *  - Grid points are x_j = -L/2 + j L/n along each axis (periodic).
 *  - Device pointers are HIP device addresses (e.g. torch tensor data_ptr());
 *    host pointers are ordinary host memory owned by the caller.
 *  - Every call enqueues its work on the plan's stream.  Calls that return
 *    host arrays synchronise that stream before returning.
 *  - Calls return a status code and never abort or throw across the ABI; the
 *    plan keeps a message for the last failure (mpe_last_error).
 *  - A plan must not be used from two host threads at once.
 */
#ifndef MPE_H_
#define MPE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPE_ABI_VERSION 1

typedef struct mpe_plan_s* mpe_plan;

typedef enum {
  MPE_OK = 0,
  MPE_ERR_INVALID_ARGUMENT = 1,   /* null pointer, bad size, bad order ...          */
  MPE_ERR_UNSUPPORTED = 2,        /* grid size / precision without a kernel          */
  MPE_ERR_OUT_OF_MEMORY = 3,      /* device workspace allocation failed              */
  MPE_ERR_NOT_POSITIVE_DEFINITE = 4, /* overlap S not SPD: states linearly dependent */
  MPE_ERR_EIG_NO_CONVERGENCE = 5, /* Jacobi sweeps exhausted                          */
  MPE_ERR_NONFINITE = 6,          /* NaN/Inf met in the states or the overlaps       */
  MPE_ERR_DEVICE = 7,             /* a HIP runtime call failed                       */
  MPE_ERR_STATE = 8               /* call order violated (e.g. no potential set)     */
} mpe_status;

typedef enum {
  MPE_FP64 = 0,   /* float64 states, transforms and combination                       */
  MPE_FP32 = 1    /* float32 states and transforms; float64 c_k combination, overlaps,
                     Cholesky and Rayleigh-Ritz                                        */
} mpe_precision;

/* Version of this ABI (MPE_ABI_VERSION). */
int mpe_abi_version(void);

/* Static description of a status code. */
const char* mpe_status_string(mpe_status s);

/* Coefficients c_1..c_K of the order-2K multi-product expansion (Section II,
 * Eq. coef: c_i = prod_{j != i} i^2/(i^2 - j^2)), as float64 from exact
 * rational arithmetic.  order = 2K with K = 1..6; c must hold K doubles.
 * Errors: INVALID_ARGUMENT for a bad order or null c. */
mpe_status mpe_coefficients(int32_t order, double* c);

/* Create a plan (Introduction, problem statement; Section II for `order`).
 *  grid[3]  = (nx, ny, nz); each in {8,16,32,48,64,96,128,192}.  Grids with
 *             nx == ny run two passes per transform (x and y planes in one)
 *             except float64 planes of 192 points, which like every grid with
 *             nx != ny run three (see mpe_set_three_pass).  Others: UNSUPPORTED.
 *  box[3]   = (Lx, Ly, Lz) > 0, periodic box lengths.
 *  n_states = states whose convergence is checked; n_guard extra states carried
 *             along (m = n_states + n_guard <= 128 and m <= nx*ny*nz).
 *  order    = 2K, K = 1..6 (orders 2, 4, ..., 12).
 *  prec     = MPE_FP64 or MPE_FP32.
 *  hip_stream = hipStream_t to enqueue on (NULL = the null stream).
 * The plan owns its device workspace (chain spectra, propagated states, H
 * applied to them, overlap partials, small matrices) and frees it in
 * mpe_plan_destroy.  On failure *out is NULL. */
mpe_status mpe_plan_create(mpe_plan* out, const int32_t grid[3], const double box[3], int32_t n_states,
                           int32_t order, mpe_precision prec, int32_t n_guard, void* hip_stream);

mpe_status mpe_plan_destroy(mpe_plan p);

/* Message of the last failure on this plan (static storage of the plan). */
const char* mpe_last_error(mpe_plan p);

/* Device bytes held by the plan's workspace. */
int64_t mpe_workspace_bytes(mpe_plan p);

/* Set the potential V (Eq. Ham).  V: device float64 array [nz][ny][nx];
 * hbar2_over_m = hbar^2/m > 0 (1 in atomic units).  The plan keeps its own
 * copies; V may be freed afterwards.  Errors: INVALID_ARGUMENT, DEVICE. */
mpe_status mpe_set_potential(mpe_plan p, const double* V, double hbar2_over_m);

/* One multi-product step (Section II, Eq. mcomp; Section I, Eqs. so, propstep):
 * psi <- sum_k c_k T2(dt/k)^k psi for all m states, in place, with
 * T2(tau) = exp(-tau V/2) exp(-tau T) exp(-tau V/2).  dt > 0.  No ortho-
 * normalisation.  Errors: INVALID_ARGUMENT (dt <= 0, null), STATE (no V). */
mpe_status mpe_step(mpe_plan p, void* psi, double dt);

/* hpsi <- H psi for all m states (Eq. Ham; T applied spectrally).  psi and
 * hpsi are distinct device arrays of the plan's type. */
mpe_status mpe_apply_h(mpe_plan p, const void* psi, void* hpsi);

/* Orthonormalise the block in place (Section I, Eq. ortho): S = Psi Psi^T
 * (float64), S = L L^T, Psi <- L^-1 Psi.  On NOT_POSITIVE_DEFINITE or
 * NONFINITE psi is left unchanged. */
mpe_status mpe_orthonormalize(mpe_plan p, void* psi);

/* Rayleigh-Ritz rotation in span(psi) (Section III, subspace
 * orthogonalisation): solves Hs c = theta S c with S = Psi Psi^T and
 * Hs = Psi (H Psi)^T, rotates psi in place to the Ritz vectors (orthonormal,
 * ascending theta) and writes the m Ritz values to eig (host, m doubles).
 * Caches H psi for mpe_residuals; any other call drops the cache.  On
 * failure psi is left unchanged. */
mpe_status mpe_rayleigh_ritz(mpe_plan p, void* psi, double* eig);

/* Variances of Section III for the block psi with values eig (host, m):
 *   rh[j] = sum_k |H psi_j(r_k) - eig_j psi_j(r_k)|^2          (R^H)
 *   re[j] = ||phi_j - mu_j psi_j||^2, phi = T_order(dt) psi, mu_j = (psi_j|phi_j)
 *           (R^E, E_i of the paper read as the state's own value; dt is the
 *           last dt given to mpe_step or mpe_iterate; nullable)
 * rh: host, m doubles (required). */
mpe_status mpe_residuals(mpe_plan p, const void* psi, const double* eig, double* rh, double* re);

/* Drop the H psi kept by the last mpe_rayleigh_ritz / mpe_iterate (see above
 * and mpe_set_locked).  The library recognises the block only by its device
 * address, so a caller that writes the block itself (or frees it and lets the
 * address be reused) must call this before the next mpe_residuals or locked
 * mpe_iterate; they then apply H afresh.  Always MPE_OK for a valid plan. */
mpe_status mpe_forget_cached_h(mpe_plan p);

/* One fused iteration (Section I, Eqs. propstep and ortho; Section III):
 *   Phi = T_order(dt) psi; H Phi; S = Phi Phi^T, Hs = Phi (H Phi)^T,
 *   M = psi Phi^T; generalised eigenproblem Hs c = theta S c by Cholesky and
 *   Jacobi; psi <- Phi C (orthonormal Ritz vectors, ascending theta).
 * Host outputs (m doubles each, any may be NULL):
 *   eig     Ritz values theta_j
 *   rh      R^H_j of the new psi
 *   re      R^E_j = S_jj - M_jj^2       (variance of the incoming psi_j)
 *   re_perp S_jj - sum_i M_ij^2          (basis-invariant R^E)
 * re / re_perp assume the incoming psi is orthonormal.  On failure psi is
 * left unchanged. */
mpe_status mpe_iterate(mpe_plan p, void* psi, double dt, double* eig, double* rh, double* re, double* re_perp);

/* Graph replay of mpe_iterate (off by default).  On: the first call for a
 * given psi array captures the iteration's launches into a hipGraph on a
 * private stream ordered after the plan's stream; later calls with the same
 * psi, launch grouping and lock setting replay it (dt enters through tables
 * rebuilt outside the graph).  Off: every launch is enqueued eagerly on the
 * plan's stream.  Eager is the default because it measured as fast or faster
 * on MI355X at every size tried (32^3 x 8 states: 0.37 against 0.39 ms per
 * iteration; 128^3 x 125 float32: 32.1 against 32.6 ms): the GPU work of an
 * iteration hides the enqueueing, and a change of the locked states needs no
 * re-capture.  Kernel timing (below) uses the eager path. */
mpe_status mpe_set_graph(mpe_plan p, int32_t on);

/* Jacobi sweeps used by the last successful Rayleigh-Ritz solve of
 * mpe_rayleigh_ritz / mpe_iterate (diagnostic; -1 if none). */
int32_t mpe_last_jacobi_sweeps(mpe_plan p);

/* Durations in microseconds of the phases of the last small dense solve
 * (Cholesky, reduction to A = L^-1 Hs L^-T including L^-T, Jacobi sweeps,
 * eigenvalue sort, eigenvector replay as seen by the first row group), from
 * the GPU's constant clock; us must hold 5 doubles.
 * Diagnostic: synchronises the plan's stream. */
mpe_status mpe_small_dense_phases(mpe_plan p, double* us);

/* Selective propagation (Section III: only states whose variance has not
 * reached the error bound need to be propagated).  The following mpe_iterate
 * calls leave the first `locked` states of the block unpropagated: they enter
 * the overlaps, the Rayleigh-Ritz rotation and the variances as Phi_j = Psi_j
 * (so their R^E and R^E_perp come out as 0), while states locked..m-1 are
 * propagated as usual and the whole block is orthonormalised and rotated.
 * R^H is evaluated for every state.  When the previous call on this plan was
 * mpe_iterate or mpe_rayleigh_ritz on the same block (nothing has touched it
 * since), H Psi_j of the locked states is taken from that call's rotation
 * instead of applying H again; the caller must not modify the block between
 * such calls.  0 <= locked <= m, else
 * MPE_ERR_INVALID_ARGUMENT; 0 (the default) propagates every state.  Applies
 * to mpe_iterate only (mpe_step always propagates the whole block). */
mpe_status mpe_set_locked(mpe_plan p, int32_t locked);
/* Selective propagation with any set of locked states (Section III: each state
 * whose variance has reached the bound is left unpropagated, wherever it sits
 * in the block).  mask: host array of m bytes, nonzero = locked; NULL unlocks
 * every state.  A leading run (or none) is the same as mpe_set_locked(count).
 * Otherwise, with n locked states, the following mpe_iterate calls form Phi
 * with the locked states in rows 0..n-1 and the others in rows n..m-1 (a
 * state keeps its own row where that row lies in its part; the locked states
 * beyond row n-1 trade rows with the unlocked ones before row n), gathering
 * the rows of psi (one extra read and write of the unlocked states), propagate
 * rows n..m-1 in place, and proceed as with mpe_set_locked: the overlaps,
 * Rayleigh-Ritz and R^H do not depend on the order of Phi's rows, and R^E_j,
 * R^E_perp_j are reported for state j of the incoming block (0 for the locked
 * ones).  The H Psi reuse of mpe_set_locked applies alike (the cached rows of
 * the locked states that trade rows move with them).  mpe_get_locked reports
 * the number of locked states.  Copies the mask to the device and synchronises the plan's stream
 * when the set changes; replaced by the next mpe_set_locked or
 * mpe_set_locked_states call. */
mpe_status mpe_set_locked_states(mpe_plan p, const uint8_t* mask);
/* Whether the following mpe_iterate calls form the overlap M = Psi^T Phi and
 * the variances R^E, R^E_perp (on != 0, the default) or skip them (their
 * outputs are then NaN; eigenvalues and R^H are unaffected).  A driver that
 * needs the variances only now and then saves one of the three overlap
 * products in the other iterations. */
mpe_status mpe_set_variances(mpe_plan p, int32_t on);

/* Propagator of mpe_step / mpe_iterate / mpe_residuals (Section II).
 * MPE_PROP_EXPANSION (default): the order-2K multi-product expansion of the
 * plan, K(K+1)/2 T2 applications per state.  MPE_PROP_ROMBERG6 (order-4 plans
 * only, else MPE_ERR_UNSUPPORTED): the Romberg-type operator of Eq. sixp built
 * from the order-4 expansion T4,
 *   T(dt) = -T4(dt)/15 + 16 T4(dt/2)^2 / 15,
 * nine T2 applications per state; the two terms are staged in two extra state
 * blocks and combined in float64 with one rounding.  (Built on the expansion
 * T4, whose error is not an odd-power exponent, this combination has local
 * error O(dt^6), one order short of the expansion's T6.)  The first switch to
 * MPE_PROP_ROMBERG6 allocates the dt/2 tables and 2 m N staging values
 * (MPE_ERR_OUT_OF_MEMORY on failure).  MPE_ERR_INVALID_ARGUMENT for another kind. */
enum { MPE_PROP_EXPANSION = 0, MPE_PROP_ROMBERG6 = 1 };
mpe_status mpe_set_propagator(mpe_plan p, int32_t kind);
/* Current propagator kind (-1 for a null plan). */
int32_t mpe_get_propagator(mpe_plan p);

/* Pass structure of the transforms.  The default two-pass form transforms a
 * whole z plane (x and y) in one pass and z pencils in the other; it needs
 * nx == ny and a plane that fits the LDS.  The three-pass form (x rows, y
 * columns and z pencils as separate passes, more HBM traffic) serves every
 * other grid and is chosen at plan creation when the plane does not fit;
 * on != 0 forces it for any grid with row and column passes (the chain output
 * buffers are then allocated, MPE_ERR_OUT_OF_MEMORY on failure), on == 0
 * returns to two passes where they are possible (else MPE_ERR_UNSUPPORTED).
 * Both forms compute the same transforms; results agree to rounding. */
mpe_status mpe_set_three_pass(mpe_plan p, int32_t on);
/* 1 for a three-pass plan, 0 for two passes, -1 for a null plan. */
int32_t mpe_get_three_pass(mpe_plan p);

/* Current number of locked states (-1 for a null plan). */
int32_t mpe_get_locked(mpe_plan p);

/* Launch-shape knob: states per propagation launch (0 = all m). */
mpe_status mpe_set_states_per_launch(mpe_plan p, int32_t states);

/* Launch shape of the forward (kernel_class MPE_KC_PLANE_FWD) or link
 * (MPE_KC_PLANE_LINK) plane passes.  mode = persistence + 3 * order:
 *   persistence 0: one work-group per (z, state) plane (the default);
 *   persistence 1: blocks_per_cu work-groups per CU loop over the planes, each
 *                  loading the next plane's input while it transforms the
 *                  current one, compiled with the register budget of one
 *                  work-group per CU (grids with nx >= 64; smaller grids fall
 *                  back to persistence 0);
 *   persistence 2: the same loop at the register budget of persistence 0;
 *   order 0: z planes fastest; order 1: states fastest (the work-groups in
 *            flight share a few z planes of the potential-factor table).
 * The forward launch forms the first half-step and transform of all K chains;
 * in modes 0..5 one work item per chain and plane, the K chains of a plane on
 * one XCD.  Forward modes 6 and 7 (the chain loop, z planes / states fastest,
 * blocks_per_cu ignored) give each work-group one plane and have it form the K
 * chains one after the other, reading the plane's rows again from its own
 * CU's caches (grids with nx >= 64; smaller grids run them as modes 0 and 3).
 * The H application's last pass and the single-chain output passes follow
 * the link pass's order.
 * Results are bitwise identical for every shape.  MPE_ERR_INVALID_ARGUMENT
 * for another class, a mode outside 0..7 (forward) or 0..5 (link), or
 * blocks_per_cu outside 1..16 (persistent modes). */
mpe_status mpe_set_plane_shape(mpe_plan p, int32_t kernel_class, int32_t mode, int32_t blocks_per_cu);

/* Precision of the overlap GEMMs (S = Phi Phi^T, Hs, the variance overlaps):
 * MPE_GEMM_FP64 (default): float64 MFMA on the states (exact products of
 * float32 states); MPE_GEMM_FP32 (float32 plans only): float32 MFMA with float32
 * accumulation over slabs of 32 points and float64 sums across slabs and
 * chunks -- the float32 half of the precision split; overlaps then carry
 * ~1e-7 relative error, so the Cholesky pivot test becomes 1e-5 of the
 * diagonal.  MPE_GEMM_BF16X3 / MPE_GEMM_BF16X6 (float32 plans only): every
 * float32 value is split into 2 / 3 bfloat16 parts and the products of parts
 * up to the matching order (3 / 6 products) run on bf16 MFMA with float32
 * accumulation over 32-point slabs and float64 sums: ~1e-5 / ~1e-7 relative
 * error, pivot tests 1e-3 / 1e-5 (two parts leave the variances R^E, which
 * subtract overlaps near 1, as noise below ~1e-6).  The rotation of float32 plans always runs on
 * float32 MFMA.  MPE_ERR_UNSUPPORTED for any mode but MPE_GEMM_FP64 on a
 * float64 plan; MPE_ERR_INVALID_ARGUMENT for an unknown mode. */
enum { MPE_GEMM_FP64 = 0, MPE_GEMM_FP32 = 1, MPE_GEMM_BF16X3 = 2, MPE_GEMM_BF16X6 = 3 };
mpe_status mpe_set_gemm_precision(mpe_plan p, int32_t mode);

/* Work-group shape of the pencil (z) passes: tile 0 = 256 threads (default),
 * 1 = 128 threads, 2 = 512 threads, the columns per work-group scaling alike
 * (shapes a grid cannot take, such as 512 threads where the exchange rows would
 * not fit 64 KB of LDS, run as tile 0).  Results are bitwise identical for
 * every shape.  MPE_ERR_INVALID_ARGUMENT outside 0..2. */
mpe_status mpe_set_pencil_shape(mpe_plan p, int32_t tile);
/* Current pencil tile (-1 for a null plan). */
int32_t mpe_get_pencil_shape(mpe_plan p);

/* Current shapes: shape[4] = {fwd mode, fwd blocks_per_cu, link mode, link blocks_per_cu}. */
mpe_status mpe_get_plane_shape(mpe_plan p, int32_t* shape);

/* Autotuner: times the candidate plane shapes (mode, blocks per CU) in
 * {(0,0), (1,1), (2,1), (2,2), (2,4)}, the same five with states fastest
 * (modes 3..5) and, for the forward pass, the chain loop (modes 6, 7), then
 * the pencil tiles 0..2 with the chosen plane shapes, on `reps` steps of psi
 * (read only; the steps write the plan's workspace) at dt, and keeps the
 * fastest shape per pass.  With cache_path (may be NULL), a line
 * "key|fwd_mode fwd_bpc link_mode link_bpc pencil_tile" keyed by device, CU
 * count, grid, precision, block size and order is looked up first (no timing
 * on a hit; a line without the pencil tile reads as tile 0) and appended after
 * tuning.  ms_out (may be NULL) receives the chosen plane shapes'
 * milliseconds per step for the forward and link passes (-1 on a cache hit).
 * Synchronises. */
mpe_status mpe_autotune(mpe_plan p, const void* psi, double dt, int32_t reps, const char* cache_path,
                        double* ms_out);

/* Per-kernel timing.  When enabled, every launch is bracketed by HIP events
 * on the plan's stream; mpe_get_kernel_times synchronises and returns, per
 * kernel class (MPE_KC_*), the accumulated milliseconds and launch counts
 * since the last reset. */
enum {
  MPE_KC_PLANE_FWD = 0, MPE_KC_PENCIL = 1, MPE_KC_PLANE_LINK = 2, MPE_KC_PLANE_TAIL = 3,
  MPE_KC_H_APPLY = 4, MPE_KC_GRAM = 5, MPE_KC_SMALL_DENSE = 6, MPE_KC_ROTATE = 7,
  MPE_KC_OTHER = 8, MPE_KC_COUNT = 9
};
mpe_status mpe_profile_enable(mpe_plan p, int32_t on);
mpe_status mpe_get_kernel_times(mpe_plan p, double* ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Allocation-free orthonormalisation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the work of mpe_orthonormalize without a plan.
 *
 * psi: device array [m][n_points] of double (MPE_FP64) or float (MPE_FP32),
 * orthonormalised in place (S = Psi Psi^T on float64 MFMA, S = L L^T,
 * Psi <- L^-1 Psi) on hip_stream (NULL = null stream); the call synchronises
 * that stream to read the status.  Limits: 1 <= m <= 128 and m <= n_points,
 * else MPE_ERR_UNSUPPORTED (m > 128) or MPE_ERR_INVALID_ARGUMENT, with a
 * message in mpe_noalloc_last_error().
 *
 * Every intermediate (overlap partials of up to 64 point chunks, S, L^-T,
 * status) lives in one file-scope device array of MPE_NOALLOC_SCRATCH_BYTES
 * bytes that each GPU the library runs on holds until the process ends; no
 * call allocates or frees memory.  All calls on one GPU share that array, so
 * calls that overlap in time on one GPU (two host threads, or two streams
 * without ordering) race and must not be issued.  Up to 64 * 4096 points the
 * overlap is chunked exactly as in a plan and the result equals
 * mpe_orthonormalize bitwise; beyond, the sums are grouped into 64 chunks
 * instead of up to 256 (float64 rounding differences only).
 * On NOT_POSITIVE_DEFINITE or NONFINITE psi is left unchanged.
 *
 * Set-up: the array's device address is resolved once per GPU, by
 * mpe_noalloc_prepare() or else by the first call on that GPU; the HIP runtime
 * may materialise the array's storage at that moment (once per GPU, for the
 * life of the process).  Callers that must not allocate at all call
 * mpe_noalloc_prepare() with each GPU current beforehand. */
#define MPE_NOALLOC_SCRATCH_BYTES 8656912
mpe_status mpe_orthonormalize_noalloc(void* psi, int32_t m, int64_t n_points, mpe_precision prec, void* hip_stream);
/* Resolve the scratch array on the current GPU (see above).  MPE_ERR_DEVICE on a
 * HIP failure, with a message in mpe_noalloc_last_error(). */
mpe_status mpe_noalloc_prepare(void);
/* Message of the calling thread's last failed mpe_orthonormalize_noalloc or
 * mpe_noalloc_prepare ("" after success). */
const char* mpe_noalloc_last_error(void);

/* ---------------------------------------------------------------------------
 * Batched uneven systems: many independent eigenproblems (different grids,
 * state counts and potentials, one order and precision) advanced together.
 * Systems with the same grid share every propagation and H launch (one launch
 * per pass over all their states); the overlaps, small dense solves and
 * rotations of all systems share one launch per kernel and tile class (see
 * mpe_batch_set_batched_la); one iteration of all systems is one hipGraph
 * replay.  Results equal those of separate plans bitwise.  Every system needs
 * a grid with two-pass transforms (nx == ny), else MPE_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------- */
typedef struct mpe_batch_s* mpe_batch;

typedef struct {
  int32_t grid[3];     /* as for mpe_plan_create                                  */
  double box[3];
  int32_t n_states;
  int32_t n_guard;
  const double* V;     /* device float64 [nz][ny][nx]; copied at creation          */
} mpe_system_desc;

/* Create plans for `count` systems on one stream.  Errors as mpe_plan_create. */
mpe_status mpe_batch_create(mpe_batch* out, int32_t count, const mpe_system_desc* systems, int32_t order,
                            mpe_precision prec, double hbar2_over_m, void* hip_stream);
mpe_status mpe_batch_destroy(mpe_batch b);
const char* mpe_batch_last_error(mpe_batch b);

/* psi[i] <- T_order(dt) psi[i] for every system (psi: `count` device state
 * blocks, each [m_i][nz][ny][nx]). */
mpe_status mpe_batch_step(mpe_batch b, void* const* psi, double dt);

/* One fused iteration (as mpe_iterate) of every system.  Host outputs hold
 * sum_i m_i doubles, system i's values at offset sum_{k<i} m_k; any may be
 * NULL.  The first failing system's status is returned (others still ran). */
mpe_status mpe_batch_iterate(mpe_batch b, void* const* psi, double dt, double* eig, double* rh, double* re,
                             double* re_perp);

/* Kernel launches in the captured iteration graph (diagnostic). */
int32_t mpe_batch_launches_per_step(mpe_batch b);

/* How mpe_batch_iterate issues the per-system linear algebra (overlaps,
 * variances, small dense solves, eigenvector replays, rotations): on != 0 (the
 * default) as one launch per kernel and 16-state tile class for all systems,
 * each launch walking a device table of (system, chunk) work items; on == 0 as
 * separate launches per system on parallel graph branches.  Results are bitwise
 * identical either way. */
mpe_status mpe_batch_set_batched_la(mpe_batch b, int32_t on);

/* ---------------------------------------------------------------------------
 * Learned warm start (an addition outside the paper, whose Section III starts
 * from random or plane-wave states): a small 3-D U-Net maps a coarse potential
 * on a d^3 grid (d = 32 for the cage workload) to n_out starting orbitals on
 * the same grid; wsn_upsample_periodic carries them to the solver's grid,
 * after which the solver's own residual R^H judges them.  The network is
 * trained on the GPU with these calls.
 *
 * Architecture: channels 16/32/64 over three levels (d, d/2, d/4); every
 * convolution has 3x3x3 periodic taps, weights W[co][tz][ty][tx][ci] and a
 * bias; ReLU after every convolution but the head; two stride-2 convolutions
 * down, nearest-neighbour doubling plus channel concatenation up:
 *   e1 = relu(c1b(relu(c1a(v))))  e2 = relu(c2b(relu(c2a_s2(e1))))
 *   e3 = relu(c3b(relu(c3a_s2(e2))))  d2 = relu(cd2([up(e3) | e2]))
 *   d1 = relu(cd1([up(d2) | e1]))     y = head(d1)
 * Parameters form one float32 vector, layer by layer (c1a, c1b, c2a, c2b,
 * c3a, c3b, d2, d1, head), each layer's weights [co][27][ci] then its bias.
 * Convolutions run on bfloat16 MFMA with float32 accumulation (operands
 * rounded to bfloat16, float32 master weights).
 * ------------------------------------------------------------------------- */
typedef struct wsn_net_s* wsn_net;

/* Create a network for d = grid (a multiple of 4, >= 8), n_out output orbitals
 * (a multiple of 8, <= 128), batches up to max_batch; He-normal weights drawn
 * from seed, zero biases, zero Adam moments.  All device memory (weights,
 * activations for max_batch, gradients) is allocated here and owned by the
 * network.  hip_stream may be NULL (default stream). */
mpe_status wsn_create(wsn_net* out, int32_t grid, int32_t n_out, int32_t max_batch, uint64_t seed,
                      void* hip_stream);
mpe_status wsn_destroy(wsn_net n);
const char* wsn_last_error(wsn_net n);

/* Length of the parameter vector (-1 for a null network). */
int64_t wsn_num_params(wsn_net n);

/* Copy the parameters (which = 0) or the accumulated gradients (which = 1) to
 * host float32 [wsn_num_params]; synchronises. */
mpe_status wsn_get_params(wsn_net n, float* host, int32_t which);
/* Replace the parameters from host float32 [wsn_num_params]; synchronises. */
mpe_status wsn_set_params(wsn_net n, const float* host);
/* Clear the accumulated gradients. */
mpe_status wsn_zero_grads(wsn_net n);

/* Forward pass.  v: device float32 [batch][d][d][d] potentials, multiplied by
 * vscale on input; y: device float32 [batch][n_out][d][d][d] orbitals (state
 * layout, z slowest), the head's output multiplied by yscale.  Keeps the
 * activations (and yscale) for wsn_backward.  MPE_ERR_INVALID_ARGUMENT for a
 * batch outside [1, max_batch]. */
mpe_status wsn_forward(wsn_net n, const float* v, float vscale, float yscale, int32_t batch, float* y);

/* Backward pass of the last forward: dy is device float32 shaped like y
 * (dL/dy); parameter gradients are ADDED to the accumulated ones.
 * MPE_ERR_STATE before any forward. */
mpe_status wsn_backward(wsn_net n, const float* dy);

/* One convolution layer alone (layer = 0..8 in parameter order c1a .. head),
 * for checking each layer at its own shape.  info (wsn_layer_info) receives
 * {ci, co, ci_pad, stride, relu}.  wsn_layer runs the layer's forward
 *   y = act(conv(x) + b)     (act = ReLU unless the layer is the head)
 * on x, device float32 channels-last [batch][din^3][ci_pad] (channels ci..
 * ci_pad-1 zero), into y [batch][dout^3][co], dout = din / stride.  When dz is
 * not NULL it holds dL/dy ([batch][dout^3][co]) and the backward follows: dz
 * is overwritten by the pre-activation gradient, the layer's weight and bias
 * gradients are ADDED to the accumulated ones (wsn_get_params which = 1), and,
 * when dx is not NULL, dx [batch][din^3][ci] receives dL/dx.  The same bfloat16
 * MFMA kernels as wsn_forward / wsn_backward.  MPE_ERR_INVALID_ARGUMENT for a
 * bad layer, a batch outside [1, max_batch] or din not a multiple of
 * 2 * stride. */
mpe_status wsn_layer_info(wsn_net n, int32_t layer, int32_t* info);
mpe_status wsn_layer(wsn_net n, int32_t layer, int32_t batch, int32_t din, const float* x, float* y, float* dz,
                     float* dx);

/* Adam step with bias correction (t = 1, 2, ...) on the accumulated
 * gradients, which it then clears. */
mpe_status wsn_adam_step(wsn_net n, float lr, float beta1, float beta2, float eps, int32_t t);

/* Rotation-invariant subspace loss of one prediction y (device float32
 * [n_states][P]) against targets (device float32 [n_states][P]): with
 * M = y target^T,
 *   L = ||y - M target||^2 + ||M M^T - I||^2,
 * zero exactly when y = R target with R orthogonal and orthonormal targets.
 * Writes into dy (device, same shape; must not alias y) the gradient
 * 2(y - M target) + 4(M M^T - I) M target, which is dL/dy when the target
 * rows are orthonormal (the intended use), and, when loss_host is not NULL,
 * {L, ||M M^T - I||^2} into loss_host[2].  Overlaps and M are float64
 * (||y - M target||^2 = ||y||^2 - 2||M||^2 + tr(M target target^T M^T)).
 * Synchronises. */
mpe_status wsn_subspace_loss(wsn_net n, const float* y, const float* target, int32_t n_states, int64_t P,
                             double* loss_host, float* dy);

/* Procrustes loss of one prediction y (device float32 [n_states][P]) against
 * targets with orthonormal rows (device float32 [n_states][P]): with M =
 * y target^T and its polar factor Q = M (M^T M)^(-1/2),
 *   L = ||y - Q target||^2,
 * the distance from y to the nearest rotation of the targets.  Writes
 * dL/dy = 2(y - Q target) into dy (device, same shape; must not alias y) and,
 * when loss_host is not NULL, {L, sum of the singular values of M} into
 * loss_host[2].  Overlaps, M^T M, its eigenpairs (the plan's Jacobi solver)
 * and Q are float64; eigenvalues below 1e-12 of the largest are raised to it.
 * MPE_ERR_EIG_NO_CONVERGENCE / MPE_ERR_NONFINITE when the eigenpairs fail.
 * Synchronises. */
mpe_status wsn_procrustes_loss(wsn_net n, const float* y, const float* target, int32_t n_states, int64_t P,
                               double* loss_host, float* dy);

/* Periodic trilinear interpolation of u (device float32 [channels][d][d][d])
 * onto the grid of (d*factor)^3 points: fine point j of an axis sits at coarse
 * coordinate j/factor.  out: device float32 [channels][D][D][D], D = d*factor.
 * Enqueued on hip_stream (may be NULL). */
mpe_status wsn_upsample_periodic(const float* u, int32_t channels, int32_t d, int32_t factor, float* out,
                                 void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MPE_H_ */
