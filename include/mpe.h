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
 *  grid[3]  = (nx, ny, nz); supported: nx == ny in {8,16,32,48,64,96,128,192}
 *             (192 for MPE_FP32 only), nz in the same set.  Others: UNSUPPORTED.
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

/* Graph replay of mpe_iterate (on by default).  The first call for a given
 * psi array captures the iteration's launches into a hipGraph on a private
 * stream ordered after the plan's stream; later calls with the same psi and
 * launch grouping replay it (dt enters through tables rebuilt outside the
 * graph).  Off: every launch is enqueued eagerly. Kernel timing (below) uses
 * the eager path. */
mpe_status mpe_set_graph(mpe_plan p, int32_t on);

/* Jacobi sweeps used by the last successful Rayleigh-Ritz solve of
 * mpe_rayleigh_ritz / mpe_iterate (diagnostic; -1 if none). */
int32_t mpe_last_jacobi_sweeps(mpe_plan p);

/* Durations in microseconds of the phases of the last small dense solve
 * (Cholesky, triangular solves, Jacobi sweeps, eigenvector rebuild, back
 * substitution), from the GPU's constant clock; us must hold 5 doubles.
 * Diagnostic: synchronises the plan's stream. */
mpe_status mpe_small_dense_phases(mpe_plan p, double* us);

/* Launch-shape knob: states per propagation launch (0 = all m). */
mpe_status mpe_set_states_per_launch(mpe_plan p, int32_t states);

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
 * Batched uneven systems: many independent eigenproblems (different grids,
 * state counts and potentials, one order and precision) advanced together.
 * Systems with the same grid share every propagation and H launch (one launch
 * per pass over all their states); overlaps, the small dense solve and the
 * rotation run per system; one iteration of all systems is one hipGraph
 * replay.  Results equal those of separate plans bitwise.
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

#ifdef __cplusplus
}
#endif

#endif /* MPE_H_ */
