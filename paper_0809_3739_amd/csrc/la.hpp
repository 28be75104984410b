// Host-visible descriptors of the subspace linear-algebra kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mpe {

constexpr int MAXM = 128;  // states (incl. guards) per system handled by one plan

enum SmallDenseMode { SD_ORTHO = 0, SD_RR = 1 };

// Jacobi rotation log of the small dense solve: per step a flag and (c, s) for
// every pair; the rotation buffer (SmallDenseArgs::rot) holds max_sweeps sweeps.
constexpr int SD_LOG_STRIDE = 1 + 2 * (MAXM / 2 + 1);
inline size_t small_dense_rot_doubles(int max_sweeps) { return (size_t)max_sweeps * (MAXM + 1) * SD_LOG_STRIDE; }
enum SmallDenseStatus { ST_OK = 0, ST_NOT_SPD = 1, ST_EIG_NO_CONV = 2, ST_NONFINITE = 3 };

// partial[prod][chunk][mp][mp] = X_prod Y_prod^T over the chunk's points
// Gram product modes (see gram_partial_kernel)
enum { GRAM_FULL = 0, GRAM_SELF = 1, GRAM_UPPER = 2 };

struct GramArgs {
  const void* X[3];
  const void* Y[3];
  int upper_mask;       // bit i: product i is symmetric in exact arithmetic (upper tiles only)
  double* partials;
  long N;
  long chunk;
  int m, mp;
};

struct SmallDenseArgs {
  const double* S;      // mp x mp overlap
  const double* Hs;     // mp x mp projected H (SD_RR)
  double* L;            // mp x mp workspace (holds Hs L^-T during SD_RR)
  double* rot;          // workspace: the Jacobi rotation log (small_dense_rot_doubles(max_sweeps))
  double* scratch;      // >= 2*MAXM doubles
  double* C;            // out: mp x mp, Psi_j = sum_i C[i][j] Phi_i
  double* theta;        // out: m Ritz values ascending (SD_RR)
  int* status;          // out: [code, detail]
  long long* ticks;     // optional out: constant-clock stamps at phase ends (8 entries)
  int m, mp, mode, max_sweeps;
  double tol;           // Jacobi: converged when |a_ij| <= tol * max(sqrt|a_ii a_jj|, floor)
  double pivot_tol;     // Cholesky: pivot must exceed pivot_tol * original diagonal
};

struct RotateArgs {
  const void* Phi;
  const void* HPhi;     // may be null when no H rotation is wanted
  const double* C;      // mp x mp
  const double* theta;  // m (with H)
  void* Psi;            // out
  void* HPsi;           // optional out
  double* res_partials; // [chunk][mp]
  const int* status;    // small-dense status; the kernel does nothing unless it is ST_OK
  long N;
  long chunk;
  int m, mp;
};

// Point chunks of the overlap kernels: at most max_chunks chunks of >= 4096
// points (multiples of 16), one work-group each; returns the count, *chunk
// the chunk length.
inline int gram_chunking(long N, long max_chunks, long* chunk) {
  long nch = N / 4096 + (N % 4096 != 0);
  nch = nch < 1 ? 1 : (nch > max_chunks ? max_chunks : nch);
  long c = (N + nch - 1) / nch;
  c = (c + 15) / 16 * 16;
  *chunk = c;
  return (int)((N + c - 1) / c);
}
// Point chunks of the rotation: at most 1024 chunks of >= 256 points (multiples of 64).
inline int rot_chunking(long N, long* chunk) {
  long nch = N / 256 + (N % 256 != 0);
  nch = nch < 1 ? 1 : (nch > 1024 ? 1024 : nch);
  long c = (N + nch - 1) / nch;
  c = (c + 63) / 64 * 64;
  *chunk = c;
  return (int)((N + c - 1) / c);
}

// Batched launches over many systems (job tables in device memory, sorted by
// block0, the first work-group of each job).  The kernels run the same code per
// chunk / system as the single-system launches, so results are bitwise equal.
struct GramJob {       // one product X Y^T of one system: partials [chunk][mp][mp]
  const void* X;
  const void* Y;
  double* partials;
  long N, chunk;
  int m, block0;
};
struct RotateJob {     // one system's rotation: its chunks are consecutive work-groups
  RotateArgs r;
  int block0;
};
struct ReduceJob {     // out[c][e] = sum_q in[c][q][e]: ceil(count / 64) * ncomp work-groups
  const double* in;
  double* out;
  long count;
  int nparts, ncomp, block0;
};
struct ReplayJob {     // eigenvector replay of one system: ceil(m / 4) work-groups
  SmallDenseArgs d;
  int block0;
};
struct VarianceJob {   // R^E and R^E_perp of one system (one work-group of 128 threads)
  const double* S;
  const double* M;
  double* re;
  double* re_perp;
  int m, mp;
};
hipError_t launch_gram_jobs(int is_double, int nt, int mode, const GramJob* jobs, int njobs, int nblocks,
                            hipStream_t st);
hipError_t launch_rotate_jobs(int is_double, bool with_h, int nt, const RotateJob* jobs, int njobs, int nblocks,
                              hipStream_t st);
hipError_t launch_reduce_jobs(const ReduceJob* jobs, int njobs, int nblocks, hipStream_t st);
hipError_t launch_small_dense_jobs(const SmallDenseArgs* jobs, int njobs, int max_mp, hipStream_t st);
hipError_t launch_replay_jobs(const ReplayJob* jobs, int njobs, int nblocks, hipStream_t st);
hipError_t launch_variance_jobs(const VarianceJob* jobs, int njobs, hipStream_t st);
constexpr int REPLAY_ROWS = 4;   // rows of C per replay work-group

hipError_t launch_gram(int is_double, const GramArgs& g, int nprod, int nchunks, hipStream_t st);
// float32 states only: float32 MFMA, float64 slab sums and partials
hipError_t launch_gram32(const GramArgs& g, int nprod, int nchunks, hipStream_t st);
// float32 states only: BF16-split products (split = 2 or 3 parts) on bf16 MFMA
hipError_t launch_gramb(const GramArgs& g, int nprod, int nchunks, int split, hipStream_t st);
hipError_t launch_reduce(const double* in, int nparts, long count, int ncomp, double* out, hipStream_t st);
hipError_t prepare_small_dense();
hipError_t launch_small_dense(const SmallDenseArgs& d, hipStream_t st);
hipError_t launch_rotate(int is_double, bool with_h, const RotateArgs& r, int nchunks, hipStream_t st);
hipError_t launch_fill(double* p, long n, double v, hipStream_t st);
hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t st);
// row i of dst <- row rows[i] of src (device index table), i < nrows; rows of
// row_bytes (a multiple of 16); dst and src must not overlap
hipError_t launch_gather_rows(void* dst, const void* src, const int* rows, int nrows, size_t row_bytes,
                              hipStream_t st);
// in place: row i of buf <- row rows[i] for i < nrows with rows[i] != i; no
// destination row may be the source of another move
hipError_t launch_move_rows(void* buf, const int* rows, int nrows, size_t row_bytes, hipStream_t st);
// rows: optional (nullptr = identity) table of the state each column of phi propagates
hipError_t launch_variance(const double* S, const double* M, int m, int mp, const int* rows, double* re,
                           double* re_perp, hipStream_t st);

}  // namespace mpe
