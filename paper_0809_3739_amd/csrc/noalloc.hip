// Allocation-free orthonormalisation: the work of mpe_orthonormalize (overlap
// S = Psi Psi^T on float64 MFMA, Cholesky S = L L^T, Psi <- L^-1 Psi) for
// callers that cannot allocate device memory, with every intermediate in one
// file-scope device array instead of a plan's workspace.
//
// The array `scratch` holds, at fixed offsets: the overlap partials of up to
// NA_MAX_CHUNKS point chunks (mp x mp float64 each), S, the triangular factor's
// inverse W = L^-T (C of the small dense solve), the small dense solve's
// scratch and its status words.  Every region is written before it is read in
// each call, so nothing has to be cleared.  Each GPU holds its own copy of the
// array; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (kept per device on first use).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/mpe.h"
#include "la.hpp"

using namespace mpe;

namespace {

constexpr long NA_MAX_CHUNKS = 64;
constexpr size_t NA_PARTIALS = (size_t)NA_MAX_CHUNKS * MAXM * MAXM;   // doubles
constexpr size_t NA_MAT = (size_t)MAXM * MAXM;                        // doubles per matrix
constexpr size_t NA_SD_SCRATCH = 6 * (size_t)MAXM;                    // doubles
constexpr size_t NA_OFF_S = NA_PARTIALS;
constexpr size_t NA_OFF_C = NA_OFF_S + NA_MAT;
constexpr size_t NA_OFF_SD = NA_OFF_C + NA_MAT;
constexpr size_t NA_OFF_STATUS = NA_OFF_SD + NA_SD_SCRATCH;           // 4 ints (2 doubles)
constexpr size_t NA_DOUBLES = NA_OFF_STATUS + 2;
constexpr size_t NA_BYTES = NA_DOUBLES * sizeof(double);
static_assert(NA_BYTES == MPE_NOALLOC_SCRATCH_BYTES, "header states the scratch size");

}  // namespace

static __device__ __align__(256) double scratch[NA_DOUBLES];

namespace {

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
double* na_ptr[NA_MAX_DEVICES] = {nullptr};
thread_local std::string na_err;

mpe_status na_fail(mpe_status s, const std::string& msg) {
  na_err = msg;
  return s;
}

// The device address of `scratch` on the current device (looked up once per
// device), or an error.
mpe_status na_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return na_fail(MPE_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= NA_MAX_DEVICES) return na_fail(MPE_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(na_mutex);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return na_fail(MPE_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    e = prepare_small_dense();   // the small dense kernel's LDS limit, once per device
    if (e != hipSuccess) return na_fail(MPE_ERR_DEVICE, std::string("small dense set-up: ") + hipGetErrorString(e));
    na_ptr[dev] = static_cast<double*>(p);
  }
  *out = na_ptr[dev];
  return MPE_OK;
}

}  // namespace

extern "C" {

const char* mpe_noalloc_last_error(void) { return na_err.c_str(); }

mpe_status mpe_noalloc_prepare(void) {
  na_err.clear();
  double* base = nullptr;
  return na_scratch(&base);
}

mpe_status mpe_orthonormalize_noalloc(void* psi, int32_t m, int64_t n_points, mpe_precision prec, void* hip_stream) {
  na_err.clear();
  if (!psi) return na_fail(MPE_ERR_INVALID_ARGUMENT, "psi is null");
  if (prec != MPE_FP64 && prec != MPE_FP32) return na_fail(MPE_ERR_INVALID_ARGUMENT, "unknown precision");
  if (m < 1 || n_points < 1) return na_fail(MPE_ERR_INVALID_ARGUMENT, "m and n_points must be positive");
  if (m > MAXM) {
    char b[128];
    std::snprintf(b, sizeof b, "m = %d exceeds the %d states the scratch array holds", (int)m, MAXM);
    return na_fail(MPE_ERR_UNSUPPORTED, b);
  }
  if (m > n_points) return na_fail(MPE_ERR_INVALID_ARGUMENT, "more states than grid points");
  double* base = nullptr;
  mpe_status s = na_scratch(&base);
  if (s != MPE_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int dbl = prec == MPE_FP64;
  const int mp = (m + 15) / 16 * 16;
  double* partials = base;
  double* S = base + NA_OFF_S;
  double* C = base + NA_OFF_C;
  double* sd = base + NA_OFF_SD;
  int* status = reinterpret_cast<int*>(base + NA_OFF_STATUS);

  // S = Psi Psi^T: chunk partials, then their fixed-order sum
  GramArgs g;
  std::memset(&g, 0, sizeof(g));
  g.X[0] = g.Y[0] = psi;
  long chunk;
  const int nch = gram_chunking(n_points, NA_MAX_CHUNKS, &chunk);
  g.partials = partials;
  g.N = n_points;
  g.chunk = chunk;
  g.m = m;
  g.mp = mp;
  hipError_t e = launch_gram(dbl, g, 1, nch, st);
  if (e == hipSuccess) e = launch_reduce(partials, nch, (long)mp * mp, 1, S, st);
  // Cholesky and W = L^-T (status written in every case)
  SmallDenseArgs d;
  std::memset(&d, 0, sizeof(d));
  d.S = S;
  d.C = C;
  d.scratch = sd;
  d.status = status;
  d.m = m;
  d.mp = mp;
  d.mode = SD_ORTHO;
  d.max_sweeps = 1;
  d.tol = 1e-13;
  d.pivot_tol = 1e-13;
  if (e == hipSuccess) e = launch_small_dense(d, st);
  // Psi <- W^T Psi in place (skipped by the kernel unless the status is OK)
  RotateArgs r;
  std::memset(&r, 0, sizeof(r));
  long rchunk;
  const int nrch = rot_chunking(n_points, &rchunk);
  r.Phi = psi;
  r.Psi = psi;
  r.C = C;
  r.status = status;
  r.N = n_points;
  r.chunk = rchunk;
  r.m = m;
  r.mp = mp;
  if (e == hipSuccess) e = launch_rotate(dbl, false, r, nrch, st);
  int hs[2] = {-1, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hs, status, sizeof hs, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return na_fail(MPE_ERR_DEVICE, std::string("HIP: ") + hipGetErrorString(e));
  char b[128];
  switch (hs[0]) {
    case ST_OK: return MPE_OK;
    case ST_NOT_SPD:
      std::snprintf(b, sizeof b, "overlap matrix not positive definite at pivot %d", hs[1]);
      return na_fail(MPE_ERR_NOT_POSITIVE_DEFINITE, b);
    case ST_NONFINITE:
      std::snprintf(b, sizeof b, "non-finite value in the overlap matrix at pivot %d", hs[1]);
      return na_fail(MPE_ERR_NONFINITE, b);
    default: return na_fail(MPE_ERR_DEVICE, "unknown device status");
  }
}

}  // extern "C"
