// C ABI of libmpe: plan management and the launch sequences of one
// multi-product step, the H application, orthonormalisation, Rayleigh-Ritz,
// the variances and the fused iteration.  See include/mpe.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpe.h"
#include "la.hpp"
#include "prop.hpp"

using namespace mpe;

namespace {

// ------------------------------------------------------------------ device table kernels
// fac[j][p] = exp(-dt V[p] / (j + 1)), j = 0..ntab-1: the potential half- and
// full-steps exp(-tau V/2) and exp(-tau V) of every chain (tau = dt/k).
template <typename F>
__global__ void factor_tables_kernel(const double* __restrict__ V, long N, double dt, int ntab, F* __restrict__ out) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double v = V[p];
  for (int j = 0; j < ntab; ++j) out[(long)j * N + p] = (F)exp(-dt * v / (double)(j + 1));
}

template <typename F>
__global__ void cast_kernel(const double* __restrict__ in, long n, F* __restrict__ out) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[p] = (F)in[p];
}

__device__ __forceinline__ double wavenumber(int k, int n, double L) {
  const int mfreq = (k <= n / 2) ? k : k - n;
  return 2.0 * 3.14159265358979323846 * (double)mfreq / L;
}

// Per-axis kinetic tables on the half spectrum.  For chain k (tau = dt/k):
//   ex[kx] = exp(-tau hbar^2/2m qx^2), ey, ez likewise, ez also carrying 1/(nx ny nz)
// (the three unnormalised inverse transforms); and the additive tables of T itself:
//   hx[kx] = hbar^2/2m qx^2 / (nx ny nz), ...
template <typename F>
__global__ void kinetic_tables_kernel(int nx, int ny, int nz, double Lx, double Ly, double Lz, double h2m, double dt,
                                      int K, F* __restrict__ exp_tab, F* __restrict__ add_tab) {
  const int nxh = nx / 2 + 1, len = nxh + ny + nz;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double inv_n = 1.0 / ((double)nx * ny * nz);
  double q;
  bool is_z = false;
  if (i < nxh) q = wavenumber(i, nx, Lx);
  else if (i < nxh + ny) q = wavenumber(i - nxh, ny, Ly);
  else { q = wavenumber(i - nxh - ny, nz, Lz); is_z = true; }
  const double t = 0.5 * h2m * q * q;
  for (int k = 1; k <= K; ++k) {
    double e = exp(-(dt / k) * t);
    if (is_z) e *= inv_n;
    exp_tab[(long)(k - 1) * len + i] = (F)e;
  }
  add_tab[i] = (F)(t * inv_n);
}

// R^H partials for a block with given values: part[c][j] = sum over chunk c of (hpsi - e_j psi)^2
template <typename F>
__global__ __launch_bounds__(256) void residual_kernel(const F* __restrict__ psi, const F* __restrict__ hpsi,
                                                       const double* __restrict__ eig, long N, long chunk, int mp,
                                                       double* __restrict__ part) {
  const int j = blockIdx.y;
  const long b = (long)blockIdx.x * chunk, e = min(N, b + chunk);
  const double ej = eig[j];
  double s = 0.0;
  for (long p = b + threadIdx.x; p < e; p += 256) {
    const double d = (double)hpsi[(long)j * N + p] - ej * (double)psi[(long)j * N + p];
    s += d * d;
  }
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(long)blockIdx.x * mp + j] = red[0] + red[1] + red[2] + red[3];
}

// ------------------------------------------------------------------ host-side exact coefficients
long long gcdll(long long a, long long b) {
  a = a < 0 ? -a : a;
  b = b < 0 ? -b : b;
  while (b) { long long t = a % b; a = b; b = t; }
  return a;
}

// c_i = prod_{j != i} i^2/(i^2 - j^2) as a reduced fraction, then rounded once.
bool mpe_coeffs(int K, double* c) {
  if (K < 1 || K > MAX_K) return false;
  for (int i = 1; i <= K; ++i) {
    long long num = 1, den = 1;
    for (int j = 1; j <= K; ++j) {
      if (j == i) continue;
      num *= (long long)i * i;
      den *= (long long)i * i - (long long)j * j;
      const long long g = gcdll(num, den);
      num /= g;
      den /= g;
    }
    if (den < 0) { den = -den; num = -num; }
    c[i - 1] = (double)num / (double)den;   // num, den < 2^53: one rounding
  }
  return true;
}

struct Timer {
  hipEvent_t a, b;
  int kc;
};

}  // namespace

// ------------------------------------------------------------------ the plan
struct mpe_plan_s {
  int nx = 0, ny = 0, nz = 0, nxh = 0;
  double Lx = 0, Ly = 0, Lz = 0;
  int n = 0, g = 0, m = 0, mp = 0, K = 0, dbl = 0;
  long N = 0, M = 0, spec = 0;            // points, columns per z, spectrum elements per state
  size_t fsz = 0;                         // sizeof data type
  hipStream_t st = nullptr;
  std::string err;

  // workspace
  void* W = nullptr;           // K chains x m states x spec complex
  void* tailbuf = nullptr;     // split tail: K chains x m states x N real (when tail_split)
  bool split_tail = false;
  bool three_pass = false;     // x rows, y columns and z pencils as separate passes
  void* phi = nullptr;         // m x N
  void* hphi = nullptr;        // m x N
  double* V64 = nullptr;       // N
  void* Vf = nullptr;          // N, data type
  void* fac = nullptr;         // 2K x N
  void* kin = nullptr;         // K x (nxh+ny+nz)
  // Romberg propagator (mpe_set_propagator): tables at dt/2 and two staging blocks
  int prop = MPE_PROP_EXPANSION;
  void* fac2 = nullptr;        // 2K x N at dt/2
  void* kin2 = nullptr;        // K x (nxh+ny+nz) at dt/2
  void* rtmp = nullptr;        // 2 x m x N: T4(dt) psi | T4(dt/2)^2 psi
  void* hk = nullptr;          // nxh+ny+nz
  void* roots = nullptr;       // rx | ry | rz | wpost
  size_t off_ry = 0, off_rz = 0, off_wp = 0;
  double* partials = nullptr;  // gram / residual partials
  size_t partials_bytes = 0;
  double* mats = nullptr;      // S, Hs, M, L, C (mp x mp each)
  double* rot = nullptr;       // Jacobi eigenvector accumulator U (mp x mp)
  size_t rot_count = 0;
  double* res = nullptr;       // theta | rh | re | re_perp (MAXM each) | scratch (2 MAXM) | status
  int* status = nullptr;
  double* host_res = nullptr;  // pinned mirror of res + status
  size_t res_bytes = 0;
  int64_t ws_bytes = 0;
  long long* ticks = nullptr;  // small-dense phase stamps (device, 8 entries; diagnostics)

  bool have_v = false;
  double h2m = 1.0;
  double tab_dt = -1.0;
  double last_dt = -1.0;
  int states_per_launch = 0;
  int locked = 0;                    // states mpe_iterate leaves unpropagated
  // locked states that are not a leading run (mpe_set_locked_states): Phi is
  // formed in the order lock_perm (the locked states in rows 0..locked-1, the
  // others after them, each state in its own row where its part allows),
  // gathered from psi through the device copy perm
  bool lock_mapped = false;
  std::vector<int> lock_perm;
  int* perm = nullptr;               // device, MAXM entries
  int hfirst = 0;                    // first state whose H phi the next iteration computes
  // launch shapes of the forward [0] and link [1] plane passes (PlaneArgs::persist_mode,
  // work-groups per CU); shape_ver counts changes so a captured graph can notice them
  int pmode[2] = {0, 0};
  int pbpc[2] = {0, 0};
  int ptile = 0;               // pencil work-group shape (PencilArgs::tile)
  int shape_ver = 0;
  int n_cu = 0;
  int gemm = 0;                 // overlap GEMMs: 0 = float64 MFMA, 1 = float32 MFMA (float32 plans)
  int max_sweeps = 60;
  double jacobi_tol = 1e-13;
  double pivot_tol = 1e-13;
  const void* rr_cache_psi = nullptr;   // H psi cached in hphi for this psi

  // graph replay of the fused iteration
  bool use_graph = false;      // replay a captured iteration (mpe_set_graph); eager launches by default
  hipStream_t gst = nullptr;         // private stream for capture and replay
  // one captured iteration per variance setting (slot = variances on)
  struct IterGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* psi = nullptr;       // the graph bakes in this state block ...
    int spl = -1;                    // ... and this launch grouping
    int locked = -1;                 // ... and this number of locked states
    int mapped = -1;                 // ... locked as a leading run (0) or through perm (1)
    int hfirst = -1;                 // ... and this first H state
    int shape = -1;                  // ... and these plane-pass shapes
  } ig[2];
  bool variances = true;             // mpe_iterate forms M = Psi^T Phi and the variances R^E
  hipEvent_t ev_in = nullptr;
  int64_t graph_launches = 0;

  // timing
  bool prof = false;
  std::vector<Timer> timers;
  std::vector<hipEvent_t> pool;
  double kms[MPE_KC_COUNT] = {0};
  int64_t kcount[MPE_KC_COUNT] = {0};

  double* S() { return mats; }
  double* Hs() { return mats + (size_t)mp * mp; }
  double* Mm() { return mats + 2 * (size_t)mp * mp; }
  double* L() { return mats + 3 * (size_t)mp * mp; }
  double* C() { return mats + 4 * (size_t)mp * mp; }
  double* theta() { return res; }
  double* rh() { return res + MAXM; }
  double* re() { return res + 2 * MAXM; }
  double* reperp() { return res + 3 * MAXM; }
  double* scratch() { return res + 4 * MAXM; }
  const void* rx() const { return roots; }
  const void* ry() const { return (const char*)roots + off_ry; }
  const void* rz() const { return (const char*)roots + off_rz; }
  const void* wpost() const { return (const char*)roots + off_wp; }
  size_t cx_size() const { return 2 * fsz; }
};

namespace {

mpe_status fail(mpe_plan p, mpe_status s, const std::string& msg) {
  if (p) p->err = msg;
  return s;
}

#define HIPCHK(p, expr)                                                                           \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return fail(p, MPE_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

hipEvent_t get_event(mpe_plan p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void tic(mpe_plan p, Timer& t, int kc) {
  t.kc = kc;
  t.a = t.b = nullptr;
  if (!p->prof) return;
  t.a = get_event(p);
  t.b = get_event(p);
  if (t.a) (void)hipEventRecord(t.a, p->st);
}

void toc(mpe_plan p, Timer& t) {
  if (!p->prof || !t.a || !t.b) return;
  (void)hipEventRecord(t.b, p->st);
  p->timers.push_back(t);
}

void collect_times(mpe_plan p) {
  if (p->timers.empty()) return;
  (void)hipStreamSynchronize(p->st);
  for (auto& t : p->timers) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      p->kms[t.kc] += ms;
      p->kcount[t.kc] += 1;
    }
    p->pool.push_back(t.a);
    p->pool.push_back(t.b);
  }
  p->timers.clear();
}

template <typename F>
hipError_t launch_factor_tables(mpe_plan p, double dt, void* fac, void* kin) {
  const long N = p->N;
  hipLaunchKernelGGL(factor_tables_kernel<F>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, p->st, p->V64, N, dt,
                     2 * p->K, reinterpret_cast<F*>(fac));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int len = p->nxh + p->ny + p->nz;
  hipLaunchKernelGGL(kinetic_tables_kernel<F>, dim3((len + 255) / 256), dim3(256), 0, p->st, p->nx, p->ny, p->nz, p->Lx,
                     p->Ly, p->Lz, p->h2m, dt, p->K, reinterpret_cast<F*>(kin), reinterpret_cast<F*>(p->hk));
  return hipGetLastError();
}

mpe_status ensure_tables(mpe_plan p, double dt) {
  if (!p->have_v) return fail(p, MPE_ERR_STATE, "no potential set (mpe_set_potential)");
  if (p->tab_dt == dt) return MPE_OK;
  HIPCHK(p, p->dbl ? launch_factor_tables<double>(p, dt, p->fac, p->kin)
                   : launch_factor_tables<float>(p, dt, p->fac, p->kin));
  if (p->prop == MPE_PROP_ROMBERG6)   // the two half steps of Eq. sixp
    HIPCHK(p, p->dbl ? launch_factor_tables<double>(p, 0.5 * dt, p->fac2, p->kin2)
                     : launch_factor_tables<float>(p, 0.5 * dt, p->fac2, p->kin2));
  p->tab_dt = dt;
  return MPE_OK;
}

// Launch groups of states: [s0, s0 + count) covering [first, m) with count <= states_per_launch.
template <typename Fn>
hipError_t for_groups(mpe_plan p, Fn fn, int first = 0) {
  const int G = (p->states_per_launch > 0 && p->states_per_launch < p->m) ? p->states_per_launch : p->m;
  for (int s0 = first; s0 < p->m; s0 += G) {
    hipError_t e = fn(s0, std::min(G, p->m - s0));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// forward-pass shape: modes 0..5 as for the link pass (persist kind mode % 3,
// states fastest for mode / 3); 6 / 7 = the chain loop with z / states fastest
void set_fwd_shape(mpe_plan p, PlaneArgs& a) {
  const int m = p->pmode[0];
  a.fwd_loop = m >= 6;
  a.persist_mode = m >= 6 ? 0 : m % 3;
  a.states_fast = m >= 6 ? m - 6 : m / 3;
  a.persist_blocks = p->pbpc[0] * p->n_cu;
}

PlaneArgs plane_base(mpe_plan p) {
  PlaneArgs a;
  std::memset(&a, 0, sizeof(a));
  a.rx = p->rx();
  a.ry = p->ry();
  a.wpost = p->wpost();
  a.real_state_stride = p->N;
  a.spec_state_stride = p->spec;
  a.fac_table_stride = p->N;
  a.fac_index = -1;
  return a;
}

PencilArgs pencil_base(mpe_plan p, void* data, const void* tab) {
  PencilArgs a;
  std::memset(&a, 0, sizeof(a));
  a.tile = p->ptile;
  a.data = data;
  a.rz = p->rz();
  a.tab = tab;
  a.state_stride = p->spec;
  a.M = (int)p->M;
  a.NXH = p->nxh;
  a.NY = p->ny;
  return a;
}

void* chain_spec(mpe_plan p, int k) {  // k = 0..K-1
  return (char*)p->W + (size_t)k * p->m * p->spec * p->cx_size();
}

mpe_status enqueue_step3(mpe_plan p, const void* src, void* dst, int first, const void* fac, const void* kin);

// dst <- T_2K(dt) src, all m states (src may equal dst); tables for dt must be current.
// Propagation of states [first, m) of src into dst (the rows below first are
// not touched).
mpe_status enqueue_step(mpe_plan p, const void* src, void* dst, int first = 0, const void* fac = nullptr,
                        const void* kin = nullptr) {
  if (!fac) fac = p->fac;
  if (!kin) kin = p->kin;
  if (p->three_pass) return enqueue_step3(p, src, dst, first, fac, kin);
  const size_t f = p->fsz;
  double c[MAX_K];
  mpe_coeffs(p->K, c);
  // every chain's first potential half-step exp(-dt V / 2k) (table 2k - 1) and
  // forward transform, from one read of src
  {
    Timer t;
    tic(p, t, MPE_KC_PLANE_FWD);
    HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
             PlaneArgs a = plane_base(p);
             a.real_in = src;
             a.fac = fac;
             a.fac_index = 1;
             a.fwd_chains = p->K;
             a.spec = chain_spec(p, 0);
             a.chain_stride = (long)p->m * p->spec;
             a.state0 = s0;
             set_fwd_shape(p, a);
             return launch_plane(p->dbl, PM_FWD, p->nx, a, p->nz, cnt, p->st);
           }, first));
    toc(p, t);
  }
  for (int k = 1; k <= p->K; ++k) {
    void* Wk = chain_spec(p, k - 1);
    const int full = k - 1;       // table exp(-dt V / k)
    const void* ktab = (const char*)kin + (size_t)(k - 1) * (p->nxh + p->ny + p->nz) * f;
    Timer t;
    for (int l = 1; l <= k; ++l) {
      tic(p, t, MPE_KC_PENCIL);
      HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
               PencilArgs a = pencil_base(p, Wk, ktab);
               a.state0 = s0;
               return launch_pencil(p->dbl, PK_EXP, p->nz, a, cnt, p->st);
             }, first));
      toc(p, t);
      if (l < k) {
        tic(p, t, MPE_KC_PLANE_LINK);
        HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
                 PlaneArgs a = plane_base(p);
                 a.spec = Wk;
                 a.fac = fac;
                 a.fac_index = full;
                 a.state0 = s0;
                 a.persist_mode = p->pmode[1] % 3;
                 a.states_fast = p->pmode[1] / 3;
                 a.persist_blocks = p->pbpc[1] * p->n_cu;
                 return launch_plane(p->dbl, PM_LINK, p->nx, a, p->nz, cnt, p->st);
               }, first));
        toc(p, t);
      }
    }
  }
  Timer t;
  tic(p, t, MPE_KC_PLANE_TAIL);
  if (p->split_tail) {
    // each chain leaves through its own pass, then the float64 combination
    for (int k = 0; k < p->K; ++k) {
      void* out_k = (char*)p->tailbuf + (size_t)k * p->m * p->N * f;
      HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
               PlaneArgs a = plane_base(p);
               a.spec = chain_spec(p, k);
               a.fac = fac;
               a.fac_index = 2 * k + 1;
               a.real_out = out_k;
               a.state0 = s0;
               a.states_fast = p->pmode[1] / 3;
               return launch_plane(p->dbl, PM_OUT, p->nx, a, p->nz, cnt, p->st);
             }, first));
    }
    const size_t off = (size_t)first * p->N * f;
    HIPCHK(p, launch_combine(p->dbl, (const char*)p->tailbuf + off, (long)p->m * p->N, p->K, c, (char*)dst + off,
                             (long)(p->m - first) * p->N, p->st));
  } else {
    HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
             PlaneArgs a = plane_base(p);
             a.spec = chain_spec(p, 0);
             a.chain_stride = (long)p->m * p->spec;
             a.fac = fac;
             a.real_out = dst;
             a.K = p->K;
             for (int k = 0; k < p->K; ++k) a.coef[k] = c[k];
             a.state0 = s0;
             return launch_plane(p->dbl, PM_TAIL, p->nx, a, p->nz, cnt, p->st);
           }, first));
  }
  toc(p, t);
  return MPE_OK;
}

// y transforms of every z plane of states [s0, s0 + cnt): the pencil kernel
// along y (stride NX/2+1), one "state" per (state, z) plane.
hipError_t launch_ypass(mpe_plan p, int kind, void* spec, int s0, int cnt) {
  PencilArgs a;
  std::memset(&a, 0, sizeof(a));
  a.data = spec;
  a.rz = p->ry();
  a.state_stride = (long)p->ny * p->nxh;
  a.M = p->nxh;
  a.NXH = p->nxh;
  a.NY = p->ny;
  a.state0 = s0 * p->nz;
  return launch_pencil(p->dbl, kind, p->ny, a, cnt * p->nz, p->st);
}

PlaneArgs row_base(mpe_plan p, void* spec, const void* fac, int fac_index, int s0) {
  PlaneArgs a = plane_base(p);
  a.spec = spec;
  a.fac = fac;
  a.fac_index = fac_index;
  a.state0 = s0;
  return a;
}

// Three-pass form of enqueue_step: per T2 application a z pencil pass and
// row / column passes in place of the plane pass; each chain leaves through a
// row pass into its real buffer, combined in float64.
mpe_status enqueue_step3(mpe_plan p, const void* src, void* dst, int first, const void* fac, const void* kin) {
  const size_t f = p->fsz;
  double c[MAX_K];
  mpe_coeffs(p->K, c);
  for (int k = 1; k <= p->K; ++k) {
    void* Wk = chain_spec(p, k - 1);
    const void* ktab = (const char*)kin + (size_t)(k - 1) * (p->nxh + p->ny + p->nz) * f;
    void* out_k = (char*)p->tailbuf + (size_t)(k - 1) * p->m * p->N * f;
    Timer t;
    tic(p, t, MPE_KC_PLANE_FWD);
    HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
             PlaneArgs a = row_base(p, Wk, fac, 2 * k - 1, s0);
             a.real_in = src;
             hipError_t e = launch_rows(p->dbl, RW_FWD, p->nx, a, p->ny, p->nz, cnt, p->st);
             return e == hipSuccess ? launch_ypass(p, PK_FFT_FWD, Wk, s0, cnt) : e;
           }, first));
    toc(p, t);
    for (int l = 1; l <= k; ++l) {
      tic(p, t, MPE_KC_PENCIL);
      HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
               PencilArgs a = pencil_base(p, Wk, ktab);
               a.state0 = s0;
               return launch_pencil(p->dbl, PK_EXP, p->nz, a, cnt, p->st);
             }, first));
      toc(p, t);
      tic(p, t, l < k ? MPE_KC_PLANE_LINK : MPE_KC_PLANE_TAIL);
      HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
               hipError_t e = launch_ypass(p, PK_FFT_INV, Wk, s0, cnt);
               if (e != hipSuccess) return e;
               if (l < k) {
                 PlaneArgs a = row_base(p, Wk, fac, k - 1, s0);
                 e = launch_rows(p->dbl, RW_LINK, p->nx, a, p->ny, p->nz, cnt, p->st);
                 return e == hipSuccess ? launch_ypass(p, PK_FFT_FWD, Wk, s0, cnt) : e;
               }
               PlaneArgs a = row_base(p, Wk, fac, 2 * k - 1, s0);
               a.real_out = out_k;
               return launch_rows(p->dbl, RW_OUT, p->nx, a, p->ny, p->nz, cnt, p->st);
             }, first));
      toc(p, t);
    }
  }
  Timer t;
  tic(p, t, MPE_KC_PLANE_TAIL);
  const size_t off = (size_t)first * p->N * f;
  HIPCHK(p, launch_combine(p->dbl, (const char*)p->tailbuf + off, (long)p->m * p->N, p->K, c, (char*)dst + off,
                           (long)(p->m - first) * p->N, p->st));
  toc(p, t);
  return MPE_OK;
}

// dst <- T(dt) src for states [first, m) with the plan's propagator: the
// order-2K expansion, or the Romberg-type T6 of Section II (Eq. sixp) built
// from the order-4 expansion T4 (K = 2): -T4(dt)/15 + 16 T4(dt/2)^2/15, the
// two terms staged in rtmp and combined in float64 with one rounding.
mpe_status enqueue_propagate(mpe_plan p, const void* src, void* dst, int first = 0) {
  if (p->prop != MPE_PROP_ROMBERG6) return enqueue_step(p, src, dst, first);
  const size_t blk = (size_t)p->m * p->N;
  void* full = p->rtmp;
  void* half = (char*)p->rtmp + blk * p->fsz;
  mpe_status s = enqueue_step(p, src, full, first);
  if (s == MPE_OK) s = enqueue_step(p, src, half, first, p->fac2, p->kin2);
  if (s == MPE_OK) s = enqueue_step(p, half, half, first, p->fac2, p->kin2);
  if (s != MPE_OK) return s;
  const double w[2] = {-1.0 / 15.0, 16.0 / 15.0};
  const size_t off = (size_t)first * p->N * p->fsz;
  HIPCHK(p, launch_combine(p->dbl, (const char*)p->rtmp + off, (long)blk, 2, w, (char*)dst + off,
                           (long)(p->m - first) * p->N, p->st));
  return MPE_OK;
}

mpe_status run_step(mpe_plan p, const void* src, void* dst, double dt) {
  mpe_status s = ensure_tables(p, dt);
  if (s != MPE_OK) return s;
  s = enqueue_propagate(p, src, dst);
  if (s == MPE_OK) p->last_dt = dt;
  return s;
}

// hdst <- H src for states [first, m) (src != hdst); uses chain 0's spectrum buffer as scratch.
mpe_status run_h(mpe_plan p, const void* src, void* hdst, int first = 0) {
  if (!p->have_v) return fail(p, MPE_ERR_STATE, "no potential set (mpe_set_potential)");
  if (p->tab_dt < 0) {
    mpe_status s = ensure_tables(p, 1.0);  // builds the additive table (independent of dt)
    if (s != MPE_OK) return s;
  }
  void* Wh = chain_spec(p, 0);
  Timer t;
  tic(p, t, MPE_KC_H_APPLY);
  if (p->three_pass) {
    HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
             PlaneArgs a = row_base(p, Wh, nullptr, -1, s0);
             a.real_in = src;
             hipError_t e = launch_rows(p->dbl, RW_FWD, p->nx, a, p->ny, p->nz, cnt, p->st);
             if (e == hipSuccess) e = launch_ypass(p, PK_FFT_FWD, Wh, s0, cnt);
             if (e != hipSuccess) return e;
             PencilArgs b = pencil_base(p, Wh, p->hk);
             b.state0 = s0;
             e = launch_pencil(p->dbl, PK_ADD, p->nz, b, cnt, p->st);
             if (e == hipSuccess) e = launch_ypass(p, PK_FFT_INV, Wh, s0, cnt);
             if (e != hipSuccess) return e;
             PlaneArgs c = row_base(p, Wh, p->Vf, -1, s0);
             c.real_in = src;
             c.real_out = hdst;
             return launch_rows(p->dbl, RW_HTAIL, p->nx, c, p->ny, p->nz, cnt, p->st);
           }, first));
    toc(p, t);
    return MPE_OK;
  }
  HIPCHK(p, for_groups(p, [&](int s0, int cnt) {
           PlaneArgs a = plane_base(p);
           a.real_in = src;
           a.fac = nullptr;
           a.fac_index = -1;
           a.spec = Wh;
           a.state0 = s0;
           hipError_t e = launch_plane(p->dbl, PM_FWD, p->nx, a, p->nz, cnt, p->st);
           if (e != hipSuccess) return e;
           PencilArgs b = pencil_base(p, Wh, p->hk);
           b.state0 = s0;
           e = launch_pencil(p->dbl, PK_ADD, p->nz, b, cnt, p->st);
           if (e != hipSuccess) return e;
           PlaneArgs c = plane_base(p);
           c.spec = Wh;
           c.real_in = src;
           c.fac = p->Vf;
           c.real_out = hdst;
           c.state0 = s0;
           c.states_fast = p->pmode[1] / 3;   // the link pass's plane order
           return launch_plane(p->dbl, PM_HTAIL, p->nx, c, p->nz, cnt, p->st);
         }, first));
  toc(p, t);
  return MPE_OK;
}

int gram_chunks(mpe_plan p, long* chunk) { return gram_chunking(p->N, 256, chunk); }

int rot_chunks(mpe_plan p, long* chunk) { return rot_chunking(p->N, chunk); }

// Overlaps X_i Y_i^T (i < nprod) reduced into outs[i] (mp x mp float64 each, contiguous from out0).
mpe_status run_gram(mpe_plan p, const void* const* X, const void* const* Y, int nprod, double* out0,
                    int upper_mask = 0) {
  GramArgs g;
  std::memset(&g, 0, sizeof(g));
  g.upper_mask = upper_mask;
  for (int i = 0; i < nprod; ++i) {
    g.X[i] = X[i];
    g.Y[i] = Y[i];
  }
  long chunk;
  const int nch = gram_chunks(p, &chunk);
  g.partials = p->partials;
  g.N = p->N;
  g.chunk = chunk;
  g.m = p->m;
  g.mp = p->mp;
  Timer t;
  tic(p, t, MPE_KC_GRAM);
  if (!p->dbl && p->gemm == 1) HIPCHK(p, launch_gram32(g, nprod, nch, p->st));
  else if (!p->dbl && p->gemm >= 2) HIPCHK(p, launch_gramb(g, nprod, nch, p->gemm == 2 ? 2 : 3, p->st));
  else HIPCHK(p, launch_gram(p->dbl, g, nprod, nch, p->st));
  HIPCHK(p, launch_reduce(p->partials, nch, (long)p->mp * p->mp, nprod, out0, p->st));
  toc(p, t);
  return MPE_OK;
}

mpe_status run_small_dense(mpe_plan p, int mode) {
  SmallDenseArgs d;
  std::memset(&d, 0, sizeof(d));
  d.S = p->S();
  d.Hs = p->Hs();
  d.L = p->L();
  d.rot = p->rot;
  d.scratch = p->scratch();
  d.C = p->C();
  d.theta = p->theta();
  d.status = p->status;
  d.m = p->m;
  d.mp = p->mp;
  d.mode = mode;
  d.max_sweeps = p->max_sweeps;
  d.ticks = p->ticks;
  d.tol = p->jacobi_tol;
  d.pivot_tol = p->pivot_tol;
  Timer t;
  tic(p, t, MPE_KC_SMALL_DENSE);
  HIPCHK(p, launch_small_dense(d, p->st));
  toc(p, t);
  return MPE_OK;
}

mpe_status run_rotate(mpe_plan p, const void* Phi, const void* HPhi, void* Psi, void* HPsi) {
  RotateArgs r;
  std::memset(&r, 0, sizeof(r));
  long chunk;
  const int nch = rot_chunks(p, &chunk);
  r.Phi = Phi;
  r.HPhi = HPhi;
  r.C = p->C();
  r.theta = p->theta();
  r.Psi = Psi;
  r.HPsi = HPsi;
  r.res_partials = p->partials;
  r.status = p->status;
  r.N = p->N;
  r.chunk = chunk;
  r.m = p->m;
  r.mp = p->mp;
  Timer t;
  tic(p, t, MPE_KC_ROTATE);
  HIPCHK(p, launch_rotate(p->dbl, HPhi != nullptr, r, nch, p->st));
  if (HPhi) HIPCHK(p, launch_reduce(p->partials, nch, (long)p->mp, 1, p->rh(), p->st));
  toc(p, t);
  return MPE_OK;
}

// Copy results + status to the pinned mirror and wait.
mpe_status fetch(mpe_plan p) {
  HIPCHK(p, hipMemcpyAsync(p->host_res, p->res, p->res_bytes, hipMemcpyDeviceToHost, p->st));
  HIPCHK(p, hipStreamSynchronize(p->st));
  collect_times(p);
  return MPE_OK;
}

mpe_status status_to_error(mpe_plan p) {
  const int* hs = reinterpret_cast<const int*>(p->host_res + 6 * MAXM);
  switch (hs[0]) {
    case ST_OK: return MPE_OK;
    case ST_NOT_SPD: {
      char b[128];
      snprintf(b, sizeof b, "overlap matrix not positive definite at pivot %d", hs[1]);
      return fail(p, MPE_ERR_NOT_POSITIVE_DEFINITE, b);
    }
    case ST_NONFINITE: {
      char b[128];
      snprintf(b, sizeof b, "non-finite value in the overlap matrix at pivot %d", hs[1]);
      return fail(p, MPE_ERR_NONFINITE, b);
    }
    case ST_EIG_NO_CONV: {
      char b[128];
      snprintf(b, sizeof b, "Jacobi eigensolver did not converge in %d sweeps", hs[1]);
      return fail(p, MPE_ERR_EIG_NO_CONVERGENCE, b);
    }
    default: return fail(p, MPE_ERR_DEVICE, "unknown device status");
  }
}

void copy_out(double* dst, const double* src, int m) {
  if (dst) std::memcpy(dst, src, sizeof(double) * m);
}

bool size_ok(int n) {
  switch (n) {
    case 8: case 16: case 32: case 48: case 64: case 96: case 128: case 192: return true;
    default: return false;
  }
}

void host_roots(int L, std::vector<double>& out) {
  for (int j = 0; j < L; ++j) {
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)L;
    out.push_back((double)cosl(ang));
    out.push_back((double)sinl(ang));
  }
}

// Device work of one fused iteration on p->st, ending with the copy of the
// results to the pinned mirror (no synchronisation).  Tables must be current.
mpe_status enqueue_iterate(mpe_plan p, void* psi) {
  // locked states (Section III: only states not yet converged need propagating)
  // enter the overlaps and the rotation unpropagated: Phi_j = Psi_j
  const size_t row = (size_t)p->N * p->fsz;
  const bool mapped = p->lock_mapped && p->locked > 0;
  mpe_status s = MPE_OK;
  if (mapped) {
    // any locked set: Phi holds the states in the order perm (locked first), so
    // the propagation covers one contiguous run; the overlaps, the Rayleigh-Ritz
    // rotation and R^H do not depend on the order of Phi's rows, and the
    // variances are written back to each state's own entry
    // the cached H Psi of the locked states outside rows 0..locked-1 moves into
    // the rows there of unlocked states (whose H the propagation replaces)
    if (p->hfirst > 0) HIPCHK(p, launch_move_rows(p->hphi, p->perm, p->locked, row, p->st));
    HIPCHK(p, launch_gather_rows(p->phi, psi, p->perm, p->m, row, p->st));
    s = enqueue_propagate(p, p->phi, p->phi, p->locked);
  } else {
    if (p->locked > 0) HIPCHK(p, launch_copy16(p->phi, psi, (size_t)p->locked * row, p->st));
    s = enqueue_propagate(p, psi, p->phi, p->locked);
  }
  // H Phi_j = H Psi_j of the locked states is still in hphi from the previous
  // rotation when nothing touched psi since (p->hfirst > 0 only then)
  if (s == MPE_OK) s = run_h(p, p->phi, p->hphi, p->hfirst);
  const void* X[3] = {p->phi, p->phi, psi};
  const void* Y[3] = {p->phi, p->hphi, p->phi};
  // S, Hs (upper tiles) and, with the variances, M; contiguous
  if (s == MPE_OK) s = run_gram(p, X, Y, p->variances ? 3 : 2, p->S(), 2);
  if (s == MPE_OK && p->variances) {
    hipError_t e = launch_variance(p->S(), p->Mm(), p->m, p->mp, mapped ? p->perm : nullptr, p->re(), p->reperp(),
                                   p->st);
    if (e != hipSuccess) s = fail(p, MPE_ERR_DEVICE, hipGetErrorString(e));
  }
  if (s == MPE_OK) s = run_small_dense(p, SD_RR);
  if (s == MPE_OK) s = run_rotate(p, p->phi, p->hphi, psi, p->hphi);
  if (s != MPE_OK) return s;
  HIPCHK(p, hipMemcpyAsync(p->host_res, p->res, p->res_bytes, hipMemcpyDeviceToHost, p->st));
  return MPE_OK;
}

void drop_graph_slot(mpe_plan_s::IterGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = mpe_plan_s::IterGraph();
}

void drop_graph(mpe_plan p) {
  drop_graph_slot(p->ig[0]);
  drop_graph_slot(p->ig[1]);
}

// Capture enqueue_iterate(psi) on the private stream into an executable graph.
mpe_status capture_iterate(mpe_plan p, void* psi) {
  mpe_plan_s::IterGraph& ig = p->ig[p->variances ? 1 : 0];
  drop_graph_slot(ig);
  if (!p->gst) HIPCHK(p, hipStreamCreateWithFlags(&p->gst, hipStreamNonBlocking));
  if (!p->ev_in) HIPCHK(p, hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
  HIPCHK(p, hipStreamBeginCapture(p->gst, hipStreamCaptureModeRelaxed));
  hipStream_t user = p->st;
  p->st = p->gst;
  mpe_status s = enqueue_iterate(p, psi);
  p->st = user;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p->gst, &g);
  if (s != MPE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(p, MPE_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  ig.graph = g;
  HIPCHK(p, hipGraphInstantiate(&ig.exec, ig.graph, nullptr, nullptr, 0));
  ig.psi = psi;
  ig.spl = p->states_per_launch;
  ig.locked = p->locked;
  ig.mapped = p->lock_mapped ? 1 : 0;
  ig.hfirst = p->hfirst;
  ig.shape = p->shape_ver;
  return MPE_OK;
}

mpe_status finish_iterate(mpe_plan p, void* psi, double* eig, double* rh, double* re, double* re_perp) {
  mpe_status s = status_to_error(p);
  if (s != MPE_OK) return s;
  copy_out(eig, p->host_res, p->m);
  copy_out(rh, p->host_res + MAXM, p->m);
  if (p->variances) {
    copy_out(re, p->host_res + 2 * MAXM, p->m);
    copy_out(re_perp, p->host_res + 3 * MAXM, p->m);
  } else {
    for (int j = 0; j < p->m; ++j) {
      if (re) re[j] = std::numeric_limits<double>::quiet_NaN();
      if (re_perp) re_perp[j] = std::numeric_limits<double>::quiet_NaN();
    }
  }
  p->rr_cache_psi = psi;   // hphi now holds H psi (rotated)
  return MPE_OK;
}

}  // namespace

// ------------------------------------------------------------------ exported API
extern "C" {

int mpe_abi_version(void) { return MPE_ABI_VERSION; }

const char* mpe_status_string(mpe_status s) {
  switch (s) {
    case MPE_OK: return "ok";
    case MPE_ERR_INVALID_ARGUMENT: return "invalid argument";
    case MPE_ERR_UNSUPPORTED: return "unsupported configuration";
    case MPE_ERR_OUT_OF_MEMORY: return "out of device memory";
    case MPE_ERR_NOT_POSITIVE_DEFINITE: return "overlap matrix not positive definite";
    case MPE_ERR_EIG_NO_CONVERGENCE: return "eigensolver did not converge";
    case MPE_ERR_NONFINITE: return "non-finite values";
    case MPE_ERR_DEVICE: return "HIP runtime error";
    case MPE_ERR_STATE: return "invalid call order";
  }
  return "unknown status";
}

mpe_status mpe_coefficients(int32_t order, double* c) {
  if (!c || order < 2 || order > 2 * MAX_K || order % 2) return MPE_ERR_INVALID_ARGUMENT;
  return mpe_coeffs(order / 2, c) ? MPE_OK : MPE_ERR_INVALID_ARGUMENT;
}

mpe_status mpe_plan_destroy(mpe_plan p) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  (void)hipStreamSynchronize(p->st);
  for (auto& t : p->timers) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : p->pool) (void)hipEventDestroy(e);
  drop_graph(p);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->gst) (void)hipStreamDestroy(p->gst);
  void* bufs[] = {p->W, p->tailbuf, p->phi, p->hphi, p->V64, p->Vf, p->fac, p->kin, p->hk, p->roots,
                  p->partials, p->mats, p->rot, p->res, p->ticks, p->fac2, p->kin2, p->rtmp, p->perm};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (p->host_res) (void)hipHostFree(p->host_res);
  delete p;
  return MPE_OK;
}

mpe_status mpe_plan_create(mpe_plan* out, const int32_t grid[3], const double box[3], int32_t n_states, int32_t order,
                           mpe_precision prec, int32_t n_guard, void* hip_stream) {
  if (!out) return MPE_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!grid || !box) return MPE_ERR_INVALID_ARGUMENT;
  if (order < 2 || order > 2 * MAX_K || order % 2) return MPE_ERR_INVALID_ARGUMENT;
  if (prec != MPE_FP64 && prec != MPE_FP32) return MPE_ERR_INVALID_ARGUMENT;
  if (n_states < 1 || n_guard < 0) return MPE_ERR_INVALID_ARGUMENT;
  for (int i = 0; i < 3; ++i) {
    if (grid[i] < 2 || grid[i] % 2) return MPE_ERR_INVALID_ARGUMENT;
    if (!(box[i] > 0.0) || !std::isfinite(box[i])) return MPE_ERR_INVALID_ARGUMENT;
  }
  const long N = (long)grid[0] * grid[1] * grid[2];
  const int m = n_states + n_guard;
  if (m > N) return MPE_ERR_INVALID_ARGUMENT;
  if (m > MAXM) return MPE_ERR_UNSUPPORTED;
  if (!size_ok(grid[0]) || !size_ok(grid[1]) || !size_ok(grid[2])) return MPE_ERR_UNSUPPORTED;
  const bool planes_fit = plane_supported(prec == MPE_FP64, grid[0], grid[1]);
  if (!pencil_supported(grid[2]) || (!planes_fit && (!row_supported(grid[0]) || !pencil_supported(grid[1]))))
    return MPE_ERR_UNSUPPORTED;

  mpe_plan p = new mpe_plan_s();
  p->nx = grid[0];
  p->ny = grid[1];
  p->nz = grid[2];
  p->nxh = p->nx / 2 + 1;
  p->Lx = box[0];
  p->Ly = box[1];
  p->Lz = box[2];
  p->n = n_states;
  p->g = n_guard;
  p->m = m;
  p->mp = (m + 15) / 16 * 16;
  p->K = order / 2;
  p->dbl = prec == MPE_FP64;
  // Jacobi convergence (|a_ij| <= tol sqrt|a_ii a_jj|): 1e-13 for float64 states;
  // 1e-7 for float32 states, the level of their own ~6e-8 relative rounding (a
  // coupling that small adds ~(1e-7 |theta|)^2 to R^H, far below any bound the
  // float32 floor allows).  R^H keeps any off-diagonal coupling that is left, so
  // convergence checks stay conservative.
  p->jacobi_tol = p->dbl ? 1e-13 : 1e-7;
  p->N = N;
  p->M = (long)p->ny * p->nxh;
  p->spec = (long)p->nz * p->M;
  p->fsz = p->dbl ? sizeof(double) : sizeof(float);
  p->st = reinterpret_cast<hipStream_t>(hip_stream);

  auto alloc = [&](void** ptr, size_t bytes) -> bool {
    if (hipMalloc(ptr, bytes) != hipSuccess) {
      *ptr = nullptr;
      return false;
    }
    p->ws_bytes += (int64_t)bytes;
    return true;
  };
  const size_t f = p->fsz, cxs = 2 * f;
  long gch;
  const int ngch = gram_chunks(p, &gch);
  long rch;
  const int nrch = rot_chunks(p, &rch);
  p->partials_bytes = std::max((size_t)3 * ngch * p->mp * p->mp, (size_t)nrch * p->mp) * sizeof(double);
  p->rot_count = small_dense_rot_doubles(p->max_sweeps) / 4 + 4;   // Jacobi rotation log
  p->res_bytes = 6 * MAXM * sizeof(double) + 4 * sizeof(int);
  const int tablen = p->nxh + p->ny + p->nz;
  std::vector<double> r;
  host_roots(p->nx / 2, r);
  p->off_ry = r.size() / 2 * cxs;
  host_roots(p->ny, r);
  p->off_rz = r.size() / 2 * cxs;
  host_roots(p->nz, r);
  p->off_wp = r.size() / 2 * cxs;
  {
    std::vector<double> w;
    host_roots(p->nx, w);
    for (int k = 0; k <= p->nx / 4; ++k) {
      r.push_back(w[2 * k]);
      r.push_back(w[2 * k + 1]);
    }
  }
  bool ok = alloc(&p->W, (size_t)p->K * m * p->spec * cxs) && alloc(&p->phi, (size_t)m * N * f) &&
            alloc(&p->hphi, (size_t)m * N * f) && alloc((void**)&p->V64, N * sizeof(double)) &&
            alloc(&p->Vf, N * f) && alloc(&p->fac, (size_t)2 * p->K * N * f) &&
            alloc(&p->kin, (size_t)p->K * tablen * f) && alloc(&p->hk, (size_t)tablen * f) &&
            alloc(&p->roots, r.size() / 2 * cxs) && alloc((void**)&p->partials, p->partials_bytes) &&
            alloc((void**)&p->mats, 5 * (size_t)p->mp * p->mp * sizeof(double)) &&
            alloc((void**)&p->rot, p->rot_count * 4 * sizeof(double)) && alloc((void**)&p->res, p->res_bytes) &&
            alloc((void**)&p->ticks, 8 * sizeof(long long)) && alloc((void**)&p->perm, MAXM * sizeof(int));
  p->three_pass = !planes_fit;
  p->split_tail = p->three_pass || tail_split(p->dbl, p->nx);
  if (ok && p->split_tail) ok = alloc(&p->tailbuf, (size_t)p->K * m * N * f);
  if (!ok) {
    mpe_plan_destroy(p);
    return MPE_ERR_OUT_OF_MEMORY;
  }
  p->status = reinterpret_cast<int*>(p->res + 6 * MAXM);
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || p->n_cu < 1) {
      mpe_plan_destroy(p);
      return MPE_ERR_DEVICE;
    }
  }
  if (prepare_small_dense() != hipSuccess) {
    mpe_plan_destroy(p);
    return MPE_ERR_DEVICE;
  }
  if (hipHostMalloc((void**)&p->host_res, p->res_bytes, hipHostMallocDefault) != hipSuccess) {
    mpe_plan_destroy(p);
    return MPE_ERR_OUT_OF_MEMORY;
  }
  // roots in the data type
  hipError_t e;
  if (p->dbl) {
    e = hipMemcpyAsync(p->roots, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice, p->st);
  } else {
    std::vector<float> rf(r.begin(), r.end());
    e = hipMemcpyAsync(p->roots, rf.data(), rf.size() * sizeof(float), hipMemcpyHostToDevice, p->st);
    if (e == hipSuccess) e = hipStreamSynchronize(p->st);
  }
  if (e == hipSuccess) e = hipMemsetAsync(p->res, 0, p->res_bytes, p->st);
  if (e == hipSuccess) e = hipMemsetAsync(p->mats, 0, 5 * (size_t)p->mp * p->mp * sizeof(double), p->st);
  if (e == hipSuccess) e = hipStreamSynchronize(p->st);
  if (e != hipSuccess) {
    mpe_plan_destroy(p);
    return MPE_ERR_DEVICE;
  }
  *out = p;
  return MPE_OK;
}

const char* mpe_last_error(mpe_plan p) { return p ? p->err.c_str() : "null plan"; }

int64_t mpe_workspace_bytes(mpe_plan p) { return p ? p->ws_bytes : 0; }

mpe_status mpe_set_potential(mpe_plan p, const double* V, double hbar2_over_m) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!V) return fail(p, MPE_ERR_INVALID_ARGUMENT, "V is null");
  if (!(hbar2_over_m > 0.0) || !std::isfinite(hbar2_over_m))
    return fail(p, MPE_ERR_INVALID_ARGUMENT, "hbar2_over_m must be positive");
  HIPCHK(p, hipMemcpyAsync(p->V64, V, p->N * sizeof(double), hipMemcpyDeviceToDevice, p->st));
  const unsigned nb = (unsigned)((p->N + 255) / 256);
  if (p->dbl)
    hipLaunchKernelGGL(cast_kernel<double>, dim3(nb), dim3(256), 0, p->st, p->V64, p->N, (double*)p->Vf);
  else
    hipLaunchKernelGGL(cast_kernel<float>, dim3(nb), dim3(256), 0, p->st, p->V64, p->N, (float*)p->Vf);
  HIPCHK(p, hipGetLastError());
  p->h2m = hbar2_over_m;
  p->have_v = true;
  p->tab_dt = -1.0;
  p->rr_cache_psi = nullptr;
  return MPE_OK;
}

mpe_status mpe_step(mpe_plan p, void* psi, double dt) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!psi) return fail(p, MPE_ERR_INVALID_ARGUMENT, "psi is null");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, MPE_ERR_INVALID_ARGUMENT, "dt must be positive");
  p->rr_cache_psi = nullptr;
  mpe_status s = run_step(p, psi, psi, dt);
  collect_times(p);
  return s;
}

mpe_status mpe_apply_h(mpe_plan p, const void* psi, void* hpsi) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!psi || !hpsi) return fail(p, MPE_ERR_INVALID_ARGUMENT, "null array");
  if (psi == hpsi) return fail(p, MPE_ERR_INVALID_ARGUMENT, "psi and hpsi must differ");
  p->rr_cache_psi = nullptr;
  mpe_status s = run_h(p, psi, hpsi);
  collect_times(p);
  return s;
}

mpe_status mpe_orthonormalize(mpe_plan p, void* psi) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!psi) return fail(p, MPE_ERR_INVALID_ARGUMENT, "psi is null");
  p->rr_cache_psi = nullptr;
  const void* X[1] = {psi};
  mpe_status s = run_gram(p, X, X, 1, p->S());
  if (s == MPE_OK) s = run_small_dense(p, SD_ORTHO);
  if (s == MPE_OK) s = run_rotate(p, psi, nullptr, psi, nullptr);
  if (s != MPE_OK) return s;
  s = fetch(p);
  if (s != MPE_OK) return s;
  return status_to_error(p);
}

mpe_status mpe_rayleigh_ritz(mpe_plan p, void* psi, double* eig) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!psi || !eig) return fail(p, MPE_ERR_INVALID_ARGUMENT, "null array");
  p->rr_cache_psi = nullptr;
  mpe_status s = run_h(p, psi, p->hphi);
  const void* X[2] = {psi, psi};
  const void* Y[2] = {psi, p->hphi};
  if (s == MPE_OK) s = run_gram(p, X, Y, 2, p->S(), 2);   // Hs from its upper tiles
  if (s == MPE_OK) s = run_small_dense(p, SD_RR);
  if (s == MPE_OK) s = run_rotate(p, psi, p->hphi, psi, p->hphi);
  if (s != MPE_OK) return s;
  s = fetch(p);
  if (s != MPE_OK) return s;
  s = status_to_error(p);
  if (s != MPE_OK) return s;
  copy_out(eig, p->host_res, p->m);
  p->rr_cache_psi = psi;
  return MPE_OK;
}

mpe_status mpe_residuals(mpe_plan p, const void* psi, const double* eig, double* rh, double* re) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!psi || !eig || !rh) return fail(p, MPE_ERR_INVALID_ARGUMENT, "null array");
  if (p->rr_cache_psi != psi) {
    mpe_status s = run_h(p, psi, p->hphi);
    if (s != MPE_OK) return s;
    p->rr_cache_psi = psi;
  }
  // values to the device (theta slot), then R^H partials
  HIPCHK(p, hipMemcpyAsync(p->scratch(), eig, sizeof(double) * p->m, hipMemcpyHostToDevice, p->st));
  long chunk;
  const int nch = rot_chunks(p, &chunk);
  Timer t;
  tic(p, t, MPE_KC_OTHER);
  if (p->dbl)
    hipLaunchKernelGGL(residual_kernel<double>, dim3(nch, p->m), dim3(256), 0, p->st, (const double*)psi,
                       (const double*)p->hphi, (const double*)p->scratch(), p->N, chunk, p->mp, p->partials);
  else
    hipLaunchKernelGGL(residual_kernel<float>, dim3(nch, p->m), dim3(256), 0, p->st, (const float*)psi,
                       (const float*)p->hphi, (const double*)p->scratch(), p->N, chunk, p->mp, p->partials);
  HIPCHK(p, hipGetLastError());
  HIPCHK(p, launch_reduce(p->partials, nch, (long)p->mp, 1, p->rh(), p->st));
  toc(p, t);
  if (re) {
    if (p->last_dt <= 0) return fail(p, MPE_ERR_STATE, "R^E needs a previous step size");
    mpe_status s = run_step(p, psi, p->phi, p->last_dt);
    if (s != MPE_OK) return s;
    const void* X[2] = {p->phi, psi};
    const void* Y[2] = {p->phi, p->phi};
    s = run_gram(p, X, Y, 2, p->S());   // S = phi phi^T, Hs slot = psi phi^T
    if (s != MPE_OK) return s;
    HIPCHK(p, launch_variance(p->S(), p->Hs(), p->m, p->mp, nullptr, p->re(), p->reperp(), p->st));
  }
  // the H psi cache stays valid (psi unchanged)
  HIPCHK(p, hipMemsetAsync(p->status, 0, 4 * sizeof(int), p->st));
  mpe_status s = fetch(p);
  if (s != MPE_OK) return s;
  copy_out(rh, p->host_res + MAXM, p->m);
  if (re) copy_out(re, p->host_res + 2 * MAXM, p->m);
  return MPE_OK;
}

mpe_status mpe_forget_cached_h(mpe_plan p) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  p->rr_cache_psi = nullptr;
  return MPE_OK;
}

mpe_status mpe_iterate(mpe_plan p, void* psi, double dt, double* eig, double* rh, double* re, double* re_perp) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!psi) return fail(p, MPE_ERR_INVALID_ARGUMENT, "psi is null");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, MPE_ERR_INVALID_ARGUMENT, "dt must be positive");
  // hphi holds H psi (the previous iteration's or Rayleigh-Ritz rotation) only
  // when no call has touched psi since: then locked states reuse it
  p->hfirst = (p->locked > 0 && p->rr_cache_psi == psi) ? p->locked : 0;
  p->rr_cache_psi = nullptr;
  mpe_status s = ensure_tables(p, dt);
  if (s != MPE_OK) return s;
  p->last_dt = dt;
  if (p->use_graph && !p->prof) {
    const mpe_plan_s::IterGraph& ig = p->ig[p->variances ? 1 : 0];
    if (!ig.exec || ig.psi != psi || ig.spl != p->states_per_launch || ig.shape != p->shape_ver ||
        ig.locked != p->locked || ig.mapped != (p->lock_mapped ? 1 : 0) || ig.hfirst != p->hfirst) {
      s = capture_iterate(p, psi);
      if (s != MPE_OK) return s;
    }
    HIPCHK(p, hipEventRecord(p->ev_in, p->st));           // tables and earlier work on the user stream
    HIPCHK(p, hipStreamWaitEvent(p->gst, p->ev_in, 0));
    HIPCHK(p, hipGraphLaunch(p->ig[p->variances ? 1 : 0].exec, p->gst));
    HIPCHK(p, hipStreamSynchronize(p->gst));
    p->graph_launches++;
  } else {
    s = enqueue_iterate(p, psi);
    if (s != MPE_OK) return s;
    HIPCHK(p, hipStreamSynchronize(p->st));
    collect_times(p);
  }
  return finish_iterate(p, psi, eig, rh, re, re_perp);
}

mpe_status mpe_small_dense_phases(mpe_plan p, double* us) {
  if (!p || !us) return MPE_ERR_INVALID_ARGUMENT;
  long long t[8];
  HIPCHK(p, hipStreamSynchronize(p->st));
  HIPCHK(p, hipMemcpy(t, p->ticks, sizeof t, hipMemcpyDeviceToHost));
  for (int i = 0; i < 5; ++i) us[i] = (double)(t[i + 1] - t[i]) / 100.0;   // 100 MHz clock
  return MPE_OK;
}

int32_t mpe_last_jacobi_sweeps(mpe_plan p) {
  if (!p || !p->host_res) return -1;
  const int* hs = reinterpret_cast<const int*>(p->host_res + 6 * MAXM);
  return hs[0] == ST_OK ? hs[1] : -1;
}

mpe_status mpe_set_graph(mpe_plan p, int32_t on) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  p->use_graph = on != 0;
  if (!p->use_graph) drop_graph(p);
  return MPE_OK;
}

mpe_status mpe_set_propagator(mpe_plan p, int32_t kind) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (kind != MPE_PROP_EXPANSION && kind != MPE_PROP_ROMBERG6)
    return fail(p, MPE_ERR_INVALID_ARGUMENT, "kind must be MPE_PROP_EXPANSION or MPE_PROP_ROMBERG6");
  if (kind == MPE_PROP_ROMBERG6 && p->K != 2)
    return fail(p, MPE_ERR_UNSUPPORTED, "the Romberg T6 is built from T4: it needs a plan of order 4");
  if (kind == MPE_PROP_ROMBERG6 && !p->rtmp) {
    const size_t tablen = (size_t)(p->nxh + p->ny + p->nz);
    hipError_t e = hipMalloc(&p->fac2, (size_t)2 * p->K * p->N * p->fsz);
    if (e == hipSuccess) e = hipMalloc(&p->kin2, (size_t)p->K * tablen * p->fsz);
    if (e == hipSuccess) e = hipMalloc(&p->rtmp, (size_t)2 * p->m * p->N * p->fsz);
    if (e != hipSuccess) {
      for (void** b : {&p->fac2, &p->kin2, &p->rtmp})
        if (*b) (void)hipFree(*b), *b = nullptr;
      return fail(p, MPE_ERR_OUT_OF_MEMORY, "Romberg tables and staging blocks");
    }
    p->ws_bytes += (int64_t)((size_t)2 * p->K * p->N * p->fsz + (size_t)p->K * tablen * p->fsz +
                             (size_t)2 * p->m * p->N * p->fsz);
  }
  p->prop = kind;
  p->tab_dt = -1.0;   // rebuild the tables (the dt/2 set)
  p->shape_ver++;     // re-capture the iteration graph
  p->rr_cache_psi = nullptr;
  return MPE_OK;
}

int32_t mpe_get_propagator(mpe_plan p) { return p ? p->prop : -1; }

mpe_status mpe_set_three_pass(mpe_plan p, int32_t on) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (!on && !plane_supported(p->dbl, p->nx, p->ny))
    return fail(p, MPE_ERR_UNSUPPORTED, "the plane pass does not hold this grid's planes");
  if (on && !(row_supported(p->nx) && pencil_supported(p->ny)))
    return fail(p, MPE_ERR_UNSUPPORTED, "no row or column pass for this grid");
  if (on && !p->tailbuf) {
    const size_t bytes = (size_t)p->K * p->m * p->N * p->fsz;
    if (hipMalloc(&p->tailbuf, bytes) != hipSuccess) {
      p->tailbuf = nullptr;
      return fail(p, MPE_ERR_OUT_OF_MEMORY, "chain output buffers of the three-pass plan");
    }
    p->ws_bytes += (int64_t)bytes;
  }
  p->three_pass = on != 0;
  p->split_tail = p->three_pass || tail_split(p->dbl, p->nx);
  p->shape_ver++;
  return MPE_OK;
}

int32_t mpe_get_three_pass(mpe_plan p) { return p ? (p->three_pass ? 1 : 0) : -1; }

mpe_status mpe_set_variances(mpe_plan p, int32_t on) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  p->variances = on != 0;
  return MPE_OK;
}

mpe_status mpe_set_locked(mpe_plan p, int32_t locked) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (locked < 0 || locked > p->m) return fail(p, MPE_ERR_INVALID_ARGUMENT, "locked must lie in [0, m]");
  p->locked = locked;
  p->lock_mapped = false;
  return MPE_OK;
}

mpe_status mpe_set_locked_states(mpe_plan p, const uint8_t* mask) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  int n = 0, lead = 0;
  if (mask) {
    for (int j = 0; j < p->m; ++j) n += mask[j] ? 1 : 0;
    while (lead < p->m && mask[lead]) ++lead;
  }
  if (lead == n) return mpe_set_locked(p, n);   // none, or a leading run
  // rows 0..n-1 take the locked states, rows n..m-1 the others; a state stays
  // in its own row where that row is in its part, so only the locked states
  // beyond row n-1 and the unlocked ones before row n trade places (their
  // rows: destinations below n, sources from n on, as launch_move_rows needs)
  std::vector<int> lk_hi, un_lo, perm(p->m);
  for (int j = 0; j < n; ++j)
    if (!mask[j]) un_lo.push_back(j);
  for (int j = n; j < p->m; ++j)
    if (mask[j]) lk_hi.push_back(j);
  size_t a = 0, c = 0;
  for (int i = 0; i < n; ++i) perm[i] = mask[i] ? i : lk_hi[a++];
  for (int i = n; i < p->m; ++i) perm[i] = !mask[i] ? i : un_lo[c++];
  if (!p->lock_mapped || perm != p->lock_perm) {
    // no replay of a captured iteration is in flight here: mpe_iterate
    // synchronises before it returns
    HIPCHK(p, hipMemcpyAsync(p->perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, p->st));
    HIPCHK(p, hipStreamSynchronize(p->st));
    p->lock_perm = perm;
  }
  p->locked = n;
  p->lock_mapped = true;
  return MPE_OK;
}

int32_t mpe_get_locked(mpe_plan p) { return p ? p->locked : -1; }

mpe_status mpe_set_states_per_launch(mpe_plan p, int32_t states) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (states < 0) return fail(p, MPE_ERR_INVALID_ARGUMENT, "states must be >= 0");
  p->states_per_launch = states;
  return MPE_OK;
}

mpe_status mpe_set_plane_shape(mpe_plan p, int32_t kernel_class, int32_t mode, int32_t blocks_per_cu) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  const int c = kernel_class == MPE_KC_PLANE_FWD ? 0 : kernel_class == MPE_KC_PLANE_LINK ? 1 : -1;
  if (c < 0) return fail(p, MPE_ERR_INVALID_ARGUMENT, "kernel_class must be MPE_KC_PLANE_FWD or MPE_KC_PLANE_LINK");
  if (mode < 0 || mode > (c == 0 ? 7 : 5))
    return fail(p, MPE_ERR_INVALID_ARGUMENT, c == 0 ? "forward mode must lie in 0..7" : "link mode must lie in 0..5");
  const bool persistent = mode < 6 && mode % 3 > 0;
  if (persistent && (blocks_per_cu < 1 || blocks_per_cu > 16))
    return fail(p, MPE_ERR_INVALID_ARGUMENT, "blocks_per_cu must be in [1, 16] for a persistent shape");
  p->pmode[c] = mode;
  p->pbpc[c] = persistent ? blocks_per_cu : 0;
  p->shape_ver++;
  return MPE_OK;
}

mpe_status mpe_set_gemm_precision(mpe_plan p, int32_t mode) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (mode < MPE_GEMM_FP64 || mode > MPE_GEMM_BF16X6)
    return fail(p, MPE_ERR_INVALID_ARGUMENT, "mode must be one of MPE_GEMM_FP64, FP32, BF16X3, BF16X6");
  if (mode != MPE_GEMM_FP64 && p->dbl)
    return fail(p, MPE_ERR_UNSUPPORTED, "float32 and BF16-split overlap GEMMs are for float32 plans");
  p->gemm = mode;
  // overlaps now carry ~1e-7 (float32, BF16x6) or ~1e-5 (BF16x3) relative error: a
  // pivot below 1e-5 (1e-3) of its diagonal marks linearly dependent states
  p->pivot_tol = p->gemm == MPE_GEMM_FP64 ? 1e-13 : (p->gemm == MPE_GEMM_BF16X3 ? 1e-3 : 1e-5);
  p->shape_ver++;   // re-capture the iteration graph
  return MPE_OK;
}

mpe_status mpe_set_pencil_shape(mpe_plan p, int32_t tile) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  if (tile < 0 || tile > 2) return fail(p, MPE_ERR_INVALID_ARGUMENT, "tile must be 0, 1 or 2");
  p->ptile = tile;
  p->shape_ver++;
  return MPE_OK;
}

int32_t mpe_get_pencil_shape(mpe_plan p) { return p ? p->ptile : -1; }

mpe_status mpe_get_plane_shape(mpe_plan p, int32_t* shape) {
  if (!p || !shape) return MPE_ERR_INVALID_ARGUMENT;
  shape[0] = p->pmode[0];
  shape[1] = p->pbpc[0];
  shape[2] = p->pmode[1];
  shape[3] = p->pbpc[1];
  return MPE_OK;
}

mpe_status mpe_autotune(mpe_plan p, const void* psi, double dt, int32_t reps, const char* cache_path,
                        double* ms_out) {
  if (!p || !psi) return MPE_ERR_INVALID_ARGUMENT;
  if (!(dt > 0.0) || !std::isfinite(dt) || reps < 1) return fail(p, MPE_ERR_INVALID_ARGUMENT, "dt > 0, reps >= 1");
  if (!p->have_v) return fail(p, MPE_ERR_STATE, "no potential set (mpe_set_potential)");
  // cache key: device, grid, precision, block size, order
  std::string key;
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return fail(p, MPE_ERR_DEVICE, "device query failed");
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s/%d %d %d %d %s m%d K%d", prop.gcnArchName, p->n_cu, p->nx, p->ny, p->nz,
                  p->dbl ? "fp64" : "fp32", p->m, p->K);
    key = buf;
    for (char& ch : key)
      if (ch == '\n' || ch == '|') ch = ' ';
  }
  if (cache_path && *cache_path) {
    std::FILE* f = std::fopen(cache_path, "r");
    if (f) {
      char line[512];
      int best[5] = {0, 0, 0, 0, 0};
      bool hit = false;
      while (std::fgets(line, sizeof line, f)) {
        char* bar = std::strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        int v[5] = {0, 0, 0, 0, 0};
        const int n = std::sscanf(bar + 1, "%d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4]);
        if (key == line && n >= 4) {   // the last matching line wins; a missing fifth field is tile 0
          hit = true;
          std::memcpy(best, v, sizeof best);
        }
      }
      std::fclose(f);
      if (hit) {
        mpe_status s = mpe_set_plane_shape(p, MPE_KC_PLANE_FWD, best[0], best[1]);
        if (s == MPE_OK) s = mpe_set_plane_shape(p, MPE_KC_PLANE_LINK, best[2], best[3]);
        if (s == MPE_OK) s = mpe_set_pencil_shape(p, best[4]);
        if (s == MPE_OK) {
          if (ms_out) ms_out[0] = ms_out[1] = -1.0;
          return MPE_OK;
        }
      }
    }
  }
  mpe_status s = ensure_tables(p, dt);
  if (s != MPE_OK) return s;
  // candidate shapes (mode, work-groups per CU), timed on steps psi -> phi;
  // the forward pass's chain loop (modes 6, 7) is timed beside link modes 0, 3
  const int cand[][2] = {{0, 0}, {1, 1}, {2, 1}, {2, 2}, {2, 4}, {3, 0}, {4, 1}, {5, 1}, {5, 2}, {5, 4}, {6, 0}, {7, 0}};
  const int nc = (int)(sizeof cand / sizeof cand[0]);
  double best_ms[2] = {1e300, 1e300};
  int best_c[2] = {0, 0};
  const bool prof0 = p->prof;
  collect_times(p);
  double saved_ms[MPE_KC_COUNT];
  int64_t saved_n[MPE_KC_COUNT];
  for (int i = 0; i < MPE_KC_COUNT; ++i) saved_ms[i] = p->kms[i], saved_n[i] = p->kcount[i];
  p->prof = true;
  for (int c = 0; c < nc; ++c) {
    const bool loop = cand[c][0] >= 6;
    p->pmode[0] = cand[c][0];
    p->pmode[1] = loop ? 3 * (cand[c][0] - 6) : cand[c][0];
    p->pbpc[0] = p->pbpc[1] = cand[c][1];
    s = enqueue_step(p, psi, p->phi);   // warm-up
    if (s != MPE_OK) break;
    collect_times(p);
    for (int i = 0; i < MPE_KC_COUNT; ++i) p->kms[i] = 0, p->kcount[i] = 0;
    for (int r = 0; r < reps && s == MPE_OK; ++r) s = enqueue_step(p, psi, p->phi);
    if (s != MPE_OK) break;
    collect_times(p);
    const double t[2] = {p->kms[MPE_KC_PLANE_FWD], p->kms[MPE_KC_PLANE_LINK]};
    for (int k = 0; k < (loop ? 1 : 2); ++k)
      if (t[k] < best_ms[k]) best_ms[k] = t[k], best_c[k] = c;
  }
  for (int i = 0; i < MPE_KC_COUNT; ++i) p->kms[i] = saved_ms[i], p->kcount[i] = saved_n[i];
  p->prof = prof0;
  if (s != MPE_OK) {
    p->pmode[0] = p->pmode[1] = p->pbpc[0] = p->pbpc[1] = 0;
    p->shape_ver++;
    return s;
  }
  p->pmode[0] = cand[best_c[0]][0];
  p->pbpc[0] = cand[best_c[0]][1];
  p->pmode[1] = cand[best_c[1]][0];
  p->pbpc[1] = cand[best_c[1]][1];
  // pencil work-group shapes, timed with the chosen plane shapes
  {
    double best_pm = 1e300;
    int best_t = 0;
    p->prof = true;
    for (int tile = 0; tile < 3 && s == MPE_OK; ++tile) {
      p->ptile = tile;
      s = enqueue_step(p, psi, p->phi);   // warm-up
      if (s != MPE_OK) break;
      collect_times(p);
      for (int i = 0; i < MPE_KC_COUNT; ++i) p->kms[i] = 0, p->kcount[i] = 0;
      for (int r = 0; r < reps && s == MPE_OK; ++r) s = enqueue_step(p, psi, p->phi);
      collect_times(p);
      if (p->kms[MPE_KC_PENCIL] < best_pm) best_pm = p->kms[MPE_KC_PENCIL], best_t = tile;
    }
    for (int i = 0; i < MPE_KC_COUNT; ++i) p->kms[i] = saved_ms[i], p->kcount[i] = saved_n[i];
    p->prof = prof0;
    p->ptile = best_t;
    if (s != MPE_OK) {
      p->ptile = 0;
      p->shape_ver++;
      return s;
    }
  }
  p->shape_ver++;
  if (ms_out) {
    ms_out[0] = best_ms[0] / reps;
    ms_out[1] = best_ms[1] / reps;
  }
  if (cache_path && *cache_path) {
    std::FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s|%d %d %d %d %d\n", key.c_str(), p->pmode[0], p->pbpc[0], p->pmode[1], p->pbpc[1],
                   p->ptile);
      std::fclose(f);
    }
  }
  return MPE_OK;
}

mpe_status mpe_profile_enable(mpe_plan p, int32_t on) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  collect_times(p);
  p->prof = on != 0;
  return MPE_OK;
}

mpe_status mpe_get_kernel_times(mpe_plan p, double* ms, int64_t* launches) {
  if (!p) return MPE_ERR_INVALID_ARGUMENT;
  collect_times(p);
  for (int i = 0; i < MPE_KC_COUNT; ++i) {
    if (ms) ms[i] = p->kms[i];
    if (launches) launches[i] = p->kcount[i];
    p->kms[i] = 0;
    p->kcount[i] = 0;
  }
  return MPE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched uneven systems
// Systems are grouped by grid.  Every propagation and H pass of a group is one
// launch over all states of all its systems: the kernels read each state's
// addresses (its system's spectra, tables and potential) from a descriptor
// table.  Overlaps, the small dense solve and the rotation run per system.
// The whole iteration for every system is captured as one hipGraph.
namespace {

struct BatchGroup {
  int nx = 0, ny = 0, nz = 0;
  std::vector<int> sys;            // plan indices
  int nstates = 0;
  StateDesc* d_step = nullptr;     // device descriptors: propagation (psi -> phi)
  StateDesc* d_h = nullptr;        // device descriptors: H (phi -> hphi)
  std::vector<StateDesc> h_step, h_h;
};

}  // namespace

struct mpe_batch_s {
  int count = 0, K = 0, dbl = 0;
  hipStream_t st = nullptr;
  std::string err;
  std::vector<mpe_plan> plans;
  std::vector<BatchGroup> groups;
  hipStream_t gst = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<void*> g_psi;
  hipEvent_t ev_in = nullptr;
  int launches = 0;
  // branches of the captured iteration: the per-system overlaps, small dense
  // solves and rotations of different systems run on these streams side by side
  // (used when per-system launches are selected)
  std::vector<hipStream_t> br;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  // batched linear algebra: one launch per kernel (and tile class) for all systems
  bool batched_la = true;
  struct JobSet {
    char* dev = nullptr;   // device job table
    size_t bytes = 0;
    int njobs = 0, nblocks = 0, nt = 0, mode = 0;
  };
  std::vector<JobSet> gram_sets, rot_sets;
  JobSet red_gram, red_rh, var, sd, rep;
  int max_mp = 16;
  void* job_mem = nullptr;
  size_t job_cap = 0;
};

namespace {

mpe_status bfail(mpe_batch b, mpe_status s, const std::string& msg) {
  if (b) b->err = msg;
  return s;
}

#define BHIPCHK(b, expr)                                                                          \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return bfail(b, MPE_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

void batch_drop_graph(mpe_batch b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->g_psi.clear();
}

// Descriptors of one group for the given state blocks.
void fill_descs(mpe_batch b, BatchGroup& g, void* const* psi, bool step_inplace) {
  g.h_step.clear();
  g.h_h.clear();
  for (int si : g.sys) {
    mpe_plan p = b->plans[si];
    const size_t rs = (size_t)p->N * p->fsz, ss = (size_t)p->spec * p->cx_size();
    for (int j = 0; j < p->m; ++j) {
      StateDesc d;
      d.real_in = (const char*)psi[si] + j * rs;
      d.real_out = step_inplace ? (char*)psi[si] + j * rs : (char*)p->phi + j * rs;
      d.spec = (char*)p->W + j * ss;
      d.fac = p->fac;
      d.V = p->Vf;
      d.kin = p->kin;
      d.hk = p->hk;
      d.chain_stride = (long)p->m * p->spec;
      g.h_step.push_back(d);
      StateDesc e = d;
      e.real_in = (const char*)p->phi + j * rs;
      e.real_out = (char*)p->hphi + j * rs;
      g.h_h.push_back(e);
    }
  }
}

// Job tables of the batched linear algebra for the state blocks psi (one per
// system), laid out in one device allocation (kept between calls, grown as needed).
mpe_status build_jobs(mpe_batch b, void* const* psi) {
  std::vector<std::vector<GramJob>> gj(3 * 9);     // [mode][nt]
  std::vector<std::vector<RotateJob>> rj(9);
  std::vector<ReduceJob> rg, rr;
  std::vector<VarianceJob> vj;
  std::vector<SmallDenseArgs> dj;
  std::vector<ReplayJob> pj;
  int brg = 0, brr = 0, bpj = 0;
  std::vector<int> bg(3 * 9, 0), br(9, 0);
  b->max_mp = 16;
  for (int i = 0; i < b->count; ++i) {
    mpe_plan p = b->plans[i];
    const int nt = p->mp / 16;
    b->max_mp = std::max(b->max_mp, p->mp);
    long chunk;
    const int nch = gram_chunks(p, &chunk);
    const void* X[3] = {p->phi, p->phi, psi[i]};
    const void* Y[3] = {p->phi, p->hphi, p->phi};
    const int modes[3] = {GRAM_SELF, GRAM_UPPER, GRAM_FULL};
    for (int k = 0; k < 3; ++k) {
      GramJob g;
      g.X = X[k];
      g.Y = Y[k];
      g.partials = p->partials + (size_t)k * nch * p->mp * p->mp;
      g.N = p->N;
      g.chunk = chunk;
      g.m = p->m;
      const int slot = modes[k] * 9 + nt;
      g.block0 = bg[slot];
      bg[slot] += nch;
      gj[slot].push_back(g);
    }
    ReduceJob r1;
    r1.in = p->partials;
    r1.out = p->S();                        // S, Hs, M contiguous
    r1.count = (long)p->mp * p->mp;
    r1.nparts = nch;
    r1.ncomp = 3;
    r1.block0 = brg;
    brg += (int)((r1.count + 63) / 64) * 3;
    rg.push_back(r1);
    VarianceJob v;
    v.S = p->S();
    v.M = p->Mm();
    v.re = p->re();
    v.re_perp = p->reperp();
    v.m = p->m;
    v.mp = p->mp;
    vj.push_back(v);
    SmallDenseArgs d;
    std::memset(&d, 0, sizeof(d));
    d.S = p->S();
    d.Hs = p->Hs();
    d.L = p->L();
    d.rot = p->rot;
    d.scratch = p->scratch();
    d.C = p->C();
    d.theta = p->theta();
    d.status = p->status;
    d.m = p->m;
    d.mp = p->mp;
    d.mode = SD_RR;
    d.max_sweeps = p->max_sweeps;
    d.tol = p->jacobi_tol;
    d.pivot_tol = p->pivot_tol;
    dj.push_back(d);
    ReplayJob q;
    q.d = d;
    q.block0 = bpj;
    bpj += (p->m + REPLAY_ROWS - 1) / REPLAY_ROWS;
    pj.push_back(q);
    long rchunk;
    const int nrch = rot_chunks(p, &rchunk);
    RotateJob t;
    std::memset(&t, 0, sizeof(t));
    t.r.Phi = p->phi;
    t.r.HPhi = p->hphi;
    t.r.C = p->C();
    t.r.theta = p->theta();
    t.r.Psi = psi[i];
    t.r.HPsi = p->hphi;
    t.r.res_partials = p->partials;
    t.r.status = p->status;
    t.r.N = p->N;
    t.r.chunk = rchunk;
    t.r.m = p->m;
    t.r.mp = p->mp;
    t.block0 = br[nt];
    br[nt] += nrch;
    rj[nt].push_back(t);
    ReduceJob r2;
    r2.in = p->partials;
    r2.out = p->rh();
    r2.count = p->mp;
    r2.nparts = nrch;
    r2.ncomp = 1;
    r2.block0 = brr;
    brr += (int)((r2.count + 63) / 64);
    rr.push_back(r2);
  }
  // one host image of every table, then one upload
  std::vector<char> img;
  auto put = [&](mpe_batch_s::JobSet& js, const void* data, size_t bytes, int njobs, int nblocks) {
    const size_t off = (img.size() + 255) / 256 * 256;
    img.resize(off + bytes);
    std::memcpy(img.data() + off, data, bytes);
    js.dev = reinterpret_cast<char*>(off);   // offset until the allocation is known
    js.bytes = bytes;
    js.njobs = njobs;
    js.nblocks = nblocks;
  };
  b->gram_sets.clear();
  b->rot_sets.clear();
  for (int mode = 0; mode < 3; ++mode)
    for (int nt = 1; nt <= 8; ++nt) {
      auto& v = gj[mode * 9 + nt];
      if (v.empty()) continue;
      mpe_batch_s::JobSet js;
      put(js, v.data(), v.size() * sizeof(GramJob), (int)v.size(), bg[mode * 9 + nt]);
      js.nt = nt;
      js.mode = mode;
      b->gram_sets.push_back(js);
    }
  for (int nt = 1; nt <= 8; ++nt) {
    auto& v = rj[nt];
    if (v.empty()) continue;
    mpe_batch_s::JobSet js;
    put(js, v.data(), v.size() * sizeof(RotateJob), (int)v.size(), br[nt]);
    js.nt = nt;
    b->rot_sets.push_back(js);
  }
  put(b->red_gram, rg.data(), rg.size() * sizeof(ReduceJob), (int)rg.size(), brg);
  put(b->red_rh, rr.data(), rr.size() * sizeof(ReduceJob), (int)rr.size(), brr);
  put(b->var, vj.data(), vj.size() * sizeof(VarianceJob), (int)vj.size(), (int)vj.size());
  put(b->sd, dj.data(), dj.size() * sizeof(SmallDenseArgs), (int)dj.size(), (int)dj.size());
  put(b->rep, pj.data(), pj.size() * sizeof(ReplayJob), (int)pj.size(), bpj);
  if (img.size() > b->job_cap) {
    if (b->job_mem) (void)hipFree(b->job_mem);
    b->job_mem = nullptr;
    b->job_cap = 0;
    BHIPCHK(b, hipMalloc(&b->job_mem, img.size()));
    b->job_cap = img.size();
  }
  auto fix = [&](mpe_batch_s::JobSet& js) { js.dev = static_cast<char*>(b->job_mem) + reinterpret_cast<size_t>(js.dev); };
  for (auto& js : b->gram_sets) fix(js);
  for (auto& js : b->rot_sets) fix(js);
  for (auto* js : {&b->red_gram, &b->red_rh, &b->var, &b->sd, &b->rep}) fix(*js);
  BHIPCHK(b, hipMemcpyAsync(b->job_mem, img.data(), img.size(), hipMemcpyHostToDevice, b->st));
  BHIPCHK(b, hipStreamSynchronize(b->st));   // the host image goes out of scope
  return MPE_OK;
}

// Overlaps, variances, small dense solves, replays and rotations of every
// system, batched: one launch per kernel and tile class.
mpe_status enqueue_batch_la(mpe_batch b, hipStream_t st) {
  for (auto& js : b->gram_sets) {
    BHIPCHK(b, launch_gram_jobs(b->dbl, js.nt, js.mode, reinterpret_cast<const GramJob*>(js.dev), js.njobs,
                                js.nblocks, st));
    ++b->launches;
  }
  BHIPCHK(b, launch_reduce_jobs(reinterpret_cast<const ReduceJob*>(b->red_gram.dev), b->red_gram.njobs,
                                b->red_gram.nblocks, st));
  BHIPCHK(b, launch_variance_jobs(reinterpret_cast<const VarianceJob*>(b->var.dev), b->var.njobs, st));
  BHIPCHK(b, launch_small_dense_jobs(reinterpret_cast<const SmallDenseArgs*>(b->sd.dev), b->sd.njobs, b->max_mp, st));
  BHIPCHK(b, launch_replay_jobs(reinterpret_cast<const ReplayJob*>(b->rep.dev), b->rep.njobs, b->rep.nblocks, st));
  b->launches += 4;
  for (auto& js : b->rot_sets) {
    BHIPCHK(b, launch_rotate_jobs(b->dbl, true, js.nt, reinterpret_cast<const RotateJob*>(js.dev), js.njobs,
                                  js.nblocks, st));
    ++b->launches;
  }
  BHIPCHK(b, launch_reduce_jobs(reinterpret_cast<const ReduceJob*>(b->red_rh.dev), b->red_rh.njobs,
                                b->red_rh.nblocks, st));
  ++b->launches;
  for (int i = 0; i < b->count; ++i) {
    mpe_plan p = b->plans[i];
    BHIPCHK(b, hipMemcpyAsync(p->host_res, p->res, p->res_bytes, hipMemcpyDeviceToHost, st));
  }
  return MPE_OK;
}

mpe_status upload_descs(mpe_batch b) {
  for (auto& g : b->groups) {
    BHIPCHK(b, hipMemcpyAsync(g.d_step, g.h_step.data(), g.h_step.size() * sizeof(StateDesc), hipMemcpyHostToDevice,
                              b->st));
    BHIPCHK(b, hipMemcpyAsync(g.d_h, g.h_h.data(), g.h_h.size() * sizeof(StateDesc), hipMemcpyHostToDevice, b->st));
  }
  BHIPCHK(b, hipStreamSynchronize(b->st));   // host vectors may change after this call
  return MPE_OK;
}

// Propagation of every state of the group: phi (or psi in place) <- T_2K psi.
mpe_status enqueue_group_step(mpe_batch b, BatchGroup& g, hipStream_t st) {
  mpe_plan p0 = b->plans[g.sys[0]];
  double c[MAX_K];
  mpe_coeffs(b->K, c);
  {
    // every chain's first half-step and forward transform from one read of psi
    PlaneArgs a = plane_base(p0);
    a.desc = g.d_step;
    a.chain = 0;
    a.fac_index = 1;
    a.fwd_chains = b->K;
    BHIPCHK(b, launch_plane(b->dbl, PM_FWD, g.nx, a, g.nz, g.nstates, st));
    ++b->launches;
  }
  for (int k = 1; k <= b->K; ++k) {
    for (int l = 1; l <= k; ++l) {
      PencilArgs pa = pencil_base(p0, nullptr, nullptr);
      pa.desc = g.d_step;
      pa.chain = k - 1;
      pa.desc_tables = 0;
      BHIPCHK(b, launch_pencil(b->dbl, PK_EXP, g.nz, pa, g.nstates, st));
      ++b->launches;
      if (l < k) {
        PlaneArgs la = plane_base(p0);
        la.desc = g.d_step;
        la.chain = k - 1;
        la.fac_index = k - 1;
        BHIPCHK(b, launch_plane(b->dbl, PM_LINK, g.nx, la, g.nz, g.nstates, st));
        ++b->launches;
      }
    }
  }
  PlaneArgs t = plane_base(p0);
  t.desc = g.d_step;
  t.chain = 0;
  t.K = b->K;
  for (int k = 0; k < b->K; ++k) t.coef[k] = c[k];
  BHIPCHK(b, launch_plane(b->dbl, PM_TAIL, g.nx, t, g.nz, g.nstates, st));
  ++b->launches;
  return MPE_OK;
}

mpe_status enqueue_group_h(mpe_batch b, BatchGroup& g, hipStream_t st) {
  mpe_plan p0 = b->plans[g.sys[0]];
  PlaneArgs a = plane_base(p0);
  a.desc = g.d_h;
  a.chain = 0;
  a.fac_index = -1;
  BHIPCHK(b, launch_plane(b->dbl, PM_FWD, g.nx, a, g.nz, g.nstates, st));
  PencilArgs pa = pencil_base(p0, nullptr, nullptr);
  pa.desc = g.d_h;
  pa.chain = 0;
  pa.desc_tables = 1;
  BHIPCHK(b, launch_pencil(b->dbl, PK_ADD, g.nz, pa, g.nstates, st));
  PlaneArgs c = plane_base(p0);
  c.desc = g.d_h;
  c.chain = 0;
  BHIPCHK(b, launch_plane(b->dbl, PM_HTAIL, g.nx, c, g.nz, g.nstates, st));
  b->launches += 3;
  return MPE_OK;
}

// All device work of one batched iteration on stream st (plans temporarily enqueue on st).
// Propagation (and with_h: H) passes of every grid group, ordered after the
// work on st and before what st receives next.  The groups touch disjoint
// systems: each runs on a branch stream of its own, so the launches of small
// grids (few work-groups, latency-bound) overlap those of large ones.
mpe_status enqueue_groups(mpe_batch b, hipStream_t st, bool with_h) {
  const int nbr = (int)b->br.size(), ngr = (int)b->groups.size();
  const int gbr = (nbr > 1 && ngr > 1) ? std::min(nbr, ngr) : 0;
  if (gbr > 0) {
    BHIPCHK(b, hipEventRecord(b->ev_fork, st));
    for (int j = 0; j < gbr; ++j) BHIPCHK(b, hipStreamWaitEvent(b->br[j], b->ev_fork, 0));
  }
  for (int gi = 0; gi < ngr; ++gi) {
    const hipStream_t sg = gbr > 0 ? b->br[gi % gbr] : st;
    mpe_status s = enqueue_group_step(b, b->groups[gi], sg);
    if (s == MPE_OK && with_h) s = enqueue_group_h(b, b->groups[gi], sg);
    if (s != MPE_OK) return s;
  }
  for (int j = 0; j < gbr; ++j) {
    BHIPCHK(b, hipEventRecord(b->ev_join[j], b->br[j]));
    BHIPCHK(b, hipStreamWaitEvent(st, b->ev_join[j], 0));
  }
  return MPE_OK;
}

mpe_status enqueue_batch_iterate(mpe_batch b, void* const* psi, hipStream_t st) {
  b->launches = 0;
  mpe_status gs = enqueue_groups(b, st, true);
  if (gs != MPE_OK) return gs;
  if (b->batched_la) return enqueue_batch_la(b, st);
  // fork: system i's chain goes to branch i % nbr
  const int nbr = (int)b->br.size();
  if (nbr > 0) {
    BHIPCHK(b, hipEventRecord(b->ev_fork, st));
    for (auto s2 : b->br) BHIPCHK(b, hipStreamWaitEvent(s2, b->ev_fork, 0));
  }
  for (int i = 0; i < b->count; ++i) {
    mpe_plan p = b->plans[i];
    hipStream_t keep = p->st;
    const hipStream_t si = nbr > 0 ? b->br[i % nbr] : st;
    p->st = si;
    const void* X[3] = {p->phi, p->phi, psi[i]};
    const void* Y[3] = {p->phi, p->hphi, p->phi};
    mpe_status s = run_gram(p, X, Y, 3, p->S(), 2);
    if (s == MPE_OK) {
      hipError_t e = launch_variance(p->S(), p->Mm(), p->m, p->mp, nullptr, p->re(), p->reperp(), si);
      if (e != hipSuccess) s = fail(p, MPE_ERR_DEVICE, hipGetErrorString(e));
    }
    if (s == MPE_OK) s = run_small_dense(p, SD_RR);
    if (s == MPE_OK) s = run_rotate(p, p->phi, p->hphi, psi[i], p->hphi);
    if (s == MPE_OK) {
      hipError_t e = hipMemcpyAsync(p->host_res, p->res, p->res_bytes, hipMemcpyDeviceToHost, si);
      if (e != hipSuccess) s = fail(p, MPE_ERR_DEVICE, hipGetErrorString(e));
    }
    p->st = keep;
    if (s != MPE_OK) return bfail(b, s, "system " + std::to_string(i) + ": " + p->err);
    b->launches += 7;
  }
  // join
  for (int j = 0; j < nbr; ++j) {
    BHIPCHK(b, hipEventRecord(b->ev_join[j], b->br[j]));
    BHIPCHK(b, hipStreamWaitEvent(st, b->ev_join[j], 0));
  }
  return MPE_OK;
}

}  // namespace

extern "C" {

mpe_status mpe_batch_destroy(mpe_batch b) {
  if (!b) return MPE_ERR_INVALID_ARGUMENT;
  (void)hipStreamSynchronize(b->st);
  batch_drop_graph(b);
  for (auto& g : b->groups) {
    if (g.d_step) (void)hipFree(g.d_step);
    if (g.d_h) (void)hipFree(g.d_h);
  }
  for (auto p : b->plans)
    if (p) mpe_plan_destroy(p);
  if (b->job_mem) (void)hipFree(b->job_mem);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->gst) (void)hipStreamDestroy(b->gst);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  for (auto e : b->ev_join) (void)hipEventDestroy(e);
  for (auto s2 : b->br) (void)hipStreamDestroy(s2);
  delete b;
  return MPE_OK;
}

mpe_status mpe_batch_create(mpe_batch* out, int32_t count, const mpe_system_desc* systems, int32_t order,
                            mpe_precision prec, double hbar2_over_m, void* hip_stream) {
  if (!out) return MPE_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (count < 1 || !systems) return MPE_ERR_INVALID_ARGUMENT;
  mpe_batch b = new mpe_batch_s();
  b->count = count;
  b->K = order / 2;
  b->dbl = prec == MPE_FP64;
  b->st = reinterpret_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < count; ++i) {
    const mpe_system_desc& sd = systems[i];
    mpe_plan p = nullptr;
    mpe_status s = mpe_plan_create(&p, sd.grid, sd.box, sd.n_states, order, prec, sd.n_guard, hip_stream);
    if (s != MPE_OK) {
      mpe_batch_destroy(b);
      return s;
    }
    b->plans.push_back(p);
    if (p->three_pass) {   // batched launches are plane passes
      mpe_batch_destroy(b);
      return MPE_ERR_UNSUPPORTED;
    }
    s = mpe_set_potential(p, sd.V, hbar2_over_m);
    if (s != MPE_OK) {
      mpe_batch_destroy(b);
      return s;
    }
    int gi = -1;
    for (size_t k = 0; k < b->groups.size(); ++k)
      if (b->groups[k].nx == p->nx && b->groups[k].ny == p->ny && b->groups[k].nz == p->nz) gi = (int)k;
    if (gi < 0) {
      BatchGroup g;
      g.nx = p->nx;
      g.ny = p->ny;
      g.nz = p->nz;
      b->groups.push_back(g);
      gi = (int)b->groups.size() - 1;
    }
    b->groups[gi].sys.push_back(i);
    b->groups[gi].nstates += p->m;
  }
  for (auto& g : b->groups) {
    if (hipMalloc((void**)&g.d_step, g.nstates * sizeof(StateDesc)) != hipSuccess ||
        hipMalloc((void**)&g.d_h, g.nstates * sizeof(StateDesc)) != hipSuccess) {
      mpe_batch_destroy(b);
      return MPE_ERR_OUT_OF_MEMORY;
    }
  }
  if (hipStreamCreateWithFlags(&b->gst, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) {
    mpe_batch_destroy(b);
    return MPE_ERR_DEVICE;
  }
  const int nbr = std::min(b->count, 8);
  for (int j = 0; nbr > 1 && j < nbr; ++j) {   // default-priority streams
    hipStream_t s2 = nullptr;
    hipEvent_t e2 = nullptr;
    if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) {
      mpe_batch_destroy(b);
      return MPE_ERR_DEVICE;
    }
    b->br.push_back(s2);
    if (hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess) {
      mpe_batch_destroy(b);
      return MPE_ERR_DEVICE;
    }
    b->ev_join.push_back(e2);
  }
  *out = b;
  return MPE_OK;
}

const char* mpe_batch_last_error(mpe_batch b) { return b ? b->err.c_str() : "null batch"; }

int32_t mpe_batch_launches_per_step(mpe_batch b) { return b ? b->launches : -1; }

mpe_status mpe_batch_set_batched_la(mpe_batch b, int32_t on) {
  if (!b) return MPE_ERR_INVALID_ARGUMENT;
  b->batched_la = on != 0;
  batch_drop_graph(b);
  return MPE_OK;
}

mpe_status mpe_batch_step(mpe_batch b, void* const* psi, double dt) {
  if (!b || !psi) return MPE_ERR_INVALID_ARGUMENT;
  if (!(dt > 0.0) || !std::isfinite(dt)) return bfail(b, MPE_ERR_INVALID_ARGUMENT, "dt must be positive");
  for (int i = 0; i < b->count; ++i) {
    if (!psi[i]) return bfail(b, MPE_ERR_INVALID_ARGUMENT, "null state block");
    mpe_plan p = b->plans[i];
    p->rr_cache_psi = nullptr;
    mpe_status s = ensure_tables(p, dt);
    if (s != MPE_OK) return bfail(b, s, p->err);
    p->last_dt = dt;
  }
  batch_drop_graph(b);   // descriptors are rewritten for the in-place step
  for (auto& g : b->groups) fill_descs(b, g, psi, true);
  mpe_status s = upload_descs(b);
  if (s != MPE_OK) return s;
  const int keep = b->launches;   // the count reported is the iteration graph's
  s = enqueue_groups(b, b->st, false);
  b->launches = keep;
  if (s != MPE_OK) return s;
  BHIPCHK(b, hipStreamSynchronize(b->st));
  return MPE_OK;
}

mpe_status mpe_batch_iterate(mpe_batch b, void* const* psi, double dt, double* eig, double* rh, double* re,
                             double* re_perp) {
  if (!b || !psi) return MPE_ERR_INVALID_ARGUMENT;
  if (!(dt > 0.0) || !std::isfinite(dt)) return bfail(b, MPE_ERR_INVALID_ARGUMENT, "dt must be positive");
  bool same = b->gexec != nullptr && (int)b->g_psi.size() == b->count;
  for (int i = 0; i < b->count; ++i) {
    if (!psi[i]) return bfail(b, MPE_ERR_INVALID_ARGUMENT, "null state block");
    if (same && b->g_psi[i] != psi[i]) same = false;
    mpe_plan p = b->plans[i];
    p->rr_cache_psi = nullptr;
    mpe_status s = ensure_tables(p, dt);
    if (s != MPE_OK) return bfail(b, s, p->err);
    p->last_dt = dt;
  }
  if (!same) {
    batch_drop_graph(b);
    for (auto& g : b->groups) fill_descs(b, g, psi, false);
    mpe_status s = upload_descs(b);
    if (s == MPE_OK && b->batched_la) s = build_jobs(b, psi);
    if (s != MPE_OK) return s;
    BHIPCHK(b, hipStreamBeginCapture(b->gst, hipStreamCaptureModeRelaxed));
    s = enqueue_batch_iterate(b, psi, b->gst);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->gst, &g);
    if (s != MPE_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return bfail(b, MPE_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    b->graph = g;
    BHIPCHK(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->g_psi.assign(psi, psi + b->count);
  }
  BHIPCHK(b, hipEventRecord(b->ev_in, b->st));
  BHIPCHK(b, hipStreamWaitEvent(b->gst, b->ev_in, 0));
  BHIPCHK(b, hipGraphLaunch(b->gexec, b->gst));
  BHIPCHK(b, hipStreamSynchronize(b->gst));
  long off = 0;
  mpe_status first = MPE_OK;
  for (int i = 0; i < b->count; ++i) {
    mpe_plan p = b->plans[i];
    mpe_status s = finish_iterate(p, psi[i], eig ? eig + off : nullptr, rh ? rh + off : nullptr,
                                  re ? re + off : nullptr, re_perp ? re_perp + off : nullptr);
    if (s != MPE_OK && first == MPE_OK) {
      first = s;
      b->err = "system " + std::to_string(i) + ": " + p->err;
    }
    off += p->m;
  }
  return first;
}

}  // extern "C"
