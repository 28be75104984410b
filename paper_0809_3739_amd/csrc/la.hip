// Subspace linear algebra on the GPU: overlap matrices, Cholesky
// orthonormalisation and the Rayleigh-Ritz rotation (Section I, Eq. ortho;
// Section III, subspace orthogonalisation; variances R^H and R^E).
//
// States are rows of an [m][N] array (m = states incl. guards, N grid points).
//  * gram_partial_kernel : X Y^T over a chunk of points on float64 MFMA
//    (v_mfma_f64_16x16x4f64); inputs of either precision are widened exactly.
//  * gram32_partial_kernel / gramb_partial_kernel : the same for float32 states
//    on float32 MFMA, or on bf16 MFMA with the values split into bf16 parts.
//  * reduce_kernel       : fixed-order float64 sum of chunk partials.
//  * small_dense_kernel  : one work-group; S = L L^T, A = L^-1 Hs L^-T,
//    cyclic parallel Jacobi on A (rotations logged), eigenvalues sorted, L^-T.
//  * sd_replay_kernel    : C = L^-T U, the logged rotations applied to the rows
//    of L^-T (one wavefront per row), columns sorted by eigenvalue.
//  * rotate_kernel       : Psi = Phi C and (H Phi) C on float64 MFMA with the
//    residual sum_p ((H Psi)_j - theta_j Psi_j)^2 accumulated in the epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "la.hpp"

namespace mpe {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f64_16x16x4f64 (one block, 64 lanes), measured on gfx950:
//   A (16x4) : lane l holds A[l % 16][l / 16]
//   B (4x16) : lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, register r holds D[4 * r + l / 16][l % 16]
// (the float32 16x16x4 variant instead holds D[4 * (l / 16) + r][l % 16]).
__device__ __forceinline__ int drow(int lane, int r) { return 4 * r + (lane >> 4); }
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ Gram partials
// Work-group: 256 threads (4 waves).  The 16x16 output tiles of an mp x mp
// product (NT = mp/16 per side, compile time) are dealt round-robin to the
// waves.  Modes: GRAM_FULL forms all tiles; GRAM_SELF (X == Y) and GRAM_UPPER
// (X != Y, a product symmetric in exact arithmetic, such as Psi (H Psi)^T) form
// only tiles ti <= tj and mirror them on store, GRAM_SELF staging one array.
// Points are staged through LDS in slabs of GSLAB, transposed to
// [point][state]; the next slab is loaded into registers while the MFMAs of
// the current one run.
constexpr int GSLAB = 32;
constexpr int GLD = MAXM + 1;   // LDS row: consecutive points of a state land in distinct banks

template <int NT, bool SYM>
struct GramTiles {
  static constexpr int count = SYM ? NT * (NT + 1) / 2 : NT * NT;
  static constexpr int per_wave = (count + 3) / 4;
};

static int gram_mode(const GramArgs& g, int i) {
  if (g.X[i] == g.Y[i]) return GRAM_SELF;
  return (g.upper_mask >> i) & 1 ? GRAM_UPPER : GRAM_FULL;
}

__device__ __forceinline__ void tile_coords(int u, int nt, bool sym, int& ti, int& tj) {
  if (!sym) {
    ti = u / nt;
    tj = u - ti * nt;
    return;
  }
  ti = 0;
  while (u >= nt - ti) {
    u -= nt - ti;
    ++ti;
  }
  tj = ti + u;
}

// One chunk of points [p_begin, p_end) of X Y^T into out (mp x mp float64).
template <typename F, int NT, int MODE>
__device__ __forceinline__ void gram_chunk(const F* __restrict__ X, const F* __restrict__ Y, int m, long N,
                                           long p_begin, long p_end, double* __restrict__ out) {
  constexpr bool ONE = MODE == GRAM_SELF, TRI = MODE != GRAM_FULL;
  constexpr int mp = NT * 16;
  constexpr int TPW = GramTiles<NT, TRI>::per_wave;
  constexpr int NTILE = GramTiles<NT, TRI>::count;
  constexpr int PER = (mp * GSLAB + 255) / 256;   // staged elements per thread and array
  __shared__ double xs[GSLAB][GLD];
  __shared__ double ys[ONE ? 1 : GSLAB][ONE ? 1 : GLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  int tiv[TPW], tjv[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int u = wave + 4 * t;
    tile_coords(u < NTILE ? u : 0, NT, TRI, tiv[t], tjv[t]);
  }
  d4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  F px[PER], py[PER];
  auto load = [&](long p0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      const int st = e / GSLAB, q = e - st * GSLAB;
      const long p = p0 + q;
      const bool ok = e < mp * GSLAB && st < m && p < p_end;
      px[r] = ok ? X[(long)st * N + p] : F(0);
      if (!ONE) py[r] = ok ? Y[(long)st * N + p] : F(0);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      if (e < mp * GSLAB) {
        const int st = e / GSLAB, q = e - st * GSLAB;
        xs[q][st] = (double)px[r];
        if (!ONE) ys[q][st] = (double)py[r];
      }
    }
  };
  load(p_begin);
  for (long p0 = p_begin; p0 < p_end; p0 += GSLAB) {
    stage();
    __syncthreads();
    if (p0 + GSLAB < p_end) load(p0 + GSLAB);   // in flight during the MFMAs below
#pragma unroll
    for (int k0 = 0; k0 < GSLAB; k0 += 4) {
      const int kq = k0 + (lane >> 4);
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (TPW * 4 == NTILE || wave + 4 * t < NTILE) {
          const double a = xs[kq][tiv[t] * 16 + (lane & 15)];
          const double b = ONE ? xs[kq][tjv[t] * 16 + (lane & 15)] : ys[kq][tjv[t] * 16 + (lane & 15)];
          acc[t] = mfma16(a, b, acc[t]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (wave + 4 * t < NTILE) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = tiv[t] * 16 + drow(lane, r), j = tjv[t] * 16 + (lane & 15);
        out[(long)i * mp + j] = acc[t][r];
        if (TRI && tiv[t] != tjv[t]) out[(long)j * mp + i] = acc[t][r];
      }
    }
  }
}

template <typename F, int NT, int MODE>
__global__ __launch_bounds__(256) void gram_partial_kernel(GramArgs g) {
  const int prod = blockIdx.y;
  const long p_begin = (long)blockIdx.x * g.chunk;
  gram_chunk<F, NT, MODE>(reinterpret_cast<const F*>(g.X[prod]), reinterpret_cast<const F*>(g.Y[prod]), g.m, g.N,
                          p_begin, min(g.N, p_begin + g.chunk),
                          g.partials + ((long)prod * gridDim.x + blockIdx.x) * (long)(NT * 16) * (NT * 16));
}

// Job-table lookup for batched launches: the job whose first work-group is the
// largest one not above this work-group (jobs sorted by block0).
template <typename J>
__device__ __forceinline__ const J& find_job(const J* __restrict__ jobs, int njobs) {
  int lo = 0, hi = njobs - 1;
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return jobs[lo];
}

// Many systems' overlap products of one tile class in one launch: each job is
// one product of one system, its chunks consecutive work-groups.
template <typename F, int NT, int MODE>
__global__ __launch_bounds__(256) void gram_jobs_kernel(const GramJob* __restrict__ jobs, int njobs) {
  const GramJob& J = find_job(jobs, njobs);
  const int c = (int)blockIdx.x - J.block0;
  const long p_begin = (long)c * J.chunk;
  gram_chunk<F, NT, MODE>(reinterpret_cast<const F*>(J.X), reinterpret_cast<const F*>(J.Y), J.m, J.N, p_begin,
                          min(J.N, p_begin + J.chunk), J.partials + (long)c * (NT * 16) * (NT * 16));
}

// Float32-MFMA variant for float32 states (the precision split of the overlap
// GEMMs): 512 threads (8 waves), points staged as float, v_mfma_f32_16x16x4f32
// with float32 accumulation over one slab of GSLAB points, then added into
// float64 per-tile sums (one rounding per 32 products), float64 partials out.
template <int NT, int MODE>
__global__ __launch_bounds__(512) void gram32_partial_kernel(GramArgs g) {
  constexpr bool ONE = MODE == GRAM_SELF, TRI = MODE != GRAM_FULL;
  constexpr int W = 8;
  constexpr int mp = NT * 16;
  constexpr int NTILE = GramTiles<NT, TRI>::count;
  constexpr int TPW = (NTILE + W - 1) / W;
  constexpr int PER = (mp * GSLAB + 511) / 512;
  __shared__ float xs[GSLAB][GLD];
  __shared__ float ys[ONE ? 1 : GSLAB][ONE ? 1 : GLD];
  const int prod = blockIdx.y;
  const float* __restrict__ X = reinterpret_cast<const float*>(g.X[prod]);
  const float* __restrict__ Y = reinterpret_cast<const float*>(g.Y[prod]);
  const int m = g.m;
  const long N = g.N;
  const long p_begin = (long)blockIdx.x * g.chunk;
  const long p_end = min(N, p_begin + g.chunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int tiv[TPW], tjv[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int u = wave + W * t;
    tile_coords(u < NTILE ? u : 0, NT, TRI, tiv[t], tjv[t]);
  }
  d4 sum[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) sum[t] = d4{0.0, 0.0, 0.0, 0.0};
  float px[PER], py[PER];
  auto load = [&](long p0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 512 * r;
      const int st = e / GSLAB, q = e - st * GSLAB;
      const long p = p0 + q;
      const bool ok = e < mp * GSLAB && st < m && p < p_end;
      px[r] = ok ? X[(long)st * N + p] : 0.f;
      if (!ONE) py[r] = ok ? Y[(long)st * N + p] : 0.f;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 512 * r;
      if (e < mp * GSLAB) {
        const int st = e / GSLAB, q = e - st * GSLAB;
        xs[q][st] = px[r];
        if (!ONE) ys[q][st] = py[r];
      }
    }
  };
  load(p_begin);
  for (long p0 = p_begin; p0 < p_end; p0 += GSLAB) {
    stage();
    __syncthreads();
    if (p0 + GSLAB < p_end) load(p0 + GSLAB);
    f4 acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < GSLAB; k0 += 4) {
      const int kq = k0 + (lane >> 4);
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (TPW * W == NTILE || wave + W * t < NTILE) {
          const float a = xs[kq][tiv[t] * 16 + (lane & 15)];
          const float b = ONE ? xs[kq][tjv[t] * 16 + (lane & 15)] : ys[kq][tjv[t] * 16 + (lane & 15)];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) sum[t][r] += (double)acc[t][r];
    __syncthreads();
  }
  double* out = g.partials + ((long)prod * gridDim.x + blockIdx.x) * (long)mp * mp;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (wave + W * t < NTILE) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = tiv[t] * 16 + 4 * (lane >> 4) + r, j = tjv[t] * 16 + (lane & 15);   // f32 D layout
        out[(long)i * mp + j] = sum[t][r];
        if (TRI && tiv[t] != tjv[t]) out[(long)j * mp + i] = sum[t][r];
      }
    }
  }
}

// BF16-split variant for float32 states: every staged value x is split into
// SPLIT bfloat16 parts (x = h + m + l up to the last bits: h = bf16(x), then the
// exact float32 remainder is split again), and X Y^T is formed from the
// products of parts whose orders add up to at most SPLIT - 1 (SPLIT = 2: hh,
// hl, lh, ~16 significant bits; SPLIT = 3: hh, hm, mh, hl, mm, lh, ~24 bits)
// on v_mfma_f32_16x16x32_bf16, smallest terms first, float32 accumulation over
// the 32-point slab and float64 sums across slabs.  Parts are staged in LDS as
// [part][state][point] (rows padded to 40 bf16), so the 8 consecutive points a
// lane feeds to one MFMA are one 16-byte read.
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan kept
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int NT, int MODE, int SPLIT>
__global__ __launch_bounds__(512) void gramb_partial_kernel(GramArgs g) {
  constexpr bool ONE = MODE == GRAM_SELF, TRI = MODE != GRAM_FULL;
  constexpr int W = 8;
  constexpr int mp = NT * 16;
  constexpr int NTILE = GramTiles<NT, TRI>::count;
  constexpr int TPW = (NTILE + W - 1) / W;
  constexpr int PER = (mp * GSLAB + 511) / 512;
  constexpr int RS = GSLAB + 8;   // bf16 per staged row (80 bytes)
  static_assert(GSLAB == 32, "one 16x16x32 MFMA per slab and part pair");
  __shared__ __align__(16) unsigned short xs[SPLIT][mp][RS];
  __shared__ __align__(16) unsigned short ys[ONE ? 1 : SPLIT][ONE ? 1 : mp][ONE ? 8 : RS];
  const int prod = blockIdx.y;
  const float* __restrict__ X = reinterpret_cast<const float*>(g.X[prod]);
  const float* __restrict__ Y = reinterpret_cast<const float*>(g.Y[prod]);
  const int m = g.m;
  const long N = g.N;
  const long p_begin = (long)blockIdx.x * g.chunk;
  const long p_end = min(N, p_begin + g.chunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int tiv[TPW], tjv[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int u = wave + W * t;
    tile_coords(u < NTILE ? u : 0, NT, TRI, tiv[t], tjv[t]);
  }
  d4 sum[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) sum[t] = d4{0.0, 0.0, 0.0, 0.0};
  float px[PER], py[PER];
  auto load = [&](long p0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 512 * r;
      const int st = e / GSLAB, q = e - st * GSLAB;
      const long p = p0 + q;
      const bool ok = e < mp * GSLAB && st < m && p < p_end;
      const long idx = ok ? (long)st * N + p : 0;   // unconditional loads, no exec-mask branches
      const float vx = X[idx];
      px[r] = ok ? vx : 0.f;
      if (!ONE) {
        const float vy = Y[idx];
        py[r] = ok ? vy : 0.f;
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 512 * r;
      if (e < mp * GSLAB) {
        const int st = e / GSLAB, q = e - st * GSLAB;
        float x = px[r];
#pragma unroll
        for (int s = 0; s < SPLIT; ++s) {
          const unsigned short h = bf16_rne(x);
          xs[s][st][q] = h;
          x -= bf16_f(h);
        }
        if (!ONE) {
          float y = py[r];
#pragma unroll
          for (int s = 0; s < SPLIT; ++s) {
            const unsigned short h = bf16_rne(y);
            ys[s][st][q] = h;
            y -= bf16_f(h);
          }
        }
      }
    }
  };
  auto part = [&](int s, int state, bool from_y) -> bf16x8 {
    const unsigned short* row = (ONE || !from_y) ? &xs[s][state][0] : &ys[s][state][0];
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(row + 8 * (lane >> 4)));
  };
  load(p_begin);
  for (long p0 = p_begin; p0 < p_end; p0 += GSLAB) {
    stage();
    __syncthreads();
    if (p0 + GSLAB < p_end) load(p0 + GSLAB);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      if (TPW * W == NTILE || wave + W * t < NTILE) {
        const int si = tiv[t] * 16 + (lane & 15), sj = tjv[t] * 16 + (lane & 15);
        f4 acc = f4{0.f, 0.f, 0.f, 0.f};
        // part pairs by decreasing order sum (smallest products first)
#pragma unroll
        for (int o = SPLIT - 1; o >= 0; --o)
#pragma unroll
          for (int a = o; a >= 0; --a)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(part(a, si, false), part(o - a, sj, true), acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) sum[t][r] += (double)acc[r];
      }
    }
    __syncthreads();
  }
  double* out = g.partials + ((long)prod * gridDim.x + blockIdx.x) * (long)mp * mp;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (wave + W * t < NTILE) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = tiv[t] * 16 + 4 * (lane >> 4) + r, j = tjv[t] * 16 + (lane & 15);   // f32 D layout
        out[(long)i * mp + j] = sum[t][r];
        if (TRI && tiv[t] != tjv[t]) out[(long)j * mp + i] = sum[t][r];
      }
    }
  }
}

// out[c][e] = sum_{q < nparts} in[c][q][e], e < count, fixed order.
// Work-group: 64 elements x RD_SLICES wavefronts; wavefront w sums the parts
// q = w, w + RD_SLICES, ... of its lane's element, then the slices are added
// in slice order (a fixed order for every call).
constexpr int RD_SLICES = 8;
__device__ __forceinline__ void reduce_block(const double* __restrict__ in, int nparts, long count,
                                             double* __restrict__ out, long e0, int c) {
  __shared__ double part[RD_SLICES][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long e = e0 + lane;
  double s = 0.0;
  if (e < count) {
    const double* src = in + (long)c * nparts * count + e;
#pragma unroll 8
    for (int q = w; q < nparts; q += RD_SLICES) s += src[(long)q * count];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && e < count) {
    double t = part[0][lane];
#pragma unroll
    for (int k = 1; k < RD_SLICES; ++k) t += part[k][lane];
    out[(long)c * count + e] = t;
  }
}

__global__ __launch_bounds__(64 * RD_SLICES) void reduce_kernel(const double* __restrict__ in, int nparts, long count,
                                                                double* __restrict__ out) {
  reduce_block(in, nparts, count, out, (long)blockIdx.x * 64, blockIdx.y);
}

// Many reductions in one launch: job j covers ceil(count / 64) * ncomp work-groups.
__global__ __launch_bounds__(64 * RD_SLICES) void reduce_jobs_kernel(const ReduceJob* __restrict__ jobs, int njobs) {
  const ReduceJob& J = find_job(jobs, njobs);
  const int b = (int)blockIdx.x - J.block0;
  const int per = (int)((J.count + 63) / 64);
  reduce_block(J.in, J.nparts, J.count, J.out, (long)(b % per) * 64, b / per);
}

// ------------------------------------------------------------------ small dense problem
// One work-group of 1024 threads.  LDS holds one mp x (mp+1) float64 matrix
// (S, then L, then A); W = L^-T, the product Hs W, the Jacobi rotation log and
// scratch live in global memory (L2 resident).
constexpr int SD_THREADS = 1024;

__device__ __forceinline__ double block_max(double v, double* red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid < 64) {
    double w = tid < SD_THREADS / 64 ? red[tid] : 0.0;
    for (int o = 32; o > 0; o >>= 1) w = fmax(w, __shfl_xor(w, o));
    if (tid == 0) red[16] = w;
  }
  __syncthreads();
  const double r = red[16];
  __syncthreads();
  return r;
}

// phase stamps from the 100 MHz constant clock (diagnostics only)
__device__ __forceinline__ void stamp(const SmallDenseArgs& d, int i) {
  if (d.ticks && threadIdx.x == 0) d.ticks[i] = (long long)__builtin_amdgcn_s_memrealtime();
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __hiloint2double(hi, lo);
}

// out(i, j, sum_k P(i, k) Q(k, j)) for i, j, k < mp (mp a multiple of 16), float64
// MFMA, the 16x16 output tiles dealt round-robin to the work-group's wavefronts;
// P and Q are read through the accessors (entries beyond the matrices are zero).
template <typename PA, typename QA, typename OUT>
__device__ void mfma_product(int mp, PA P, QA Q, OUT out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nt = mp / 16;
  for (int t = wv; t < nt * nt; t += SD_THREADS / 64) {
    const int i0 = (t / nt) * 16, j0 = (t % nt) * 16;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int k0 = 0; k0 < mp; k0 += 4) {
      const double a = P(i0 + (lane & 15), k0 + (lane >> 4));
      const double b = Q(k0 + (lane >> 4), j0 + (lane & 15));
      acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) out(i0 + drow(lane, r), j0 + (lane & 15), acc[r]);
  }
}

__device__ __forceinline__ void small_dense_body(const SmallDenseArgs& d) {
  extern __shared__ double sh[];  // mp x LD
  __shared__ double red[20];
  __shared__ int flag;
  __shared__ double cs[MAXM / 2 + 1][2];
  __shared__ int pq[MAXM / 2 + 1][2];
  __shared__ double dg[MAXM];
  const int m = d.m, LD = d.mp + 1;
  const int tid = threadIdx.x;
  double* L = d.L;            // mp x mp global workspace (the product Hs W)
  auto A = [&](int i, int j) -> double& { return sh[i * LD + j]; };

  if (tid == 0) flag = -1;
  stamp(d, 0);
  __syncthreads();
  // ---- Cholesky of S in LDS (right-looking, one barrier per pivot): step k
  // updates the trailing lower triangle with column k unscaled,
  // a_ij -= a_ik a_jk / p_k, and every column is scaled by 1/sqrt(p_k) once at
  // the end.  Each thread owns fixed elements of the lower triangle.
  for (int e = tid; e < m * m; e += SD_THREADS) A(e / m, e % m) = d.S[(e / m) * (long)d.mp + e % m];
  for (int i = tid; i < m; i += SD_THREADS) dg[i] = d.S[i * (long)d.mp + i];
  constexpr int CH_EL = (MAXM * (MAXM + 1) / 2 + SD_THREADS - 1) / SD_THREADS;
  int el_i[CH_EL], el_j[CH_EL];
#pragma unroll
  for (int r = 0; r < CH_EL; ++r) {
    const int t = tid + r * SD_THREADS;   // row-major index into the lower triangle
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    const bool ok = t < m * (m + 1) / 2;
    el_i[r] = ok ? i : 0;
    el_j[r] = ok ? t - i * (i + 1) / 2 : m;   // j = m: never updated
  }
  __syncthreads();
  // A pivot that has lost all but ~13 digits of its original diagonal means the
  // states are linearly dependent to working precision: reported, not factored.
  for (int k = 0; k < m; ++k) {
    const double piv = A(k, k);
    const bool bad = !(piv > d.pivot_tol * dg[k]) || !isfinite(piv);
    if (bad) {
      if (tid == 0 && flag < 0) flag = isfinite(piv) ? k : -2 - k;
      break;  // uniform: every thread sees the same pivot
    }
    const double inv = 1.0 / piv;
#pragma unroll
    for (int r = 0; r < CH_EL; ++r) {
      const int i = el_i[r], j = el_j[r];
      if (j > k && j < m) A(i, j) -= A(i, k) * A(j, k) * inv;
    }
    __syncthreads();
  }
  if (flag == -1) {   // scale the columns: L_ij = a_ij / sqrt(p_j), L_jj = sqrt(p_j)
#pragma unroll
    for (int r = 0; r < CH_EL; ++r) {
      const int i = el_i[r], j = el_j[r];
      if (j < m) {
        const double pj = A(j, j);   // diagonal entries are only rewritten below, after the barrier
        if (i != j) A(i, j) /= sqrt(pj);
      }
    }
  }
  __syncthreads();
  if (flag == -1)
    for (int i = tid; i < m; i += SD_THREADS) A(i, i) = sqrt(A(i, i));
  __syncthreads();
  if (flag != -1) {
    if (tid == 0) {
      d.status[0] = flag >= 0 ? ST_NOT_SPD : ST_NONFINITE;
      d.status[1] = flag >= 0 ? flag : -2 - flag;
    }
    return;
  }
  stamp(d, 1);
  // ---- W = L^-T into C (the whole output for SD_ORTHO; for SD_RR the replay
  // kernel turns it into C = W U).  One column per wavefront at a time, from L
  // in LDS: column j solves L^T w = e_j backwards, lane l carries rows l and
  // l + 64; the pivot being eliminated is read from its lane with readlane.
  for (int i = tid; i < m; i += SD_THREADS) dg[i] = 1.0 / A(i, i);   // reciprocal pivots
  __syncthreads();
  {
    const int wv = tid >> 6, ln = tid & 63;
    for (int j = wv; j < d.mp; j += SD_THREADS / 64) {
      double b0 = ln == j ? 1.0 : 0.0, b1 = ln + 64 == j ? 1.0 : 0.0;
      if (j < m) {
        for (int k = j; k >= 0; --k) {
          const double wk = readlane_d(k < 64 ? b0 : b1, k & 63) * dg[k];
          if (ln == k) b0 = wk;
          if (ln + 64 == k) b1 = wk;
          if (ln < k) b0 -= A(k, ln) * wk;
          if (ln + 64 < k) b1 -= A(k, ln + 64) * wk;
        }
      }
      if (ln < d.mp) d.C[(long)ln * d.mp + j] = (ln < m && ln <= j && j < m) ? b0 : 0.0;
      if (ln + 64 < d.mp) d.C[(long)(ln + 64) * d.mp + j] = (ln + 64 < m && ln + 64 <= j && j < m) ? b1 : 0.0;
    }
  }
  if (d.mode == SD_ORTHO) {
    if (tid == 0) d.status[0] = ST_OK, d.status[1] = 0;
    return;
  }
  __threadfence();   // W visible to every wavefront of the work-group
  __syncthreads();

  // ---- A = W^T Hs W on float64 MFMA from L2-resident operands: Y = Hs W into
  // the (no longer needed) global L, then A = W^T Y into LDS
  mfma_product(d.mp, [&](int i, int k) { return (i < m && k < m) ? d.Hs[(long)i * d.mp + k] : 0.0; },
               [&](int k, int j) { return d.C[(long)k * d.mp + j]; },
               [&](int i, int j, double v) { L[(long)i * d.mp + j] = v; });
  __threadfence();
  __syncthreads();
  mfma_product(d.mp, [&](int i, int k) { return d.C[(long)k * d.mp + i]; },
               [&](int k, int j) { return L[(long)k * d.mp + j]; },
               [&](int i, int j, double v) {
                 if (i < m && j < m) A(i, j) = v;
               });
  __syncthreads();
  for (int e = tid; e < m * m; e += SD_THREADS) {   // symmetrise (Hs is symmetric up to rounding)
    const int i = e / m, j = e % m;
    if (i < j) {
      const double v = 0.5 * (A(i, j) + A(j, i));
      A(i, j) = v;
      A(j, i) = v;
    }
  }
  __syncthreads();

  stamp(d, 2);
  // ---- cyclic Jacobi, round-robin ordering over n = m rounded up to even.
  // One step rotates n/2 disjoint pairs at once.  A' = J^T A J is applied as
  // independent 2x2 blocks: block (k, l) = rows {p_k, q_k} x columns {p_l, q_l}
  // becomes J_k^T B J_l, so every element is read and written once per step.
  const int n = (m + 1) & ~1, half = n / 2;
  if (n > m) {   // zero padding row / column: the identity "rotations" of it stay exact
    for (int i = tid; i < n; i += SD_THREADS) {
      A(m, i) = 0.0;
      A(i, m) = 0.0;
    }
  }
  __shared__ int step_active[2];
  if (tid == 0) step_active[0] = step_active[1] = 0;
  __syncthreads();
  // absolute floor: rotations regenerate off-diagonal roundoff of order eps * max|a_ii|.
  // Rotations are applied above tol/8 and convergence is declared at tol, so the
  // roundoff a rotation leaves behind cannot keep a sweep from finishing.
  double dmax = 0.0;
  for (int i = tid; i < m; i += SD_THREADS) dmax = fmax(dmax, fabs(A(i, i)));
  const double floor_abs = 32.0 * 2.220446049250313e-16 * fmax(block_max(dmax, red), 1e-300) / d.tol;
  const double rot_tol = 0.125 * d.tol;
  // the rotations of every step are logged (flag, then (c, s) per pair) and the
  // eigenvectors are rebuilt from the log once the sweeps are done
  double* lg = d.rot;
  // the 2x2 blocks (k, l), k <= l, of this thread, fixed for every step; A stays
  // symmetric, so block (l, k) is written as the transpose of block (k, l)
  constexpr int SD_BLOCKS = ((MAXM / 2) * (MAXM / 2 + 1) / 2 + SD_THREADS - 1) / SD_THREADS;
  const int nbt = half * (half + 1) / 2;
  int blk_k[SD_BLOCKS], blk_l[SD_BLOCKS], nblk = 0;
#pragma unroll
  for (int b = 0; b < SD_BLOCKS; ++b) {
    const int e = tid + b * SD_THREADS;   // row-major index into the triangle l >= k
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    blk_l[b] = e < nbt ? i : 0;
    blk_k[b] = e < nbt ? e - i * (i + 1) / 2 : 0;
    if (e < nbt) nblk = b + 1;
  }
  int sweep = 0;
  bool converged = false;
  int gstep = 0;
  for (; sweep < d.max_sweeps; ++sweep) {
    // convergence test: every off-diagonal |a_ij| <= tol * max(sqrt(|a_ii a_jj|), floor)
    double worst = 0.0;
    for (int e = tid; e < m * m; e += SD_THREADS) {
      const int i = e / m, j = e % m;
      if (i != j) {
        const double den = fmax(sqrt(fabs(A(i, i) * A(j, j))), floor_abs);
        worst = fmax(worst, fabs(A(i, j)) / den);
      }
    }
    worst = block_max(worst, red);
    if (worst <= d.tol) {
      converged = true;
      break;
    }
    for (int step = 0; step < n - 1; ++step, ++gstep) {
      const int cur = gstep & 1;
      if (tid == 0) step_active[cur ^ 1] = 0;   // last read before the previous step's final barrier
      for (int k = tid; k < half; k += SD_THREADS) {
        int p, q;
        if (k == 0) {
          p = 0;
          q = (step % (n - 1)) + 1;
        } else {
          p = ((k + step) % (n - 1)) + 1;
          q = ((n - 1 - k + step) % (n - 1)) + 1;
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, sn = 0.0;
        if (q < m) {
          const double apq = A(p, q), app = A(p, p), aqq = A(q, q);
          if (fabs(apq) > rot_tol * fmax(sqrt(fabs(app * aqq)), floor_abs) && apq != 0.0) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            step_active[cur] = 1;
          }
        }
        cs[k][0] = c;
        cs[k][1] = sn;
        pq[k][0] = p;
        pq[k][1] = q;
        lg[(long)gstep * SD_LOG_STRIDE + 1 + 2 * k] = c;
        lg[(long)gstep * SD_LOG_STRIDE + 2 + 2 * k] = sn;
      }
      __syncthreads();
      if (tid == 0) lg[(long)gstep * SD_LOG_STRIDE] = step_active[cur] ? 1.0 : 0.0;
      if (step_active[cur]) {   // uniform
#pragma unroll
        for (int b = 0; b < SD_BLOCKS; ++b) {
          if (b >= nblk) break;
          const int k = blk_k[b], l = blk_l[b];
          const double ck = cs[k][0], sk = cs[k][1], cl = cs[l][0], sl = cs[l][1];
          if (sk == 0.0 && sl == 0.0) continue;   // both rotations are the identity
          const int pk = pq[k][0], qk = pq[k][1], pl = pq[l][0], ql = pq[l][1];
          const double b00 = A(pk, pl), b01 = A(pk, ql), b10 = A(qk, pl), b11 = A(qk, ql);
          // rows: J_k^T
          const double r00 = ck * b00 - sk * b10, r01 = ck * b01 - sk * b11;
          const double r10 = sk * b00 + ck * b10, r11 = sk * b01 + ck * b11;
          // columns: J_l
          const double n00 = cl * r00 - sl * r01, n01 = sl * r00 + cl * r01;
          const double n10 = cl * r10 - sl * r11, n11 = sl * r10 + cl * r11;
          A(pk, pl) = n00;
          A(pk, ql) = n01;
          A(qk, pl) = n10;
          A(qk, ql) = n11;
          if (k != l) {   // the mirrored block
            A(pl, pk) = n00;
            A(ql, pk) = n01;
            A(pl, qk) = n10;
            A(ql, qk) = n11;
          }
        }
      }
      __syncthreads();
    }
  }
  stamp(d, 3);
  if (!converged) {
    if (tid == 0) d.status[0] = ST_EIG_NO_CONV, d.status[1] = sweep;
    return;
  }
  // eigenvalues and their ascending order (rank sort, ties by index)
  double* theta_tmp = d.scratch;          // m
  int* rank = reinterpret_cast<int*>(d.scratch + MAXM);
  for (int i = tid; i < m; i += SD_THREADS) theta_tmp[i] = A(i, i);
  __threadfence_block();
  __syncthreads();
  for (int i = tid; i < m; i += SD_THREADS) {
    const double ti = theta_tmp[i];
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double tj = theta_tmp[j];
      r += (tj < ti) || (tj == ti && j < i);
    }
    rank[i] = r;
    d.theta[r] = ti;
  }
  __threadfence_block();
  __syncthreads();
  // C = W U with U = J_1 J_2 ... J_G: the replay kernel applies the logged
  // rotations to the rows of W (already in C)
  if (tid == 0) d.status[0] = ST_OK, d.status[1] = sweep;
  stamp(d, 4);
}

__global__ __launch_bounds__(SD_THREADS) void small_dense_kernel(SmallDenseArgs d) { small_dense_body(d); }

// Many systems' small dense solves in one launch: work-group i solves system i
// (dynamic LDS sized for the largest block of the launch).
__global__ __launch_bounds__(SD_THREADS) void small_dense_jobs_kernel(const SmallDenseArgs* __restrict__ jobs) {
  small_dense_body(jobs[blockIdx.x]);
}

// Eigenvector replay: row r of C (holding W = L^-T) becomes W_r J_1 J_2 ... J_G
// with the Jacobi rotations of the log, columns then permuted to ascending
// Ritz values.  Rows are independent: one wavefront per row, 4 rows per
// work-group; the log is staged through LDS in chunks shared by the 4 rows.
// Lane l carries row elements l and l + 64; in step s of the round-robin
// ordering it needs the partner element of each and the pair index k that
// holds the (c, s) of that pair in the log.
constexpr int RP_ROWS = REPLAY_ROWS, RP_CHUNK = 24;

__device__ __forceinline__ void rr_partner(int e, int step, int n, int half, int& k, int& f) {
  if (e == 0) {           // pair 0 is (0, step + 1)
    k = 0;
    f = step + 1;
    return;
  }
  int a = e - 1 - step;   // pair k (k > 0) is (1 + (k + step) mod (n-1), 1 + (n-1-k+step) mod (n-1))
  if (a < 0) a += n - 1;
  if (a == 0) {
    k = 0;
    f = 0;
  } else if (a < half) {
    k = a;
    int b = n - 1 - k + step;
    if (b >= n - 1) b -= n - 1;
    f = b + 1;
  } else {
    k = n - 1 - a;
    int b = k + step;
    if (b >= n - 1) b -= n - 1;
    f = b + 1;
  }
}

__device__ __forceinline__ void sd_replay_rows(const SmallDenseArgs& d, int rb) {
  __shared__ double lgbuf[RP_CHUNK * SD_LOG_STRIDE];
  __shared__ double rowv[RP_ROWS][MAXM];
  if (d.status[0] != ST_OK) return;   // uniform
  const int m = d.m, mp = d.mp, n = (m + 1) & ~1, half = n / 2;
  const int G = d.status[1] * (n - 1);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = rb * RP_ROWS + w;
  const bool act = r < m;
  double* ur = rowv[w];
  const int e0 = lane, e1 = lane + 64;
  const bool h0 = e0 < n, h1 = e1 < n;
  double u0 = (act && e0 < m) ? d.C[(long)r * mp + e0] : 0.0;
  double u1 = (act && e1 < m) ? d.C[(long)r * mp + e1] : 0.0;
  if (h0) ur[e0] = u0;
  if (h1) ur[e1] = u1;
  int step = 0;
  for (int g0 = 0; g0 < G; g0 += RP_CHUNK) {
    const int cnt = min(RP_CHUNK, G - g0);
    __syncthreads();   // the previous chunk is consumed
    for (int e = tid; e < cnt * SD_LOG_STRIDE; e += 64 * RP_ROWS) lgbuf[e] = d.rot[(long)g0 * SD_LOG_STRIDE + e];
    __syncthreads();
    for (int gg = 0; gg < cnt; ++gg) {
      const double* lgs = lgbuf + gg * SD_LOG_STRIDE;
      if (lgs[0] != 0.0) {   // same value for every lane
        int k0 = 0, f0 = 0, k1 = 0, f1 = 0;
        if (h0) rr_partner(e0, step, n, half, k0, f0);
        if (h1) rr_partner(e1, step, n, half, k1, f1);
        const double v0 = h0 ? ur[f0] : 0.0, v1 = h1 ? ur[f1] : 0.0;
        const double c0 = lgs[1 + 2 * k0], s0 = lgs[2 + 2 * k0];
        const double c1 = lgs[1 + 2 * k1], s1 = lgs[2 + 2 * k1];
        // pair (p, q), p < q: u_p <- c u_p - s u_q, u_q <- s u_p + c u_q
        u0 = e0 < f0 ? c0 * u0 - s0 * v0 : s0 * v0 + c0 * u0;
        u1 = e1 < f1 ? c1 * u1 - s1 * v1 : s1 * v1 + c1 * u1;
        // every lane has read its partners before any lane writes (in-order LDS
        // within the wavefront; the fence keeps the compiler from reordering)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (h0) ur[e0] = u0;
        if (h1) ur[e1] = u1;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      if (++step == n - 1) step = 0;
    }
  }
  if (act) {
    const int* rank = reinterpret_cast<const int*>(d.scratch + MAXM);
    if (e0 < m) d.C[(long)r * mp + rank[e0]] = u0;
    if (e1 < m) d.C[(long)r * mp + rank[e1]] = u1;
  }
  if (rb == 0) stamp(d, 5);
}

__global__ __launch_bounds__(64 * RP_ROWS) void sd_replay_kernel(SmallDenseArgs d) { sd_replay_rows(d, blockIdx.x); }

// Many systems' replays in one launch: job j covers ceil(m_j / RP_ROWS) work-groups.
__global__ __launch_bounds__(64 * RP_ROWS) void sd_replay_jobs_kernel(const ReplayJob* __restrict__ jobs, int njobs) {
  const ReplayJob& J = find_job(jobs, njobs);
  sd_replay_rows(J.d, (int)blockIdx.x - J.block0);
}

// ------------------------------------------------------------------ rotation + residual epilogue
// Work-group: 256 threads = 4 waves; each wave owns strips of 16 points and all
// mp/16 output tiles of states.  Psi[j][p] = sum_i C[i][j] Phi[i][p].
// MT is the MFMA operand type: double (v_mfma_f64_16x16x4f64, float64 plans)
// or float (v_mfma_f32_16x16x4f32, float32 plans: C rounded to float32, the
// rotation of float32 states then loses nothing beyond float32 storage).

template <typename MT>
struct Mfma;
template <>
struct Mfma<double> {
  using acc = d4;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) { return mfma16(a, b, c); }
  static __device__ __forceinline__ int row(int lane, int r) { return drow(lane, r); }
};
// float32 16x16x4 layout (measured): D[4 * (l / 16) + r][l % 16]
template <>
struct Mfma<float> {
  using acc = f4;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Chunk c of the points (work-group of 256 threads).
template <typename F, typename MT, bool WITH_H, int NT>
__device__ __forceinline__ void rotate_chunk(const RotateArgs& r, int c) {
  // C in LDS.  float32: row-major, rows padded by 16 words so that the two
  // 16-lane row segments of one ds_read land in disjoint banks.  float64:
  // transposed (cs[j * mp + i] = C[i][j]), measured faster for the 64-bit reads.
  constexpr bool F32 = sizeof(MT) == 4;
  constexpr int PAD = F32 ? 16 : 0;
  __shared__ MT cs[MAXM * (MAXM + PAD)];
  __shared__ double thl[MAXM];
  __shared__ double rs[4][MAXM];
  if (r.status && r.status[0] != ST_OK) return;   // uniform: leave the states untouched
  using M = Mfma<MT>;
  using acc_t = typename M::acc;
  // NT = mp / 16 output tiles at compile time: no predicated MFMAs
  constexpr int mp = NT * 16, nk = NT * 4;
  const int m = r.m;
  const long N = r.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int LS = mp + PAD;
  for (int e = tid; e < mp * mp; e += 256) {
    const int i = e / mp, j = e - i * mp;
    cs[F32 ? i * LS + j : j * mp + i] = (MT)r.C[e];
  }
  for (int j = tid; j < mp; j += 256) thl[j] = (WITH_H && j < m) ? r.theta[j] : 0.0;
  __syncthreads();
  // Psi may alias Phi (in-place rotation): every output point depends only on
  // the same point of the inputs, and each 16-point strip is read completely
  // by one wave before that wave writes it.
  const F* Phi = reinterpret_cast<const F*>(r.Phi);
  const F* HPhi = reinterpret_cast<const F*>(r.HPhi);
  F* Psi = reinterpret_cast<F*>(r.Psi);
  F* HPsi = reinterpret_cast<F*>(r.HPsi);

  float res[NT][4];   // residual partial sums (a convergence measure: float32 suffices)
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) res[t][q] = 0.f;

  const long p_begin = (long)c * r.chunk;
  const long p_end = min(N, p_begin + r.chunk);
  // B operands in groups of KG k-steps; each group's loads are issued before
  // the MFMAs of the group before it, across strip boundaries too (the next
  // strip's first group is in flight while this strip's last MFMAs and its
  // stores run), so a wave waits on HBM only for its very first group.
  constexpr int KG = F32 ? (nk < 4 ? nk : 4) : 2;
  constexpr int NG = (nk + KG - 1) / KG;
  MT b[KG], bh[KG], nb[KG], nbh[KG];
  // float32: unconditional loads (masked lanes read element 0 and discard it),
  // so no exec-mask branches surround them; the k-step offsets 4 k N are
  // wave-uniform.  float64 keeps predicated loads (measured faster there).
  auto load_group = [&](long p0, int k0, MT (&x)[KG], MT (&xh)[KG]) {
    const long p = p0 + (lane & 15);
    const bool pok = p < p_end;
    const long lane_off = (long)(lane >> 4) * N + p;
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
      const int k = k0 + kk;
      const bool ok = k < nk && pok && 4 * k + (lane >> 4) < m;
      if constexpr (F32) {
        const long idx = ok ? lane_off + (long)(4 * k) * N : 0;
        const F v = Phi[idx];
        x[kk] = ok ? (MT)v : MT(0);
        if (WITH_H) {
          const F vh = HPhi[idx];
          xh[kk] = ok ? (MT)vh : MT(0);
        } else {
          xh[kk] = MT(0);
        }
      } else {
        const long idx = lane_off + (long)(4 * k) * N;
        x[kk] = ok ? (MT)Phi[idx] : MT(0);
        xh[kk] = (WITH_H && ok) ? (MT)HPhi[idx] : MT(0);
      }
    }
  };
  const long p_first = p_begin + 16 * wave;
  if (p_first < p_end) load_group(p_first, 0, b, bh);
  for (long p0 = p_first; p0 < p_end; p0 += 64) {
    const long p = p0 + (lane & 15);
    const bool pok = p < p_end;
    acc_t ap[NT], ah[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) ap[t] = ah[t] = acc_t{0, 0, 0, 0};
#pragma unroll 1
    for (int gq = 0; gq < NG; ++gq) {
      if (gq + 1 < NG) {
        load_group(p0, (gq + 1) * KG, nb, nbh);
      } else if (p0 + 64 < p_end) {
        load_group(p0 + 64, 0, nb, nbh);
      }
      const int k0 = gq * KG;
#pragma unroll
      for (int kk = 0; kk < KG; ++kk) {
        const int k = k0 + kk;
        if (KG * NG == nk || k < nk) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            // A (16x4) = C^T tile: A[jj][kk] = C[4k + kk][t*16 + jj]
            const MT a = F32 ? cs[(4 * k + (lane >> 4)) * LS + t * 16 + (lane & 15)]
                             : cs[(t * 16 + (lane & 15)) * mp + 4 * k + (lane >> 4)];
            ap[t] = M::mma(a, b[kk], ap[t]);
            if (WITH_H) ah[t] = M::mma(a, bh[kk], ah[t]);
          }
        }
      }
#pragma unroll
      for (int kk = 0; kk < KG; ++kk) {
        b[kk] = nb[kk];
        bh[kk] = nbh[kk];
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = t * 16 + M::row(lane, q);
        if (j < m && pok) {
          const F ps = (F)ap[t][q];
          Psi[(long)j * N + p] = ps;
          if (WITH_H) {
            const F hs = (F)ah[t][q];
            if (HPsi) HPsi[(long)j * N + p] = hs;
            const double dv = (double)hs - thl[j] * (double)ps;
            res[t][q] += (float)(dv * dv);
          }
        }
      }
    }
  }
  if (!WITH_H) return;
  // reduce residual partials over the 16 lanes sharing a state, then over waves
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = res[t][q];
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
      const int j = t * 16 + M::row(lane, q);
      if ((lane & 15) == 0) rs[wave][j] = v;
    }
  __syncthreads();
  for (int j = tid; j < mp; j += 256) {
    const double v = rs[0][j] + rs[1][j] + rs[2][j] + rs[3][j];
    r.res_partials[(long)c * mp + j] = v;
  }
}

template <typename F, typename MT, bool WITH_H, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(MT) == 4 ? 2 : 1))) void rotate_kernel(
    RotateArgs r) {
  rotate_chunk<F, MT, WITH_H, NT>(r, (int)blockIdx.x);
}

// Many systems' rotations of one tile class in one launch (one job per system).
template <typename F, typename MT, bool WITH_H, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(MT) == 4 ? 2 : 1))) void rotate_jobs_kernel(
    const RotateJob* __restrict__ jobs, int njobs) {
  const RotateJob& J = find_job(jobs, njobs);
  rotate_chunk<F, MT, WITH_H, NT>(J.r, (int)blockIdx.x - J.block0);
}

// ------------------------------------------------------------------ small helpers
__global__ void fill_kernel(double* p, long n, double v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// R^E_j = S_jj - M_jj^2 and R^E_perp_j = S_jj - sum_i M_ij^2 (psi_old orthonormal),
// with M_ij = (psi_i | phi_j); float64 on mp x mp matrices.  With a row table,
// phi_j is the propagated psi_(rows[j]): its variances go to entry rows[j].
__global__ void variance_kernel(const double* S, const double* M, int m, int mp, const int* rows, double* re,
                                double* re_perp) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int r = rows ? rows[j] : j;
  const double sjj = S[(long)j * mp + j];
  const double mrj = M[(long)r * mp + j];
  double s2 = 0.0;
  for (int i = 0; i < m; ++i) {
    const double v = M[(long)i * mp + j];
    s2 += v * v;
  }
  re[r] = sjj - mrj * mrj;
  re_perp[r] = sjj - s2;
}

// Many systems' variances in one launch: work-group j handles job j (m <= 128).
__global__ void variance_jobs_kernel(const VarianceJob* __restrict__ jobs) {
  const VarianceJob& J = jobs[blockIdx.x];
  const int j = threadIdx.x;
  if (j >= J.m) return;
  const double sjj = J.S[(long)j * J.mp + j];
  const double mjj = J.M[(long)j * J.mp + j];
  double s2 = 0.0;
  for (int i = 0; i < J.m; ++i) {
    const double v = J.M[(long)i * J.mp + j];
    s2 += v * v;
  }
  J.re[j] = sjj - mjj * mjj;
  J.re_perp[j] = sjj - s2;
}

// ------------------------------------------------------------------ launchers
template <typename F, int MODE>
static hipError_t launch_gram_t(const GramArgs& g, int nprod, int nchunks, hipStream_t st) {
  dim3 grid(nchunks, nprod), block(256);
  switch (g.mp / 16) {
    case 1: hipLaunchKernelGGL((gram_partial_kernel<F, 1, MODE>), grid, block, 0, st, g); break;
    case 2: hipLaunchKernelGGL((gram_partial_kernel<F, 2, MODE>), grid, block, 0, st, g); break;
    case 3: hipLaunchKernelGGL((gram_partial_kernel<F, 3, MODE>), grid, block, 0, st, g); break;
    case 4: hipLaunchKernelGGL((gram_partial_kernel<F, 4, MODE>), grid, block, 0, st, g); break;
    case 5: hipLaunchKernelGGL((gram_partial_kernel<F, 5, MODE>), grid, block, 0, st, g); break;
    case 6: hipLaunchKernelGGL((gram_partial_kernel<F, 6, MODE>), grid, block, 0, st, g); break;
    case 7: hipLaunchKernelGGL((gram_partial_kernel<F, 7, MODE>), grid, block, 0, st, g); break;
    case 8: hipLaunchKernelGGL((gram_partial_kernel<F, 8, MODE>), grid, block, 0, st, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Products with X == Y (overlaps of one block with itself) run as symmetric
// launches; the others as general ones.  Partials land in g.partials[prod].
template <int MODE>
static hipError_t launch_gram32_t(const GramArgs& g, int nchunks, hipStream_t st) {
  dim3 grid(nchunks, 1), block(512);
  switch (g.mp / 16) {
    case 1: hipLaunchKernelGGL((gram32_partial_kernel<1, MODE>), grid, block, 0, st, g); break;
    case 2: hipLaunchKernelGGL((gram32_partial_kernel<2, MODE>), grid, block, 0, st, g); break;
    case 3: hipLaunchKernelGGL((gram32_partial_kernel<3, MODE>), grid, block, 0, st, g); break;
    case 4: hipLaunchKernelGGL((gram32_partial_kernel<4, MODE>), grid, block, 0, st, g); break;
    case 5: hipLaunchKernelGGL((gram32_partial_kernel<5, MODE>), grid, block, 0, st, g); break;
    case 6: hipLaunchKernelGGL((gram32_partial_kernel<6, MODE>), grid, block, 0, st, g); break;
    case 7: hipLaunchKernelGGL((gram32_partial_kernel<7, MODE>), grid, block, 0, st, g); break;
    case 8: hipLaunchKernelGGL((gram32_partial_kernel<8, MODE>), grid, block, 0, st, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE, int SPLIT>
static hipError_t launch_gramb_t(const GramArgs& g, int nchunks, hipStream_t st) {
  dim3 grid(nchunks, 1), block(512);
  switch (g.mp / 16) {
    case 1: hipLaunchKernelGGL((gramb_partial_kernel<1, MODE, SPLIT>), grid, block, 0, st, g); break;
    case 2: hipLaunchKernelGGL((gramb_partial_kernel<2, MODE, SPLIT>), grid, block, 0, st, g); break;
    case 3: hipLaunchKernelGGL((gramb_partial_kernel<3, MODE, SPLIT>), grid, block, 0, st, g); break;
    case 4: hipLaunchKernelGGL((gramb_partial_kernel<4, MODE, SPLIT>), grid, block, 0, st, g); break;
    case 5: hipLaunchKernelGGL((gramb_partial_kernel<5, MODE, SPLIT>), grid, block, 0, st, g); break;
    case 6: hipLaunchKernelGGL((gramb_partial_kernel<6, MODE, SPLIT>), grid, block, 0, st, g); break;
    case 7: hipLaunchKernelGGL((gramb_partial_kernel<7, MODE, SPLIT>), grid, block, 0, st, g); break;
    case 8: hipLaunchKernelGGL((gramb_partial_kernel<8, MODE, SPLIT>), grid, block, 0, st, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int SPLIT>
static hipError_t launch_gramb_split(const GramArgs& g, int nprod, int nchunks, hipStream_t st) {
  for (int i = 0; i < nprod; ++i) {
    GramArgs one = g;
    one.X[0] = g.X[i];
    one.Y[0] = g.Y[i];
    one.partials = g.partials + (long)i * nchunks * g.mp * g.mp;
    const int mode = gram_mode(g, i);
    const hipError_t e = mode == GRAM_SELF    ? launch_gramb_t<GRAM_SELF, SPLIT>(one, nchunks, st)
                         : mode == GRAM_UPPER ? launch_gramb_t<GRAM_UPPER, SPLIT>(one, nchunks, st)
                                              : launch_gramb_t<GRAM_FULL, SPLIT>(one, nchunks, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gramb(const GramArgs& g, int nprod, int nchunks, int split, hipStream_t st) {
  if (split == 2) return launch_gramb_split<2>(g, nprod, nchunks, st);
  if (split == 3) return launch_gramb_split<3>(g, nprod, nchunks, st);
  return hipErrorInvalidValue;
}

hipError_t launch_gram32(const GramArgs& g, int nprod, int nchunks, hipStream_t st) {
  for (int i = 0; i < nprod; ++i) {
    GramArgs one = g;
    one.X[0] = g.X[i];
    one.Y[0] = g.Y[i];
    one.partials = g.partials + (long)i * nchunks * g.mp * g.mp;
    const int mode = gram_mode(g, i);
    const hipError_t e = mode == GRAM_SELF    ? launch_gram32_t<GRAM_SELF>(one, nchunks, st)
                         : mode == GRAM_UPPER ? launch_gram32_t<GRAM_UPPER>(one, nchunks, st)
                                              : launch_gram32_t<GRAM_FULL>(one, nchunks, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gram(int is_double, const GramArgs& g, int nprod, int nchunks, hipStream_t st) {
  for (int i = 0; i < nprod; ++i) {
    GramArgs one = g;
    one.X[0] = g.X[i];
    one.Y[0] = g.Y[i];
    one.partials = g.partials + (long)i * nchunks * g.mp * g.mp;
    const int mode = gram_mode(g, i);
    hipError_t e;
    if (is_double)
      e = mode == GRAM_SELF    ? launch_gram_t<double, GRAM_SELF>(one, 1, nchunks, st)
          : mode == GRAM_UPPER ? launch_gram_t<double, GRAM_UPPER>(one, 1, nchunks, st)
                               : launch_gram_t<double, GRAM_FULL>(one, 1, nchunks, st);
    else
      e = mode == GRAM_SELF    ? launch_gram_t<float, GRAM_SELF>(one, 1, nchunks, st)
          : mode == GRAM_UPPER ? launch_gram_t<float, GRAM_UPPER>(one, 1, nchunks, st)
                               : launch_gram_t<float, GRAM_FULL>(one, 1, nchunks, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reduce(const double* in, int nparts, long count, int ncomp, double* out, hipStream_t st) {
  dim3 grid((unsigned)((count + 63) / 64), ncomp);
  hipLaunchKernelGGL(reduce_kernel, grid, dim3(64 * RD_SLICES), 0, st, in, nparts, count, out);
  return hipGetLastError();
}

hipError_t prepare_small_dense() {
  const int lds = (int)((size_t)MAXM * (MAXM + 1) * sizeof(double));
  hipError_t e = hipFuncSetAttribute((const void*)small_dense_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)small_dense_jobs_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// ---- batched launchers
template <typename F, int MODE>
static hipError_t launch_gram_jobs_t(int nt, const GramJob* jobs, int njobs, int nblocks, hipStream_t st) {
  dim3 grid(nblocks), block(256);
  switch (nt) {
    case 1: hipLaunchKernelGGL((gram_jobs_kernel<F, 1, MODE>), grid, block, 0, st, jobs, njobs); break;
    case 2: hipLaunchKernelGGL((gram_jobs_kernel<F, 2, MODE>), grid, block, 0, st, jobs, njobs); break;
    case 3: hipLaunchKernelGGL((gram_jobs_kernel<F, 3, MODE>), grid, block, 0, st, jobs, njobs); break;
    case 4: hipLaunchKernelGGL((gram_jobs_kernel<F, 4, MODE>), grid, block, 0, st, jobs, njobs); break;
    case 5: hipLaunchKernelGGL((gram_jobs_kernel<F, 5, MODE>), grid, block, 0, st, jobs, njobs); break;
    case 6: hipLaunchKernelGGL((gram_jobs_kernel<F, 6, MODE>), grid, block, 0, st, jobs, njobs); break;
    case 7: hipLaunchKernelGGL((gram_jobs_kernel<F, 7, MODE>), grid, block, 0, st, jobs, njobs); break;
    case 8: hipLaunchKernelGGL((gram_jobs_kernel<F, 8, MODE>), grid, block, 0, st, jobs, njobs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram_jobs(int is_double, int nt, int mode, const GramJob* jobs, int njobs, int nblocks,
                            hipStream_t st) {
  if (njobs <= 0 || nblocks <= 0) return hipSuccess;
  if (is_double)
    return mode == GRAM_SELF    ? launch_gram_jobs_t<double, GRAM_SELF>(nt, jobs, njobs, nblocks, st)
           : mode == GRAM_UPPER ? launch_gram_jobs_t<double, GRAM_UPPER>(nt, jobs, njobs, nblocks, st)
                                : launch_gram_jobs_t<double, GRAM_FULL>(nt, jobs, njobs, nblocks, st);
  return mode == GRAM_SELF    ? launch_gram_jobs_t<float, GRAM_SELF>(nt, jobs, njobs, nblocks, st)
         : mode == GRAM_UPPER ? launch_gram_jobs_t<float, GRAM_UPPER>(nt, jobs, njobs, nblocks, st)
                              : launch_gram_jobs_t<float, GRAM_FULL>(nt, jobs, njobs, nblocks, st);
}

template <typename F, typename MT, bool H>
static hipError_t launch_rotate_jobs_t(int nt, const RotateJob* jobs, int njobs, int nblocks, hipStream_t st) {
  dim3 grid(nblocks), block(256);
  switch (nt) {
    case 1: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 1>), grid, block, 0, st, jobs, njobs); break;
    case 2: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 2>), grid, block, 0, st, jobs, njobs); break;
    case 3: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 3>), grid, block, 0, st, jobs, njobs); break;
    case 4: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 4>), grid, block, 0, st, jobs, njobs); break;
    case 5: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 5>), grid, block, 0, st, jobs, njobs); break;
    case 6: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 6>), grid, block, 0, st, jobs, njobs); break;
    case 7: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 7>), grid, block, 0, st, jobs, njobs); break;
    case 8: hipLaunchKernelGGL((rotate_jobs_kernel<F, MT, H, 8>), grid, block, 0, st, jobs, njobs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rotate_jobs(int is_double, bool with_h, int nt, const RotateJob* jobs, int njobs, int nblocks,
                              hipStream_t st) {
  if (njobs <= 0 || nblocks <= 0) return hipSuccess;
  if (is_double)
    return with_h ? launch_rotate_jobs_t<double, double, true>(nt, jobs, njobs, nblocks, st)
                  : launch_rotate_jobs_t<double, double, false>(nt, jobs, njobs, nblocks, st);
  return with_h ? launch_rotate_jobs_t<float, float, true>(nt, jobs, njobs, nblocks, st)
                : launch_rotate_jobs_t<float, float, false>(nt, jobs, njobs, nblocks, st);
}

hipError_t launch_reduce_jobs(const ReduceJob* jobs, int njobs, int nblocks, hipStream_t st) {
  if (njobs <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_jobs_kernel, dim3(nblocks), dim3(64 * RD_SLICES), 0, st, jobs, njobs);
  return hipGetLastError();
}

hipError_t launch_small_dense_jobs(const SmallDenseArgs* jobs, int njobs, int max_mp, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  const size_t lds = (size_t)max_mp * (max_mp + 1) * sizeof(double);
  hipLaunchKernelGGL(small_dense_jobs_kernel, dim3(njobs), dim3(SD_THREADS), lds, st, jobs);
  return hipGetLastError();
}

hipError_t launch_replay_jobs(const ReplayJob* jobs, int njobs, int nblocks, hipStream_t st) {
  if (njobs <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(sd_replay_jobs_kernel, dim3(nblocks), dim3(64 * RP_ROWS), 0, st, jobs, njobs);
  return hipGetLastError();
}

hipError_t launch_variance_jobs(const VarianceJob* jobs, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(variance_jobs_kernel, dim3(njobs), dim3(MAXM), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_small_dense(const SmallDenseArgs& d, hipStream_t st) {
  const size_t lds = (size_t)d.mp * (d.mp + 1) * sizeof(double);
  hipLaunchKernelGGL(small_dense_kernel, dim3(1), dim3(SD_THREADS), lds, st, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || d.mode != SD_RR) return e;
  hipLaunchKernelGGL(sd_replay_kernel, dim3((d.m + RP_ROWS - 1) / RP_ROWS), dim3(64 * RP_ROWS), 0, st, d);
  return hipGetLastError();
}

template <typename F, typename MT, bool H>
static hipError_t launch_rotate_t(const RotateArgs& r, int nchunks, hipStream_t st) {
  dim3 grid(nchunks), block(256);
  switch (r.mp / 16) {
    case 1: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 1>), grid, block, 0, st, r); break;
    case 2: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 2>), grid, block, 0, st, r); break;
    case 3: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 3>), grid, block, 0, st, r); break;
    case 4: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 4>), grid, block, 0, st, r); break;
    case 5: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 5>), grid, block, 0, st, r); break;
    case 6: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 6>), grid, block, 0, st, r); break;
    case 7: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 7>), grid, block, 0, st, r); break;
    case 8: hipLaunchKernelGGL((rotate_kernel<F, MT, H, 8>), grid, block, 0, st, r); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rotate(int is_double, bool with_h, const RotateArgs& r, int nchunks, hipStream_t st) {
  if (is_double)
    return with_h ? launch_rotate_t<double, double, true>(r, nchunks, st)
                  : launch_rotate_t<double, double, false>(r, nchunks, st);
  return with_h ? launch_rotate_t<float, float, true>(r, nchunks, st)
                : launch_rotate_t<float, float, false>(r, nchunks, st);
}

// dst <- src, n16 16-byte words (a plain kernel: usable inside captured graphs)
__global__ void copy16_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src, long n16) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (long)gridDim.x * blockDim.x) dst[i] = src[i];
}

hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 16) return hipErrorInvalidValue;
  const long n16 = (long)(bytes / 16);
  const long blocks = std::min<long>(8192, (n16 + 255) / 256);
  hipLaunchKernelGGL(copy16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<uint4*>(dst),
                     reinterpret_cast<const uint4*>(src), n16);
  return hipGetLastError();
}

// Row gather: row i of dst <- row rows[i] of src, i < nrows, rows of row16
// 16-byte words; work-group (x, i) copies a strided share of row i.  Rows of
// dst and src must not overlap (the rows are read and written concurrently).
__global__ void gather_rows16_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                     const int* __restrict__ rows, long row16) {
  const long i = blockIdx.y;
  const uint4* s = src + (long)rows[i] * row16;
  uint4* d = dst + i * row16;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < row16; k += (long)gridDim.x * blockDim.x) d[k] = s[k];
}

hipError_t launch_gather_rows(void* dst, const void* src, const int* rows, int nrows, size_t row_bytes,
                              hipStream_t st) {
  if (nrows <= 0 || row_bytes == 0) return hipSuccess;
  if (row_bytes % 16 || nrows > 65535) return hipErrorInvalidValue;
  const long row16 = (long)(row_bytes / 16);
  const long bx = std::max<long>(1, std::min<long>(64, (row16 + 255) / 256));
  hipLaunchKernelGGL(gather_rows16_kernel, dim3((unsigned)bx, (unsigned)nrows), dim3(256), 0, st,
                     reinterpret_cast<uint4*>(dst), reinterpret_cast<const uint4*>(src), rows, row16);
  return hipGetLastError();
}

// In-place row moves: row i of buf <- row rows[i] where rows[i] != i, i < nrows.
// No row that is moved into may be the source of another move (the moves run
// concurrently).
__global__ void move_rows16_kernel(uint4* __restrict__ buf, const int* __restrict__ rows, long row16) {
  const long i = blockIdx.y;
  const long r = rows[i];
  if (r == i) return;
  const uint4* s = buf + r * row16;
  uint4* d = buf + i * row16;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < row16; k += (long)gridDim.x * blockDim.x) d[k] = s[k];
}

hipError_t launch_move_rows(void* buf, const int* rows, int nrows, size_t row_bytes, hipStream_t st) {
  if (nrows <= 0 || row_bytes == 0) return hipSuccess;
  if (row_bytes % 16 || nrows > 65535) return hipErrorInvalidValue;
  const long row16 = (long)(row_bytes / 16);
  const long bx = std::max<long>(1, std::min<long>(64, (row16 + 255) / 256));
  hipLaunchKernelGGL(move_rows16_kernel, dim3((unsigned)bx, (unsigned)nrows), dim3(256), 0, st,
                     reinterpret_cast<uint4*>(buf), rows, row16);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_variance(const double* S, const double* M, int m, int mp, const int* rows, double* re,
                           double* re_perp, hipStream_t st) {
  hipLaunchKernelGGL(variance_kernel, dim3((m + 127) / 128), dim3(128), 0, st, S, M, m, mp, rows, re, re_perp);
  return hipGetLastError();
}

}  // namespace mpe
