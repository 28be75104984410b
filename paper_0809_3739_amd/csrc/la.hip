// Subspace linear algebra on the GPU: overlap matrices, Cholesky
// orthonormalisation and the Rayleigh-Ritz rotation (Section I, Eq. ortho;
// Section III, subspace orthogonalisation; variances R^H and R^E).
//
// States are rows of an [m][N] array (m = states incl. guards, N grid points).
//  * gram_partial_kernel : X Y^T over a chunk of points on float64 MFMA
//    (v_mfma_f64_16x16x4f64); inputs of either precision are widened exactly.
//  * reduce_kernel       : fixed-order float64 sum of chunk partials.
//  * small_dense_kernel  : one work-group; S = L L^T, A = L^-1 Hs L^-T,
//    cyclic parallel Jacobi on A, C = L^-T U with columns sorted by eigenvalue.
//  * rotate_kernel       : Psi = Phi C and (H Phi) C on float64 MFMA with the
//    residual sum_p ((H Psi)_j - theta_j Psi_j)^2 accumulated in the epilogue.
#include <hip/hip_runtime.h>

#include <cmath>

#include "la.hpp"

namespace mpe {

typedef double d4 __attribute__((ext_vector_type(4)));

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
// Work-group: 256 threads (4 waves).  Output tiles of 16x16 over mp x mp are
// dealt round-robin to the waves (<= 16 tiles each for mp <= 128).  Points are
// staged through LDS in slabs of GSLAB, transposed to [point][state].
constexpr int GSLAB = 16;
constexpr int GMAXT = 16;

template <typename F>
__global__ __launch_bounds__(256) void gram_partial_kernel(GramArgs g) {
  __shared__ double xs[GSLAB][MAXM + 2];
  __shared__ double ys[GSLAB][MAXM + 2];
  const int prod = blockIdx.y;
  const F* __restrict__ X = reinterpret_cast<const F*>(g.X[prod]);
  const F* __restrict__ Y = reinterpret_cast<const F*>(g.Y[prod]);
  const bool same = X == Y;
  const int m = g.m, mp = g.mp, nt = mp / 16;
  const long N = g.N;
  const long p_begin = (long)blockIdx.x * g.chunk;
  const long p_end = min(N, p_begin + g.chunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  d4 acc[GMAXT];
#pragma unroll
  for (int t = 0; t < GMAXT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  for (long p0 = p_begin; p0 < p_end; p0 += GSLAB) {
    // stage: element (state s, point p0 + q) -> xs[q][s]
    for (int e = tid; e < mp * GSLAB; e += 256) {
      const int s = e / GSLAB, q = e - s * GSLAB;
      const long p = p0 + q;
      const bool ok = s < m && p < p_end;
      xs[q][s] = ok ? (double)X[(long)s * N + p] : 0.0;
      if (!same) ys[q][s] = ok ? (double)Y[(long)s * N + p] : 0.0;
    }
    __syncthreads();
    const double(*yy)[MAXM + 2] = same ? xs : ys;
#pragma unroll
    for (int k0 = 0; k0 < GSLAB; k0 += 4) {
      const int kq = k0 + (lane >> 4);
#pragma unroll
      for (int t = 0; t < GMAXT; ++t) {
        const int tile = wave + 4 * t;
        if (tile < nt * nt) {
          const int ti = tile / nt, tj = tile - ti * nt;
          const double a = xs[kq][ti * 16 + (lane & 15)];
          const double b = yy[kq][tj * 16 + (lane & 15)];
          acc[t] = mfma16(a, b, acc[t]);
        }
      }
    }
    __syncthreads();
  }
  double* out = g.partials + ((long)prod * gridDim.x + blockIdx.x) * (long)mp * mp;
#pragma unroll
  for (int t = 0; t < GMAXT; ++t) {
    const int tile = wave + 4 * t;
    if (tile < nt * nt) {
      const int ti = tile / nt, tj = tile - ti * nt;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti * 16 + drow(lane, r), j = tj * 16 + (lane & 15);
        out[(long)i * mp + j] = acc[t][r];
      }
    }
  }
}

// out[c][e] = sum_{q < nparts} in[c][q][e], e < count, fixed order.
__global__ void reduce_kernel(const double* __restrict__ in, int nparts, long count, double* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= count) return;
  const double* src = in + (long)c * nparts * count + e;
  double s = 0.0;
  for (int q = 0; q < nparts; ++q) s += src[(long)q * count];
  out[(long)c * count + e] = s;
}

// ------------------------------------------------------------------ small dense problem
// One work-group of 1024 threads.  LDS holds one mp x (mp+1) float64 matrix;
// L, the Jacobi rotation log and scratch live in global memory (L2 resident).
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

__global__ __launch_bounds__(SD_THREADS) void small_dense_kernel(SmallDenseArgs d) {
  extern __shared__ double sh[];  // mp x LD
  __shared__ double red[20];
  __shared__ int flag;
  __shared__ double cs[MAXM / 2 + 1][2];
  __shared__ int pq[MAXM / 2 + 1][2];
  __shared__ double dg[MAXM];
  const int m = d.m, LD = d.mp + 1;
  const int tid = threadIdx.x;
  double* L = d.L;            // mp x mp, lower triangle
  auto A = [&](int i, int j) -> double& { return sh[i * LD + j]; };

  if (tid == 0) flag = -1;
  __syncthreads();
  // ---- Cholesky of S in LDS (right-looking)
  for (int e = tid; e < m * m; e += SD_THREADS) A(e / m, e % m) = d.S[(e / m) * (long)d.mp + e % m];
  for (int i = tid; i < m; i += SD_THREADS) dg[i] = d.S[i * (long)d.mp + i];
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
    const double lkk = sqrt(piv);
    __syncthreads();
    for (int i = k + tid; i < m; i += SD_THREADS) A(i, k) = (i == k) ? lkk : A(i, k) / lkk;
    __syncthreads();
    const int rem = m - k - 1;
    for (int e = tid; e < rem * rem; e += SD_THREADS) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      if (j <= i) A(i, j) -= A(i, k) * A(j, k);
    }
    __syncthreads();
  }
  __syncthreads();
  if (flag != -1) {
    if (tid == 0) {
      d.status[0] = flag >= 0 ? ST_NOT_SPD : ST_NONFINITE;
      d.status[1] = flag >= 0 ? flag : -2 - flag;
    }
    return;
  }
  for (int e = tid; e < m * m; e += SD_THREADS) {
    const int i = e / m, j = e % m;
    L[(long)i * d.mp + j] = j <= i ? A(i, j) : 0.0;
  }
  __threadfence_block();
  __syncthreads();

  if (d.mode == SD_ORTHO) {
    // C = L^-T: back substitution on the identity, one column per thread
    for (int e = tid; e < m * m; e += SD_THREADS) A(e / m, e % m) = (e / m == e % m) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = tid; j < m; j += SD_THREADS) {
      for (int i = m - 1; i >= 0; --i) {
        double s = A(i, j);
        for (int k = i + 1; k < m; ++k) s -= L[(long)k * d.mp + i] * A(k, j);
        A(i, j) = s / L[(long)i * d.mp + i];
      }
    }
    __syncthreads();
    for (int e = tid; e < d.mp * d.mp; e += SD_THREADS) {
      const int i = e / d.mp, j = e % d.mp;
      d.C[e] = (i < m && j < m) ? A(i, j) : 0.0;
    }
    if (tid == 0) d.status[0] = ST_OK, d.status[1] = 0;
    return;
  }

  // ---- X = L^-1 Hs (column per thread), then A = L^-1 X^T (row per thread, in place)
  for (int e = tid; e < m * m; e += SD_THREADS) A(e / m, e % m) = d.Hs[(e / m) * (long)d.mp + e % m];
  __syncthreads();
  for (int e = tid; e < m * m; e += SD_THREADS) {   // symmetrise Hs
    const int i = e / m, j = e % m;
    if (i < j) {
      const double v = 0.5 * (A(i, j) + A(j, i));
      A(i, j) = v;
      A(j, i) = v;
    }
  }
  __syncthreads();
  for (int j = tid; j < m; j += SD_THREADS) {
    for (int i = 0; i < m; ++i) {
      double s = A(i, j);
      for (int k = 0; k < i; ++k) s -= L[(long)i * d.mp + k] * A(k, j);
      A(i, j) = s / L[(long)i * d.mp + i];
    }
  }
  __syncthreads();
  for (int j = tid; j < m; j += SD_THREADS) {
    for (int i = 0; i < m; ++i) {
      double s = A(j, i);
      for (int k = 0; k < i; ++k) s -= L[(long)i * d.mp + k] * A(j, k);
      A(j, i) = s / L[(long)i * d.mp + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += SD_THREADS) {
    const int i = e / m, j = e % m;
    if (i < j) {
      const double v = 0.5 * (A(i, j) + A(j, i));
      A(i, j) = v;
      A(j, i) = v;
    }
  }
  __syncthreads();

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
  long nrot = 0;
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
      }
      __syncthreads();
      if (step_active[cur]) {   // uniform
        for (int k = tid; k < half; k += SD_THREADS) {
          double* slot = d.rot + (nrot + k) * 4;
          slot[0] = cs[k][0];
          slot[1] = cs[k][1];
          slot[2] = (double)pq[k][0];
          slot[3] = (double)pq[k][1];
        }
        for (int e = tid; e < half * half; e += SD_THREADS) {
          const int k = e / half, l = e - k * half;
          const int pk = pq[k][0], qk = pq[k][1], pl = pq[l][0], ql = pq[l][1];
          const double ck = cs[k][0], sk = cs[k][1], cl = cs[l][0], sl = cs[l][1];
          const double b00 = A(pk, pl), b01 = A(pk, ql), b10 = A(qk, pl), b11 = A(qk, ql);
          // rows: J_k^T
          const double r00 = ck * b00 - sk * b10, r01 = ck * b01 - sk * b11;
          const double r10 = sk * b00 + ck * b10, r11 = sk * b01 + ck * b11;
          // columns: J_l
          A(pk, pl) = cl * r00 - sl * r01;
          A(pk, ql) = sl * r00 + cl * r01;
          A(qk, pl) = cl * r10 - sl * r11;
          A(qk, ql) = sl * r10 + cl * r11;
        }
        nrot += half;
      }
      __syncthreads();
    }
  }
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
  // U = product of the logged rotations, rebuilt in LDS
  for (int e = tid; e < m * m; e += SD_THREADS) A(e / m, e % m) = (e / m == e % m) ? 1.0 : 0.0;
  __syncthreads();
  for (long base = 0; base < nrot; base += half) {
    for (int e = tid; e < half * m; e += SD_THREADS) {
      const int k = e / m, r = e % m;
      const double* rr = d.rot + (base + k) * 4;
      const int p = (int)rr[2], q = (int)rr[3];
      if (q < m) {
        const double c = rr[0], s = rr[1];
        const double ap = A(r, p), aq = A(r, q);
        A(r, p) = c * ap - s * aq;
        A(r, q) = s * ap + c * aq;
      }
    }
    __syncthreads();
  }
  // C = L^-T U (column per thread, in place, bottom up)
  for (int j = tid; j < m; j += SD_THREADS) {
    for (int i = m - 1; i >= 0; --i) {
      double s = A(i, j);
      for (int k = i + 1; k < m; ++k) s -= L[(long)k * d.mp + i] * A(k, j);
      A(i, j) = s / L[(long)i * d.mp + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < d.mp * d.mp; e += SD_THREADS) d.C[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < m * m; e += SD_THREADS) {
    const int i = e / m, j = e % m;
    d.C[(long)i * d.mp + rank[j]] = A(i, j);
  }
  if (tid == 0) d.status[0] = ST_OK, d.status[1] = sweep;
}

// ------------------------------------------------------------------ rotation + residual epilogue
// Work-group: 256 threads = 4 waves; each wave owns strips of 16 points and all
// mp/16 output tiles of states.  Psi[j][p] = sum_i C[i][j] Phi[i][p].
constexpr int RMAXT = MAXM / 16;

template <typename F, bool WITH_H>
__global__ __launch_bounds__(256) void rotate_kernel(RotateArgs r) {
  __shared__ double cT[MAXM * MAXM];  // cT[j * mp + i] = C[i][j]
  if (r.status && r.status[0] != ST_OK) return;   // uniform: leave the states untouched
  const int m = r.m, mp = r.mp, nt = mp / 16;
  const long N = r.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < mp * mp; e += 256) {
    const int i = e / mp, j = e - i * mp;
    cT[j * mp + i] = r.C[e];
  }
  __syncthreads();
  // Psi may alias Phi (in-place rotation): every output point depends only on
  // the same point of the inputs, and each 16-point strip is read completely
  // by one wave before that wave writes it.
  const F* Phi = reinterpret_cast<const F*>(r.Phi);
  const F* HPhi = reinterpret_cast<const F*>(r.HPhi);
  F* Psi = reinterpret_cast<F*>(r.Psi);
  F* HPsi = reinterpret_cast<F*>(r.HPsi);

  double res[RMAXT][4];
#pragma unroll
  for (int t = 0; t < RMAXT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) res[t][q] = 0.0;
  double th[RMAXT][4];
#pragma unroll
  for (int t = 0; t < RMAXT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = t * 16 + drow(lane, q);
      th[t][q] = (WITH_H && j < m) ? r.theta[j] : 0.0;
    }

  const long p_begin = (long)blockIdx.x * r.chunk;
  const long p_end = min(N, p_begin + r.chunk);
  for (long p0 = p_begin + 16 * wave; p0 < p_end; p0 += 64) {
    const long p = p0 + (lane & 15);
    const bool pok = p < p_end;
    d4 ap[RMAXT], ah[RMAXT];
#pragma unroll
    for (int t = 0; t < RMAXT; ++t) ap[t] = ah[t] = d4{0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < mp; i0 += 4) {
      const int i = i0 + (lane >> 4);
      const bool ok = pok && i < m;
      const double b = ok ? (double)Phi[(long)i * N + p] : 0.0;
      const double bh = (WITH_H && ok) ? (double)HPhi[(long)i * N + p] : 0.0;
#pragma unroll
      for (int t = 0; t < RMAXT; ++t) {
        if (t < nt) {
          // A (16x4) = C^T tile: A[jj][kk] = C[i0 + kk][t*16 + jj]
          const double a = cT[(t * 16 + (lane & 15)) * mp + i0 + (lane >> 4)];
          ap[t] = mfma16(a, b, ap[t]);
          if (WITH_H) ah[t] = mfma16(a, bh, ah[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RMAXT; ++t) {
      if (t < nt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = t * 16 + drow(lane, q);
          if (j < m && pok) {
            const F ps = (F)ap[t][q];
            Psi[(long)j * N + p] = ps;
            if (WITH_H) {
              const F hs = (F)ah[t][q];
              if (HPsi) HPsi[(long)j * N + p] = hs;
              const double dv = (double)hs - th[t][q] * (double)ps;
              res[t][q] += dv * dv;
            }
          }
        }
      }
    }
  }
  if (!WITH_H) return;
  // reduce residual partials over the 16 lanes sharing a state, then over waves
  __shared__ double rs[4][MAXM];
#pragma unroll
  for (int t = 0; t < RMAXT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = res[t][q];
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
      const int j = t * 16 + drow(lane, q);
      if ((lane & 15) == 0 && t < nt) rs[wave][j] = v;
    }
  __syncthreads();
  for (int j = tid; j < mp; j += 256) {
    const double v = rs[0][j] + rs[1][j] + rs[2][j] + rs[3][j];
    r.res_partials[(long)blockIdx.x * mp + j] = v;
  }
}

// ------------------------------------------------------------------ small helpers
__global__ void fill_kernel(double* p, long n, double v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// R^E_j = S_jj - M_jj^2 and R^E_perp_j = S_jj - sum_i M_ij^2 (psi_old orthonormal),
// with M_ij = (psi_i | phi_j); float64 on mp x mp matrices.
__global__ void variance_kernel(const double* S, const double* M, int m, int mp, double* re, double* re_perp) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const double sjj = S[(long)j * mp + j];
  const double mjj = M[(long)j * mp + j];
  double s2 = 0.0;
  for (int i = 0; i < m; ++i) {
    const double v = M[(long)i * mp + j];
    s2 += v * v;
  }
  re[j] = sjj - mjj * mjj;
  re_perp[j] = sjj - s2;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_gram(int is_double, const GramArgs& g, int nprod, int nchunks, hipStream_t st) {
  dim3 grid(nchunks, nprod);
  if (is_double)
    hipLaunchKernelGGL(gram_partial_kernel<double>, grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL(gram_partial_kernel<float>, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* in, int nparts, long count, int ncomp, double* out, hipStream_t st) {
  dim3 grid((unsigned)((count + 255) / 256), ncomp);
  hipLaunchKernelGGL(reduce_kernel, grid, dim3(256), 0, st, in, nparts, count, out);
  return hipGetLastError();
}

hipError_t prepare_small_dense() {
  return hipFuncSetAttribute((const void*)small_dense_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)((size_t)MAXM * (MAXM + 1) * sizeof(double)));
}

hipError_t launch_small_dense(const SmallDenseArgs& d, hipStream_t st) {
  const size_t lds = (size_t)d.mp * (d.mp + 1) * sizeof(double);
  hipLaunchKernelGGL(small_dense_kernel, dim3(1), dim3(SD_THREADS), lds, st, d);
  return hipGetLastError();
}

hipError_t launch_rotate(int is_double, bool with_h, const RotateArgs& r, int nchunks, hipStream_t st) {
  dim3 grid(nchunks);
  if (is_double) {
    if (with_h) hipLaunchKernelGGL((rotate_kernel<double, true>), grid, dim3(256), 0, st, r);
    else hipLaunchKernelGGL((rotate_kernel<double, false>), grid, dim3(256), 0, st, r);
  } else {
    if (with_h) hipLaunchKernelGGL((rotate_kernel<float, true>), grid, dim3(256), 0, st, r);
    else hipLaunchKernelGGL((rotate_kernel<float, false>), grid, dim3(256), 0, st, r);
  }
  return hipGetLastError();
}

hipError_t launch_fill(double* p, long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_variance(const double* S, const double* M, int m, int mp, double* re, double* re_perp, hipStream_t st) {
  hipLaunchKernelGGL(variance_kernel, dim3((m + 127) / 128), dim3(128), 0, st, S, M, m, mp, re, re_perp);
  return hipGetLastError();
}

}  // namespace mpe
