// Learned warm start: a small 3-D U-Net mapping a coarse potential (32^3) to
// starting orbitals, trained on the GPU by these kernels.
//
// Tensors are channels-last float32, periodic.  Convolutions (3x3x3 taps) are
// implicit GEMMs on v_mfma_f32_16x16x32_bf16: bfloat16 operands (weights and
// activations rounded on load), float32 accumulation.  Weights keep a float32
// master copy for Adam and bfloat16 copies in the two layouts the kernels read:
//   forward       Wf[co_pad][27][ci_pad]        k = tap * ci_pad + ci
//   data gradient Wb[ci_pad][27][co_pad]        (taps mirrored for stride 1)
// Architecture (channels 16/32/64, ReLU after every convolution but the head):
//   e1 = relu(c1b(relu(c1a(v))))            32^3, 16
//   e2 = relu(c2b(relu(c2a_s2(e1))))        16^3, 32
//   e3 = relu(c3b(relu(c3a_s2(e2))))         8^3, 64
//   d2 = relu(cd2([up(e3) | e2]))           16^3, 32
//   d1 = relu(cd1([up(d2) | e1]))           32^3, 16
//   y  = head(d1)                           32^3, n_out
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/mpe.h"
#include "la.hpp"

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan kept
  u += 0x7fffu + ((u >> 16) & 1u);                                          // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ unsigned int pack2(float a, float b) {
  return (unsigned int)f2bf(a) | ((unsigned int)f2bf(b) << 16);
}

enum ConvMode { CM_S1 = 0, CM_S2 = 1, CM_S2T = 2 };

struct ConvArgs {
  const float* x;            // input, channels-last [batch][din^3][x_cs]
  int x_cs, x_co;            // channel stride and offset of the input slice
  const unsigned short* w;   // bf16 weights [co_pad][27][cin_pad]
  const float* bias;         // nullable
  float* y;                  // output [batch][dout^3][y_cs]
  int y_cs, y_co;
  int cin_pad, co, co_pad;
  int din, dout, batch;
  int mode, relu, accumulate;
};

// source voxel of output voxel (oz, oy, ox) for tap (tz, ty, tx); -1 when the tap
// does not contribute (transposed stride-2 parity)
__device__ __forceinline__ int src_voxel(int mode, int din, int oz, int oy, int ox, int tz, int ty, int tx) {
  int sz, sy, sx;
  if (mode == CM_S1) {
    sz = oz + tz - 1; sy = oy + ty - 1; sx = ox + tx - 1;
  } else if (mode == CM_S2) {
    sz = 2 * oz + tz - 1; sy = 2 * oy + ty - 1; sx = 2 * ox + tx - 1;
  } else {
    const int qz = oz - tz + 1, qy = oy - ty + 1, qx = ox - tx + 1;
    if ((qz | qy | qx) & 1) return -1;
    sz = qz >> 1; sy = qy >> 1; sx = qx >> 1;
  }
  sz = (sz % din + din) % din;
  sy = (sy % din + din) % din;
  sx = (sx % din + din) % din;
  return (sz * din + sy) * din + sx;
}

// One work-group: 64 output voxels (16 per wave) x all output channels.
template <int MT>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int D3 = a.dout * a.dout * a.dout;
  const long nvox = (long)a.batch * D3;
  const long v = (long)blockIdx.x * 64 + wave * 16 + (lane & 15);
  const bool vok = v < nvox;
  const long vv = vok ? v : 0;
  const int b = (int)(vv / D3), o = (int)(vv % D3);
  const int oz = o / (a.dout * a.dout), oy = (o / a.dout) % a.dout, ox = o % a.dout;
  const int din3 = a.din * a.din * a.din;
  const int K = 27 * a.cin_pad;
  const int g = lane >> 4;
  f4v acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int k = k0 + 8 * g;          // this lane's 8 consecutive k (one tap, 8 channels)
    u4v bw = u4v{0u, 0u, 0u, 0u};
    if (k < K && vok) {
      const int tap = k / a.cin_pad, ci = k - tap * a.cin_pad;
      const int sv = src_voxel(a.mode, a.din, oz, oy, ox, tap / 9, (tap / 3) % 3, tap % 3);
      if (sv >= 0) {
        const float4* px = reinterpret_cast<const float4*>(a.x + ((long)b * din3 + sv) * a.x_cs + a.x_co + ci);
        const float4 lo = px[0], hi = px[1];
        bw = u4v{pack2(lo.x, lo.y), pack2(lo.z, lo.w), pack2(hi.x, hi.y), pack2(hi.z, hi.w)};
      }
    }
    const bf8 bv = __builtin_bit_cast(bf8, bw);
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      u4v aw = u4v{0u, 0u, 0u, 0u};
      if (k < K) aw = *reinterpret_cast<const u4v*>(a.w + (long)(t * 16 + (lane & 15)) * K + k);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, aw), bv, acc[t], 0, 0, 0);
    }
  }
  if (!vok) return;
  float* yo = a.y + ((long)b * D3 + o) * a.y_cs + a.y_co;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = t * 16 + 4 * g + r;   // D[4(l/16)+r][l%16]: row = channel, column = voxel
      if (co < a.co) {
        float val = acc[t][r] + (a.bias ? a.bias[co] : 0.f);
        if (a.accumulate) val += yo[co];
        if (a.relu) val = fmaxf(val, 0.f);
        yo[co] = val;
      }
    }
}

// dW[co][tap][ci] += sum_v dz[v][co] * x[src(v, tap)][ci]   (float32 atomics)
struct WgradArgs {
  const float* dz; int dz_cs;          // gradient of the pre-activation [batch][dout^3][dz_cs]
  const float* x; int x_cs, x_co;      // layer input slice
  float* dw;                           // [co][27][ci]
  int ci, cin_pad, co;
  int din, dout, batch, mode;
  long vox_per_block;
};

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int ncol = 27 * a.ci;                               // real (tap, ci) columns
  const int col_tiles = (ncol + 15) / 16, co_tiles = (a.co + 15) / 16;
  const int tile = blockIdx.y * 4 + wave;
  if (tile >= col_tiles * co_tiles) return;
  const int ti = tile / col_tiles, tj = tile % col_tiles;
  const int D3 = a.dout * a.dout * a.dout, din3 = a.din * a.din * a.din;
  const long nvox = (long)a.batch * D3;
  const long v_begin = (long)blockIdx.x * a.vox_per_block;
  const long v_end = v_begin + a.vox_per_block < nvox ? v_begin + a.vox_per_block : nvox;
  const int co_a = ti * 16 + j;                             // A row (channel) of this lane
  const int cj = tj * 16 + j;                               // B column of this lane
  const int tap = cj / a.ci, ci = cj - tap * a.ci;
  const bool col_ok = cj < ncol, co_ok = co_a < a.co;
  f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
  for (long v0 = v_begin; v0 < v_end; v0 += 32) {
    float av[8], bv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const long v = v0 + 8 * g + e;
      av[e] = 0.f;
      bv[e] = 0.f;
      if (v < v_end) {
        const int b = (int)(v / D3), o = (int)(v % D3);
        if (co_ok) av[e] = a.dz[v * a.dz_cs + co_a];
        if (col_ok) {
          const int oz = o / (a.dout * a.dout), oy = (o / a.dout) % a.dout, ox = o % a.dout;
          const int sv = src_voxel(a.mode, a.din, oz, oy, ox, tap / 9, (tap / 3) % 3, tap % 3);
          bv[e] = a.x[((long)b * din3 + sv) * a.x_cs + a.x_co + ci];
        }
      }
    }
    const u4v aw = u4v{pack2(av[0], av[1]), pack2(av[2], av[3]), pack2(av[4], av[5]), pack2(av[6], av[7])};
    const u4v bw = u4v{pack2(bv[0], bv[1]), pack2(bv[2], bv[3]), pack2(bv[4], bv[5]), pack2(bv[6], bv[7])};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, aw), __builtin_bit_cast(bf8, bw), acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int co = ti * 16 + 4 * g + r, c = tj * 16 + j;
    if (co < a.co && c < ncol) {
      const int tp = c / a.ci, cc = c - tp * a.ci;
      atomicAdd(a.dw + ((long)co * 27 + tp) * a.ci + cc, acc[r]);
    }
  }
}

// db[co] += sum_v dz[v][co]
__global__ void bgrad_kernel(const float* dz, int dz_cs, long nvox, int co, float* db) {
  __shared__ float red[256];
  const int c = blockIdx.y;
  float s = 0.f;
  for (long v = (long)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (long)gridDim.x * 256) s += dz[v * dz_cs + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(db + c, red[0]);
}

// g[v][c] *= (out[v][c] > 0)
__global__ void relu_back_kernel(float* g, int g_cs, const float* out, int out_cs, int out_co, long nvox, int c) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * c) return;
  const long v = i / c;
  const int ch = (int)(i - v * c);
  if (!(out[v * out_cs + out_co + ch] > 0.f)) g[v * g_cs + ch] = 0.f;
}

// nearest doubling into a channel slice: y[b][2o + d][y_co + ch] = x[b][o][x_co + ch]
__global__ void up2_kernel(const float* x, int x_cs, int x_co, float* y, int y_cs, int y_co, int din, int batch, int c) {
  const int dout = 2 * din;
  const long n = (long)batch * dout * dout * dout * c;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ch = (int)(i % c);
  const long v = i / c;
  const int D3 = dout * dout * dout;
  const int b = (int)(v / D3), o = (int)(v % D3);
  const int z = o / (dout * dout), yy = (o / dout) % dout, xx = o % dout;
  const long s = (long)b * din * din * din + ((z / 2) * din + yy / 2) * din + xx / 2;
  y[v * y_cs + y_co + ch] = x[s * x_cs + x_co + ch];
}

// adjoint of up2: x[b][o][ch] (+)= sum over the 8 children of g[child][g_co + ch]
__global__ void up2_back_kernel(const float* g, int g_cs, int g_co, float* x, int x_cs, int din, int batch, int c,
                                int accumulate) {
  const long n = (long)batch * din * din * din * c;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ch = (int)(i % c);
  const long v = i / c;
  const int D3 = din * din * din, dout = 2 * din;
  const int b = (int)(v / D3), o = (int)(v % D3);
  const int z = o / (din * din), yy = (o / din) % din, xx = o % din;
  float s = 0.f;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const long cidx = (long)b * dout * dout * dout + ((2 * z + dz) * dout + 2 * yy + dy) * dout + 2 * xx + dx;
        s += g[cidx * g_cs + g_co + ch];
      }
  if (accumulate) x[v * x_cs + ch] += s;
  else x[v * x_cs + ch] = s;
}

// y[v][ch] = x[v][x_co + ch]
__global__ void copy_slice_kernel(const float* x, int x_cs, int x_co, float* y, int y_cs, long nvox, int c) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * c) return;
  const long v = i / c;
  const int ch = (int)(i - v * c);
  y[v * y_cs + ch] = x[v * x_cs + x_co + ch];
}

// scale * ([b][P][n] <-> [b][n][P])
__global__ void transpose_kernel(const float* x, float* y, long P, int n, int batch, int to_states, float scale) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)batch * P * n) return;
  const long b = i / (P * n), r = i - b * P * n;
  if (to_states) {            // x [b][P][n] -> y [b][n][P], i runs over y
    const long s = r / P, p = r - s * P;
    y[i] = scale * x[b * P * n + p * n + s];
  } else {                    // x [b][n][P] -> y [b][P][n], i runs over y
    const long p = r / n, s = r - p * n;
    y[i] = scale * x[b * P * n + s * P + p];
  }
}

// potential [b][P] -> channels-last input [b][P][8] (channel 0, the rest zero), scaled
__global__ void input_kernel(const float* vin, float scale, float* x, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * 8) return;
  x[i] = (i % 8 == 0) ? vin[i / 8] * scale : 0.f;
}

// Adam with bias correction on float32 master weights
__global__ void adam_kernel(float* p, float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  g[i] = 0.f;
}

// bf16 weight copies: forward Wf[co_pad][27][ci_pad]; data-gradient Wb[ci_rows][27][co]
// (ci_rows = ci rounded up to 16; co is a multiple of 8 for every layer)
__global__ void pack_weights_kernel(const float* w, int co, int ci, int co_pad, int ci_pad, int ci_rows, int mirror,
                                    unsigned short* wf, unsigned short* wb) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nf = (long)co_pad * 27 * ci_pad;
  if (i < nf) {
    const int o = (int)(i / (27 * ci_pad)), r = (int)(i % (27 * ci_pad)), t = r / ci_pad, c = r % ci_pad;
    wf[i] = (o < co && c < ci) ? f2bf(w[((long)o * 27 + t) * ci + c]) : 0;
  }
  const long nb = (long)ci_rows * 27 * co;
  if (i < nb && wb) {
    const int c = (int)(i / (27 * co)), r = (int)(i % (27 * co)), t = r / co, o = r % co;
    const int ts = mirror ? 26 - t : t;
    wb[i] = (c < ci) ? f2bf(w[((long)o * 27 + ts) * ci + c]) : 0;
  }
}

// periodic trilinear up-sampling of [C][d^3] by `factor` per axis
__global__ void upsample_kernel(const float* u, int C, int d, int factor, float* out) {
  const int D = d * factor;
  const long n = (long)C * D * D * D;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long c = i / ((long)D * D * D);
  const int r = (int)(i - c * (long)D * D * D);
  const int Z = r / (D * D), Y = (r / D) % D, X = r % D;
  const float inv = 1.f / factor;
  const int z0 = Z / factor, y0 = Y / factor, x0 = X / factor;
  const float wz = (Z - z0 * factor) * inv, wy = (Y - y0 * factor) * inv, wx = (X - x0 * factor) * inv;
  const int z1 = (z0 + 1) % d, y1 = (y0 + 1) % d, x1 = (x0 + 1) % d;
  const float* uc = u + c * (long)d * d * d;
  auto at = [&](int z, int y, int x) { return uc[(z * d + y) * d + x]; };
  const float v00 = (1 - wx) * at(z0, y0, x0) + wx * at(z0, y0, x1);
  const float v01 = (1 - wx) * at(z0, y1, x0) + wx * at(z0, y1, x1);
  const float v10 = (1 - wx) * at(z1, y0, x0) + wx * at(z1, y0, x1);
  const float v11 = (1 - wx) * at(z1, y1, x0) + wx * at(z1, y1, x1);
  out[i] = (1 - wz) * ((1 - wy) * v00 + wy * v01) + wz * ((1 - wy) * v10 + wy * v11);
}

// subspace-loss helpers ------------------------------------------------------
// One work-group.  M = Y T^T and S = T T^T (mp x mp, float64).  G = M M^T - I and
// B = 4 G M - 2 M (n x n; G kept in global scratch, visible to the work-group
// after the barrier); B is stored transposed for the rotation kernel.
//   ||Y - M T||^2 = ||Y||^2 - 2 ||M||^2 + tr(M S M^T)
// loss = {||Y - M T||^2 + ||G||^2, ||G||^2}.
__global__ __launch_bounds__(1024) void loss_small_kernel(const double* M, const double* S, int n, int mp,
                                                          const double* y2, double* G, double* Bt, double* loss) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  double l2 = 0.0, r2 = 0.0;
  for (int e = tid; e < n * n; e += 1024) {
    const int i = e / n, j = e % n;
    double s = 0.0, ms = 0.0;
    for (int k = 0; k < n; ++k) {
      s += M[(long)i * mp + k] * M[(long)j * mp + k];
      ms += M[(long)i * mp + k] * S[(long)k * mp + j];
    }
    if (i == j) s -= 1.0;
    G[e] = s;
    l2 += s * s;
    const double mij = M[(long)i * mp + j];
    r2 += ms * mij - 2.0 * mij * mij;
  }
  __syncthreads();
  for (int e = tid; e < mp * mp; e += 1024) {
    const int i = e / mp, j = e % mp;
    double s = 0.0;
    if (i < n && j < n) {
      for (int k = 0; k < n; ++k) s += G[i * n + k] * M[(long)k * mp + j];
      s = 4.0 * s - 2.0 * M[(long)i * mp + j];
    }
    Bt[(long)j * mp + i] = s;
  }
  red[tid] = l2;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double L2 = red[0];
  __syncthreads();
  red[tid] = r2;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    loss[0] = y2[0] + red[0] + L2;
    loss[1] = L2;
  }
}

// A = M^T M (n x n in an mp x mp buffer, zero padded); Sid = identity
__global__ __launch_bounds__(256) void ata_kernel(const double* M, int n, int mp, double* A, double* Sid) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < mp * mp; e += gridDim.x * 256) {
    const int i = e / mp, j = e % mp;
    double s = 0.0;
    if (i < n && j < n)
      for (int k = 0; k < n; ++k) s += M[(long)k * mp + i] * M[(long)k * mp + j];
    A[e] = s;
    Sid[e] = (i == j) ? 1.0 : 0.0;
  }
}

// Polar factor Q = M U diag(theta)^(-1/2) U^T from the eigenpairs (theta, U) of
// M^T M (U's columns in an mp x mp buffer), then
//   loss = {||Y||^2 - 2 tr(Q^T M) + tr(Q S Q^T), sum_k sqrt(theta_k)}
// and Bt[j][i] = -2 Q[i][j] (the rotation kernel then forms -2 Q T).
// One work-group; W and Q in global scratch (visible after the barriers).
__global__ __launch_bounds__(1024) void polar_kernel(const double* M, const double* S, const double* U,
                                                     const double* theta, const int* status, int n, int mp,
                                                     const double* y2, double* W, double* Q, double* Bt,
                                                     double* loss) {
  __shared__ double red[1024];
  __shared__ double isq[mpe::MAXM];
  const int tid = threadIdx.x;
  if (status[0] != 0) {
    if (tid == 0) loss[0] = loss[1] = __builtin_nan("");
    return;
  }
  double tmax = 0.0;
  for (int k = 0; k < n; ++k) tmax = fmax(tmax, theta[k]);
  const double floor_ = 1e-12 * tmax;
  double nuc = 0.0;
  for (int k = tid; k < n; k += 1024) {
    const double t = fmax(theta[k], floor_);
    isq[k] = 1.0 / sqrt(t);
  }
  if (tid == 0)
    for (int k = 0; k < n; ++k) nuc += sqrt(fmax(theta[k], 0.0));
  __syncthreads();
  for (int e = tid; e < n * n; e += 1024) {   // W = M U diag(theta^-1/2)
    const int i = e / n, k = e % n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += M[(long)i * mp + j] * U[(long)j * mp + k];
    W[e] = s * isq[k];
  }
  __syncthreads();
  double tqm = 0.0;
  for (int e = tid; e < n * n; e += 1024) {   // Q = W U^T
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += W[i * n + k] * U[(long)j * mp + k];
    Q[e] = s;
    tqm += s * M[(long)i * mp + j];
  }
  __syncthreads();
  double tqsq = 0.0;
  for (int e = tid; e < mp * mp; e += 1024) {
    const int i = e / mp, j = e % mp;
    double b = 0.0;
    if (i < n && j < n) {
      b = -2.0 * Q[i * n + j];
      double qs = 0.0;
      for (int l = 0; l < n; ++l) qs += S[(long)j * mp + l] * Q[i * n + l];
      tqsq += Q[i * n + j] * qs;
    }
    Bt[(long)j * mp + i] = b;
  }
  red[tid] = tqsq - 2.0 * tqm;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    loss[0] = y2[0] + red[0];
    loss[1] = nuc;
  }
}

__global__ void sumsq_kernel(const float* y, long n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) s += (double)y[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// dy = 2 y + t   (t = B T from the rotation kernel)
__global__ void axpy2_kernel(const float* y, float* t, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] += 2.f * y[i];
}

unsigned nblk(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------ network description
struct Layer {
  const char* name;
  int ci, co, stride, relu;
  int ci_pad, co_pad;
  long w_off, b_off;            // offsets in the parameter vector
  unsigned short *wf, *wb;      // bf16 copies
};

}  // namespace

struct wsn_net_s {
  int D = 32, n_out = 120, max_batch = 1;
  hipStream_t st = nullptr;
  std::string err;
  std::vector<Layer> layers;
  long nparam = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  // activations (channels-last) for max_batch
  float *x0 = nullptr, *a1 = nullptr, *cat1 = nullptr, *a2 = nullptr, *cat2 = nullptr, *a3 = nullptr, *e3 = nullptr,
        *d2 = nullptr, *d1 = nullptr, *yo = nullptr;
  // gradients
  float *g_y = nullptr, *g_d1 = nullptr, *g_cat1 = nullptr, *g_d2 = nullptr, *g_cat2 = nullptr, *g_e3 = nullptr,
        *g_a3 = nullptr, *g_e2 = nullptr, *g_a2 = nullptr, *g_e1 = nullptr, *g_a1 = nullptr;
  double* scratch = nullptr;   // loss: gram partials, M, B, loss values
  size_t scratch_bytes = 0;
  int batch = 0;               // batch of the last forward
  float yscale = 1.f;          // output scale of the last forward
  std::vector<void*> allocs;
};

namespace {

mpe_status wfail(wsn_net n, mpe_status s, const std::string& msg) {
  if (n) n->err = msg;
  return s;
}

#define WHIP(n, expr)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return wfail(n, MPE_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

hipError_t conv(wsn_net n, const Layer& L, const float* x, int x_cs, int x_co, float* y, int y_cs, int y_co, int din,
                int dout, int mode, bool fwd_weights, int co, int cin_pad, int relu, int acc, const float* bias) {
  ConvArgs a;
  a.x = x;
  a.x_cs = x_cs;
  a.x_co = x_co;
  a.w = fwd_weights ? L.wf : L.wb;
  a.bias = bias;
  a.y = y;
  a.y_cs = y_cs;
  a.y_co = y_co;
  a.cin_pad = cin_pad;
  a.co = co;
  a.co_pad = (co + 15) / 16 * 16;
  a.din = din;
  a.dout = dout;
  a.batch = n->batch;
  a.mode = mode;
  a.relu = relu;
  a.accumulate = acc;
  const long nvox = (long)n->batch * dout * dout * dout;
  dim3 grid(nblk(nvox, 64)), block(256);
  switch (a.co_pad / 16) {
    case 1: hipLaunchKernelGGL(conv_kernel<1>, grid, block, 0, n->st, a); break;
    case 2: hipLaunchKernelGGL(conv_kernel<2>, grid, block, 0, n->st, a); break;
    case 3: hipLaunchKernelGGL(conv_kernel<3>, grid, block, 0, n->st, a); break;
    case 4: hipLaunchKernelGGL(conv_kernel<4>, grid, block, 0, n->st, a); break;
    case 5: hipLaunchKernelGGL(conv_kernel<5>, grid, block, 0, n->st, a); break;
    case 6: hipLaunchKernelGGL(conv_kernel<6>, grid, block, 0, n->st, a); break;
    case 7: hipLaunchKernelGGL(conv_kernel<7>, grid, block, 0, n->st, a); break;
    case 8: hipLaunchKernelGGL(conv_kernel<8>, grid, block, 0, n->st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// forward layer: y = act(conv(x) + b)
hipError_t fwd(wsn_net n, int li, const float* x, int x_cs, int x_co, float* y, int y_cs, int y_co, int din) {
  const Layer& L = n->layers[li];
  const int dout = din / L.stride;
  return conv(n, L, x, x_cs, x_co, y, y_cs, y_co, din, dout, L.stride == 2 ? CM_S2 : CM_S1, true, L.co, L.ci_pad,
              L.relu, 0, n->p + L.b_off);
}

// backward of layer li: gz (its output gradient, channels-last, stride gz_cs) is
// turned into the pre-activation gradient in place; weight and bias gradients
// accumulate; the input gradient is written (or added) to gx (stride gx_cs)
// unless gx is null.
hipError_t bwd(wsn_net n, int li, float* gz, int gz_cs, const float* out, int out_cs, int out_co, const float* x,
               int x_cs, int x_co, float* gx, int gx_cs, int gx_acc, int din) {
  const Layer& L = n->layers[li];
  const int dout = din / L.stride;
  const long nvox = (long)n->batch * dout * dout * dout;
  if (L.relu) {
    hipLaunchKernelGGL(relu_back_kernel, dim3(nblk(nvox * L.co)), dim3(256), 0, n->st, gz, gz_cs, out, out_cs, out_co,
                       nvox, L.co);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  WgradArgs w;
  w.dz = gz;
  w.dz_cs = gz_cs;
  w.x = x;
  w.x_cs = x_cs;
  w.x_co = x_co;
  w.dw = n->g + L.w_off;
  w.ci = L.ci;
  w.cin_pad = L.ci_pad;
  w.co = L.co;
  w.din = din;
  w.dout = dout;
  w.batch = n->batch;
  w.mode = L.stride == 2 ? CM_S2 : CM_S1;
  w.vox_per_block = 4096;
  const int tiles = ((27 * L.ci + 15) / 16) * ((L.co + 15) / 16);
  hipLaunchKernelGGL(wgrad_kernel, dim3(nblk(nvox, 4096), (tiles + 3) / 4), dim3(256), 0, n->st, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bgrad_kernel, dim3(64, L.co), dim3(256), 0, n->st, (const float*)gz, gz_cs, nvox, L.co,
                     n->g + L.b_off);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!gx) return hipSuccess;
  // data gradient: a convolution of gz with the mirrored / transposed weights
  return conv(n, L, gz, gz_cs, 0, gx, gx_cs, 0, dout, din, L.stride == 2 ? CM_S2T : CM_S1, false, L.ci, L.co,
              0, gx_acc, nullptr);
}

hipError_t pack_all(wsn_net n) {
  for (auto& L : n->layers) {
    const int ci_rows = (L.ci + 15) / 16 * 16;
    const long nmax = std::max((long)L.co_pad * 27 * L.ci_pad, (long)ci_rows * 27 * L.co);
    hipLaunchKernelGGL(pack_weights_kernel, dim3(nblk(nmax)), dim3(256), 0, n->st, (const float*)(n->p + L.w_off), L.co,
                       L.ci, L.co_pad, L.ci_pad, ci_rows, L.stride == 1 ? 1 : 0, L.wf, L.wb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

mpe_status wsn_destroy(wsn_net n) {
  if (!n) return MPE_ERR_INVALID_ARGUMENT;
  (void)hipStreamSynchronize(n->st);
  for (void* a : n->allocs) (void)hipFree(a);
  delete n;
  return MPE_OK;
}

mpe_status wsn_create(wsn_net* out, int32_t grid, int32_t n_out, int32_t max_batch, uint64_t seed, void* hip_stream) {
  if (!out) return MPE_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (grid < 8 || grid % 4 || n_out < 1 || n_out > mpe::MAXM || n_out % 8 || max_batch < 1)
    return MPE_ERR_INVALID_ARGUMENT;
  wsn_net n = new wsn_net_s();
  n->D = grid;
  n->n_out = n_out;
  n->max_batch = max_batch;
  n->st = reinterpret_cast<hipStream_t>(hip_stream);
  if (mpe::prepare_small_dense() != hipSuccess) {
    delete n;
    return MPE_ERR_DEVICE;
  }
  struct Spec { const char* name; int ci, co, stride, relu, ci_pad; };
  const Spec spec[] = {{"c1a", 1, 16, 1, 1, 8},   {"c1b", 16, 16, 1, 1, 16}, {"c2a", 16, 32, 2, 1, 16},
                       {"c2b", 32, 32, 1, 1, 32}, {"c3a", 32, 64, 2, 1, 32}, {"c3b", 64, 64, 1, 1, 64},
                       {"d2", 96, 32, 1, 1, 96},  {"d1", 48, 16, 1, 1, 48},  {"head", 16, n_out, 1, 0, 16}};
  long off = 0;
  for (const auto& s : spec) {
    Layer L;
    L.name = s.name;
    L.ci = s.ci;
    L.co = s.co;
    L.stride = s.stride;
    L.relu = s.relu;
    L.ci_pad = s.ci_pad;
    L.co_pad = (s.co + 15) / 16 * 16;
    L.w_off = off;
    off += (long)s.co * 27 * s.ci;
    L.b_off = off;
    off += s.co;
    L.wf = L.wb = nullptr;
    n->layers.push_back(L);
  }
  n->nparam = off;
  auto alloc = [&](void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) return false;
    n->allocs.push_back(*p);
    return hipMemsetAsync(*p, 0, bytes, n->st) == hipSuccess;
  };
  const long B = max_batch, D = grid, v32 = D * D * D, v16 = v32 / 8, v8 = v16 / 8;
  bool ok = alloc((void**)&n->p, off * 4) && alloc((void**)&n->g, off * 4) && alloc((void**)&n->m, off * 4) &&
            alloc((void**)&n->v, off * 4);
  for (auto& L : n->layers) {
    ok = ok && alloc((void**)&L.wf, (size_t)L.co_pad * 27 * L.ci_pad * 2) &&
         alloc((void**)&L.wb, (size_t)((L.ci + 15) / 16 * 16) * 27 * L.co * 2);
  }
  ok = ok && alloc((void**)&n->x0, B * v32 * 8 * 4) && alloc((void**)&n->a1, B * v32 * 16 * 4) &&
       alloc((void**)&n->cat1, B * v32 * 48 * 4) && alloc((void**)&n->a2, B * v16 * 32 * 4) &&
       alloc((void**)&n->cat2, B * v16 * 96 * 4) && alloc((void**)&n->a3, B * v8 * 64 * 4) &&
       alloc((void**)&n->e3, B * v8 * 64 * 4) && alloc((void**)&n->d2, B * v16 * 32 * 4) &&
       alloc((void**)&n->d1, B * v32 * 16 * 4) && alloc((void**)&n->yo, B * v32 * n_out * 4);
  ok = ok && alloc((void**)&n->g_y, B * v32 * n_out * 4) && alloc((void**)&n->g_d1, B * v32 * 16 * 4) &&
       alloc((void**)&n->g_cat1, B * v32 * 48 * 4) && alloc((void**)&n->g_d2, B * v16 * 32 * 4) &&
       alloc((void**)&n->g_cat2, B * v16 * 96 * 4) && alloc((void**)&n->g_e3, B * v8 * 64 * 4) &&
       alloc((void**)&n->g_a3, B * v8 * 64 * 4) && alloc((void**)&n->g_e2, B * v16 * 32 * 4) &&
       alloc((void**)&n->g_a2, B * v16 * 32 * 4) && alloc((void**)&n->g_e1, B * v32 * 16 * 4) &&
       alloc((void**)&n->g_a1, B * v32 * 16 * 4);
  // loss scratch: gram partials (2 products x <= 128 chunks), M and S, B^T, G (then W), A, Sid, L, rot, U, Q,
  // theta, small-dense scratch, status, loss values
  n->scratch_bytes = ((size_t)256 * 128 * 128 + 11 * 128 * 128 + 128 + 256 + 16 + 16 +
                      mpe::small_dense_rot_doubles(60)) * sizeof(double);
  ok = ok && alloc((void**)&n->scratch, n->scratch_bytes);
  if (!ok) {
    wsn_destroy(n);
    return MPE_ERR_OUT_OF_MEMORY;
  }
  // He-normal initial weights from the seed (host generator), zero biases
  std::vector<float> hp(off, 0.f);
  std::mt19937_64 rng(seed);
  for (auto& L : n->layers) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (27.f * L.ci)));
    for (long i = 0; i < (long)L.co * 27 * L.ci; ++i) hp[L.w_off + i] = nd(rng);
  }
  if (hipMemcpyAsync(n->p, hp.data(), off * 4, hipMemcpyHostToDevice, n->st) != hipSuccess || pack_all(n) != hipSuccess ||
      hipStreamSynchronize(n->st) != hipSuccess) {
    wsn_destroy(n);
    return MPE_ERR_DEVICE;
  }
  *out = n;
  return MPE_OK;
}

const char* wsn_last_error(wsn_net n) { return n ? n->err.c_str() : "null network"; }

int64_t wsn_num_params(wsn_net n) { return n ? n->nparam : -1; }

mpe_status wsn_get_params(wsn_net n, float* host, int32_t which) {
  if (!n || !host) return MPE_ERR_INVALID_ARGUMENT;
  const float* src = which == 0 ? n->p : which == 1 ? n->g : nullptr;
  if (!src) return wfail(n, MPE_ERR_INVALID_ARGUMENT, "which must be 0 (parameters) or 1 (gradients)");
  WHIP(n, hipMemcpyAsync(host, src, n->nparam * 4, hipMemcpyDeviceToHost, n->st));
  WHIP(n, hipStreamSynchronize(n->st));
  return MPE_OK;
}

mpe_status wsn_set_params(wsn_net n, const float* host) {
  if (!n || !host) return MPE_ERR_INVALID_ARGUMENT;
  WHIP(n, hipMemcpyAsync(n->p, host, n->nparam * 4, hipMemcpyHostToDevice, n->st));
  WHIP(n, pack_all(n));
  WHIP(n, hipStreamSynchronize(n->st));
  return MPE_OK;
}

mpe_status wsn_zero_grads(wsn_net n) {
  if (!n) return MPE_ERR_INVALID_ARGUMENT;
  WHIP(n, hipMemsetAsync(n->g, 0, n->nparam * 4, n->st));
  return MPE_OK;
}

mpe_status wsn_forward(wsn_net n, const float* v, float vscale, float yscale, int32_t batch, float* y) {
  if (!n || !v || !y) return MPE_ERR_INVALID_ARGUMENT;
  if (batch < 1 || batch > n->max_batch) return wfail(n, MPE_ERR_INVALID_ARGUMENT, "batch out of range");
  n->batch = batch;
  n->yscale = yscale;
  const int D = n->D, h = D / 2, q = D / 4;
  const long v32 = (long)D * D * D;
  hipLaunchKernelGGL(input_kernel, dim3(nblk(batch * v32 * 8)), dim3(256), 0, n->st, v, vscale, n->x0, batch * v32);
  WHIP(n, hipGetLastError());
  WHIP(n, fwd(n, 0, n->x0, 8, 0, n->a1, 16, 0, D));         // c1a
  WHIP(n, fwd(n, 1, n->a1, 16, 0, n->cat1, 48, 32, D));     // c1b -> e1 = cat1[32:48]
  WHIP(n, fwd(n, 2, n->cat1, 48, 32, n->a2, 32, 0, D));     // c2a (stride 2)
  WHIP(n, fwd(n, 3, n->a2, 32, 0, n->cat2, 96, 64, h));     // c2b -> e2 = cat2[64:96]
  WHIP(n, fwd(n, 4, n->cat2, 96, 64, n->a3, 64, 0, h));     // c3a (stride 2)
  WHIP(n, fwd(n, 5, n->a3, 64, 0, n->e3, 64, 0, q));        // c3b -> e3
  hipLaunchKernelGGL(up2_kernel, dim3(nblk(batch * (v32 / 8) * 64)), dim3(256), 0, n->st, (const float*)n->e3, 64, 0,
                     n->cat2, 96, 0, q, batch, 64);
  WHIP(n, hipGetLastError());
  WHIP(n, fwd(n, 6, n->cat2, 96, 0, n->d2, 32, 0, h));      // d2
  hipLaunchKernelGGL(up2_kernel, dim3(nblk(batch * v32 * 32)), dim3(256), 0, n->st, (const float*)n->d2, 32, 0,
                     n->cat1, 48, 0, h, batch, 32);
  WHIP(n, hipGetLastError());
  WHIP(n, fwd(n, 7, n->cat1, 48, 0, n->d1, 16, 0, D));      // d1
  WHIP(n, fwd(n, 8, n->d1, 16, 0, n->yo, n->n_out, 0, D));  // head
  hipLaunchKernelGGL(transpose_kernel, dim3(nblk(batch * v32 * n->n_out)), dim3(256), 0, n->st, (const float*)n->yo, y,
                     v32, n->n_out, batch, 1, yscale);
  WHIP(n, hipGetLastError());
  return MPE_OK;
}

mpe_status wsn_backward(wsn_net n, const float* dy) {
  if (!n || !dy) return MPE_ERR_INVALID_ARGUMENT;
  if (n->batch < 1) return wfail(n, MPE_ERR_STATE, "backward before forward");
  const int B = n->batch, D = n->D, h = D / 2, q = D / 4;
  const long v32 = (long)D * D * D, v16 = v32 / 8, v8 = v16 / 8;
  hipLaunchKernelGGL(transpose_kernel, dim3(nblk(B * v32 * n->n_out)), dim3(256), 0, n->st, dy, n->g_y, v32, n->n_out, B,
                     0, n->yscale);
  WHIP(n, hipGetLastError());
  WHIP(n, bwd(n, 8, n->g_y, n->n_out, n->yo, n->n_out, 0, n->d1, 16, 0, n->g_d1, 16, 0, D));            // head
  WHIP(n, bwd(n, 7, n->g_d1, 16, n->d1, 16, 0, n->cat1, 48, 0, n->g_cat1, 48, 0, D));                  // d1
  hipLaunchKernelGGL(up2_back_kernel, dim3(nblk(B * v16 * 32)), dim3(256), 0, n->st, (const float*)n->g_cat1, 48, 0,
                     n->g_d2, 32, h, B, 32, 0);
  WHIP(n, hipGetLastError());
  hipLaunchKernelGGL(copy_slice_kernel, dim3(nblk(B * v32 * 16)), dim3(256), 0, n->st, (const float*)n->g_cat1, 48, 32,
                     n->g_e1, 16, B * v32, 16);
  WHIP(n, hipGetLastError());
  WHIP(n, bwd(n, 6, n->g_d2, 32, n->d2, 32, 0, n->cat2, 96, 0, n->g_cat2, 96, 0, h));                  // d2
  hipLaunchKernelGGL(up2_back_kernel, dim3(nblk(B * v8 * 64)), dim3(256), 0, n->st, (const float*)n->g_cat2, 96, 0,
                     n->g_e3, 64, q, B, 64, 0);
  WHIP(n, hipGetLastError());
  hipLaunchKernelGGL(copy_slice_kernel, dim3(nblk(B * v16 * 32)), dim3(256), 0, n->st, (const float*)n->g_cat2, 96, 64,
                     n->g_e2, 32, B * v16, 32);
  WHIP(n, hipGetLastError());
  WHIP(n, bwd(n, 5, n->g_e3, 64, n->e3, 64, 0, n->a3, 64, 0, n->g_a3, 64, 0, q));                      // c3b
  WHIP(n, bwd(n, 4, n->g_a3, 64, n->a3, 64, 0, n->cat2, 96, 64, n->g_e2, 32, 1, h));                   // c3a
  WHIP(n, bwd(n, 3, n->g_e2, 32, n->cat2, 96, 64, n->a2, 32, 0, n->g_a2, 32, 0, h));                   // c2b
  WHIP(n, bwd(n, 2, n->g_a2, 32, n->a2, 32, 0, n->cat1, 48, 32, n->g_e1, 16, 1, D));                   // c2a
  WHIP(n, bwd(n, 1, n->g_e1, 16, n->cat1, 48, 32, n->a1, 16, 0, n->g_a1, 16, 0, D));                   // c1b
  WHIP(n, bwd(n, 0, n->g_a1, 16, n->a1, 16, 0, n->x0, 8, 0, nullptr, 0, 0, D));                        // c1a
  return MPE_OK;
}

mpe_status wsn_layer_info(wsn_net n, int32_t layer, int32_t* info) {
  if (!n || !info || layer < 0 || layer >= (int)n->layers.size()) return MPE_ERR_INVALID_ARGUMENT;
  const Layer& L = n->layers[layer];
  info[0] = L.ci;
  info[1] = L.co;
  info[2] = L.ci_pad;
  info[3] = L.stride;
  info[4] = L.relu;
  return MPE_OK;
}

mpe_status wsn_layer(wsn_net n, int32_t layer, int32_t batch, int32_t din, const float* x, float* y, float* dz,
                     float* dx) {
  if (!n || !x || !y) return MPE_ERR_INVALID_ARGUMENT;
  if (layer < 0 || layer >= (int)n->layers.size()) return wfail(n, MPE_ERR_INVALID_ARGUMENT, "no such layer");
  const Layer& L = n->layers[layer];
  if (batch < 1 || batch > n->max_batch) return wfail(n, MPE_ERR_INVALID_ARGUMENT, "batch out of range");
  if (din < 2 * L.stride || din % (2 * L.stride)) return wfail(n, MPE_ERR_INVALID_ARGUMENT, "bad grid size");
  n->batch = batch;
  WHIP(n, fwd(n, layer, x, L.ci_pad, 0, y, L.co, 0, din));
  if (!dz) return MPE_OK;
  WHIP(n, bwd(n, layer, dz, L.co, y, L.co, 0, x, L.ci_pad, 0, dx, L.ci, 0, din));
  return MPE_OK;
}

mpe_status wsn_adam_step(wsn_net n, float lr, float beta1, float beta2, float eps, int32_t t) {
  if (!n || t < 1) return MPE_ERR_INVALID_ARGUMENT;
  const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3(nblk(n->nparam)), dim3(256), 0, n->st, n->p, n->g, n->m, n->v, n->nparam, lr,
                     beta1, beta2, eps, c1, c2);
  WHIP(n, hipGetLastError());
  WHIP(n, pack_all(n));
  return MPE_OK;
}

mpe_status wsn_subspace_loss(wsn_net n, const float* y, const float* target, int32_t n_states, int64_t P,
                             double* loss_host, float* dy) {
  if (!n || !y || !target || !dy || n_states < 1 || n_states > mpe::MAXM || P < 1)
    return MPE_ERR_INVALID_ARGUMENT;
  if ((const float*)dy == y) return wfail(n, MPE_ERR_INVALID_ARGUMENT, "dy must not alias y");
  const int mp = (n_states + 15) / 16 * 16;
  long nch = std::min<long>(128, std::max<long>(1, (P + 4095) / 4096));
  long chunk = ((P + nch - 1) / nch + 31) / 32 * 32;
  nch = (P + chunk - 1) / chunk;
  double* partials = n->scratch;             // [2][nch][mp][mp]
  double* M = partials + 256L * 128 * 128;   // M then S, each mp x mp
  double* S = M + (long)mp * mp;
  double* Bt = M + 2L * 128 * 128;
  double* G = Bt + 128 * 128;
  double* lv = G + 128 * 128;                // [||y||^2, loss, ||G||^2]
  mpe::GramArgs g;
  std::memset(&g, 0, sizeof(g));
  g.X[0] = y;
  g.Y[0] = target;
  g.X[1] = target;
  g.Y[1] = target;
  g.partials = partials;
  g.N = P;
  g.chunk = chunk;
  g.m = n_states;
  g.mp = mp;
  WHIP(n, mpe::launch_gram(0, g, 2, (int)nch, n->st));
  WHIP(n, mpe::launch_reduce(partials, (int)nch, (long)mp * mp, 2, M, n->st));
  WHIP(n, hipMemsetAsync(lv, 0, sizeof(double), n->st));
  hipLaunchKernelGGL(sumsq_kernel, dim3(256), dim3(256), 0, n->st, y, (long)n_states * P, lv);
  WHIP(n, hipGetLastError());
  hipLaunchKernelGGL(loss_small_kernel, dim3(1), dim3(1024), 0, n->st, (const double*)M, (const double*)S, n_states,
                     mp, (const double*)lv, G, Bt, lv + 1);
  WHIP(n, hipGetLastError());
  // dy = B T + 2 y : the rotation kernel forms sum_i C[i][j] T[i][p], here with C = B^T
  mpe::RotateArgs r;
  std::memset(&r, 0, sizeof(r));
  r.Phi = target;
  r.C = Bt;
  r.Psi = dy;
  r.N = P;
  long rch = std::min<long>(1024, std::max<long>(1, (P + 255) / 256));
  r.chunk = ((P + rch - 1) / rch + 63) / 64 * 64;
  rch = (P + r.chunk - 1) / r.chunk;
  r.m = n_states;
  r.mp = mp;
  WHIP(n, mpe::launch_rotate(0, false, r, (int)rch, n->st));
  hipLaunchKernelGGL(axpy2_kernel, dim3(nblk((long)n_states * P)), dim3(256), 0, n->st, y, dy, (long)n_states * P);
  WHIP(n, hipGetLastError());
  double lh[2];
  WHIP(n, hipMemcpyAsync(lh, lv + 1, sizeof lh, hipMemcpyDeviceToHost, n->st));
  WHIP(n, hipStreamSynchronize(n->st));
  if (loss_host) {
    loss_host[0] = lh[0];
    loss_host[1] = lh[1];
  }
  return MPE_OK;
}

mpe_status wsn_procrustes_loss(wsn_net n, const float* y, const float* target, int32_t n_states, int64_t P,
                               double* loss_host, float* dy) {
  if (!n || !y || !target || !dy || n_states < 1 || n_states > mpe::MAXM || P < 1)
    return MPE_ERR_INVALID_ARGUMENT;
  if ((const float*)dy == y) return wfail(n, MPE_ERR_INVALID_ARGUMENT, "dy must not alias y");
  const int mp = (n_states + 15) / 16 * 16;
  long nch = std::min<long>(128, std::max<long>(1, (P + 4095) / 4096));
  long chunk = ((P + nch - 1) / nch + 31) / 32 * 32;
  nch = (P + chunk - 1) / chunk;
  const long q = 128L * 128;
  double* partials = n->scratch;   // [2][nch][mp][mp]
  double* M = partials + 256 * q;  // M then S
  double* S = M + (long)mp * mp;
  double* Bt = M + 2 * q;
  double* W = Bt + q;
  double* A = W + q;
  double* Sid = A + q;
  double* Lb = Sid + q;
  double* rot = Lb + q;
  double* U = rot + q;
  double* Q = U + q;
  double* theta = Q + q;
  double* sds = theta + 128;
  int* status = reinterpret_cast<int*>(sds + 256);
  double* lv = sds + 256 + 16;     // [||y||^2, loss, nuclear norm]
  double* jlog = lv + 16;          // Jacobi rotation log
  mpe::GramArgs g;
  std::memset(&g, 0, sizeof(g));
  g.X[0] = y;
  g.Y[0] = target;
  g.X[1] = target;
  g.Y[1] = target;
  g.partials = partials;
  g.N = P;
  g.chunk = chunk;
  g.m = n_states;
  g.mp = mp;
  WHIP(n, mpe::launch_gram(0, g, 2, (int)nch, n->st));
  WHIP(n, mpe::launch_reduce(partials, (int)nch, (long)mp * mp, 2, M, n->st));
  WHIP(n, hipMemsetAsync(lv, 0, sizeof(double), n->st));
  hipLaunchKernelGGL(sumsq_kernel, dim3(256), dim3(256), 0, n->st, y, (long)n_states * P, lv);
  WHIP(n, hipGetLastError());
  hipLaunchKernelGGL(ata_kernel, dim3((mp * mp + 255) / 256), dim3(256), 0, n->st, (const double*)M, n_states, mp, A,
                     Sid);
  WHIP(n, hipGetLastError());
  // eigenpairs of M^T M: the plan's small dense solver with S = I (Cholesky factor I, C = U)
  mpe::SmallDenseArgs d;
  std::memset(&d, 0, sizeof(d));
  d.S = Sid;
  d.Hs = A;
  d.L = Lb;
  d.rot = jlog;
  d.scratch = sds;
  d.C = U;
  d.theta = theta;
  d.status = status;
  d.m = n_states;
  d.mp = mp;
  d.mode = mpe::SD_RR;
  d.max_sweeps = 60;
  d.tol = 1e-13;
  d.pivot_tol = 1e-13;
  WHIP(n, mpe::launch_small_dense(d, n->st));
  hipLaunchKernelGGL(polar_kernel, dim3(1), dim3(1024), 0, n->st, (const double*)M, (const double*)S,
                     (const double*)U, (const double*)theta, (const int*)status, n_states, mp, (const double*)lv, W,
                     Q, Bt, lv + 1);
  WHIP(n, hipGetLastError());
  mpe::RotateArgs r;
  std::memset(&r, 0, sizeof(r));
  r.Phi = target;
  r.C = Bt;
  r.Psi = dy;
  r.N = P;
  r.status = status;
  long rch = std::min<long>(1024, std::max<long>(1, (P + 255) / 256));
  r.chunk = ((P + rch - 1) / rch + 63) / 64 * 64;
  rch = (P + r.chunk - 1) / r.chunk;
  r.m = n_states;
  r.mp = mp;
  WHIP(n, mpe::launch_rotate(0, false, r, (int)rch, n->st));
  hipLaunchKernelGGL(axpy2_kernel, dim3(nblk((long)n_states * P)), dim3(256), 0, n->st, y, dy, (long)n_states * P);
  WHIP(n, hipGetLastError());
  double lh[2];
  int st[2];
  WHIP(n, hipMemcpyAsync(lh, lv + 1, sizeof lh, hipMemcpyDeviceToHost, n->st));
  WHIP(n, hipMemcpyAsync(st, status, sizeof st, hipMemcpyDeviceToHost, n->st));
  WHIP(n, hipStreamSynchronize(n->st));
  if (st[0] != 0)
    return wfail(n, st[0] == mpe::ST_NONFINITE ? MPE_ERR_NONFINITE : MPE_ERR_EIG_NO_CONVERGENCE,
                 "eigenpairs of M^T M failed (status " + std::to_string(st[0]) + ")");
  if (loss_host) {
    loss_host[0] = lh[0];
    loss_host[1] = lh[1];
  }
  return MPE_OK;
}

mpe_status wsn_upsample_periodic(const float* u, int32_t channels, int32_t d, int32_t factor, float* out,
                                 void* hip_stream) {
  if (!u || !out || channels < 1 || d < 1 || factor < 1) return MPE_ERR_INVALID_ARGUMENT;
  const long D = (long)d * factor;
  hipLaunchKernelGGL(upsample_kernel, dim3(nblk(channels * D * D * D)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(hip_stream), u, channels, d, factor, out);
  return hipGetLastError() == hipSuccess ? MPE_OK : MPE_ERR_DEVICE;
}

}  // extern "C"
