// Propagation kernels: the split operator T2 (Section I, Eq. so) as two HBM
// passes per application, chained into the multi-product expansion
// (Section II, Eq. mcomp) with the c_k combination in float64 registers.
//
// A real 3-D field psi[z][y][x] is transformed as
//   plane pass : per z-plane, x real-to-complex (as an NX/2-point complex FFT
//                plus a split step) then y complex FFT, all inside LDS;
//   pencil pass: per tile of C half-spectrum columns, z complex FFT forward,
//                the kinetic factor, z complex FFT inverse, in place.
// The half spectrum is stored [z][ky][kx], kx = 0..NX/2 (NXH = NX/2+1).
//
// Plane pass modes:
//   PM_FWD   real rows (x optional factor table) -> half spectrum
//   PM_LINK  half spectrum -> real rows in registers -> x factor -> half spectrum
//            (the two potential half-steps of consecutive T2 merged into one)
//   PM_TAIL  K half spectra -> sum_k c_k * factor_k * real rows, float64
//            accumulation in registers, one rounding on store
//   PM_HTAIL half spectrum -> real rows + V*phi   (H application)
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "prop.hpp"

namespace mpe {

// ------------------------------------------------------------------ plane pass
// One work-group per (z-plane, state).  The plane lives in LDS as
// Z[y][k], k = 0..NX/2-1, the NX/2-point complex FFTs of the packed rows
// x[2k] + i x[2k+1].  The real-to-half-spectrum split
//   X[k] = (Z[k] + conj Z[NX/2-k])/2 - i W^k (Z[k] - conj Z[NX/2-k])/2,  W = exp(-2 pi i/NX)
// is fused into the y-column phase: column FFT f (f = 0..NX/2-1) is carried by
// TY threads; f = 2g + h with g >= 1 handles kx = g (h = 0) or kx = NX/2-g
// (h = 1), so the two columns a split couples sit in neighbouring lanes.  f = 0
// carries kx = 0 and kx = NX/2 packed as one complex column (both real along
// y), f = 1 carries kx = NX/4.  That is NX/2 column FFTs for NX/2+1 columns,
// done in a single round.
__host__ __device__ constexpr int round64(int x) { return (x + 63) / 64 * 64; }
template <int NX>
struct PlaneShape {
  static constexpr int LX = NX / 2;
  static constexpr int COLT = LX * Plan<NX>::T;            // column-phase thread tasks (NY == NX)
  static constexpr int BLOCK = round64(COLT) > 1024 ? 1024 : (round64(COLT) < 64 ? 64 : round64(COLT));
};
// Waves per SIMD that the LDS footprint admits (2 work-groups per CU for a
// float32 128^2 plane): the register budget is capped to match, so that one
// work-group's loads overlap another's LDS work.
// LDS row stride (complex elements) of the plane: the row phase maps TX lanes to
// each of 32/TX rows of a half-wave, so rows are offset by TX (mod 32) complex
// slots to land in distinct LDS banks.
template <int NX>
constexpr int plane_srow() {
  constexpr int nxh = NX / 2 + 1, tx = Plan<NX / 2>::T;
  int s = nxh;
  while (!((s % 32) % tx == 0 && ((s % 32) / tx) % 2 == 1)) ++s;
  return s;
}

template <typename F, int NX>
struct PlaneOcc {
  static constexpr int LDS = NX * plane_srow<NX>() * 2 * (int)sizeof(F);
  static constexpr int WG = (160 * 1024 / LDS) < 1 ? 1 : (160 * 1024 / LDS);
  static constexpr int W = WG * (PlaneShape<NX>::BLOCK / 64) / 4;
  // register floor: at least 128 VGPRs (float) / 256 (double) per lane, the
  // working set of a row or column transform plus its twiddles and addresses
  // (a one-lane row transform, as for NX = 48, holds a whole row: half that)
  static constexpr int WMAX = (sizeof(F) == 4 ? 4 : 2) / (Plan<NX / 2>::T == 1 ? 2 : 1);
  static constexpr int value = W < 1 ? 1 : (W > WMAX ? WMAX : W);
};

template <typename F, int NX, int MODE>
struct PlaneWaves {
  static constexpr int one_wg = (PlaneShape<NX>::BLOCK / 64 + 3) / 4;
  static constexpr int value = MODE == PM_TAIL ? one_wg : PlaneOcc<F, NX>::value;
};

template <typename F, int NX, int MODE>
__global__ __launch_bounds__(PlaneShape<NX>::BLOCK) __attribute__((amdgpu_waves_per_eu(PlaneWaves<F, NX, MODE>::value)))
void plane_kernel(PlaneArgs a) {
  constexpr int NY = NX;
  constexpr int BLOCK = PlaneShape<NX>::BLOCK;
  constexpr int LX = NX / 2, NXH = LX + 1, HALF = LX / 2;
  using PX = Plan<LX>;
  using PY = Plan<NY>;
  constexpr int TX = PX::T, EX = PX::E, TY = PY::T, EY = PY::E;
  constexpr int NCF = LX;                          // column FFTs
  constexpr int RPR = BLOCK / TX;                  // rows per round
  constexpr int XR = (NY + RPR - 1) / RPR;         // row rounds
  constexpr int SROW = plane_srow<NX>();           // LDS row stride (complex), bank-spread
  static_assert(BLOCK % TX == 0, "block must hold whole row transforms");
  // a row's TX lanes are consecutive lanes of one wavefront (tx = tid % TX)
  constexpr bool ROWWAVE = (64 % TX == 0);
  static_assert(NCF * TY <= BLOCK, "one column round");
  static_assert(NCF % 2 == 0, "column pairs");
  constexpr bool TAIL_PREFETCH = sizeof(F) == 4 && EY <= 16;

  __shared__ cx<F> lds[NY * SROW];
  // twiddle tables staged in LDS (they sit on the FFT critical path)
  __shared__ cx<F> tw_x[LX], tw_y[NY], tw_w[HALF + 1];

  const int tid = threadIdx.x;
  const int z = blockIdx.x;
  const long s = (long)blockIdx.y + a.state0;
  const long plane_real = (long)NY * NX;
  const long plane_spec = (long)NY * NXH;
  const long z_real = (long)z * plane_real;
  const long z_spec = (long)z * plane_spec;
  // this state's arrays (plane z offsets added below)
  const F* rin;
  F* rout;
  cx<F>* spec;
  long chain_stride;
  const F* facb;
  if (a.desc) {
    const StateDesc& d = a.desc[s];
    rin = reinterpret_cast<const F*>(d.real_in);
    rout = reinterpret_cast<F*>(d.real_out);
    chain_stride = d.chain_stride;
    spec = reinterpret_cast<cx<F>*>(d.spec) + (long)a.chain * chain_stride;
    facb = reinterpret_cast<const F*>(MODE == PM_HTAIL ? d.V : d.fac);
  } else {
    rin = reinterpret_cast<const F*>(a.real_in) + s * a.real_state_stride;
    rout = reinterpret_cast<F*>(a.real_out) + s * a.real_state_stride;
    spec = reinterpret_cast<cx<F>*>(a.spec) + s * a.spec_state_stride;
    chain_stride = a.chain_stride;
    facb = reinterpret_cast<const F*>(a.fac);
  }
  const F* facz = (MODE == PM_HTAIL || MODE == PM_TAIL || a.fac_index < 0 || !facb)
                      ? facb
                      : facb + (long)a.fac_index * a.fac_table_stride;

  {
    const cx<F>* gx = reinterpret_cast<const cx<F>*>(a.rx);
    const cx<F>* gy = reinterpret_cast<const cx<F>*>(a.ry);
    const cx<F>* gw = reinterpret_cast<const cx<F>*>(a.wpost);
    for (int i = tid; i < LX; i += BLOCK) tw_x[i] = gx[i];
    for (int i = tid; i < NY; i += BLOCK) tw_y[i] = gy[i];
    for (int i = tid; i <= HALF; i += BLOCK) tw_w[i] = gw[i];
  }
  const cx<F>* rx = tw_x;
  const cx<F>* ry = tw_y;
  const cx<F>* wpost = tw_w;   // W^k, k = 0..NX/4
  __syncthreads();

  // row phase mapping
  const int tx = tid % TX, rloc = tid / TX;
  // column phase mapping
  const int f = tid % NCF, ty = tid / NCF;
  const bool cact = ty < TY;                       // threads beyond NCF*TY idle in the column phase
  const int g = f >> 1, h = f & 1;
  const bool packed = (g == 0 && h == 0);
  const int col = (g == 0) ? (h ? HALF : 0) : (h ? LX - g : g);   // LDS / spectrum column
  const int tyc = cact ? ty : 0;
  auto cbuf = [&](int i) { return &lds[i * SROW + col]; };

  // W^k for k = 0..LX (W^(LX-j) = -conj W^j)
  auto wk = [&](int k) -> cx<F> {
    return k <= HALF ? wpost[k] : cx<F>{-wpost[LX - k].x, wpost[LX - k].y};
  };

  // ---- spectrum in: column loads (issued early when pipelined), inverse y FFT,
  //      c2r split in registers, Z rows to LDS
  auto column_load = [&](const cx<F>* __restrict__ spec, cx<F>* v) {
    if (cact) {
#pragma unroll
      for (int m = 0; m < EY; ++m) {
        const long o = (long)(tyc + TY * m) * NXH;
        if (packed) {
          const cx<F> y0 = spec[o], yl = spec[o + LX];
          v[m] = cx<F>{y0.x - yl.y, y0.y + yl.x};            // Y0 + i Y_LX
        } else {
          v[m] = spec[o + col];
        }
      }
    }
  };
  auto column_inverse_regs = [&](cx<F>* v) {
    fft<NY, +1>(v, tyc, cact, cbuf, ry);
    // split: needs X[LX - col] at the same y, held by the neighbouring lane
    const cx<F> w = wk(col);
#pragma unroll
    for (int m = 0; m < EY; ++m) {
      const cx<F> pr{__shfl_xor(v[m].x, 1), __shfl_xor(v[m].y, 1)};
      cx<F> zv;
      if (packed) {
        zv = cx<F>{v[m].x + v[m].y, v[m].x - v[m].y};         // X0 = Re, X_LX = Im
      } else if (col == HALF) {
        zv = scale(conj(v[m]), F(2));
      } else {
        const cx<F> X2 = conj(pr);
        const cx<F> Fe = v[m] + X2;
        const cx<F> Fo = cmulc(v[m] - X2, w);
        zv = Fe + muli<+1>(Fo);
      }
      v[m] = zv;
    }
    if (cact) {
#pragma unroll
      for (int m = 0; m < EY; ++m) lds[(tyc + TY * m) * SROW + col] = v[m];
    }
    __syncthreads();
  };
  auto column_inverse = [&](const cx<F>* __restrict__ spec) {
    cx<F> v[EY];
    column_load(spec, v);
    column_inverse_regs(v);
  };

  // ---- columns forward out: r2c split on load, forward y FFT, store
  auto column_forward_store = [&](cx<F>* __restrict__ spec) {
    __syncthreads();
    cx<F> v[EY];
    if (cact) {
      const cx<F> w = wk(col);
#pragma unroll
      for (int m = 0; m < EY; ++m) {
        const cx<F>* r = lds + (tyc + TY * m) * SROW;
        if (packed) {
          const cx<F> z0 = r[0];
          v[m] = cx<F>{z0.x + z0.y, z0.x - z0.y};             // X0 + i X_LX (both real)
        } else {
          const cx<F> A = r[col], B = conj(r[LX - col]);
          const cx<F> E = scale(A + B, F(0.5));
          const cx<F> O = muli<-1>(scale(A - B, F(0.5)));
          v[m] = E + cmul(O, w);
        }
      }
    }
    __syncthreads();   // every Z value read before the exchanges reuse the columns
    fft<NY, -1>(v, tyc, cact, cbuf, ry);
    if (cact && !packed) {
#pragma unroll
      for (int m = 0; m < EY; ++m) spec[(long)(tyc + TY * m) * NXH + col] = v[m];
    }
    // unpack the DC / Nyquist column: X0[k] = (C[k] + conj C[-k])/2, X_LX[k] = -i (C[k] - conj C[-k])/2
    if (cact && packed) {
#pragma unroll
      for (int m = 0; m < EY; ++m) lds[(tyc + TY * m) * SROW] = v[m];
    }
    __syncthreads();
    if (cact && packed) {
#pragma unroll
      for (int m = 0; m < EY; ++m) {
        const int ky = tyc + TY * m;
        const cx<F> c = v[m], cm = conj(lds[((NY - ky) % NY) * SROW]);
        spec[(long)ky * NXH] = scale(c + cm, F(0.5));
        spec[(long)ky * NXH + LX] = muli<-1>(scale(c - cm, F(0.5)));
      }
    }
  };

  if constexpr (MODE == PM_FWD) {
    const F* __restrict__ src = rin + z_real;
    const F* __restrict__ fac = (a.fac_index >= 0 && facz) ? facz + z_real : nullptr;
#pragma unroll
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      const bool act = row < NY;
      const int rowc = act ? row : 0;
      cx<F> v[EX];
      if (act) {
        const cx<F>* s2 = reinterpret_cast<const cx<F>*>(src + (long)row * NX);
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = s2[tx + TX * m];
        if (fac) {
          const cx<F>* f2 = reinterpret_cast<const cx<F>*>(fac + (long)row * NX);
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> fv = f2[tx + TX * m];
            v[m].x *= fv.x;
            v[m].y *= fv.y;
          }
        }
      }
      fft<LX, -1, ROWWAVE>(v, tx, act, [&](int i) { return &lds[rowc * SROW + i]; }, rx);
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) lds[row * SROW + tx + TX * m] = v[m];
      }
    }
    column_forward_store(spec + z_spec);
  } else if constexpr (MODE == PM_LINK) {
    column_inverse(spec + z_spec);
    const F* __restrict__ fac = facz + z_real;
#pragma unroll
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      const bool act = row < NY;
      const int rowc = act ? row : 0;
      cx<F> v[EX];
      cx<F> fv[EX];
      if (act) {
        const cx<F>* f2 = reinterpret_cast<const cx<F>*>(fac + (long)row * NX);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          v[m] = lds[row * SROW + tx + TX * m];
          fv[m] = f2[tx + TX * m];
        }
      }
      fft<LX, +1, ROWWAVE>(v, tx, act, [&](int i) { return &lds[rowc * SROW + i]; }, rx);
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        v[m].x *= fv[m].x;
        v[m].y *= fv[m].y;
      }
      fft<LX, -1, ROWWAVE>(v, tx, act, [&](int i) { return &lds[rowc * SROW + i]; }, rx);
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) lds[row * SROW + tx + TX * m] = v[m];
      }
    }
    column_forward_store(spec + z_spec);
  } else if constexpr (MODE == PM_TAIL) {
    double acc[XR][EX][2];
#pragma unroll
    for (int rr = 0; rr < XR; ++rr)
#pragma unroll
      for (int m = 0; m < EX; ++m) acc[rr][m][0] = acc[rr][m][1] = 0.0;
    // the next chain's column loads are issued before this chain's row work,
    // so their latency hides behind it (one work-group per CU here)
    const cx<F>* spec0 = spec + z_spec;
    cx<F> vc[EY];
    column_load(spec0, vc);
    for (int k = 0; k < a.K; ++k) {
      const F* __restrict__ fac = facb + (long)(2 * k + 1) * a.fac_table_stride + z_real;
      const double ck = a.coef[k];
      column_inverse_regs(vc);
      // (float64 planes, and float32 planes with 24-element columns, have no
      // registers to spare for the prefetch)
      if (k + 1 < a.K) {
        if constexpr (TAIL_PREFETCH) {
          column_load(spec0 + (long)(k + 1) * chain_stride, vc);
        }
      }
#pragma unroll
      for (int rr = 0; rr < XR; ++rr) {
        const int row = rr * RPR + rloc;
        const bool act = row < NY;
        const int rowc = act ? row : 0;
        cx<F> v[EX];
        if (act) {
#pragma unroll
          for (int m = 0; m < EX; ++m) v[m] = lds[row * SROW + tx + TX * m];
        }
        fft<LX, +1, ROWWAVE>(v, tx, act, [&](int i) { return &lds[rowc * SROW + i]; }, rx);
        if (act) {
          const cx<F>* f2 = reinterpret_cast<const cx<F>*>(fac + (long)row * NX);
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> fv = f2[tx + TX * m];
            acc[rr][m][0] += ck * (double)(v[m].x * fv.x);
            acc[rr][m][1] += ck * (double)(v[m].y * fv.y);
          }
        }
      }
      __syncthreads();
      if constexpr (!TAIL_PREFETCH) {
        if (k + 1 < a.K) column_load(spec0 + (long)(k + 1) * chain_stride, vc);
      }
    }
    F* __restrict__ dst = rout + z_real;
#pragma unroll
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      if (row < NY) {
        cx<F>* d2 = reinterpret_cast<cx<F>*>(dst + (long)row * NX);
#pragma unroll
        for (int m = 0; m < EX; ++m) d2[tx + TX * m] = cx<F>{(F)acc[rr][m][0], (F)acc[rr][m][1]};
      }
    }
  } else {  // PM_HTAIL
    column_inverse(spec + z_spec);
    const F* __restrict__ phi = rin + z_real;
    const F* __restrict__ V = facb + z_real;
    F* __restrict__ dst = rout + z_real;
#pragma unroll
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      const bool act = row < NY;
      const int rowc = act ? row : 0;
      cx<F> v[EX];
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = lds[row * SROW + tx + TX * m];
      }
      fft<LX, +1, ROWWAVE>(v, tx, act, [&](int i) { return &lds[rowc * SROW + i]; }, rx);
      if (act) {
        const cx<F>* p2 = reinterpret_cast<const cx<F>*>(phi + (long)row * NX);
        const cx<F>* v2 = reinterpret_cast<const cx<F>*>(V + (long)row * NX);
        cx<F>* d2 = reinterpret_cast<cx<F>*>(dst + (long)row * NX);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          const cx<F> pv = p2[tx + TX * m], wv = v2[tx + TX * m];
          d2[tx + TX * m] = cx<F>{v[m].x + wv.x * pv.x, v[m].y + wv.y * pv.y};
        }
      }
    }
  }
}

// ------------------------------------------------------------------ pencil pass
template <int NZ>
struct PencilCols {
  static constexpr int value = 256 / Plan<NZ>::T;
};

template <typename F, int NZ, int KIND>
__global__ __launch_bounds__(256) void pencil_kernel(PencilArgs a) {
  using P = Plan<NZ>;
  constexpr int T = P::T, E = P::E;
  constexpr int C = PencilCols<NZ>::value;
  constexpr int CP = C + 1;   // padded row: the T lanes of a column hit different banks
  __shared__ cx<F> lds[T > 1 ? NZ * CP : 1];

  __shared__ cx<F> rz_s[NZ];
  __shared__ F tz_s[NZ];

  const int tid = threadIdx.x;
  const int col = tid % C, t = tid / C;
  const long s = (long)blockIdx.y + a.state0;
  const int gcol = blockIdx.x * C + col;
  const bool act = gcol < a.M;
  const int gc = act ? gcol : 0;
  cx<F>* data;
  const F* tab;
  if (a.desc) {
    const StateDesc& d = a.desc[s];
    data = reinterpret_cast<cx<F>*>(d.spec) + (long)a.chain * d.chain_stride;
    tab = a.desc_tables == 0
              ? reinterpret_cast<const F*>(d.kin) + (long)a.chain * (a.NXH + a.NY + NZ)
              : reinterpret_cast<const F*>(d.hk);
  } else {
    data = reinterpret_cast<cx<F>*>(a.data) + s * a.state_stride;
    tab = reinterpret_cast<const F*>(a.tab);
  }
  const F* tx = tab;
  const F* ty = tab + a.NXH;
  for (int i = tid; i < NZ; i += 256) {
    rz_s[i] = reinterpret_cast<const cx<F>*>(a.rz)[i];
    tz_s[i] = tab[a.NXH + a.NY + i];
  }
  const cx<F>* rz = rz_s;
  const F* tz = tz_s;

  cx<F> v[E];
  if (act) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = data[(long)(t + T * m) * a.M + gcol];
  }
  __syncthreads();   // staged tables visible
  auto buf = [&](int i) { return &lds[i * CP + col]; };
  fft<NZ, -1>(v, t, act, buf, rz);
  if (act) {
    const int ky = gc / a.NXH, kx = gc - ky * a.NXH;
    if constexpr (KIND == PK_EXP) {
      const F g = ty[ky] * tx[kx];
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = scale(v[m], tz[t + T * m] * g);
    } else {
      const F g = ty[ky] + tx[kx];
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = scale(v[m], tz[t + T * m] + g);
    }
  }
  fft<NZ, +1>(v, t, act, buf, rz);
  if (act) {
#pragma unroll
    for (int m = 0; m < E; ++m) data[(long)(t + T * m) * a.M + gcol] = v[m];
  }
}

// ------------------------------------------------------------------ launchers
template <typename F, int N>
static hipError_t launch_plane_n(int mode, const PlaneArgs& a, int nz, int nstates, hipStream_t st) {
  dim3 grid(nz, nstates);
  dim3 block(PlaneShape<N>::BLOCK);
  switch (mode) {
    case PM_FWD: hipLaunchKernelGGL((plane_kernel<F, N, PM_FWD>), grid, block, 0, st, a); break;
    case PM_LINK: hipLaunchKernelGGL((plane_kernel<F, N, PM_LINK>), grid, block, 0, st, a); break;
    case PM_TAIL: hipLaunchKernelGGL((plane_kernel<F, N, PM_TAIL>), grid, block, 0, st, a); break;
    case PM_HTAIL: hipLaunchKernelGGL((plane_kernel<F, N, PM_HTAIL>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename F, int N>
static hipError_t launch_pencil_n(int kind, const PencilArgs& a, int nstates, hipStream_t st) {
  constexpr int C = PencilCols<N>::value;
  dim3 grid((a.M + C - 1) / C, nstates);
  if (kind == PK_EXP)
    hipLaunchKernelGGL((pencil_kernel<F, N, PK_EXP>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((pencil_kernel<F, N, PK_ADD>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

bool plane_supported(int is_double, int nx, int ny) {
  if (nx != ny) return false;
  switch (nx) {
    case 8: case 16: case 32: case 48: case 64: case 96: case 128: return true;
    case 192: return !is_double;   // 192 x 97 complex doubles exceed the 160 KB LDS
    default: return false;
  }
}

bool pencil_supported(int nz) {
  switch (nz) {
    case 8: case 16: case 32: case 48: case 64: case 96: case 128: case 192: return true;
    default: return false;
  }
}

template <typename F>
static hipError_t launch_plane_t(int mode, int n, const PlaneArgs& a, int nz, int ns, hipStream_t st) {
  switch (n) {
    case 8: return launch_plane_n<F, 8>(mode, a, nz, ns, st);
    case 16: return launch_plane_n<F, 16>(mode, a, nz, ns, st);
    case 32: return launch_plane_n<F, 32>(mode, a, nz, ns, st);
    case 48: return launch_plane_n<F, 48>(mode, a, nz, ns, st);
    case 64: return launch_plane_n<F, 64>(mode, a, nz, ns, st);
    case 96: return launch_plane_n<F, 96>(mode, a, nz, ns, st);
    case 128: return launch_plane_n<F, 128>(mode, a, nz, ns, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plane(int is_double, int mode, int nx, const PlaneArgs& a, int nz, int nstates, hipStream_t st) {
  if (nstates <= 0) return hipSuccess;
  if (is_double) return launch_plane_t<double>(mode, nx, a, nz, nstates, st);
  if (nx == 192) return launch_plane_n<float, 192>(mode, a, nz, nstates, st);
  return launch_plane_t<float>(mode, nx, a, nz, nstates, st);
}

template <typename F>
static hipError_t launch_pencil_t(int kind, int nz, const PencilArgs& a, int ns, hipStream_t st) {
  switch (nz) {
    case 8: return launch_pencil_n<F, 8>(kind, a, ns, st);
    case 16: return launch_pencil_n<F, 16>(kind, a, ns, st);
    case 32: return launch_pencil_n<F, 32>(kind, a, ns, st);
    case 48: return launch_pencil_n<F, 48>(kind, a, ns, st);
    case 64: return launch_pencil_n<F, 64>(kind, a, ns, st);
    case 96: return launch_pencil_n<F, 96>(kind, a, ns, st);
    case 128: return launch_pencil_n<F, 128>(kind, a, ns, st);
    case 192: return launch_pencil_n<F, 192>(kind, a, ns, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pencil(int is_double, int kind, int nz, const PencilArgs& a, int nstates, hipStream_t st) {
  if (nstates <= 0) return hipSuccess;
  return is_double ? launch_pencil_t<double>(kind, nz, a, nstates, st)
                   : launch_pencil_t<float>(kind, nz, a, nstates, st);
}

}  // namespace mpe
