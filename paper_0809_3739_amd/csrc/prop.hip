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

// ------------------------------------------------------------------ real <-> half-spectrum split steps
// Row r holds Z = FFT_{NX/2}(x[2i] + i x[2i+1]) in slots 0..LX-1; afterwards
// slots 0..LX hold X = the NX-point real-input DFT (exact scaling).
template <typename F, int NX, int NY, int BLOCK>
__device__ __forceinline__ void r2c_split(cx<F>* lds, const cx<F>* __restrict__ wpost) {
  constexpr int LX = NX / 2, NXH = LX + 1, NP = LX / 2 + 1;
  for (int task = threadIdx.x; task < NY * NP; task += BLOCK) {
    const int row = task / NP, k = task - row * NP;
    cx<F>* r = lds + row * NXH;
    if (k == 0) {
      const cx<F> z = r[0];
      r[0] = cx<F>{z.x + z.y, F(0)};
      r[LX] = cx<F>{z.x - z.y, F(0)};
    } else if (2 * k == LX) {
      r[k] = conj(r[k]);
    } else {
      const cx<F> A = r[k], B = conj(r[LX - k]);
      const cx<F> E = scale(A + B, F(0.5));
      const cx<F> O = muli<-1>(scale(A - B, F(0.5)));
      const cx<F> WO = cmul(O, wpost[k]);
      r[k] = E + WO;
      r[LX - k] = conj(E - WO);
    }
  }
}

// Inverse of r2c_split up to a factor 2: slots 0..LX-1 receive Z' with
// IFFT_{NX/2}(Z') = NX * x (unnormalised, like the full NX-point inverse).
// The imaginary parts of the kx = 0 and kx = NX/2 bins are dropped.
template <typename F, int NX, int NY, int BLOCK>
__device__ __forceinline__ void c2r_split(cx<F>* lds, const cx<F>* __restrict__ wpost) {
  constexpr int LX = NX / 2, NXH = LX + 1, NP = LX / 2 + 1;
  for (int task = threadIdx.x; task < NY * NP; task += BLOCK) {
    const int row = task / NP, k = task - row * NP;
    cx<F>* r = lds + row * NXH;
    if (k == 0) {
      const F a = r[0].x, b = r[LX].x;
      r[0] = cx<F>{a + b, a - b};
    } else if (2 * k == LX) {
      r[k] = scale(conj(r[k]), F(2));
    } else {
      const cx<F> X1 = r[k], X2 = conj(r[LX - k]);
      const cx<F> Fe = X1 + X2;
      const cx<F> Fo = cmulc(X1 - X2, wpost[k]);
      r[k] = Fe + muli<+1>(Fo);
      r[LX - k] = conj(Fe) + muli<+1>(conj(Fo));
    }
  }
}

constexpr int plane_block(int nx, int mode) { return (mode == PM_TAIL && nx >= 96) ? 512 : 256; }

// ------------------------------------------------------------------ plane pass
template <typename F, int NX, int NY, int MODE>
__global__ __launch_bounds__(plane_block(NX, MODE)) void plane_kernel(PlaneArgs a) {
  constexpr int BLOCK = plane_block(NX, MODE);
  constexpr int LX = NX / 2, NXH = LX + 1;
  using PX = Plan<LX>;
  using PY = Plan<NY>;
  constexpr int TX = PX::T, EX = PX::E, TY = PY::T, EY = PY::E;
  constexpr int RPR = BLOCK / TX;                 // rows per round
  constexpr int XR = (NY + RPR - 1) / RPR;        // row rounds
  constexpr int CPR = BLOCK / TY;                 // columns per round
  constexpr int YR = (NXH + CPR - 1) / CPR;       // column rounds
  static_assert(BLOCK % TX == 0 && BLOCK % TY == 0, "block must hold whole transforms");

  __shared__ cx<F> lds[NY * NXH];

  const int tid = threadIdx.x;
  const int z = blockIdx.x;
  const long s = (long)blockIdx.y + a.state0;
  const long plane_real = (long)NY * NX;
  const long plane_spec = (long)NY * NXH;
  const long real_off = s * a.real_state_stride + (long)z * plane_real;
  const long spec_off = s * a.spec_state_stride + (long)z * plane_spec;
  const long fac_off = (long)z * plane_real;

  const cx<F>* rx = reinterpret_cast<const cx<F>*>(a.rx);
  const cx<F>* ry = reinterpret_cast<const cx<F>*>(a.ry);
  const cx<F>* wpost = reinterpret_cast<const cx<F>*>(a.wpost);

  const int tx = tid % TX, rloc = tid / TX;      // row-phase lane / row slot
  const int cl = tid % CPR, ty = tid / CPR;      // column-phase column slot / lane

  // ---------------- spectrum in: inverse y per column, then the c2r split
  // (PM_TAIL repeats this per chain inside its own loop)
  auto column_inverse = [&](const cx<F>* __restrict__ spec) {
    for (int cr = 0; cr < YR; ++cr) {
      const int col = cr * CPR + cl;
      const bool act = col < NXH;
      const int colc = act ? col : 0;
      cx<F> v[EY];
      if (act) {
#pragma unroll
        for (int m = 0; m < EY; ++m) v[m] = spec[(long)(ty + TY * m) * NXH + col];
      }
      fft<NY, +1>(v, ty, act, [&](int i) { return &lds[i * NXH + colc]; }, ry);
      if (act) {
#pragma unroll
        for (int m = 0; m < EY; ++m) lds[(ty + TY * m) * NXH + col] = v[m];
      }
    }
    __syncthreads();
    c2r_split<F, NX, NY, BLOCK>(lds, wpost);
    __syncthreads();
  };

  // ---------------- columns forward out: r2c split, forward y per column, store
  auto column_forward_store = [&](cx<F>* __restrict__ spec) {
    __syncthreads();
    r2c_split<F, NX, NY, BLOCK>(lds, wpost);
    __syncthreads();
    for (int cr = 0; cr < YR; ++cr) {
      const int col = cr * CPR + cl;
      const bool act = col < NXH;
      const int colc = act ? col : 0;
      cx<F> v[EY];
      if (act) {
#pragma unroll
        for (int m = 0; m < EY; ++m) v[m] = lds[(ty + TY * m) * NXH + col];
      }
      fft<NY, -1>(v, ty, act, [&](int i) { return &lds[i * NXH + colc]; }, ry);
      if (act) {
#pragma unroll
        for (int m = 0; m < EY; ++m) spec[(long)(ty + TY * m) * NXH + col] = v[m];
      }
    }
  };

  if constexpr (MODE == PM_FWD) {
    const F* __restrict__ src = reinterpret_cast<const F*>(a.real_in) + real_off;
    const F* __restrict__ fac = a.fac ? reinterpret_cast<const F*>(a.fac) + fac_off : nullptr;
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
            const cx<F> f = f2[tx + TX * m];
            v[m].x *= f.x;
            v[m].y *= f.y;
          }
        }
      }
      fft<LX, -1>(v, tx, act, [&](int i) { return &lds[rowc * NXH + i]; }, rx);
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) lds[row * NXH + tx + TX * m] = v[m];
      }
    }
    column_forward_store(reinterpret_cast<cx<F>*>(a.spec_out) + spec_off);
  } else if constexpr (MODE == PM_LINK) {
    column_inverse(reinterpret_cast<const cx<F>*>(a.spec_in) + spec_off);
    const F* __restrict__ fac = reinterpret_cast<const F*>(a.fac) + fac_off;
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      const bool act = row < NY;
      const int rowc = act ? row : 0;
      cx<F> v[EX];
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = lds[row * NXH + tx + TX * m];
      }
      fft<LX, +1>(v, tx, act, [&](int i) { return &lds[rowc * NXH + i]; }, rx);
      if (act) {
        const cx<F>* f2 = reinterpret_cast<const cx<F>*>(fac + (long)row * NX);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          const cx<F> f = f2[tx + TX * m];
          v[m].x *= f.x;
          v[m].y *= f.y;
        }
      }
      fft<LX, -1>(v, tx, act, [&](int i) { return &lds[rowc * NXH + i]; }, rx);
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) lds[row * NXH + tx + TX * m] = v[m];
      }
    }
    column_forward_store(reinterpret_cast<cx<F>*>(a.spec_out) + spec_off);
  } else if constexpr (MODE == PM_TAIL) {
    double acc[XR][EX][2];
#pragma unroll
    for (int rr = 0; rr < XR; ++rr)
#pragma unroll
      for (int m = 0; m < EX; ++m) acc[rr][m][0] = acc[rr][m][1] = 0.0;
    for (int k = 0; k < a.K; ++k) {
      const cx<F>* spec = reinterpret_cast<const cx<F>*>(a.spec_in) + spec_off + (long)k * a.chain_stride;
      const F* __restrict__ fac = reinterpret_cast<const F*>(a.fac) + (long)(2 * k + 1) * a.fac_table_stride + fac_off;
      const double ck = a.coef[k];
      column_inverse(spec);
#pragma unroll
      for (int rr = 0; rr < XR; ++rr) {
        const int row = rr * RPR + rloc;
        const bool act = row < NY;
        const int rowc = act ? row : 0;
        cx<F> v[EX];
        if (act) {
#pragma unroll
          for (int m = 0; m < EX; ++m) v[m] = lds[row * NXH + tx + TX * m];
        }
        fft<LX, +1>(v, tx, act, [&](int i) { return &lds[rowc * NXH + i]; }, rx);
        if (act) {
          const cx<F>* f2 = reinterpret_cast<const cx<F>*>(fac + (long)row * NX);
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> f = f2[tx + TX * m];
            acc[rr][m][0] += ck * (double)(v[m].x * f.x);
            acc[rr][m][1] += ck * (double)(v[m].y * f.y);
          }
        }
      }
      __syncthreads();
    }
    F* __restrict__ dst = reinterpret_cast<F*>(a.real_out) + real_off;
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
    column_inverse(reinterpret_cast<const cx<F>*>(a.spec_in) + spec_off);
    const F* __restrict__ phi = reinterpret_cast<const F*>(a.real_in) + real_off;
    const F* __restrict__ V = reinterpret_cast<const F*>(a.fac) + fac_off;
    F* __restrict__ dst = reinterpret_cast<F*>(a.real_out) + real_off;
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      const bool act = row < NY;
      const int rowc = act ? row : 0;
      cx<F> v[EX];
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = lds[row * NXH + tx + TX * m];
      }
      fft<LX, +1>(v, tx, act, [&](int i) { return &lds[rowc * NXH + i]; }, rx);
      if (act) {
        const cx<F>* p2 = reinterpret_cast<const cx<F>*>(phi + (long)row * NX);
        const cx<F>* v2 = reinterpret_cast<const cx<F>*>(V + (long)row * NX);
        cx<F>* d2 = reinterpret_cast<cx<F>*>(dst + (long)row * NX);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          const cx<F> p = p2[tx + TX * m], w = v2[tx + TX * m];
          d2[tx + TX * m] = cx<F>{v[m].x + w.x * p.x, v[m].y + w.y * p.y};
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
  __shared__ cx<F> lds[T > 1 ? NZ * C : 1];

  const int tid = threadIdx.x;
  const int col = tid % C, t = tid / C;
  const long s = (long)blockIdx.y + a.state0;
  const int gcol = blockIdx.x * C + col;
  const bool act = gcol < a.M;
  const int gc = act ? gcol : 0;
  cx<F>* data = reinterpret_cast<cx<F>*>(a.data) + s * a.state_stride;
  const cx<F>* rz = reinterpret_cast<const cx<F>*>(a.rz);
  const F* tx = reinterpret_cast<const F*>(a.tx);
  const F* ty = reinterpret_cast<const F*>(a.ty);
  const F* tz = reinterpret_cast<const F*>(a.tz);

  cx<F> v[E];
  if (act) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = data[(long)(t + T * m) * a.M + gcol];
  }
  auto buf = [&](int i) { return &lds[i * C + col]; };
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
  switch (mode) {
    case PM_FWD:
      hipLaunchKernelGGL((plane_kernel<F, N, N, PM_FWD>), grid, dim3(plane_block(N, PM_FWD)), 0, st, a);
      break;
    case PM_LINK:
      hipLaunchKernelGGL((plane_kernel<F, N, N, PM_LINK>), grid, dim3(plane_block(N, PM_LINK)), 0, st, a);
      break;
    case PM_TAIL:
      hipLaunchKernelGGL((plane_kernel<F, N, N, PM_TAIL>), grid, dim3(plane_block(N, PM_TAIL)), 0, st, a);
      break;
    case PM_HTAIL:
      hipLaunchKernelGGL((plane_kernel<F, N, N, PM_HTAIL>), grid, dim3(plane_block(N, PM_HTAIL)), 0, st, a);
      break;
    default:
      return hipErrorInvalidValue;
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
