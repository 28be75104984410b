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
//   PM_OUT   half spectrum -> real rows x exp(-tau_k V/2) of one chain (the
//            tail of a chain when the fused tail pass does not fit)
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

// PERSIST: 0 = one plane per work-group; 1 = persistent, register budget of one
// work-group per CU; 2 = persistent at the occupancy of PERSIST = 0; 3 (forward
// pass forming several chains) = one plane per work-group, every chain of it in
// turn, at the occupancy of PERSIST = 0.
template <typename F, int NX, int MODE, int PERSIST>
struct PlaneWaves {
  static constexpr int one_wg = (PlaneShape<NX>::BLOCK / 64 + 3) / 4;
  static constexpr int value = (MODE == PM_TAIL || PERSIST == 1) ? one_wg : PlaneOcc<F, NX>::value;
};

template <typename F, int NX, int MODE, int PERSIST>
__global__ __launch_bounds__(PlaneShape<NX>::BLOCK)
__attribute__((amdgpu_waves_per_eu(PlaneWaves<F, NX, MODE, PERSIST>::value))) void plane_kernel(PlaneArgs a) {
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
  static_assert(PERSIST == 0 || MODE == PM_FWD || MODE == PM_LINK, "persistent launches: forward and link passes");
  static_assert(PERSIST != 3 || MODE == PM_FWD, "the chain loop is a forward-pass form");
  constexpr bool TAIL_PREFETCH = sizeof(F) == 4 && EY <= 16;

  __shared__ cx<F> lds[NY * SROW];
  // twiddle tables staged in LDS (they sit on the FFT critical path)
  __shared__ cx<F> tw_x[LX], tw_y[NY], tw_w[HALF + 1];

  const int tid = threadIdx.x;
  const long plane_real = (long)NY * NX;
  const long plane_spec = (long)NY * NXH;
  // the arrays of state s (plane offsets added by the passes)
  // (explicitly global pointers: the loads and stores stay global_* instructions
  // after the pointers pass through this struct and the lambdas below)
  struct Ptrs {
    gp<const F> rin;
    gp<F> rout;
    gp<cx<F>> spec;
    long chain_stride;
    gp<const F> facb;
    gp<const F> facz;
  };
  auto ptrs_of = [&](long s) {
    Ptrs P;
    if (a.desc) {
      const StateDesc& d = a.desc[s];
      P.rin = (gp<const F>)reinterpret_cast<const F*>(d.real_in);
      P.rout = (gp<F>)reinterpret_cast<F*>(d.real_out);
      P.chain_stride = d.chain_stride;
      P.spec = (gp<cx<F>>)reinterpret_cast<cx<F>*>(d.spec) + (long)a.chain * P.chain_stride;
      P.facb = (gp<const F>)reinterpret_cast<const F*>(MODE == PM_HTAIL ? d.V : d.fac);
    } else {
      P.rin = (gp<const F>)reinterpret_cast<const F*>(a.real_in) + s * a.real_state_stride;
      P.rout = (gp<F>)reinterpret_cast<F*>(a.real_out) + s * a.real_state_stride;
      P.spec = (gp<cx<F>>)reinterpret_cast<cx<F>*>(a.spec) + s * a.spec_state_stride;
      P.chain_stride = a.chain_stride;
      P.facb = (gp<const F>)reinterpret_cast<const F*>(a.fac);
    }
    P.facz = (MODE == PM_HTAIL || MODE == PM_TAIL || a.fac_index < 0 || !P.facb)
                 ? P.facb
                 : P.facb + (long)a.fac_index * a.fac_table_stride;
    return P;
  };

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
  // threads beyond NCF*TY idle in the column phase; rows beyond NY in the row phase.
  // The checks stay run-time even where every thread is active: folded, they let
  // the compiler hoist loads across the transforms and raise register pressure.
  constexpr bool ALL_COLS = false, ALL_ROWS = false;
  const bool cact = ALL_COLS || ty < TY;
  const int g = f >> 1, h = f & 1;
  const bool packed = (g == 0 && h == 0);
  const int col = (g == 0) ? (h ? HALF : 0) : (h ? LX - g : g);   // LDS / spectrum column
  const int tyc = cact ? ty : 0;
  // LDS slot of spectrum column c: the upper half of the columns is rotated by
  // one slot (HALF -> LX - 1, c -> c - 1 above it).  The column phase pairs
  // columns g and LX - g on neighbouring lanes; unrotated, g and LX - g share a
  // bank for g = 0 mod 16 (and HALF shares one with 0), a two-way conflict in
  // every pass of a column exchange.  Rotated, the columns of a half-wave fill
  // distinct banks, and a row's TX consecutive columns stay in distinct ones.
  static_assert(HALF % TX == 0, "row segments do not straddle the rotated half");
  auto cslot = [&](int c) { return c < HALF ? c : (c == HALF ? LX - 1 : c - 1); };
  // slot of column tx + TX m (m unrolled: only the segment holding HALF selects)
  auto rslot = [&](int m) {
    const int c = tx + TX * m;
    if (TX * m < HALF) return c;
    if (TX * m > HALF) return c - 1;
    return tx == 0 ? LX - 1 : c - 1;
  };
  const int cs_col = cslot(col), cs_mirror = cslot(LX - col);
  // Byte offsets of the buffer accesses (see bload): one per-lane offset per
  // access pattern, the element's wave-uniform part in a compile-time offset.
  // Real rows as complex pairs: row rr * RPR + rloc, pair tx + TX m.
  constexpr unsigned CXB = sizeof(cx<F>);
  constexpr unsigned REAL_PLANE_B = (unsigned)(NY * NX * sizeof(F)), SPEC_PLANE_B = (unsigned)(NY * NXH * CXB);
  const unsigned row_vo = (unsigned)(rloc * LX + tx) * CXB;
  auto row_so = [](int rr, int m) -> unsigned { return (unsigned)(rr * RPR * LX + TX * m) * CXB; };
  // Spectrum columns: row tyc + TY m, column col (or LX, the Nyquist column).
  const unsigned col_vo = (unsigned)(tyc * NXH + col) * CXB, nyq_vo = (unsigned)(tyc * NXH + LX) * CXB;
  auto col_so = [](int m) -> unsigned { return (unsigned)(TY * m * NXH) * CXB; };
  auto cbuf = [&](int i) { return &lds[i * SROW + cs_col]; };
  // Row-transform exchange slots: element i of row r at r * SROW + i + i / EX.
  // The exchange writes lane t's outputs at E t + k; one pad slot per E
  // elements moves the T lanes of a row to different LDS banks (without it
  // they share a bank), and the strided reads t + T m stay conflict-free.
  static_assert((LX - 1) + (LX - 1) / EX < SROW, "padded row exchange fits the row stride");
  auto rowbuf = [&](int r) { return [&, r](int i) { return &lds[r * SROW + i + i / EX]; }; };

  // W^k for k = 0..LX (W^(LX-j) = -conj W^j)
  auto wk = [&](int k) -> cx<F> {
    return k <= HALF ? wpost[k] : cx<F>{-wpost[LX - k].x, wpost[LX - k].y};
  };

  // ---- spectrum in: column loads (issued early when pipelined), inverse y FFT,
  //      c2r split in registers, Z rows to LDS
  // The packed lane (DC and Nyquist columns) loads like every other lane plus
  // the row's Nyquist value, which all lanes load too (one address per row), so
  // the loads stay full-wave instructions without a divergent branch.
  auto column_load = [&](gp<const cx<F>> __restrict__ spec, cx<F>* v) {
    const brsrc r = make_brsrc(spec, SPEC_PLANE_B);
    if (cact) {
#pragma unroll
      for (int m = 0; m < EY; ++m) {
        const cx<F> y0 = bload<F>(r, col_vo, col_so(m)), yl = bload<F>(r, nyq_vo, col_so(m));
        v[m] = packed ? cx<F>{y0.x - yl.y, y0.y + yl.x} : y0;   // Y0 + i Y_LX
      }
    }
  };
  auto column_inverse_regs = [&](cx<F>* v) {
    fft<NY, +1>(v, tyc, cact, cbuf, ry);
    // split: needs X[LX - col] at the same y, held by the neighbouring lane
    const cx<F> w = wk(col);
#pragma unroll
    for (int m = 0; m < EY; ++m) {
      const cx<F> pr{lane_xor1(v[m].x), lane_xor1(v[m].y)};
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
      for (int m = 0; m < EY; ++m) lds[(tyc + TY * m) * SROW + cs_col] = v[m];
    }
    __syncthreads();
  };
  auto column_inverse = [&](gp<const cx<F>> __restrict__ spec) {
    cx<F> v[EY];
    column_load(spec, v);
    column_inverse_regs(v);
  };

  // ---- columns forward out: r2c split on load, forward y FFT, store
  auto column_forward_store = [&](gp<cx<F>> __restrict__ spec) {
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
          const cx<F> A = r[cs_col], B = conj(r[cs_mirror]);
          const cx<F> E = scale(A + B, F(0.5));
          const cx<F> O = muli<-1>(scale(A - B, F(0.5)));
          v[m] = E + cmul(O, w);
        }
      }
    }
    __syncthreads();   // every Z value read before the exchanges reuse the columns
    fft<NY, -1>(v, tyc, cact, cbuf, ry);
    // unpack the DC / Nyquist column: X0[k] = (C[k] + conj C[-k])/2, X_LX[k] = -i (C[k] - conj C[-k])/2;
    // C[-k] comes from another wave through LDS, then one store per row serves every lane
    if (cact && packed) {
#pragma unroll
      for (int m = 0; m < EY; ++m) lds[(tyc + TY * m) * SROW] = v[m];
    }
    __syncthreads();
    const brsrc r = make_brsrc(spec, SPEC_PLANE_B);
    if (cact) {
#pragma unroll
      for (int m = 0; m < EY; ++m) {
        const int ky = tyc + TY * m;
        const cx<F> c = v[m], cm = conj(lds[((NY - ky) % NY) * SROW]);
        const F hx = F(0.5) * (c.x + cm.x), hy = F(0.5) * (c.y + cm.y);
        cx<F> o;
        o.x = packed ? hx : c.x;
        o.y = packed ? hy : c.y;
        bstore<F>(r, col_vo, col_so(m), o);
      }
      if (packed) {
#pragma unroll
        for (int m = 0; m < EY; ++m) {
          const int ky = tyc + TY * m;
          const cx<F> c = v[m], cm = conj(lds[((NY - ky) % NY) * SROW]);
          bstore<F>(r, nyq_vo, col_so(m), muli<-1>(scale(c - cm, F(0.5))));
        }
      }
    }
  };

  if constexpr (MODE == PM_FWD || MODE == PM_LINK) {
    // Work items of this work-group: one (chain, z, state) item, or in a
    // persistent launch every gridDim.x-th item of the launch; the next item's input
    // (rows for the forward pass, spectrum columns for the link pass) is
    // loaded while the current plane is transformed.
    // A forward launch can form several chains (fwd_chains) from each plane of
    // rows.  The chains of one plane run on work-groups of one XCD (work-group
    // w runs on XCD w mod 8), so the plane comes from HBM once and from that
    // XCD's L2 for the other chains: item w is chain (w / 8) mod nch of plane
    // index 8 (w / 8 nch) + w mod 8, plane indices padded to a multiple of 8
    // (the padding is skipped).  With one chain the item is the plane index.
    // The plane index runs over the (z, state) pairs with z or states fastest.
    // In the chain loop (PERSIST = 3) a work-group forms every chain of its
    // plane instead, one after the other, reading the rows again from its own
    // CU's caches for each chain.
    constexpr bool PERS = PERSIST == 1 || PERSIST == 2, CHAIN_LOOP = PERSIST == 3;
    const int nch = (MODE == PM_FWD && a.fwd_chains > 1 && !CHAIN_LOOP) ? a.fwd_chains : 1;
    const long nplanes = (long)a.nz * a.nstates;
    const long nwork = nch == 1 ? nplanes : (nplanes + 7) / 8 * 8 * nch;
    auto plane_of = [&](long w, int& cw) -> long {
      if (nch == 1) {
        cw = 0;
        return w;
      }
      cw = (int)((w >> 3) % nch);
      return (w / (8L * nch)) * 8 + (w & 7);
    };
    // item q (persistent) or this work-group's item -> (z, chain, state
    // pointers); false for padding
    auto locate = [&](long q, int& zq, int& cq, Ptrs& Pq) -> bool {
      long sq;
      if constexpr (PERS) {
        const long u = plane_of(q, cq);
        if (u >= nplanes) return false;
        if (a.states_fast) {
          sq = u % a.nstates + a.state0;
          zq = (int)(u / a.nstates);
        } else {
          zq = (int)(u % a.nz);
          sq = u / a.nz + a.state0;
        }
      } else {
        const long u = plane_of((long)blockIdx.x, cq);
        if (a.states_fast) {
          if (u >= a.nstates) return false;
          zq = blockIdx.y;
          sq = u + a.state0;
        } else {
          if (u >= a.nz) return false;
          zq = (int)u;
          sq = (long)blockIdx.y + a.state0;
        }
      }
      Pq = ptrs_of(sq);
      return true;
    };
    constexpr int NPRE = MODE == PM_FWD ? XR * EX : EY;
    cx<F> pre[NPRE];
    auto prefetch = [&](int zq, const Ptrs& Pq) {
      if constexpr (MODE == PM_FWD) {
        const brsrc r = make_brsrc(Pq.rin + (long)zq * plane_real, REAL_PLANE_B);
#pragma unroll
        for (int rr = 0; rr < XR; ++rr) {
          const int row = rr * RPR + rloc;
          if (row < NY) {
#pragma unroll
            for (int m = 0; m < EX; ++m) pre[rr * EX + m] = bload<F>(r, row_vo, row_so(rr, m));
          }
        }
      } else {
        column_load(Pq.spec + (long)zq * plane_spec, pre);
      }
    };
    const long pstep = PERS ? (long)gridDim.x : 0;
    long p = PERS ? (long)blockIdx.x : 0;
    int z, ch;
    Ptrs P;
    // (a whole work-group leaves here together: no barrier has been reached)
    if constexpr (PERS) {
      while (p < nwork && !locate(p, z, ch, P)) p += pstep;
      if (p >= nwork) return;
    } else {
      if (!locate(0, z, ch, P)) return;
    }
    prefetch(z, P);
    for (;;) {
      long pn = p + pstep;
      if constexpr (PERS) {
        int cn;
        while (pn < nwork && plane_of(pn, cn) >= nplanes) pn += pstep;
      }
      const bool more = PERS && pn < nwork;
      int zn = z, chn = ch;
      Ptrs Pn = P;
      const long z_real = (long)z * plane_real;
      if constexpr (MODE == PM_FWD) {
        const bool has_fac = a.fac_index >= 0 && P.facz;
        const brsrc rf = make_brsrc(has_fac ? P.facz + (long)(2 * ch) * a.fac_table_stride + z_real : P.facz,
                                    REAL_PLANE_B);   // (not read without a factor table)
#pragma unroll
        for (int rr = 0; rr < XR; ++rr) {
          const int row = rr * RPR + rloc;
          const bool act = ALL_ROWS || row < NY;
          const int rowc = act ? row : 0;
          cx<F> v[EX];
#pragma unroll
          for (int m = 0; m < EX; ++m) v[m] = pre[rr * EX + m];
          if (act && has_fac) {
#pragma unroll
            for (int m = 0; m < EX; ++m) {
              const cx<F> fv = bload<F>(rf, row_vo, row_so(rr, m));
              v[m].x *= fv.x;
              v[m].y *= fv.y;
            }
          }
          fft<LX, -1, ROWWAVE>(v, tx, act, rowbuf(rowc), rx);
          if (act) {
#pragma unroll
            for (int m = 0; m < EX; ++m) lds[row * SROW + rslot(m)] = v[m];
          }
        }
        if (more) {
          locate(pn, zn, chn, Pn);
          prefetch(zn, Pn);
        }
      } else {
        column_inverse_regs(pre);
        if (more) {
          locate(pn, zn, chn, Pn);
          prefetch(zn, Pn);
        }
        const brsrc rf = make_brsrc(P.facz + z_real, REAL_PLANE_B);
#pragma unroll
        for (int rr = 0; rr < XR; ++rr) {
          const int row = rr * RPR + rloc;
          const bool act = ALL_ROWS || row < NY;
          const int rowc = act ? row : 0;
          cx<F> v[EX];
          if (act) {
#pragma unroll
            for (int m = 0; m < EX; ++m) v[m] = lds[row * SROW + rslot(m)];
          }
          fft<LX, +1, ROWWAVE>(v, tx, act, rowbuf(rowc), rx);
          if (act) {
#pragma unroll
            for (int m = 0; m < EX; ++m) {
              const cx<F> fv = bload<F>(rf, row_vo, row_so(rr, m));
              v[m].x *= fv.x;
              v[m].y *= fv.y;
            }
          }
          fft<LX, -1, ROWWAVE>(v, tx, act, rowbuf(rowc), rx);
          if (act) {
#pragma unroll
            for (int m = 0; m < EX; ++m) lds[row * SROW + rslot(m)] = v[m];
          }
        }
      }
      column_forward_store(P.spec + (long)ch * P.chain_stride + (long)z * plane_spec);
      if constexpr (CHAIN_LOOP) {
        // the other chains of this plane: the rows again (from this CU's
        // caches), each chain's factor table, the transforms, its own spectrum
        // (a copy of the row pass above, with the rows loaded in place: kept in
        // the loop, the prefetched rows' registers spill)
        for (int c2 = 1; c2 < a.fwd_chains; ++c2) {
          __syncthreads();   // the DC / Nyquist epilogue still reads the plane in LDS
          const brsrc rsrc = make_brsrc(P.rin + z_real, REAL_PLANE_B);
          const brsrc rf = make_brsrc(P.facz + (long)(2 * c2) * a.fac_table_stride + z_real, REAL_PLANE_B);
#pragma unroll
          for (int rr = 0; rr < XR; ++rr) {
            const int row = rr * RPR + rloc;
            const bool act = ALL_ROWS || row < NY;
            const int rowc = act ? row : 0;
            cx<F> v[EX];
#pragma unroll
            for (int m = 0; m < EX; ++m) v[m] = bload<F>(rsrc, row_vo, row_so(rr, m));
            if (act) {
#pragma unroll
              for (int m = 0; m < EX; ++m) {
                const cx<F> fv = bload<F>(rf, row_vo, row_so(rr, m));
                v[m].x *= fv.x;
                v[m].y *= fv.y;
              }
            }
            fft<LX, -1, ROWWAVE>(v, tx, act, rowbuf(rowc), rx);
            if (act) {
#pragma unroll
              for (int m = 0; m < EX; ++m) lds[row * SROW + rslot(m)] = v[m];
            }
          }
          column_forward_store(P.spec + (long)c2 * P.chain_stride + (long)z * plane_spec);
        }
      }
      if (!more) break;
      __syncthreads();   // the DC / Nyquist epilogue still reads the plane in LDS
      p = pn;
      z = zn;
      ch = chn;
      P = Pn;
    }
  } else if constexpr (MODE == PM_TAIL) {
    const int z = blockIdx.y;
    const Ptrs P = ptrs_of((long)blockIdx.x + a.state0);
    const long z_real = (long)z * plane_real, z_spec = (long)z * plane_spec;
    gp<cx<F>> spec = P.spec;
    gp<const F> facb = P.facb;
    const long chain_stride = P.chain_stride;
    gp<F> rout = P.rout;
    double acc[XR][EX][2];
#pragma unroll
    for (int rr = 0; rr < XR; ++rr)
#pragma unroll
      for (int m = 0; m < EX; ++m) acc[rr][m][0] = acc[rr][m][1] = 0.0;
    // the next chain's column loads are issued before this chain's row work,
    // so their latency hides behind it (one work-group per CU here)
    gp<const cx<F>> spec0 = spec + z_spec;
    cx<F> vc[EY];
    column_load(spec0, vc);
    for (int k = 0; k < a.K; ++k) {
      const brsrc rf = make_brsrc(facb + (long)(2 * k + 1) * a.fac_table_stride + z_real, REAL_PLANE_B);
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
        const bool act = ALL_ROWS || row < NY;
        const int rowc = act ? row : 0;
        cx<F> v[EX];
        if (act) {
#pragma unroll
          for (int m = 0; m < EX; ++m) v[m] = lds[row * SROW + rslot(m)];
        }
        fft<LX, +1, ROWWAVE>(v, tx, act, rowbuf(rowc), rx);
        if (act) {
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> fv = bload<F>(rf, row_vo, row_so(rr, m));
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
    const brsrc rd = make_brsrc(rout + z_real, REAL_PLANE_B);
#pragma unroll
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      if (row < NY) {
#pragma unroll
        for (int m = 0; m < EX; ++m)
          bstore<F>(rd, row_vo, row_so(rr, m), cx<F>{(F)acc[rr][m][0], (F)acc[rr][m][1]});
      }
    }
  } else {  // PM_HTAIL, PM_OUT
    const int z = a.states_fast ? blockIdx.y : blockIdx.x;
    const Ptrs P = ptrs_of((long)(a.states_fast ? blockIdx.x : blockIdx.y) + a.state0);
    const long z_real = (long)z * plane_real, z_spec = (long)z * plane_spec;
    gp<cx<F>> spec = P.spec;
    gp<const F> facb = P.facb;
    gp<const F> rin = P.rin;
    gp<F> rout = P.rout;
    column_inverse(spec + z_spec);
    const brsrc rp = make_brsrc(MODE == PM_OUT ? rin : rin + z_real, REAL_PLANE_B);   // (PM_OUT: not read)
    const brsrc rv = make_brsrc((MODE == PM_OUT ? P.facz : facb) + z_real, REAL_PLANE_B);
    const brsrc rd = make_brsrc(rout + z_real, REAL_PLANE_B);
#pragma unroll
    for (int rr = 0; rr < XR; ++rr) {
      const int row = rr * RPR + rloc;
      const bool act = ALL_ROWS || row < NY;
      const int rowc = act ? row : 0;
      cx<F> v[EX];
      if (act) {
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = lds[row * SROW + rslot(m)];
      }
      fft<LX, +1, ROWWAVE>(v, tx, act, rowbuf(rowc), rx);
      if (act) {
        if constexpr (MODE == PM_OUT) {
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> wv = bload<F>(rv, row_vo, row_so(rr, m));
            bstore<F>(rd, row_vo, row_so(rr, m), cx<F>{v[m].x * wv.x, v[m].y * wv.y});
          }
        } else {
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> pv = bload<F>(rp, row_vo, row_so(rr, m)), wv = bload<F>(rv, row_vo, row_so(rr, m));
            bstore<F>(rd, row_vo, row_so(rr, m), cx<F>{v[m].x + wv.x * pv.x, v[m].y + wv.y * pv.y});
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ pencil pass
// Columns per work-group: THREADS / T (the T lanes of a column transform).
template <int NZ, int THREADS>
struct PencilCols {
  static constexpr int value = THREADS / Plan<NZ>::T;
};

template <typename F, int NZ, int KIND, int THREADS = 256>
__global__ __launch_bounds__(THREADS) void pencil_kernel(PencilArgs a) {
  using P = Plan<NZ>;
  constexpr int T = P::T, E = P::E;
  constexpr int C = PencilCols<NZ, THREADS>::value;
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
  for (int i = tid; i < NZ; i += THREADS) {
    rz_s[i] = reinterpret_cast<const cx<F>*>(a.rz)[i];
    if constexpr (KIND == PK_EXP || KIND == PK_ADD) tz_s[i] = tab[a.NXH + a.NY + i];
  }
  const cx<F>* rz = rz_s;
  const F* tz = tz_s;

  // buffer accesses (see bload): element (t + T m, gcol) at byte offset
  // (t M + gcol) |cx| per lane plus T m M |cx| in a scalar register
  const brsrc rdat = make_brsrc((gp<cx<F>>)data, (unsigned)((long)NZ * a.M * (long)sizeof(cx<F>)));
  const unsigned vo = (unsigned)(t * a.M + gc) * (unsigned)sizeof(cx<F>);
  const unsigned so_m = (unsigned)(T * a.M) * (unsigned)sizeof(cx<F>);
  cx<F> v[E];
  if (act) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = bload<F>(rdat, vo, so_m * m);
  }
  __syncthreads();   // staged tables visible
  auto buf = [&](int i) { return &lds[i * CP + col]; };
  if constexpr (KIND == PK_FFT_INV) {
    fft<NZ, +1>(v, t, act, buf, rz);
  } else {
    fft<NZ, -1>(v, t, act, buf, rz);
  }
  if constexpr (KIND == PK_EXP || KIND == PK_ADD) {
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
  }
  if (act) {
#pragma unroll
    for (int m = 0; m < E; ++m) bstore<F>(rdat, vo, so_m * m, v[m]);
  }
}


// ------------------------------------------------------------------ row pass (three-pass plans)
// The x transforms alone, for grids whose planes do not fit the plane pass
// (nx != ny, or float64 planes above the LDS size): a row of NX real points and
// its half spectrum X[0..NX/2] go through the NX/2-point complex FFT of the
// packed row z_j = x_2j + i x_2j+1 and the split (W = exp(-2 pi i / NX),
// Z[NX/2] = Z[0])
//   X[k] = (Z[k] + conj Z[NX/2-k])/2 - i W^k (Z[k] - conj Z[NX/2-k])/2,
// and back (unnormalised, as the plane pass: 2 Z[k] = (X[k] + conj X[NX/2-k])
//   + i conj(W^k) (X[k] - conj X[NX/2-k])).
// A row is carried by the TX lanes of its transform (consecutive lanes of one
// wavefront); ROWS rows per work-group, each with its own LDS row for the
// transform's exchanges and the split's mirrored reads.
template <int NX>
struct RowShape {
  static constexpr int LX = NX / 2;
  static constexpr int TX = Plan<LX>::T;
  static constexpr int ROWS = 64 / TX < 16 ? 16 : 64 / TX;   // >= one wavefront of lanes
  static constexpr int BLOCK = ROWS * TX;
};

template <typename F, int NX, int MODE>
__global__ __launch_bounds__(RowShape<NX>::BLOCK) void row_kernel(PlaneArgs a) {
  constexpr int LX = NX / 2, NXH = LX + 1, HALF = LX / 2;
  using PX = Plan<LX>;
  constexpr int TX = PX::T, EX = PX::E, ROWS = RowShape<NX>::ROWS;
  constexpr int RS = LX + (LX - 1) / EX + 2;   // LDS row: padded exchange slots, or LX + 1 spectrum entries
  static_assert(RS >= NXH, "a row holds the half spectrum");
  __shared__ cx<F> lds[ROWS * RS];
  __shared__ cx<F> tw_x[LX], tw_w[HALF + 1];
  const int tid = threadIdx.x;
  {
    const cx<F>* gx = reinterpret_cast<const cx<F>*>(a.rx);
    const cx<F>* gw = reinterpret_cast<const cx<F>*>(a.wpost);
    for (int i = tid; i < LX; i += RowShape<NX>::BLOCK) tw_x[i] = gx[i];
    for (int i = tid; i <= HALF; i += RowShape<NX>::BLOCK) tw_w[i] = gw[i];
  }
  __syncthreads();
  const int tx = tid % TX, rl = tid / TX;
  const long rows_per_state = (long)a.nz * a.ny;
  const long row = (long)blockIdx.x * ROWS + rl;
  const bool act = row < (long)a.nstates * rows_per_state;
  const long rowc = act ? row : 0;
  const long s = rowc / rows_per_state + a.state0;
  const long zy = rowc % rows_per_state;          // z * ny + y
  cx<F>* R = lds + rl * RS;
  auto xbuf = [&](int i) { return R + i + i / EX; };
  auto wk = [&](int k) -> cx<F> {
    return k <= HALF ? tw_w[k] : cx<F>{-tw_w[LX - k].x, tw_w[LX - k].y};
  };
  gp<cx<F>> spec = (gp<cx<F>>)reinterpret_cast<cx<F>*>(a.spec) + s * a.spec_state_stride + zy * NXH;
  gp<const F> fac = (a.fac && a.fac_index >= 0)
                        ? (gp<const F>)reinterpret_cast<const F*>(a.fac) + (long)a.fac_index * a.fac_table_stride +
                              zy * NX
                        : nullptr;
  cx<F> v[EX];

  // half spectrum row -> 2 Z (strided order) through the LDS row
  auto inverse_split = [&]() {
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      const int k = tx + TX * m;
      if (act) R[k] = gload<F>(spec + k);
    }
    if (act && tx == 0) R[LX] = gload<F>(spec + LX);
    wave_sync();
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      const int k = tx + TX * m;
      const cx<F> X = R[k], Xm = conj(R[LX - k]);
      v[m] = (X + Xm) + muli<+1>(cmulc(X - Xm, wk(k)));
    }
    wave_sync();
  };
  // Z (strided order) -> half spectrum row through the LDS row
  auto forward_split_store = [&]() {
    wave_sync();
#pragma unroll
    for (int m = 0; m < EX; ++m) R[tx + TX * m] = v[m];
    if (tx == 0) R[LX] = v[0];
    wave_sync();
    if (act) {
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        const int k = tx + TX * m;
        const cx<F> A = R[k], B = conj(R[LX - k]);
        const cx<F> E = scale(A + B, F(0.5)), O = muli<-1>(scale(A - B, F(0.5)));
        gstore<F>(spec + k, E + cmul(O, wk(k)));
      }
      if (tx == 0) {
        const cx<F> A = R[LX], B = conj(R[0]);
        const cx<F> E = scale(A + B, F(0.5)), O = muli<-1>(scale(A - B, F(0.5)));
        gstore<F>(spec + LX, E + cmul(O, wk(LX)));
      }
    }
  };

  if constexpr (MODE == RW_FWD) {
    gp<const cx<F>> src = reinterpret_cast<gp<const cx<F>>>((gp<const F>)reinterpret_cast<const F*>(a.real_in) +
                                                          s * a.real_state_stride + zy * NX);
    gp<const cx<F>> f2 = fac ? reinterpret_cast<gp<const cx<F>>>(fac) : nullptr;
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      v[m] = act ? gload<F>(src + tx + TX * m) : cx<F>{F(0), F(0)};
      if (act && f2) {
        const cx<F> fv = gload<F>(f2 + tx + TX * m);
        v[m].x *= fv.x;
        v[m].y *= fv.y;
      }
    }
    fft<LX, -1, true>(v, tx, true, xbuf, tw_x);
    forward_split_store();
  } else {
    inverse_split();
    fft<LX, +1, true>(v, tx, true, xbuf, tw_x);
    if constexpr (MODE == RW_LINK) {
      gp<const cx<F>> f2 = reinterpret_cast<gp<const cx<F>>>(fac);
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        if (act) {
          const cx<F> fv = gload<F>(f2 + tx + TX * m);
          v[m].x *= fv.x;
          v[m].y *= fv.y;
        }
      }
      fft<LX, -1, true>(v, tx, true, xbuf, tw_x);
      forward_split_store();
    } else {
      gp<cx<F>> dst = reinterpret_cast<gp<cx<F>>>((gp<F>)reinterpret_cast<F*>(a.real_out) +
                                                s * a.real_state_stride + zy * NX);
      if (act) {
        if constexpr (MODE == RW_OUT) {
          gp<const cx<F>> f2 = reinterpret_cast<gp<const cx<F>>>(fac);
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> fv = gload<F>(f2 + tx + TX * m);
            gstore<F>(dst + tx + TX * m, cx<F>{v[m].x * fv.x, v[m].y * fv.y});
          }
        } else {   // RW_HTAIL: + V * phi
          gp<const cx<F>> ph = reinterpret_cast<gp<const cx<F>>>((gp<const F>)reinterpret_cast<const F*>(a.real_in) +
                                                               s * a.real_state_stride + zy * NX);
          gp<const cx<F>> V2 = reinterpret_cast<gp<const cx<F>>>((gp<const F>)reinterpret_cast<const F*>(a.fac) +
                                                               zy * NX);
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const cx<F> pv = gload<F>(ph + tx + TX * m), wv = gload<F>(V2 + tx + TX * m);
            gstore<F>(dst + tx + TX * m, cx<F>{v[m].x + wv.x * pv.x, v[m].y + wv.y * pv.y});
          }
        }
      }
    }
  }
}

template <typename F, int N>
static hipError_t launch_rows_n(int mode, const PlaneArgs& a0, int ny, int nz, int nstates, hipStream_t st) {
  PlaneArgs a = a0;
  a.ny = ny;
  a.nz = nz;
  a.nstates = nstates;
  const long rows = (long)nstates * nz * ny;
  constexpr int ROWS = RowShape<N>::ROWS;
  const dim3 grid((unsigned)((rows + ROWS - 1) / ROWS)), block(RowShape<N>::BLOCK);
  switch (mode) {
    case RW_FWD: hipLaunchKernelGGL((row_kernel<F, N, RW_FWD>), grid, block, 0, st, a); break;
    case RW_LINK: hipLaunchKernelGGL((row_kernel<F, N, RW_LINK>), grid, block, 0, st, a); break;
    case RW_OUT: hipLaunchKernelGGL((row_kernel<F, N, RW_OUT>), grid, block, 0, st, a); break;
    case RW_HTAIL: hipLaunchKernelGGL((row_kernel<F, N, RW_HTAIL>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename F>
static hipError_t launch_rows_t(int mode, int nx, const PlaneArgs& a, int ny, int nz, int ns, hipStream_t st) {
  switch (nx) {
    case 8: return launch_rows_n<F, 8>(mode, a, ny, nz, ns, st);
    case 16: return launch_rows_n<F, 16>(mode, a, ny, nz, ns, st);
    case 32: return launch_rows_n<F, 32>(mode, a, ny, nz, ns, st);
    case 48: return launch_rows_n<F, 48>(mode, a, ny, nz, ns, st);
    case 64: return launch_rows_n<F, 64>(mode, a, ny, nz, ns, st);
    case 96: return launch_rows_n<F, 96>(mode, a, ny, nz, ns, st);
    case 128: return launch_rows_n<F, 128>(mode, a, ny, nz, ns, st);
    case 192: return launch_rows_n<F, 192>(mode, a, ny, nz, ns, st);
    default: return hipErrorInvalidValue;
  }
}

bool row_supported(int nx) {
  switch (nx) {
    case 8: case 16: case 32: case 48: case 64: case 96: case 128: case 192: return true;
    default: return false;
  }
}

hipError_t launch_rows(int is_double, int mode, int nx, const PlaneArgs& a, int ny, int nz, int nstates,
                       hipStream_t st) {
  if (nstates <= 0) return hipSuccess;
  return is_double ? launch_rows_t<double>(mode, nx, a, ny, nz, nstates, st)
                   : launch_rows_t<float>(mode, nx, a, ny, nz, nstates, st);
}

// ------------------------------------------------------------------ launchers
template <typename F, int N>
static hipError_t launch_plane_n(int mode, const PlaneArgs& a0, int nz, int nstates, hipStream_t st) {
  dim3 block(PlaneShape<N>::BLOCK);
  PlaneArgs a = a0;
  a.nz = nz;
  a.nstates = nstates;
  if (mode != PM_FWD) a.fwd_chains = 0;
  const int nch = a.fwd_chains > 1 ? a.fwd_chains : 1;
  if constexpr (N >= 64) {
    if (a.persist_blocks > 0 && (a.persist_mode == 1 || a.persist_mode == 2) && (mode == PM_FWD || mode == PM_LINK)) {
      const PlaneArgs& b = a;
      const long nplanes = (long)nz * nstates;
      const long nwork = nch == 1 ? nplanes : (nplanes + 7) / 8 * 8 * nch;
      dim3 grid((unsigned)(a.persist_blocks < nwork ? a.persist_blocks : nwork));
      if (a.persist_mode == 1) {
        if (mode == PM_FWD) hipLaunchKernelGGL((plane_kernel<F, N, PM_FWD, 1>), grid, block, 0, st, b);
        else hipLaunchKernelGGL((plane_kernel<F, N, PM_LINK, 1>), grid, block, 0, st, b);
      } else {
        if (mode == PM_FWD) hipLaunchKernelGGL((plane_kernel<F, N, PM_FWD, 2>), grid, block, 0, st, b);
        else hipLaunchKernelGGL((plane_kernel<F, N, PM_LINK, 2>), grid, block, 0, st, b);
      }
      return hipGetLastError();
    }
  }
  // The forward, link, H-tail and single-chain passes take the order of
  // PlaneArgs::states_fast; the fused tail pass always walks states fastest,
  // so the work-groups in flight share a few z planes and the 2K
  // potential-factor planes they read stay in every XCD's L2 while the states
  // stream past
  dim3 grid(nz, nstates), grid_t(nstates, nz);
  const dim3 grid_fl = a.states_fast ? grid_t : grid;   // forward / link: either order
  if constexpr (N >= 64) {
    if (mode == PM_FWD && nch > 1 && a.fwd_loop) {
      // chain loop: one work-group per plane forms all nch chains
      hipLaunchKernelGGL((plane_kernel<F, N, PM_FWD, 3>), grid_fl, block, 0, st, a);
      return hipGetLastError();
    }
  }
  // forward launches forming several chains: nch items per plane, the fast
  // extent padded to a multiple of 8 (see the item map in plane_kernel)
  const dim3 grid_fwd = nch == 1 ? grid_fl : dim3((unsigned)((grid_fl.x + 7) / 8 * 8 * nch), grid_fl.y);
  switch (mode) {
    case PM_FWD: hipLaunchKernelGGL((plane_kernel<F, N, PM_FWD, 0>), grid_fwd, block, 0, st, a); break;
    case PM_LINK: hipLaunchKernelGGL((plane_kernel<F, N, PM_LINK, 0>), grid_fl, block, 0, st, a); break;
    case PM_TAIL: hipLaunchKernelGGL((plane_kernel<F, N, PM_TAIL, 0>), grid_t, block, 0, st, a); break;
    case PM_HTAIL: hipLaunchKernelGGL((plane_kernel<F, N, PM_HTAIL, 0>), grid_fl, block, 0, st, a); break;
    case PM_OUT: hipLaunchKernelGGL((plane_kernel<F, N, PM_OUT, 0>), grid_fl, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename F, int N, int THREADS>
static hipError_t launch_pencil_nt(int kind, const PencilArgs& a, int nstates, hipStream_t st) {
  constexpr int C = PencilCols<N, THREADS>::value;
  dim3 grid((a.M + C - 1) / C, nstates), block(THREADS);
  switch (kind) {
    case PK_EXP: hipLaunchKernelGGL((pencil_kernel<F, N, PK_EXP, THREADS>), grid, block, 0, st, a); break;
    case PK_ADD: hipLaunchKernelGGL((pencil_kernel<F, N, PK_ADD, THREADS>), grid, block, 0, st, a); break;
    case PK_FFT_FWD: hipLaunchKernelGGL((pencil_kernel<F, N, PK_FFT_FWD, THREADS>), grid, block, 0, st, a); break;
    case PK_FFT_INV: hipLaunchKernelGGL((pencil_kernel<F, N, PK_FFT_INV, THREADS>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// LDS of one pencil work-group: the transform's exchange rows plus the staged tables.
template <typename F, int N, int THREADS>
constexpr size_t pencil_lds() {
  return (Plan<N>::T > 1 ? (size_t)N * (PencilCols<N, THREADS>::value + 1) : 1) * 2 * sizeof(F) +
         (size_t)N * 3 * sizeof(F);
}

template <typename F, int N>
static hipError_t launch_pencil_n(int kind, const PencilArgs& a, int nstates, hipStream_t st) {
  // other tile shapes where the transform spans several lanes and the LDS fits
  if constexpr (Plan<N>::T >= 2) {
    if (a.tile == 1) return launch_pencil_nt<F, N, 128>(kind, a, nstates, st);
    if constexpr (pencil_lds<F, N, 512>() <= 64 * 1024) {
      if (a.tile == 2) return launch_pencil_nt<F, N, 512>(kind, a, nstates, st);
    }
  }
  return launch_pencil_nt<F, N, 256>(kind, a, nstates, st);
}

bool plane_supported(int is_double, int nx, int ny) {
  if (nx != ny) return false;
  switch (nx) {
    case 8: case 16: case 32: case 48: case 64: case 96: case 128: return true;
    case 192: return !is_double;   // 192 x 97 complex doubles exceed the 160 KB LDS
    default: return false;
  }
}

bool tail_split(int is_double, int nx) { return is_double ? nx >= 128 : nx >= 192; }

struct Coefs {
  double c[MAX_K];
};

// dst = sum_k c_k tmp_k (float64 sum, one rounding on store), 4 elements per thread
template <typename F>
__global__ __launch_bounds__(256) void combine_kernel(const F* __restrict__ tmp, long stride, int K, Coefs c,
                                                      F* __restrict__ dst, long n) {
  const long i0 = ((long)blockIdx.x * 256 + threadIdx.x) * 4;
  if (i0 >= n) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int cnt = (int)(n - i0 < 4 ? n - i0 : 4);
  for (int k = 0; k < K; ++k) {
    const F* t = tmp + k * stride + i0;
    const double ck = c.c[k];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (e < cnt) acc[e] += ck * (double)t[e];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (e < cnt) dst[i0 + e] = (F)acc[e];
}

hipError_t launch_combine(int is_double, const void* tmp, long stride, int K, const double* coef, void* dst, long n,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  Coefs c;
  for (int k = 0; k < MAX_K; ++k) c.c[k] = k < K ? coef[k] : 0.0;
  const dim3 grid((unsigned)((n + 1023) / 1024));
  if (is_double)
    hipLaunchKernelGGL(combine_kernel<double>, grid, dim3(256), 0, st, (const double*)tmp, stride, K, c,
                       (double*)dst, n);
  else
    hipLaunchKernelGGL(combine_kernel<float>, grid, dim3(256), 0, st, (const float*)tmp, stride, K, c,
                       (float*)dst, n);
  return hipGetLastError();
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
