// Work-group FFT engine for gfx950 (64-wide wavefronts, LDS exchanges).
//
// A length-L complex transform is carried by T = L/E threads, each holding E
// values in *strided* order: lane t of the transform owns elements t + T*m,
// m = 0..E-1.  The transform is a Stockham sequence of radix-R stages
// (R divides E).  The first stage reads and the last stage writes the strided
// order directly, so a one-stage transform never touches LDS and an S-stage
// transform makes S-1 exchanges through an LDS region private to it.
//
// Conventions: forward = exp(-2 pi i jk/L) (DIR = -1), inverse = exp(+...)
// (DIR = +1), both unnormalised.  Twiddles come from a table of the L roots
// W_L^m = exp(-2 pi i m / L) built on the host in double precision.
#pragma once
#include <hip/hip_runtime.h>

namespace mpe {

template <typename F>
struct alignas(2 * sizeof(F)) cx {
  F x, y;
};

// Pointer into the global address space (global_* rather than flat_* memory
// instructions when the address space cannot be inferred).
template <typename T>
using gp = T __attribute__((address_space(1)))*;

// Value of the neighbouring lane (lane ^ 1) through a DPP quad permutation
// [1, 0, 3, 2] (a VALU operand modifier, no LDS traffic).
__device__ __forceinline__ float lane_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_xor1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Complex loads and stores through global pointers, as one 2-element vector
// access (dwordx2 / dwordx4).
template <typename F>
using vec2 = F __attribute__((ext_vector_type(2)));
template <typename F>
__device__ __forceinline__ cx<F> gload(gp<const cx<F>> p) {
  const vec2<F> t = *reinterpret_cast<gp<const vec2<F>>>(p);
  return cx<F>{t.x, t.y};
}
typedef int v4i32 __attribute__((ext_vector_type(4)));
// A vector-memory store of 16 bytes per lane reads its data registers after it
// has issued.  Measured on MI355X: when the next two instruction slots write
// one of those registers (the compiler reuses them at once), the store now and
// then writes the new value into its first dword: a complex double comes out
// with the low word of its real part replaced, at random lanes and planes.
// Every such store is therefore followed by this two-slot pause that reads
// the data registers, so that they stay unchanged until after it.
__device__ __forceinline__ void hold_store_data(v4i32 t) { asm volatile("s_nop 1" ::"v"(t)); }

template <typename F>
__device__ __forceinline__ void gstore(gp<cx<F>> p, cx<F> v) {
  *reinterpret_cast<gp<vec2<F>>>(p) = vec2<F>{v.x, v.y};
}
template <>
__device__ __forceinline__ void gstore<double>(gp<cx<double>> p, cx<double> v) {
  const vec2<double> t = {v.x, v.y};
  *reinterpret_cast<gp<vec2<double>>>(p) = t;
  hold_store_data(__builtin_bit_cast(v4i32, t));
}

// Buffer (MUBUF) accesses of complex values: the wave-uniform part of an
// address (the base of a plane, a constant offset) stays in scalar registers
// and one 32-bit per-lane byte offset serves every access of a lane, so no
// 64-bit address is formed per access.  The resource's byte range bounds the
// accesses: beyond it loads read 0 and stores are dropped.  Word 3 of the
// resource (0x00020000: 32-bit data format, the untyped-access setting of
// gfx9-family parts) makes the loads valid.
// The base must be the same in every lane (the resource lives in scalar
// registers); it is passed through readfirstlane, which costs nothing where
// the compiler already holds it in scalar registers and spares a per-access
// loop over distinct resources where its analysis cannot see the uniformity
// (values carried around the persistent plane loop).
using brsrc = __amdgpu_buffer_rsrc_t;
template <typename T>
__device__ __forceinline__ brsrc make_brsrc(gp<T> base, unsigned bytes) {
  const unsigned long long b = (unsigned long long)base;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  void* u = (void*)(((unsigned long long)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(u, (short)0, (int)bytes, 0x00020000);
}
typedef int v2i32 __attribute__((ext_vector_type(2)));
template <typename F>
__device__ __forceinline__ cx<F> bload(brsrc r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ cx<float> bload<float>(brsrc r, unsigned voff, unsigned soff) {
  const v2i32 t = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
  return cx<float>{__int_as_float(t.x), __int_as_float(t.y)};
}
template <>
__device__ __forceinline__ cx<double> bload<double>(brsrc r, unsigned voff, unsigned soff) {
  const v4i32 t = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
  return cx<double>{__hiloint2double(t.y, t.x), __hiloint2double(t.w, t.z)};
}
template <typename F>
__device__ __forceinline__ void bstore(brsrc r, unsigned voff, unsigned soff, cx<F> v);
template <>
__device__ __forceinline__ void bstore<float>(brsrc r, unsigned voff, unsigned soff, cx<float> v) {
  const v2i32 t = {__float_as_int(v.x), __float_as_int(v.y)};
  __builtin_amdgcn_raw_buffer_store_b64(t, r, (int)voff, (int)soff, 0);
}
template <>
__device__ __forceinline__ void bstore<double>(brsrc r, unsigned voff, unsigned soff, cx<double> v) {
  const long long a = __double_as_longlong(v.x), b = __double_as_longlong(v.y);
  const v4i32 t = {(int)(a & 0xffffffffLL), (int)(a >> 32), (int)(b & 0xffffffffLL), (int)(b >> 32)};
  __builtin_amdgcn_raw_buffer_store_b128(t, r, (int)voff, (int)soff, 0);
  hold_store_data(t);
}

template <typename F>
__device__ __forceinline__ cx<F> mk(F a, F b) { return cx<F>{a, b}; }
template <typename F>
__device__ __forceinline__ cx<F> operator+(cx<F> a, cx<F> b) { return cx<F>{a.x + b.x, a.y + b.y}; }
template <typename F>
__device__ __forceinline__ cx<F> operator-(cx<F> a, cx<F> b) { return cx<F>{a.x - b.x, a.y - b.y}; }
template <typename F>
__device__ __forceinline__ cx<F> cmul(cx<F> a, cx<F> b) {
  return cx<F>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename F>
__device__ __forceinline__ cx<F> cmulc(cx<F> a, cx<F> b) {
  return cx<F>{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename F>
__device__ __forceinline__ cx<F> conj(cx<F> a) { return cx<F>{a.x, -a.y}; }
template <typename F>
__device__ __forceinline__ cx<F> scale(cx<F> a, F s) { return cx<F>{a.x * s, a.y * s}; }
// multiply by DIR*i : DIR=-1 gives -i*z, DIR=+1 gives +i*z
template <int DIR, typename F>
__device__ __forceinline__ cx<F> muli(cx<F> z) {
  return DIR < 0 ? cx<F>{z.y, -z.x} : cx<F>{-z.y, z.x};
}
// twiddle from the forward root table, conjugated for the inverse direction
template <int DIR, typename F>
__device__ __forceinline__ cx<F> twiddle(cx<F> a, cx<F> w) {
  return DIR < 0 ? cmul(a, w) : cmulc(a, w);
}

// ---------------------------------------------------------------- small DFTs in registers
template <int R, int DIR, typename F>
struct Dft;

template <int DIR, typename F>
struct Dft<1, DIR, F> {
  static __device__ __forceinline__ void run(cx<F>*) {}
};

template <int DIR, typename F>
struct Dft<2, DIR, F> {
  static __device__ __forceinline__ void run(cx<F>* a) {
    cx<F> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  }
};

template <int DIR, typename F>
struct Dft<3, DIR, F> {
  static __device__ __forceinline__ void run(cx<F>* a) {
    const F h = F(0.86602540378443864676372317075294);  // sqrt(3)/2
    cx<F> s = a[1] + a[2];
    cx<F> d = a[1] - a[2];
    cx<F> t = a[0] - scale(s, F(0.5));
    cx<F> r = muli<DIR>(scale(d, h));
    a[0] = a[0] + s;
    a[1] = t + r;
    a[2] = t - r;
  }
};

template <int DIR, typename F>
struct Dft<4, DIR, F> {
  static __device__ __forceinline__ void run(cx<F>* a) {
    cx<F> s0 = a[0] + a[2], d0 = a[0] - a[2];
    cx<F> s1 = a[1] + a[3], d1 = muli<DIR>(a[1] - a[3]);
    a[0] = s0 + s1;
    a[2] = s0 - s1;
    a[1] = d0 + d1;
    a[3] = d0 - d1;
  }
};

template <int DIR, typename F>
struct Dft<8, DIR, F> {
  static __device__ __forceinline__ void run(cx<F>* a) {
    const F r2 = F(0.70710678118654752440084436210485);
    cx<F> e[4] = {a[0], a[2], a[4], a[6]};
    cx<F> o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, DIR, F>::run(e);
    Dft<4, DIR, F>::run(o);
    // W8^k for k = 1, 2, 3 in direction DIR
    cx<F> o1 = cx<F>{r2 * (o[1].x - DIR * o[1].y), r2 * (o[1].y + DIR * o[1].x)};
    cx<F> o2 = muli<DIR>(o[2]);
    cx<F> o3 = cx<F>{-r2 * (o[3].x + DIR * o[3].y), r2 * (DIR * o[3].x - o[3].y)};
    a[0] = e[0] + o[0];
    a[4] = e[0] - o[0];
    a[1] = e[1] + o1;
    a[5] = e[1] - o1;
    a[2] = e[2] + o2;
    a[6] = e[2] - o2;
    a[3] = e[3] + o3;
    a[7] = e[3] - o3;
  }
};

template <int DIR, typename F>
struct Dft<16, DIR, F> {
  static __device__ __forceinline__ void run(cx<F>* a) {
    // exp(DIR * 2 pi i k / 16), k = 0..7
    const F c1 = F(0.92387953251128675612818318939679), s1 = F(0.38268343236508977172845998403040);
    const F r2 = F(0.70710678118654752440084436210485);
    cx<F> e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      e[i] = a[2 * i];
      o[i] = a[2 * i + 1];
    }
    Dft<8, DIR, F>::run(e);
    Dft<8, DIR, F>::run(o);
    const F wc[8] = {F(1), c1, r2, s1, F(0), -s1, -r2, -c1};
    const F ws[8] = {F(0), s1, r2, c1, F(1), c1, r2, s1};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      // W^0 = 1 and W^4 = DIR i exactly (a general product would multiply by 0)
      cx<F> t;
      if (k == 0) {
        t = o[0];
      } else if (k == 4) {
        t = muli<DIR>(o[4]);
      } else {
        t = cmul(o[k], cx<F>{wc[k], F(DIR) * ws[k]});
      }
      a[k] = e[k] + t;
      a[k + 8] = e[k] - t;
    }
  }
};

// ---------------------------------------------------------------- transform plans
// E values per thread, T threads per transform, S radix stages R0 R1 R2.
template <int L>
struct Plan;
template <> struct Plan<4>   { static constexpr int E = 4,  T = 1, S = 1, R0 = 4,  R1 = 1, R2 = 1; };
template <> struct Plan<8>   { static constexpr int E = 8,  T = 1, S = 1, R0 = 8,  R1 = 1, R2 = 1; };
template <> struct Plan<16>  { static constexpr int E = 16, T = 1, S = 1, R0 = 16, R1 = 1, R2 = 1; };
template <> struct Plan<24>  { static constexpr int E = 24, T = 1, S = 2, R0 = 3,  R1 = 8, R2 = 1; };
template <> struct Plan<32>  { static constexpr int E = 8,  T = 4, S = 2, R0 = 8,  R1 = 4, R2 = 1; };
template <> struct Plan<48>  { static constexpr int E = 12, T = 4, S = 3, R0 = 3,  R1 = 4, R2 = 4; };
template <> struct Plan<64>  { static constexpr int E = 16, T = 4, S = 2, R0 = 16, R1 = 4, R2 = 1; };
template <> struct Plan<96>  { static constexpr int E = 24, T = 4, S = 3, R0 = 3,  R1 = 4, R2 = 8; };
template <> struct Plan<128> { static constexpr int E = 16, T = 8, S = 2, R0 = 16, R1 = 8, R2 = 1; };
template <> struct Plan<192> { static constexpr int E = 24, T = 8, S = 3, R0 = 3,  R1 = 8, R2 = 8; };

// One Stockham stage of radix R at span NS on a length-L transform, in registers.
// On entry v[] holds this lane's inputs in strided order.  The outputs y are
// produced in v[] in the order  v[q + r*(E/R)] = y of butterfly q, output r,
// whose transform index is  out_index(q, r).
template <int L, int E, int T, int R, int NS, int DIR, typename F>
__device__ __forceinline__ void stage(cx<F>* v, int t, const cx<F>* __restrict__ roots) {
  constexpr int NB = E / R;  // butterflies per thread
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    cx<F> a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[q + r * NB];
    if constexpr (NS > 1) {
      const int j = t + T * q;
      const int k = j % NS;
      constexpr int STEP = L / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r) a[r] = twiddle<DIR>(a[r], roots[r * k * STEP]);
    }
    Dft<R, DIR, F>::run(a);
#pragma unroll
    for (int r = 0; r < R; ++r) v[q + r * NB] = a[r];
  }
}

// Transform index of output r of butterfly q (lane t) after a stage of radix R at span NS.
template <int L, int E, int T, int R, int NS>
__device__ __forceinline__ int out_index(int t, int q, int r) {
  const int j = t + T * q;
  const int k = j % NS;
  return (j / NS) * NS * R + k + r * NS;
}

// Exchange: scatter stage outputs to their transform indices, gather strided order back.
// buf(i) addresses element i of this transform in LDS.  Every thread of the
// work-group must call this (it contains barriers); it is bracketed by barriers
// so the region may be read before and written after it without further sync.
// Ordering point for an exchange whose lanes all sit in one wavefront: LDS
// operations of a wavefront execute in program order, so only the compiler
// must be kept from moving LDS accesses across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <bool WAVE>
__device__ __forceinline__ void xsync() {
  if constexpr (WAVE) wave_sync();
  else __syncthreads();
}

// WAVE = true: the T lanes of every transform are consecutive lanes of one
// wavefront, so the exchange needs no work-group barrier.
template <int L, int E, int T, int R, int NS, bool WAVE = false, typename F, typename Addr>
__device__ __forceinline__ void exchange(cx<F>* v, int t, bool active, Addr buf) {
  constexpr int NB = E / R;
  if constexpr (T == 1) {
    // single-lane transform: a register permutation resolved at compile time
    cx<F> tmp[E];
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) tmp[out_index<L, E, T, R, NS>(0, q, r)] = v[q + r * NB];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = tmp[m];
  } else {
    xsync<WAVE>();
    if (active) {
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) *buf(out_index<L, E, T, R, NS>(t, q, r)) = v[q + r * NB];
    }
    xsync<WAVE>();
    if (active) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = *buf(t + T * m);
    }
    xsync<WAVE>();
  }
}

// Full length-L transform of the values v[] (strided order in and out).
// All threads of the work-group must call it together (barriers inside when
// the transform spans several lanes).
template <int L, int DIR, bool WAVE = false, typename F, typename Addr>
__device__ __forceinline__ void fft(cx<F>* v, int t, bool active, Addr buf, const cx<F>* __restrict__ roots) {
  using P = Plan<L>;
  constexpr int E = P::E, T = P::T;
  stage<L, E, T, P::R0, 1, DIR>(v, t, roots);
  if constexpr (P::S >= 2) {
    exchange<L, E, T, P::R0, 1, WAVE>(v, t, active, buf);
    stage<L, E, T, P::R1, P::R0, DIR>(v, t, roots);
  }
  if constexpr (P::S >= 3) {
    exchange<L, E, T, P::R1, P::R0, WAVE>(v, t, active, buf);
    stage<L, E, T, P::R2, P::R0 * P::R1, DIR>(v, t, roots);
  }
}

}  // namespace mpe
