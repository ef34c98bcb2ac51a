// Device building blocks for the Core-AFD kernels on gfx950 (wave64).
//
// * Cx<T>: interleaved complex in registers (T = float or double).
// * Dif<R>: an R-point DFT (R <= 32) held in registers, radix-2 decimation in
//   frequency with compile-time twiddles; output position p holds bin
//   bitrev_R(p).
// * Stockham passes: a length-N transform is spread over TPR = N/E threads
//   holding E values each.  Before pass p a thread holds x[t + TPR*v],
//   v = 0..E-1; the pass runs E/R independent radix-R butterfly jobs
//   (job = t + u*TPR, its inputs x[job + r*N/R] = regs[u + (E/R)*r]), applies
//   the twiddle e^{+-2 pi i k r/(Ns R)} (k = job mod Ns) and the R-point DFT,
//   and its output q belongs at y[(job/Ns)*Ns*R + k + q*Ns] of the
//   self-sorting (Stockham) order.  The exchange between passes goes
//   through LDS with one pad element every 16 so that the strided writes of
//   the early passes stay free of bank conflicts.  After the last pass
//   (radix E, Ns = TPR) the thread holds output bins t + TPR*bitrev_E(p).
// The forward DFT of the samples (Sec. 3.1, eqs. term4/term3) and the
// per-radius inverse DFT (Sec. 3.1, eq. rcl and Theorem 2.1, eq. term8) are
// both this transform with SIGN = -1 and +1.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <type_traits>
#include <utility>

namespace afd {

template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
template <typename T>
__device__ __forceinline__ Cx<T> csqr(Cx<T> a) {
  return {fma(a.x, a.x, -a.y * a.y), T(2) * a.x * a.y};
}
template <typename T>
__device__ __forceinline__ Cx<T> cscale(Cx<T> a, T s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------- shape
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// LDS exchange padding: one pad element every 2^kPadShift elements
constexpr int kPadShift = 4;

// Pass structure of a length 2^LOGN transform with E values per thread: an
// optional first pass of radix 2^(LOGN mod log2 E), then passes of radix E.
template <int LOGN, int E>
struct Shape {
  static constexpr int N = 1 << LOGN;
  static constexpr int LE = ilog2c(E);
  static constexpr int Q0 = LOGN % LE;
  static constexpr int NP = LOGN / LE + (Q0 ? 1 : 0);
  static constexpr int TPR = N / E;
  static_assert(E >= 2 && (E & (E - 1)) == 0 && E <= N, "bad E");
  __host__ __device__ static constexpr int radix(int p) { return (p == 0 && Q0) ? (1 << Q0) : E; }
  __host__ __device__ static constexpr int ns(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= radix(i);
    return s;
  }
  // twiddle table: pass p >= 1 owns (radix(p) - 1) * ns(p) entries, entry
  // (r - 1) * ns(p) + k = e^{+2 pi i k r/(ns(p) radix(p))}, r = 1..radix-1
  __host__ __device__ static constexpr int twoff(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += (radix(i) - 1) * ns(i);
    return o;
  }
  __host__ __device__ static constexpr int twsize() { return twoff(NP); }
  // LDS elements for one transform (one pad element every 16)
  static constexpr int LDS_ELEMS = N + (N >> kPadShift) + 1;
};

__host__ __device__ constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> kPadShift); }

// ---------------------------------------------------------------- constant twiddles
// cos(2 pi q / 64), q = 0..16 (correctly rounded); the rest by symmetry.
constexpr double kCosQ[17] = {
    1.0,                  0.9951847266721969,  0.9807852804032304,  0.9569403357322088,
    0.9238795325112867,   0.881921264348355,   0.8314696123025452,  0.773010453362737,
    0.7071067811865476,   0.6343932841636455,  0.5555702330196022,  0.47139673682599764,
    0.3826834323650898,   0.2902846772544624,  0.19509032201612828, 0.0980171403295606,
    0.0};

__host__ __device__ constexpr double cos64(int q) {
  q = ((q % 64) + 64) % 64;
  return q <= 16 ? kCosQ[q] : q <= 32 ? -kCosQ[32 - q] : q <= 48 ? -kCosQ[q - 32] : kCosQ[64 - q];
}
__host__ __device__ constexpr double sin64(int q) { return cos64(q - 16); }

// v * e^{SIGN * 2 pi i Q / R}, R | 64
template <int R, int Q, int SIGN, typename T>
__device__ __forceinline__ Cx<T> twc(Cx<T> v) {
  constexpr int q = ((Q % R) + R) % R;
  if constexpr (q == 0) {
    return v;
  } else if constexpr (2 * q == R) {
    return {-v.x, -v.y};
  } else if constexpr (4 * q == R) {
    return {T(-SIGN) * v.y, T(SIGN) * v.x};
  } else if constexpr (4 * q == 3 * R) {
    return {T(SIGN) * v.y, T(-SIGN) * v.x};
  } else if constexpr (8 * q == R) {
    constexpr T h = T(0.7071067811865476);
    return {h * (v.x - T(SIGN) * v.y), h * (T(SIGN) * v.x + v.y)};
  } else if constexpr (8 * q == 3 * R) {
    constexpr T h = T(0.7071067811865476);
    return {h * (-v.x - T(SIGN) * v.y), h * (T(SIGN) * v.x - v.y)};
  } else if constexpr (8 * q == 5 * R) {
    constexpr T h = T(0.7071067811865476);
    return {h * (-v.x + T(SIGN) * v.y), h * (-T(SIGN) * v.x - v.y)};
  } else if constexpr (8 * q == 7 * R) {
    constexpr T h = T(0.7071067811865476);
    return {h * (v.x + T(SIGN) * v.y), h * (-T(SIGN) * v.x + v.y)};
  } else {
    constexpr int q64 = q * (64 / R);
    constexpr T c = T(cos64(q64));
    constexpr T s = T(SIGN * sin64(q64));
    return {fma(v.x, c, -v.y * s), fma(v.x, s, v.y * c)};
  }
}

// R-point DFT on a[OFF + p*STR], p = 0..R-1, in place; output position p
// holds bin bitrev_R(p).  X[q] = sum_r x[r] e^{SIGN 2 pi i r q / R}.
template <int R, int SIGN, int OFF, int STR, typename T>
struct Dif {
  template <int I>
  static __device__ __forceinline__ void bfly(Cx<T>* a) {
    constexpr int i0 = OFF + I * STR, i1 = OFF + (I + R / 2) * STR;
    const Cx<T> x = a[i0], y = a[i1];
    a[i0] = cadd(x, y);
    a[i1] = twc<R, I, SIGN>(csub(x, y));
  }
  template <int... I>
  static __device__ __forceinline__ void stage(Cx<T>* a, std::integer_sequence<int, I...>) {
    (bfly<I>(a), ...);
  }
  static __device__ __forceinline__ void run(Cx<T>* a) {
    if constexpr (R > 1) {
      stage(a, std::make_integer_sequence<int, R / 2>{});
      Dif<R / 2, SIGN, OFF, STR, T>::run(a);
      Dif<R / 2, SIGN, OFF + (R / 2) * STR, STR, T>::run(a);
    }
  }
};

// Radix-2 decimation-in-time butterfly on (e, o) with the compile-time twiddle
// W = e^{SIGN 2 pi i Q/R}: e <- e + W o, o <- e - W o, the second formed as
// 2e - (e + W o) so that a general twiddle costs six FMA-class operations.
template <int R, int Q, int SIGN, typename T>
__device__ __forceinline__ void dit_bfly(Cx<T>& e, Cx<T>& o) {
  constexpr int q = ((Q % R) + R) % R;
  if constexpr (q == 0) {
    const Cx<T> x = cadd(e, o), y = csub(e, o);
    e = x;
    o = y;
  } else if constexpr (4 * q == R) {
    // W o = SIGN i o
    const Cx<T> t{T(-SIGN) * o.y, T(SIGN) * o.x};
    const Cx<T> x = cadd(e, t), y = csub(e, t);
    e = x;
    o = y;
  } else if constexpr (8 * q == R || 8 * q == 3 * R) {
    // W = (cs + SIGN i)/sqrt2 with cs = +1 (q = R/8) or -1 (q = 3R/8)
    constexpr T h = T(0.7071067811865476);
    constexpr T cs = (8 * q == R) ? T(1) : T(-1);
    const T ur = fma(cs, o.x, -T(SIGN) * o.y);  // Re(sqrt2 W o)
    const T ui = fma(cs, o.y, T(SIGN) * o.x);   // Im(sqrt2 W o)
    const Cx<T> x{fma(h, ur, e.x), fma(h, ui, e.y)};
    o = {fma(T(2), e.x, -x.x), fma(T(2), e.y, -x.y)};
    e = x;
  } else {
    constexpr int q64 = q * (64 / R);
    constexpr T c = T(cos64(q64));
    constexpr T sn = T(SIGN * sin64(q64));
    const Cx<T> x{fma(c, o.x, fma(-sn, o.y, e.x)), fma(c, o.y, fma(sn, o.x, e.y))};
    o = {fma(T(2), e.x, -x.x), fma(T(2), e.y, -x.y)};
    e = x;
  }
}

// R-point DFT on a[OFF + p*STR], p = 0..R-1, in place, radix-2 decimation in
// time (even and odd halves first, then the combining butterflies); output
// position p holds bin bitrev_R(p), the same layout as Dif.
template <int R, int SIGN, int OFF, int STR, typename T>
struct Dit {
  template <int I>
  static __device__ __forceinline__ void bfly(Cx<T>* a) {
    // E[I] sits at position 2*bitrev_{R/2}(I), O[I] right after it
    constexpr int p = bitrev(I, ilog2c(R / 2));
    dit_bfly<R, I, SIGN>(a[OFF + (2 * p) * STR], a[OFF + (2 * p + 1) * STR]);
  }
  template <int... I>
  static __device__ __forceinline__ void stage(Cx<T>* a, std::integer_sequence<int, I...>) {
    (bfly<I>(a), ...);
  }
  static __device__ __forceinline__ void run(Cx<T>* a) {
    if constexpr (R > 1) {
      Dit<R / 2, SIGN, OFF, 2 * STR, T>::run(a);
      Dit<R / 2, SIGN, OFF + STR, 2 * STR, T>::run(a);
      stage(a, std::make_integer_sequence<int, R / 2>{});
    }
  }
};

// Twiddles of every pass of a transform held in registers, for transforms
// too short to hide a global load per pass: thread t's twiddle of pass P,
// job U, r = 1..R-1 sits at off(P) + U (R - 1) + r - 1.
template <typename T, int LOGN, int E>
struct TwRegs {
  using S = Shape<LOGN, E>;
  static constexpr int per_pass(int p) { return (E / S::radix(p)) * (S::radix(p) - 1); }
  static constexpr int off(int P) {
    int o = 0;
    for (int p = 1; p < P; ++p) o += per_pass(p);
    return o;
  }
  static constexpr int kCount = off(S::NP);
  Cx<T> w[kCount > 0 ? kCount : 1];
};

template <class X>
struct IsTwRegs : std::false_type {};
template <typename T, int LOGN, int E>
struct IsTwRegs<TwRegs<T, LOGN, E>> : std::true_type {};

// Fill R from the pass table (the entries pass_job would read for thread t).
template <typename T, int LOGN, int E, int P = 1>
__device__ __forceinline__ void tw_regs_load(TwRegs<T, LOGN, E>& R, int t, const Cx<T>* __restrict__ tw) {
  using S = Shape<LOGN, E>;
  if constexpr (P < S::NP) {
    constexpr int RX = S::radix(P), NS = S::ns(P), J = E / RX;
#pragma unroll
    for (int u = 0; u < J; ++u) {
      const int k = (t + u * S::TPR) & (NS - 1);
#pragma unroll
      for (int r = 1; r < RX; ++r)
        R.w[TwRegs<T, LOGN, E>::off(P) + u * (RX - 1) + r - 1] = tw[S::twoff(P) + (r - 1) * NS + k];
    }
    tw_regs_load<T, LOGN, E, P + 1>(R, t, tw);
  }
}

// One butterfly job u of Stockham pass P, in place on the registers: the
// twiddles e^{+-2 pi i k r/(Ns R)} come from the pass's table (exactly
// rounded; TW = const Cx<T>* reads it in memory, TW = TwRegs from
// registers), then the R-point DFT.
template <typename T, int LOGN, int E, int P, int SIGN, int U, class TW>
__device__ __forceinline__ void pass_job(Cx<T> (&v)[E], int t, const TW& tw) {
  using S = Shape<LOGN, E>;
  constexpr int R = S::radix(P);
  constexpr int NS = S::ns(P);
  constexpr int J = E / R;
  if constexpr (NS > 1) {
    if constexpr (!IsTwRegs<TW>::value) {
      const int job = t + U * S::TPR;
      const int k = job & (NS - 1);
      const Cx<T>* __restrict__ row = tw + S::twoff(P) + k;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        Cx<T> w = row[(r - 1) * NS];
        if constexpr (SIGN < 0) w.y = -w.y;
        v[U + r * J] = cmul(v[U + r * J], w);
        // bound the twiddles in flight (four in double, sixteen in single
        // precision) so the transforms stay inside their register budgets
        if ((sizeof(T) == 8 && (r % 4) == 3) || (sizeof(T) == 4 && (r % 16) == 15)) __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        Cx<T> w = tw.w[TW::off(P) + U * (R - 1) + r - 1];
        if constexpr (SIGN < 0) w.y = -w.y;
        v[U + r * J] = cmul(v[U + r * J], w);
      }
    }
  }
  Dit<R, SIGN, U, J, T>::run(v);
}

template <typename T, int LOGN, int E, int P, int SIGN, class TW, int... U>
__device__ __forceinline__ void pass_jobs(Cx<T> (&v)[E], int t, const TW& tw, std::integer_sequence<int, U...>) {
  (pass_job<T, LOGN, E, P, SIGN, U>(v, t, tw), ...);
}

// A twiddle table in memory whose address the compiler may not derive from
// before the pass that reads it: the table pointer passes through an empty
// asm at the start of every pass, so the per-thread addresses of a pass's
// twiddles are formed there and not hoisted to the start of the kernel (in
// the longest transforms they were, and were spilled).
template <typename T>
struct TwLate {
  const Cx<T>* p;
};
template <class TW>
struct IsTwLate : std::false_type {};
template <typename T>
struct IsTwLate<TwLate<T>> : std::true_type {};

// One Stockham pass P on the registers v (see the file comment).
template <typename T, int LOGN, int E, int P, int SIGN, class TW>
__device__ __forceinline__ void pass_compute(Cx<T> (&v)[E], int t, const TW& tw) {
  using S = Shape<LOGN, E>;
  if constexpr (IsTwLate<TW>::value) {
    const Cx<T>* p = tw.p;
    asm volatile("" : "+s"(p));
    pass_jobs<T, LOGN, E, P, SIGN>(v, t, p, std::make_integer_sequence<int, E / S::radix(P)>{});
  } else {
    pass_jobs<T, LOGN, E, P, SIGN>(v, t, tw, std::make_integer_sequence<int, E / S::radix(P)>{});
  }
}

// LDS addressing.  Element i lives at lds_pad(i) = i + (i >> kPadShift).  For
// every access pattern below the index is base + c with c a compile-time
// constant and (base mod 2^kPadShift) + (c mod 2^kPadShift) < 2^kPadShift, so
// lds_pad(base + c) = lds_pad(base) + pad_off(c): the padded base is computed
// once per job and the rest are immediate offsets.
__host__ __device__ constexpr int pad_off(int c) { return c + (c >> kPadShift); }

// Padded LDS index of the first output (q = 0) of job u after pass P; output
// q of the job sits pad_off(q * Ns) further on.  (Stockham destination
// (job / Ns) * Ns * R + (job mod Ns) + q * Ns.)
template <int LOGN, int E, int P>
__device__ __forceinline__ int pass_dest_base(int t, int u) {
  using S = Shape<LOGN, E>;
  constexpr int R = S::radix(P);
  constexpr int NS = S::ns(P);
  const int job = t + u * S::TPR;
  return lds_pad((job / NS) * NS * R + (job & (NS - 1)));
}

// Write the outputs of pass P to LDS (complex elements).
template <typename T, int LOGN, int E, int P>
__device__ __forceinline__ void lds_write(const Cx<T> (&v)[E], int t, Cx<T>* lds) {
  using S = Shape<LOGN, E>;
  constexpr int R = S::radix(P);
  constexpr int NS = S::ns(P);
  constexpr int J = E / R;
  constexpr int LR = ilog2c(R);
#pragma unroll
  for (int u = 0; u < J; ++u) {
    Cx<T>* b = lds + pass_dest_base<LOGN, E, P>(t, u);
#pragma unroll
    for (int q = 0; q < R; ++q) b[pad_off(q * NS)] = v[u + J * bitrev(q, LR)];
  }
}

template <typename T, int LOGN, int E, int P, int PART>
__device__ __forceinline__ void lds_write_part(const Cx<T> (&v)[E], int t, T* lds) {
  using S = Shape<LOGN, E>;
  constexpr int R = S::radix(P);
  constexpr int NS = S::ns(P);
  constexpr int J = E / R;
  constexpr int LR = ilog2c(R);
#pragma unroll
  for (int u = 0; u < J; ++u) {
    T* b = lds + pass_dest_base<LOGN, E, P>(t, u);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const Cx<T> val = v[u + J * bitrev(q, LR)];
      b[pad_off(q * NS)] = PART == 0 ? val.x : val.y;
    }
  }
}

template <typename T, int LOGN, int E>
__device__ __forceinline__ void lds_read(Cx<T> (&v)[E], int t, const Cx<T>* lds) {
  using S = Shape<LOGN, E>;
  const Cx<T>* b = lds + lds_pad(t);
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = b[pad_off(S::TPR * i)];
}

template <typename T, int LOGN, int E, int PART>
__device__ __forceinline__ void lds_read_part(Cx<T> (&v)[E], int t, const T* lds) {
  using S = Shape<LOGN, E>;
  const T* b = lds + lds_pad(t);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const T val = b[pad_off(S::TPR * i)];
    if constexpr (PART == 0) v[i].x = val; else v[i].y = val;
  }
}

// Full transform on registers: passes 0..NP-1 with LDS exchanges between
// them.  `lds` points at this transform's LDS region (Shape::LDS_ELEMS
// complex elements, or that many reals when SPLIT, which exchanges the real
// parts and then the imaginary parts through half the space).  Every thread
// of the block must call this (block-wide barriers).
//
// FIRST > 0 starts at pass FIRST with the registers already holding that
// pass's inputs (no exchange before it); see the pruned start of the radius
// transform.  `tw`: the pass table in memory (const Cx<T>*) or a TwRegs.
//
// WAVE: the threads of each transform lie in one wave (TPR divides 64), so
// an exchange needs no workgroup barrier: a wave's LDS accesses complete in
// order, and a wave-scope fence only keeps the compiler from moving them
// across one another.  The waves of a workgroup then run their transforms
// independently.
template <bool WAVE>
__device__ __forceinline__ void lds_exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <typename T, int LOGN, int E, int SIGN, bool SPLIT, int P = 0, int FIRST = 0, bool WAVE = false, class TW>
__device__ __forceinline__ void fft_regs(Cx<T> (&v)[E], int t, void* lds, const TW& tw) {
  using S = Shape<LOGN, E>;
  static_assert(!WAVE || (64 % S::TPR == 0), "a wave-synchronised transform lies in one wave");
  if constexpr (P > FIRST) {
    if constexpr (SPLIT) {
      T* l = reinterpret_cast<T*>(lds);
      lds_write_part<T, LOGN, E, P - 1, 0>(v, t, l);
      lds_exchange_sync<WAVE>();
      lds_read_part<T, LOGN, E, 0>(v, t, l);
      lds_exchange_sync<WAVE>();
      lds_write_part<T, LOGN, E, P - 1, 1>(v, t, l);
      lds_exchange_sync<WAVE>();
      lds_read_part<T, LOGN, E, 1>(v, t, l);
      lds_exchange_sync<WAVE>();
    } else {
      Cx<T>* l = reinterpret_cast<Cx<T>*>(lds);
      lds_write<T, LOGN, E, P - 1>(v, t, l);
      lds_exchange_sync<WAVE>();
      lds_read<T, LOGN, E>(v, t, l);
      lds_exchange_sync<WAVE>();
    }
  }
  pass_compute<T, LOGN, E, P, SIGN>(v, t, tw);
  if constexpr (P + 1 < S::NP) fft_regs<T, LOGN, E, SIGN, SPLIT, P + 1, FIRST, WAVE>(v, t, lds, tw);
}

// Output bin held by register p after fft_regs.
template <int LOGN, int E>
__device__ __forceinline__ int out_bin(int t, int p) {
  return t + Shape<LOGN, E>::TPR * bitrev(p, ilog2c(E));
}

// ---------------------------------------------------------------- geometry choices
// Values per thread: 32 at 2^14 points (fewer LDS exchanges: two instead of
// three; single precision keeps two workgroups per CU, double precision
// runs 512 threads in the 256-register budget of two waves per SIMD), 16
// otherwise.  From 2^12 points the
// exchange runs real and imaginary parts through half the LDS in turn: at
// 2^12..2^13 that lets four 256/512-thread workgroups share a CU (measured
// 1.4x on batches of 2^12-point signals), at 2^14 a single-precision
// workgroup leaves room for a second one and a double-precision one fits.
template <typename T, int LOGN>
__host__ __device__ constexpr int pickE() {
  return (1 << LOGN) < 16 ? (1 << LOGN) : LOGN >= 14 ? 32 : 16;
}
template <typename T, int LOGN>
__host__ __device__ constexpr bool pickSplit() {
  return LOGN >= 12;
}
__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// LDS bytes of one transform's exchange region
template <typename T, int LOGN, bool SPLIT>
__host__ __device__ constexpr size_t fft_region_bytes() {
  using S = Shape<LOGN, pickE<T, LOGN>()>;
  return align16(size_t(S::LDS_ELEMS) * (SPLIT ? sizeof(T) : sizeof(Cx<T>)));
}

// ---------------------------------------------------------------- selection keys
// Key order: larger |.|^2 first, then lower flat index.
__device__ __forceinline__ bool better64(double pa, uint32_t fa, double pb, uint32_t fb) {
  return pa > pb || (pa == pb && fa < fb);
}

// FP32 key: (float bits of P >= 0) << 32 | ~f  -- larger key = better.
__device__ __forceinline__ uint64_t key32(float p, uint32_t f) {
  return (uint64_t(__float_as_uint(p)) << 32) | uint64_t(~f);
}
__device__ __forceinline__ float key_p(uint64_t k) { return __uint_as_float(uint32_t(k >> 32)); }
__device__ __forceinline__ uint32_t key_f(uint64_t k) { return ~uint32_t(k & 0xffffffffu); }

// ---------------------------------------------------------------- wave reductions
// No LDS and no lane-address registers: DPP moves inside each row of 16 lanes
// (xor 1, xor 2, half-row mirror, row mirror) leave every lane holding its
// row's result, then the four row results are combined through readlane, so
// every lane returns the same value.  All 64 lanes of the wave must be active:
// every kernel that reduces launches whole waves (a multiple of 64 threads).
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  return (uint64_t(dpp_u32<CTRL>(uint32_t(v >> 32))) << 32) | dpp_u32<CTRL>(uint32_t(v));
}
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int lane) {
  return uint32_t(__builtin_amdgcn_readlane(int(v), lane));
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int lane) {
  return (uint64_t(lane_u32(uint32_t(v >> 32), lane)) << 32) | lane_u32(uint32_t(v), lane);
}

// OP: a struct with static T op(T, T) on the 32/64-bit pattern of the value
template <typename OP, typename U>
__device__ __forceinline__ U wave_reduce_bits(U v) {
  if constexpr (sizeof(U) == 8) {
    v = OP::op(v, dpp_u64<kDppXor1>(v));
    v = OP::op(v, dpp_u64<kDppXor2>(v));
    v = OP::op(v, dpp_u64<kDppHalfMirror>(v));
    v = OP::op(v, dpp_u64<kDppMirror>(v));
    U r = lane_u64(v, 0);
    r = OP::op(r, lane_u64(v, 16));
    r = OP::op(r, lane_u64(v, 32));
    return OP::op(r, lane_u64(v, 48));
  } else {
    v = OP::op(v, dpp_u32<kDppXor1>(v));
    v = OP::op(v, dpp_u32<kDppXor2>(v));
    v = OP::op(v, dpp_u32<kDppHalfMirror>(v));
    v = OP::op(v, dpp_u32<kDppMirror>(v));
    U r = lane_u32(v, 0);
    r = OP::op(r, lane_u32(v, 16));
    r = OP::op(r, lane_u32(v, 32));
    return OP::op(r, lane_u32(v, 48));
  }
}

struct MaxU64 {
  static __device__ __forceinline__ uint64_t op(uint64_t a, uint64_t b) { return a > b ? a : b; }
};
struct MaxF32 {  // on the bits of a float
  static __device__ __forceinline__ uint32_t op(uint32_t a, uint32_t b) {
    return __float_as_uint(fmaxf(__uint_as_float(a), __uint_as_float(b)));
  }
};
struct MinF32 {
  static __device__ __forceinline__ uint32_t op(uint32_t a, uint32_t b) {
    return __float_as_uint(fminf(__uint_as_float(a), __uint_as_float(b)));
  }
};
struct SumU32 {
  static __device__ __forceinline__ uint32_t op(uint32_t a, uint32_t b) { return a + b; }
};
struct MinU32 {
  static __device__ __forceinline__ uint32_t op(uint32_t a, uint32_t b) { return a < b ? a : b; }
};
struct SumF64 {  // on the bits of a double
  static __device__ __forceinline__ uint64_t op(uint64_t a, uint64_t b) {
    return uint64_t(__double_as_longlong(__longlong_as_double((long long)a) + __longlong_as_double((long long)b)));
  }
};
struct MaxF64 {
  static __device__ __forceinline__ uint64_t op(uint64_t a, uint64_t b) {
    return uint64_t(__double_as_longlong(fmax(__longlong_as_double((long long)a), __longlong_as_double((long long)b))));
  }
};

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) { return wave_reduce_bits<MaxU64>(v); }
__device__ __forceinline__ float wave_max_f32(float v) {
  return __uint_as_float(wave_reduce_bits<MaxF32>(__float_as_uint(v)));
}
__device__ __forceinline__ float wave_min_f32(float v) {
  return __uint_as_float(wave_reduce_bits<MinF32>(__float_as_uint(v)));
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  return __longlong_as_double((long long)wave_reduce_bits<SumF64>(uint64_t(__double_as_longlong(v))));
}
__device__ __forceinline__ double wave_max_f64(double v) {
  return __longlong_as_double((long long)wave_reduce_bits<MaxF64>(uint64_t(__double_as_longlong(v))));
}

}  // namespace afd
