// Radix-3 transforms for N = 3^K points.  The paper's closing remark notes
// that the fast algorithm carries over to N = p^K; for p = 3 the radix-2
// split of Theorem 2.1 (eqs. term8, term82) becomes a 3-point split: with
// S_r the length-N/3 DFT of the samples n = r (mod 3),
//   X[k + q N/3] = sum_{r<3} W^{r (k + q N/3)} S_r[k],   W = e^{+-2 pi i/N},
// so one level costs N/3 three-point butterflies.
//
// The layout follows the radix-2 Stockham transform of afd_device.h: a
// length-3^K transform is spread over TPR = N/E threads holding E = 3^e
// values each; pass p runs E/R radix-R jobs (job = t + u TPR, inputs
// x[job + r N/R] = regs[u + (E/R) r]), twiddles e^{+-2 pi i k r/(Ns R)}
// (k = job mod Ns) from a table, then an R-point DFT in registers whose
// output position p holds bin digrev3(p) (base-3 digit reversal), written
// to the Stockham destination (job/Ns) Ns R + (job mod Ns) + q Ns.  After
// the last pass register p holds output bin t + TPR digrev3(p).  Threads
// t >= TPR of a workgroup take part in the barriers only.  LDS needs no
// padding: every strided access steps by a power of three, which is odd,
// so the lanes of a wave fall on distinct banks.
#pragma once

#include "afd_device.h"

namespace afd {

__host__ __device__ constexpr int ipow3(int k) { return k <= 0 ? 1 : 3 * ipow3(k - 1); }
__host__ __device__ constexpr int ilog3c(int v) { return v <= 1 ? 0 : 1 + ilog3c(v / 3); }
__host__ __device__ constexpr int digrev3(int v, int digits) {
  int r = 0;
  for (int i = 0; i < digits; ++i) {
    r = r * 3 + v % 3;
    v /= 3;
  }
  return r;
}

// cos and sin of 2 pi q / R at compile time, from the Taylor series on an
// angle reduced to [0, pi/4] by the symmetries of the unit circle (accurate
// to a few units in the last place; used for the butterflies' internal
// twiddles, whose R is a power of three).
constexpr double kPi = 3.14159265358979323846264338327950288;
__host__ __device__ constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
__host__ __device__ constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
// (cos, sin)(2 pi q / R) with the angle folded into [0, pi/4]
__host__ __device__ constexpr double unit_cos(int q, int R) {
  q = ((q % R) + R) % R;
  const double t = double(q) / double(R);           // turns in [0, 1)
  const double u = t > 0.5 ? 1.0 - t : t;           // cos is even: [0, 1/2]
  const double v = u > 0.25 ? 0.5 - u : u;          // cos(pi - x) = -cos x: [0, 1/4]
  const double sgn = u > 0.25 ? -1.0 : 1.0;
  const double c = v > 0.125 ? taylor_sin(2.0 * kPi * (0.25 - v)) : taylor_cos(2.0 * kPi * v);
  return sgn * c;
}
__host__ __device__ constexpr double unit_sin(int q, int R) {
  // sin(2 pi q/R) = cos(2 pi (q/R - 1/4)) = cos(2 pi (4q - R)/(4R))
  return unit_cos(4 * (((q % R) + R) % R) - R, 4 * R);
}

// Pass structure of a length-3^K transform with E = 3^e values per thread:
// an optional first pass of radix 3^(K mod e), then passes of radix E.
template <int K, int E>
struct Shape3 {
  static constexpr int N = ipow3(K);
  static constexpr int LE = ilog3c(E);
  static constexpr int Q0 = K % LE;
  static constexpr int NP = K / LE + (Q0 ? 1 : 0);
  static constexpr int TPR = N / E;
  static_assert(ipow3(LE) == E && E <= N, "E must be a power of three, at most N");
  __host__ __device__ static constexpr int radix(int p) { return (p == 0 && Q0) ? ipow3(Q0) : E; }
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
};

// R-point DFT (R = 3^d) on a[OFF + p*STR], p = 0..R-1, in place, radix-3
// decimation in time (the three interleaved thirds first, then the
// combining butterflies); output position p holds bin digrev3(p, d).
// X[q] = sum_r x[r] e^{SIGN 2 pi i r q / R}.
template <int R, int SIGN, int OFF, int STR, typename T>
struct Dit3 {
  template <int I>
  static __device__ __forceinline__ void bfly(Cx<T>* a) {
    // sub-bin I of the three thirds sits at position 3 digrev3(I) (+1, +2)
    constexpr int p = digrev3(I, ilog3c(R / 3));
    Cx<T>& x0 = a[OFF + (3 * p) * STR];
    Cx<T>& x1 = a[OFF + (3 * p + 1) * STR];
    Cx<T>& x2 = a[OFF + (3 * p + 2) * STR];
    Cx<T> t1 = x1, t2 = x2;
    if constexpr (I != 0) {
      constexpr T c1 = T(unit_cos(I, R)), s1 = T(SIGN * unit_sin(I, R));
      constexpr T c2 = T(unit_cos(2 * I, R)), s2 = T(SIGN * unit_sin(2 * I, R));
      t1 = {fma(c1, x1.x, -s1 * x1.y), fma(c1, x1.y, s1 * x1.x)};
      t2 = {fma(c2, x2.x, -s2 * x2.y), fma(c2, x2.y, s2 * x2.x)};
    }
    // X0 = x0 + t1 + t2, X1,2 = x0 - (t1 + t2)/2 +- SIGN i (sqrt3/2)(t1 - t2)
    constexpr T h = T(0.86602540378443864676372317075293618);
    const Cx<T> s = cadd(t1, t2), d = csub(t1, t2);
    const Cx<T> m{fma(T(-0.5), s.x, x0.x), fma(T(-0.5), s.y, x0.y)};
    const Cx<T> u{T(-SIGN) * h * d.y, T(SIGN) * h * d.x};
    x0 = cadd(x0, s);
    x1 = cadd(m, u);
    x2 = csub(m, u);
  }
  template <int... I>
  static __device__ __forceinline__ void stage(Cx<T>* a, std::integer_sequence<int, I...>) {
    (bfly<I>(a), ...);
  }
  static __device__ __forceinline__ void run(Cx<T>* a) {
    if constexpr (R > 1) {
      Dit3<R / 3, SIGN, OFF, 3 * STR, T>::run(a);
      Dit3<R / 3, SIGN, OFF + STR, 3 * STR, T>::run(a);
      Dit3<R / 3, SIGN, OFF + 2 * STR, 3 * STR, T>::run(a);
      stage(a, std::make_integer_sequence<int, R / 3>{});
    }
  }
};

// One butterfly job u of Stockham pass P in place on the registers.
template <typename T, int K, int E, int P, int SIGN, int U>
__device__ __forceinline__ void pass3_job(Cx<T> (&v)[E], int t, const Cx<T>* __restrict__ tw) {
  using S = Shape3<K, E>;
  constexpr int R = S::radix(P);
  constexpr int NS = S::ns(P);
  constexpr int J = E / R;
  if constexpr (NS > 1) {
    const int job = t + U * S::TPR;
    const int k = job % NS;
    const Cx<T>* __restrict__ row = tw + S::twoff(P) + k;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      Cx<T> w = row[(r - 1) * NS];
      if constexpr (SIGN < 0) w.y = -w.y;
      v[U + r * J] = cmul(v[U + r * J], w);
    }
  }
  Dit3<R, SIGN, U, J, T>::run(v);
}

template <typename T, int K, int E, int P, int SIGN, int... U>
__device__ __forceinline__ void pass3_jobs(Cx<T> (&v)[E], int t, const Cx<T>* tw, std::integer_sequence<int, U...>) {
  (pass3_job<T, K, E, P, SIGN, U>(v, t, tw), ...);
}

// Destination of output q of job u after pass P (Stockham order).
template <int K, int E, int P>
__device__ __forceinline__ int pass3_dest(int t, int u, int q) {
  using S = Shape3<K, E>;
  constexpr int R = S::radix(P);
  constexpr int NS = S::ns(P);
  const int job = t + u * S::TPR;
  return (job / NS) * NS * R + job % NS + q * NS;
}

// The exchange between pass P - 1 and pass P: outputs to their Stockham
// destinations, then each thread reads x[t + TPR i].  SPLIT moves real and
// imaginary parts through N reals in turn.  `act`: the thread is one of the
// TPR that hold values (all threads pass the barriers).
template <typename T, int K, int E, int P, bool SPLIT>
__device__ __forceinline__ void exchange3(Cx<T> (&v)[E], int t, bool act, void* lds) {
  using S = Shape3<K, E>;
  constexpr int R = S::radix(P - 1);
  constexpr int J = E / R;
  constexpr int LR = ilog3c(R);
  if constexpr (SPLIT) {
    T* l = reinterpret_cast<T*>(lds);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      if (act) {
#pragma unroll
        for (int u = 0; u < J; ++u)
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const Cx<T> val = v[u + J * digrev3(q, LR)];
            l[pass3_dest<K, E, P - 1>(t, u, q)] = part == 0 ? val.x : val.y;
          }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const T val = l[t + S::TPR * i];
          if (part == 0) v[i].x = val; else v[i].y = val;
        }
      }
      __syncthreads();
    }
  } else {
    Cx<T>* l = reinterpret_cast<Cx<T>*>(lds);
    if (act) {
#pragma unroll
      for (int u = 0; u < J; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) l[pass3_dest<K, E, P - 1>(t, u, q)] = v[u + J * digrev3(q, LR)];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = l[t + S::TPR * i];
    }
    __syncthreads();
  }
}

// Full length-3^K transform on registers (every thread of the workgroup
// calls it; threads t >= TPR only pass the barriers).  FIRST > 0 starts at
// pass FIRST with the registers already holding that pass's inputs.
template <typename T, int K, int E, int SIGN, bool SPLIT, int P = 0, int FIRST = 0>
__device__ __forceinline__ void fft3_regs(Cx<T> (&v)[E], int t, bool act, void* lds, const Cx<T>* tw) {
  using S = Shape3<K, E>;
  if constexpr (P > FIRST) exchange3<T, K, E, P, SPLIT>(v, t, act, lds);
  if (act) pass3_jobs<T, K, E, P, SIGN>(v, t, tw, std::make_integer_sequence<int, E / S::radix(P)>{});
  if constexpr (P + 1 < S::NP) fft3_regs<T, K, E, SIGN, SPLIT, P + 1, FIRST>(v, t, act, lds, tw);
}

// Output order of the transforms for the selection: register p holds bin
// t + TPR digrev3(p) (digit reversal is its own inverse).
template <int LE>
struct DigrevOrder {
  static __host__ __device__ constexpr int bin(int p) { return digrev3(p, LE); }
  static __host__ __device__ constexpr int reg(int q) { return digrev3(q, LE); }
};

// Values per thread and threads of the length-3^K transforms (K = 1..8):
// 27 from 3^6 points (at 3^8, 243 threads), else 9 (or N).
__host__ __device__ constexpr int pickE3(int K) { return K >= 6 ? 27 : (K >= 2 ? 9 : 3); }
__host__ __device__ constexpr int threads3(int K) {
  return ((ipow3(K) / pickE3(K)) + 63) / 64 * 64;
}

}  // namespace afd
