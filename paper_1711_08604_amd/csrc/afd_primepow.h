// Radix-P transforms for N = P^K points (P = 3, 5, 7).  The paper's closing
// remark notes that the fast algorithm carries over to N = p^K for a prime
// p: the radix-2 split of Theorem 2.1 (eqs. term8, term82) becomes a P-point
// split.  With S_r the length-N/P DFT of the samples n = r (mod P),
//   X[k + q N/P] = sum_{r<P} W^{r (k + q N/P)} S_r[k],   W = e^{+-2 pi i/N},
// so one level costs N/P P-point butterflies.
//
// The layout follows the radix-2 Stockham transform of afd_device.h: a
// length-P^K transform is spread over TPR = N/E threads holding E = P^e
// values each; pass s runs E/R radix-R jobs (job = t + u TPR, inputs
// x[job + r N/R] = regs[u + (E/R) r]), twiddles e^{+-2 pi i k r/(Ns R)}
// (k = job mod Ns) from a table, then an R-point DFT in registers whose
// output position p holds bin digrev(p) (base-P digit reversal), written
// to the Stockham destination (job/Ns) Ns R + (job mod Ns) + q Ns.  After
// the last pass register p holds output bin t + TPR digrev(p).  Threads
// t >= TPR of a workgroup take part in the barriers only.  LDS needs no
// padding: every strided access steps by a power of the odd prime P, so the
// lanes of a wave fall on distinct banks.
#pragma once

#include "afd_device.h"

namespace afd {

__host__ __device__ constexpr int ipow(int p, int k) { return k <= 0 ? 1 : p * ipow(p, k - 1); }
__host__ __device__ constexpr int ilogc(int p, int v) { return v <= 1 ? 0 : 1 + ilogc(p, v / p); }
__host__ __device__ constexpr int digrev(int p, int v, int digits) {
  int r = 0;
  for (int i = 0; i < digits; ++i) {
    r = r * p + v % p;
    v /= p;
  }
  return r;
}

// cos and sin of 2 pi q / R at compile time, from the Taylor series on an
// angle reduced to [0, pi/4] by the symmetries of the unit circle (accurate
// to a few units in the last place; used for the butterflies' internal
// twiddles).
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

// Pass structure of a length-P^K transform with E = P^e values per thread:
// an optional first pass of radix P^(K mod e), then passes of radix E.
template <int P, int K, int E>
struct ShapeP {
  static constexpr int N = ipow(P, K);
  static constexpr int LE = ilogc(P, E);
  static constexpr int Q0 = K % LE;
  static constexpr int NP = K / LE + (Q0 ? 1 : 0);
  static constexpr int TPR = N / E;
  static_assert(ipow(P, LE) == E && E <= N, "E must be a power of P, at most N");
  __host__ __device__ static constexpr int radix(int s) { return (s == 0 && Q0) ? ipow(P, Q0) : E; }
  __host__ __device__ static constexpr int ns(int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= radix(i);
    return v;
  }
  // twiddle table: pass s >= 1 owns (radix(s) - 1) * ns(s) entries, entry
  // (r - 1) * ns(s) + k = e^{+2 pi i k r/(ns(s) radix(s))}, r = 1..radix-1
  __host__ __device__ static constexpr int twoff(int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += (radix(i) - 1) * ns(i);
    return o;
  }
  __host__ __device__ static constexpr int twsize() { return twoff(NP); }
};

// R-point DFT (R = P^d) on a[OFF + p*STR], p = 0..R-1, in place, radix-P
// decimation in time (the P interleaved sub-sequences first, then the
// combining butterflies); output position p holds bin digrev(P, p, d).
// X[q] = sum_r x[r] e^{SIGN 2 pi i r q / R}.
template <int P, int R, int SIGN, int OFF, int STR, typename T>
struct DitP {
  template <int I>
  static __device__ __forceinline__ void bfly(Cx<T>* a) {
    // sub-bin I of the P sub-sequences sits at position P digrev(I) + j
    constexpr int p = digrev(P, I, ilogc(P, R / P));
    if constexpr (P == 3) {
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
    } else {
      // t_j = x_j W_R^(I j); with s_j = t_j + t_(P-j), d_j = t_j - t_(P-j)
      // (j = 1..H, H = (P-1)/2):
      //   X_0 = t_0 + sum_j s_j,
      //   X_q, X_(P-q) = t_0 + sum_j cos(2 pi jq/P) s_j
      //                  +- SIGN i sum_j sin(2 pi jq/P) d_j    (q = 1..H)
      constexpr int H = (P - 1) / 2;
      Cx<T> tv[P];
#pragma unroll
      for (int j = 0; j < P; ++j) tv[j] = a[OFF + (P * p + j) * STR];
      if constexpr (I != 0) {
#pragma unroll
        for (int j = 1; j < P; ++j) {
          const T c = T(unit_cos(I * j, R)), s = T(SIGN * unit_sin(I * j, R));
          const Cx<T> x = tv[j];
          tv[j] = {fma(c, x.x, -s * x.y), fma(c, x.y, s * x.x)};
        }
      }
      Cx<T> sj[H], dj[H];
      Cx<T> x0 = tv[0];
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        sj[j - 1] = cadd(tv[j], tv[P - j]);
        dj[j - 1] = csub(tv[j], tv[P - j]);
        x0 = cadd(x0, sj[j - 1]);
      }
      a[OFF + (P * p) * STR] = x0;
#pragma unroll
      for (int q = 1; q <= H; ++q) {
        Cx<T> A = tv[0], B{T(0), T(0)};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
          const T c = T(unit_cos(j * q, P)), s = T(SIGN * unit_sin(j * q, P));
          A = {fma(c, sj[j - 1].x, A.x), fma(c, sj[j - 1].y, A.y)};
          B = {fma(s, dj[j - 1].x, B.x), fma(s, dj[j - 1].y, B.y)};
        }
        // i B = (-B.y, B.x); the sign SIGN is folded into s above
        a[OFF + (P * p + q) * STR] = {A.x - B.y, A.y + B.x};
        a[OFF + (P * p + P - q) * STR] = {A.x + B.y, A.y - B.x};
      }
    }
  }
  template <int... I>
  static __device__ __forceinline__ void stage(Cx<T>* a, std::integer_sequence<int, I...>) {
    (bfly<I>(a), ...);
  }
  template <int... J>
  static __device__ __forceinline__ void subs(Cx<T>* a, std::integer_sequence<int, J...>) {
    (DitP<P, R / P, SIGN, OFF + J * STR, P * STR, T>::run(a), ...);
  }
  static __device__ __forceinline__ void run(Cx<T>* a) {
    if constexpr (R > 1) {
      subs(a, std::make_integer_sequence<int, P>{});
      stage(a, std::make_integer_sequence<int, R / P>{});
    }
  }
};

// One butterfly job u of Stockham pass S in place on the registers.
template <typename T, int P, int K, int E, int S, int SIGN, int U>
__device__ __forceinline__ void passp_job(Cx<T> (&v)[E], int t, const Cx<T>* __restrict__ tw) {
  using Sh = ShapeP<P, K, E>;
  constexpr int R = Sh::radix(S);
  constexpr int NS = Sh::ns(S);
  constexpr int J = E / R;
  if constexpr (NS > 1) {
    const int job = t + U * Sh::TPR;
    const int k = job % NS;
    const Cx<T>* __restrict__ row = tw + Sh::twoff(S) + k;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      Cx<T> w = row[(r - 1) * NS];
      if constexpr (SIGN < 0) w.y = -w.y;
      v[U + r * J] = cmul(v[U + r * J], w);
    }
  }
  DitP<P, R, SIGN, U, J, T>::run(v);
}

template <typename T, int P, int K, int E, int S, int SIGN, int... U>
__device__ __forceinline__ void passp_jobs(Cx<T> (&v)[E], int t, const Cx<T>* tw, std::integer_sequence<int, U...>) {
  (passp_job<T, P, K, E, S, SIGN, U>(v, t, tw), ...);
}

// Destination of output q of job u after pass S (Stockham order).
template <int P, int K, int E, int S>
__device__ __forceinline__ int passp_dest(int t, int u, int q) {
  using Sh = ShapeP<P, K, E>;
  constexpr int R = Sh::radix(S);
  constexpr int NS = Sh::ns(S);
  const int job = t + u * Sh::TPR;
  return (job / NS) * NS * R + job % NS + q * NS;
}

// The exchange between pass S - 1 and pass S: outputs to their Stockham
// destinations, then each thread reads x[t + TPR i].  SPLIT moves real and
// imaginary parts through N reals in turn.  `act`: the thread is one of the
// TPR that hold values (all threads pass the barriers).
template <typename T, int P, int K, int E, int S, bool SPLIT>
__device__ __forceinline__ void exchangep(Cx<T> (&v)[E], int t, bool act, void* lds) {
  using Sh = ShapeP<P, K, E>;
  constexpr int R = Sh::radix(S - 1);
  constexpr int J = E / R;
  constexpr int LR = ilogc(P, R);
  if constexpr (SPLIT) {
    T* l = reinterpret_cast<T*>(lds);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      if (act) {
#pragma unroll
        for (int u = 0; u < J; ++u)
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const Cx<T> val = v[u + J * digrev(P, q, LR)];
            l[passp_dest<P, K, E, S - 1>(t, u, q)] = part == 0 ? val.x : val.y;
          }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const T val = l[t + Sh::TPR * i];
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
        for (int q = 0; q < R; ++q) l[passp_dest<P, K, E, S - 1>(t, u, q)] = v[u + J * digrev(P, q, LR)];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = l[t + Sh::TPR * i];
    }
    __syncthreads();
  }
}

// Full length-P^K transform on registers (every thread of the workgroup
// calls it; threads t >= TPR only pass the barriers).  FIRST > 0 starts at
// pass FIRST with the registers already holding that pass's inputs.
template <typename T, int P, int K, int E, int SIGN, bool SPLIT, int S = 0, int FIRST = 0>
__device__ __forceinline__ void fftp_regs(Cx<T> (&v)[E], int t, bool act, void* lds, const Cx<T>* tw) {
  using Sh = ShapeP<P, K, E>;
  if constexpr (S > FIRST) exchangep<T, P, K, E, S, SPLIT>(v, t, act, lds);
  if (act) passp_jobs<T, P, K, E, S, SIGN>(v, t, tw, std::make_integer_sequence<int, E / Sh::radix(S)>{});
  if constexpr (S + 1 < Sh::NP) fftp_regs<T, P, K, E, SIGN, SPLIT, S + 1, FIRST>(v, t, act, lds, tw);
}

// Output order of the transforms for the selection: register p holds bin
// t + TPR digrev(p) (digit reversal is its own inverse).
template <int P, int LE>
struct DigrevOrder {
  static __host__ __device__ constexpr int bin(int p) { return digrev(P, p, LE); }
  static __host__ __device__ constexpr int reg(int q) { return digrev(P, q, LE); }
};

// Values per thread of the length-P^K transforms.  P = 3 (K = 1..8): 27
// from 3^6 points (at 3^8, 243 threads), else 9 (or N).  P = 5 (K = 1..6):
// 25 from 5^5 points (at 5^6, 625 threads), else 5.  P = 7 (K = 1..4): 7.
__host__ __device__ constexpr int pickEp(int P, int K) {
  return P == 3 ? (K >= 6 ? 27 : (K >= 2 ? 9 : 3)) : P == 5 ? (K >= 5 ? 25 : 5) : P;
}
__host__ __device__ constexpr int threadsp(int P, int K) {
  return ((ipow(P, K) / pickEp(P, K)) + 63) / 64 * 64;
}

}  // namespace afd
