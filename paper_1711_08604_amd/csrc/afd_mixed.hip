// The decomposition for mixed-radix N: N = 2^a 3^b 5^c 7^d <= 16384 with at
// least two distinct prime factors whose product is at most 30 (e.g.
// N = 1000, 1536, 6000, 12288, 15360).  The paper's closing remark extends
// the fast algorithm beyond powers of two; only the transforms depend on the
// factorisation of N, and the records, merge, re-check and update are the
// power-of-two path's own kernels, which take N as a parameter.
//
// The transforms are Stockham passes as in afd_primepow.h, with E values per
// thread (E a multiple of every prime of N, E <= 30) and TPR = N/E threads.
// Their passes have run-time radices R_s dividing E: TPR factored greedily
// (R = gcd(rest, E)), then a last pass of radix E.  Each pass multiplies by
// the tabled twiddles and runs E/R register DFTs of size R; the kernel
// selects the pass's code by R (uniform over the workgroup), so one kernel
// per E serves every N with that E.  Because the passes before the last
// multiply to TPR, ns(s) divides TPR: a thread's jobs u share k = t mod ns
// and its twiddle row, and the Stockham destinations need one division per
// pass.  A register DFT of size R decimates in time by the smallest prime
// of R first; its output position pos holds bin mbin(R, pos).
#include "afd_select.h"
#include "afd_primepow.h"

namespace afd {

__host__ __device__ __forceinline__ constexpr int mixed_spf(int v) {
  return v % 2 == 0 ? 2 : v % 3 == 0 ? 3 : v % 5 == 0 ? 5 : v % 7 == 0 ? 7 : v;
}
// Bin held by output position pos of the size-R register DFT, and its
// inverse.  With R = p R' (p the smallest prime of R), position p p' + d
// holds bin mbin(R', p') + d R'; written as loops over the levels (loops
// fold to constants where recursion would stay a call).
__host__ __device__ __forceinline__ constexpr int mbin(int R, int pos) {
  int b = 0;
  while (R > 1) {
    const int p = mixed_spf(R);
    R /= p;
    b += (pos % p) * R;
    pos /= p;
  }
  return b;
}
__host__ __device__ __forceinline__ constexpr int mreg(int R, int q) {
  int pos = 0, mul = 1;
  while (R > 1) {
    const int p = mixed_spf(R);
    R /= p;
    pos += (q / R) * mul;
    q %= R;
    mul *= p;
  }
  return pos;
}

// Both maps of a size-R register DFT as compile-time tables (indexing them
// with an unrolled loop's counter folds to a constant).
template <int R>
struct MTab {
  int bin[R];
  int reg[R];
};
template <int R>
__host__ __device__ constexpr MTab<R> make_mtab() {
  MTab<R> t{};
  for (int p = 0; p < R; ++p) {
    t.bin[p] = mbin(R, p);
    t.reg[p] = mreg(R, p);
  }
  return t;
}

// x e^{SIGN 2 pi i Q/R}; multiples of a quarter turn exactly
template <int Q, int R, int SIGN, typename T>
__device__ __forceinline__ Cx<T> twmul(Cx<T> x) {
  constexpr int q = ((Q % R) + R) % R;
  if constexpr (q == 0) {
    return x;
  } else if constexpr ((4 * q) % R == 0) {
    constexpr int k = (4 * q) / R;  // angle k pi/2
    if constexpr (k == 2) return Cx<T>{-x.x, -x.y};
    else if constexpr ((k == 1) == (SIGN > 0)) return Cx<T>{-x.y, x.x};  // times +i
    else return Cx<T>{x.y, -x.x};                                        // times -i
  } else {
    constexpr T c = T(unit_cos(q, R)), s = T(SIGN * unit_sin(q, R));
    return Cx<T>{fma(c, x.x, -s * x.y), fma(c, x.y, s * x.x)};
  }
}

// In-place P-point DFT (P = 2, 3, 5, 7) of t[0..P) in the stored order.
template <int P, int SIGN, typename T>
__device__ __forceinline__ void prime_dft(Cx<T> (&x)[P]) {
  if constexpr (P == 2) {
    const Cx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else {
    // s_j = t_j + t_(P-j), d_j = t_j - t_(P-j) (j = 1..H):
    //   X_0 = t_0 + sum_j s_j,
    //   X_q, X_(P-q) = t_0 + sum_j cos(2 pi jq/P) s_j +- SIGN i sum_j sin(2 pi jq/P) d_j
    constexpr int H = (P - 1) / 2;
    Cx<T> sj[H], dj[H];
    Cx<T> x0 = x[0];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      sj[j - 1] = cadd(x[j], x[P - j]);
      dj[j - 1] = csub(x[j], x[P - j]);
      x0 = cadd(x0, sj[j - 1]);
    }
    const Cx<T> t0 = x[0];
    x[0] = x0;
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      Cx<T> A = t0, B{T(0), T(0)};
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const T c = T(unit_cos(j * q, P)), s = T(SIGN * unit_sin(j * q, P));
        A = {fma(c, sj[j - 1].x, A.x), fma(c, sj[j - 1].y, A.y)};
        B = {fma(s, dj[j - 1].x, B.x), fma(s, dj[j - 1].y, B.y)};
      }
      x[q] = {A.x - B.y, A.y + B.x};
      x[P - q] = {A.x + B.y, A.y - B.x};
    }
  }
}

// R-point DFT on a[OFF + p STR], p < R, in place, decimation in time by the
// smallest prime P of R: the P interleaved sub-sequences first, then the
// combining butterflies.  Output position p holds bin mbin(R, p).
template <int R, int SIGN, int OFF, int STR, typename T>
struct DitM {
  static constexpr int P = mixed_spf(R), RS = R / P;
  template <int I>
  static __device__ __forceinline__ void bfly(Cx<T>* a) {
    constexpr int p = mreg(RS, I);  // sub-bin I of every sub-sequence sits at P p + j
    Cx<T> x[P];
    x[0] = a[OFF + (P * p) * STR];
    tw_load<I, p>(a, x, std::make_integer_sequence<int, P - 1>{});
    prime_dft<P, SIGN>(x);
#pragma unroll
    for (int q = 0; q < P; ++q) a[OFF + (P * p + q) * STR] = x[q];
  }
  template <int I, int PI, int... J>
  static __device__ __forceinline__ void tw_load(Cx<T>* a, Cx<T> (&x)[P], std::integer_sequence<int, J...>) {
    ((x[J + 1] = twmul<I * (J + 1), R, SIGN>(a[OFF + (P * PI + J + 1) * STR])), ...);
  }
  template <int... I>
  static __device__ __forceinline__ void stage(Cx<T>* a, std::integer_sequence<int, I...>) {
    (bfly<I>(a), ...);
  }
  template <int... J>
  static __device__ __forceinline__ void subs(Cx<T>* a, std::integer_sequence<int, J...>) {
    (DitM<RS, SIGN, OFF + J * STR, P * STR, T>::run(a), ...);
  }
  static __device__ __forceinline__ void run(Cx<T>* a) {
    if constexpr (R > 1) {
      subs(a, std::make_integer_sequence<int, P>{});
      stage(a, std::make_integer_sequence<int, RS>{});
    }
  }
};

template <int E>
struct MixedOrder {
  static __host__ __device__ __forceinline__ constexpr int bin(int p) {
    constexpr MTab<E> tb = make_mtab<E>();
    return tb.bin[p];
  }
  static __host__ __device__ __forceinline__ constexpr int reg(int q) {
    constexpr MTab<E> tb = make_mtab<E>();
    return tb.reg[q];
  }
};

// One pass of radix R (ns = the product of the earlier radices; tw points at
// the pass's table): twiddles e^{SIGN 2 pi i k r/(ns R)}, k = t mod ns, on
// inputs r = 1..R-1 of every job, then the register DFTs.
template <typename T, int E, int SIGN, int R, int... U>
__device__ __forceinline__ void mixed_dfts(Cx<T> (&v)[E], std::integer_sequence<int, U...>) {
  (DitM<R, SIGN, U, E / R, T>::run(v), ...);
}
template <typename T, int E, int SIGN, int R>
__device__ __forceinline__ void mixed_pass(Cx<T> (&v)[E], int t, int ns, const Cx<T>* __restrict__ tw) {
  constexpr int J = E / R;
  if (ns > 1) {
    const Cx<T>* __restrict__ row = tw + t % ns;
    Cx<T> w[R - 1];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      w[r - 1] = row[(r - 1) * ns];
      if constexpr (SIGN < 0) w[r - 1].y = -w[r - 1].y;
    }
#pragma unroll
    for (int u = 0; u < J; ++u)
#pragma unroll
      for (int r = 1; r < R; ++r) v[u + r * J] = cmul(v[u + r * J], w[r - 1]);
  }
  mixed_dfts<T, E, SIGN, R>(v, std::make_integer_sequence<int, J>{});
}

// The exchange after a pass of radix R: output q of job u = t + u TPR goes to
// its Stockham destination (job/ns) ns R + (job mod ns) + q ns, then each
// thread reads x[t + TPR i].  SPLIT moves real and imaginary parts in turn.
template <typename T, int E, int R, bool SPLIT>
__device__ __forceinline__ void mixed_exchange(Cx<T> (&v)[E], int t, int tpr, int ns, bool act, void* lds) {
  constexpr int J = E / R;
  constexpr MTab<R> tb = make_mtab<R>();
  const int tq = t / ns, tr = t - tq * ns, tn = tpr / ns;
  const int base = tq * ns * R + tr, ustep = tn * ns * R;
  if constexpr (SPLIT) {
    T* l = reinterpret_cast<T*>(lds);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      if (act) {
#pragma unroll
        for (int u = 0; u < J; ++u)
#pragma unroll
          for (int q = 0; q < R; ++q) {
            const Cx<T> val = v[u + J * tb.reg[q]];
            l[base + u * ustep + q * ns] = part == 0 ? val.x : val.y;
          }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const T val = l[t + tpr * i];
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
        for (int q = 0; q < R; ++q) l[base + u * ustep + q * ns] = v[u + J * tb.reg[q]];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = l[t + tpr * i];
    }
    __syncthreads();
  }
}

// Dispatch on the run-time radix R (a divisor of E, uniform over the workgroup).
template <typename T, int E, int SIGN, int D = 2>
__device__ __forceinline__ void mixed_pass_any(int R, Cx<T> (&v)[E], int t, int ns, const Cx<T>* tw) {
  if constexpr (D <= E) {
    if constexpr (E % D == 0) {
      if (R == D) {
        mixed_pass<T, E, SIGN, D>(v, t, ns, tw);
        return;
      }
    }
    mixed_pass_any<T, E, SIGN, D + 1>(R, v, t, ns, tw);
  }
}
template <typename T, int E, bool SPLIT, int D = 2>
__device__ __forceinline__ void mixed_exchange_any(int R, Cx<T> (&v)[E], int t, int tpr, int ns, bool act,
                                                   void* lds) {
  if constexpr (D <= E) {
    if constexpr (E % D == 0) {
      if (R == D) {
        mixed_exchange<T, E, D, SPLIT>(v, t, tpr, ns, act, lds);
        return;
      }
    }
    mixed_exchange_any<T, E, SPLIT, D + 1>(R, v, t, tpr, ns, act, lds);
  }
}

// Passes first..np-1 of the transform (every thread of the workgroup calls
// it; threads t >= TPR only pass the barriers).  The registers hold pass
// `first`'s inputs; the pass table (radix, ns, twiddle offset per pass) is
// read with scalar loads.
template <typename T, int E, int SIGN, bool SPLIT>
__device__ __forceinline__ void mixed_fft(Cx<T> (&v)[E], int t, bool act, void* lds, const Cx<T>* tw,
                                          const MixedArgs& g, int first) {
  int pr = 0, pn = 0;
  for (int s = first; s < g.np; ++s) {
    const int R = __builtin_amdgcn_readfirstlane(g.passes[3 * s]);
    const int ns = __builtin_amdgcn_readfirstlane(g.passes[3 * s + 1]);
    const int off = __builtin_amdgcn_readfirstlane(g.passes[3 * s + 2]);
    if (s > first) mixed_exchange_any<T, E, SPLIT>(pr, v, t, g.tpr, pn, act, lds);
    if (act) mixed_pass_any<T, E, SIGN>(R, v, t, ns, tw + off);
    pr = R;
    pn = ns;
  }
}

// Workgroup size bound: 256 registers per thread from E = 18 (E complex
// values in registers), 128 below.
__host__ __device__ constexpr int mixed_max_threads(int E) { return E > 16 ? 512 : 1024; }

template <typename T>
__host__ __device__ constexpr bool mixed_split(int n) {
  return sizeof(T) == 8 && size_t(n) * 2 * sizeof(T) > 32768;
}
template <typename T>
__host__ __device__ constexpr size_t mixed_region(int n) {
  return size_t(n) * (mixed_split<T>(n) ? 1 : 2) * sizeof(T);
}
template <typename T>
static size_t mixed_lds(int n) {
  const size_t need = mixed_region<T>(n) + kListScratchBytes;
  return need > sizeof(MergeScratch) ? need : sizeof(MergeScratch);
}

// c_l = sum_n g_n e^{-2 pi i l n/N}, one workgroup per signal.
template <typename T, int E, bool SPLIT>
__global__ __launch_bounds__(mixed_max_threads(E)) void k_fwd_mixed(const Cx<T>* __restrict__ g,
                                                                     const Cx<T>* __restrict__ tw,
                                                                     Cx<T>* __restrict__ c, MixedArgs geom) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x, tpr = geom.tpr, n = tpr * E;
  const bool act = t < tpr;
  c += size_t(n) * blockIdx.y;
  g += size_t(n) * blockIdx.y;
  Cx<T> v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = act ? g[t + tpr * i] : Cx<T>{T(0), T(0)};
  mixed_fft<T, E, -1, SPLIT>(v, t, act, smem, tw, geom, 0);
  if (act) {
#pragma unroll
    for (int p = 0; p < E; ++p) c[t + tpr * MixedOrder<E>::bin(p)] = v[p];
  }
}

template <typename T, int E, bool SPLIT, bool LIST>
__global__ __launch_bounds__(mixed_max_threads(E)) void k_radius_mixed(RadiusParams prm, MixedArgs geom) {
  using Ord = MixedOrder<E>;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  const int b = blockIdx.y, slot = blockIdx.x;
  const int t = threadIdx.x, tpr = geom.tpr, N = tpr * E;
  const bool act = t < tpr;
  // (radius, significant length) of this workgroup, longest spectra first
  const int2 wi = reinterpret_cast<const int2*>(prm.order)[slot];
  const int m = __builtin_amdgcn_readfirstlane(wi.x);
  const int L = __builtin_amdgcn_readfirstlane(wi.y);
  const Cx<T>* __restrict__ c = reinterpret_cast<const Cx<T>*>(prm.c) + size_t(N) * b;
  const T* __restrict__ pw = reinterpret_cast<const T*>(prm.pw) + size_t(m) * tpr;
  const T* __restrict__ pv = reinterpret_cast<const T*>(prm.pv) + size_t(m) * E;
  const Cx<T>* __restrict__ tw = reinterpret_cast<const Cx<T>*>(prm.tw);
  const T sc = reinterpret_cast<const T*>(prm.scale)[m];

  // Short spectra skip passes: with at most N/ns(s) terms the first s passes
  // only replicate values, so register i of thread t starts as x[a + D i],
  // a = t / ns(s), D = TPR / ns(s).  From pass 1 the weight r^(a + D i) is
  // r^a (r^t table) times r^(D i) (the [M][E] table of r^((TPR/R0) i)); at
  // the last pass (ns = TPR, at most E terms) it is r^i (r^t table, E <= TPR).
  const int r0 = geom.np >= 2 ? __builtin_amdgcn_readfirstlane(geom.passes[4]) : 1;  // ns(1)
  int first = 0;
  if (geom.np >= 2 && L <= N / r0) first = 1;
  if (geom.np >= 3 && E <= tpr && L <= E) first = geom.np - 1;
  Cx<T> v[E];
  if (first == geom.np - 1 && first >= 2) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      v[i] = {T(0), T(0)};
      if (act && i < L) {
        const Cx<T> x = c[i];
        const T w = pw[i];
        v[i] = {x.x * w, x.y * w};
      }
    }
  } else if (first == 1) {
    const int a = t / r0, D = tpr / r0;
    const T* __restrict__ pq = reinterpret_cast<const T*>(prm.pq) + size_t(m) * E;
    const T ra = act ? pw[a] : T(0);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int l = a + D * i;
      v[i] = {T(0), T(0)};
      if (act && l < L) {
        const Cx<T> x = c[l];
        const T w = ra * pq[i];
        v[i] = {x.x * w, x.y * w};
      }
    }
  } else {
    const T rt = act ? pw[t] : T(0);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int l = t + tpr * i;
      v[i] = {T(0), T(0)};
      if (act && l < L) {
        const Cx<T> x = c[l];
        const T w = rt * pv[i];
        v[i] = {x.x * w, x.y * w};
      }
    }
  }
  mixed_fft<T, E, +1, SPLIT>(v, t, act, smem, tw, geom, first);

  unsigned char* scratch = smem + mixed_region<T>(N);
  const uint32_t fbase = uint32_t(m) * uint32_t(N);
  if constexpr (LIST) {
    const FlatOrder ord{fbase, uint32_t(N), 0u, uint32_t(N)};
    BlockList32* lists = reinterpret_cast<BlockList32*>(prm.out) + size_t(prm.nrec) * b;
    uint64_t* heads = prm.heads + size_t(prm.nrec) * b;
    uint64_t* seconds = prm.seconds + size_t(prm.nrec) * b;
    select_list_o<E, 0, Ord>(v, act, sc, fbase, 1u, t, scratch, prm.tau_band, ord, lists + slot, heads + slot,
                             seconds + slot, prm.flagword + b, tpr);
  } else {
    if (prm.probe) {
      // a replayed step: the grid value at the forced point, scaled as the
      // selection scales its best value
      const int32_t* pr = prm.probe + size_t(prm.probe_stride) * b;
      const int pm = pr[0], pj = pr[1];
      if (act && m == pm && t == pj % tpr) {
        const int q = pj / tpr;
#pragma unroll
        for (int p = 0; p < E; ++p) {
          if (Ord::bin(p) == q) {
            prm.probe_out[2 * b] = double(v[p].x * sc);
            prm.probe_out[2 * b + 1] = double(v[p].y * sc);
          }
        }
      }
    }
    select_best_o<T, E, 0, Ord>(v, act, sc, fbase, 1u, t, reinterpret_cast<Best*>(scratch),
                                reinterpret_cast<BlockBest64*>(prm.out) + size_t(prm.nrec) * b + slot, tpr);
  }
  if (!last_arrival(prm.counter + b, gridDim.x, &s_last)) return;
  MergeScratch* Sm = reinterpret_cast<MergeScratch*>(smem);
  if constexpr (LIST) {
    select32_tail<2, 8>(reinterpret_cast<const BlockList32*>(prm.out) + size_t(prm.nrec) * b,
                  prm.heads + size_t(prm.nrec) * b, prm.seconds + size_t(prm.nrec) * b, prm.nrec, prm.recheck_k,
                  prm.tau_band, prm.flagword + b, prm.cand + b, Sm);
  } else {
    merge64_tail<2, 8>(reinterpret_cast<const BlockBest64*>(prm.out) + size_t(prm.nrec) * b, prm.nrec, N, prm.winner + b,
                 Sm);
  }
}

// Values per thread the mixed-radix path is built for (each a product of
// at least two distinct primes)
#define AFD_MIXED_E(X) X(6) X(10) X(12) X(14) X(15) X(18) X(20) X(21) X(24) X(28) X(30)

static int gcd_int(int a, int b) {
  while (b) {
    const int r = a % b;
    a = b;
    b = r;
  }
  return a;
}
static int prime_set(int64_t v) {
  int s = 1;
  for (const int p : {2, 3, 5, 7}) {
    if (v % p == 0) {
      s *= p;
      while (v % p == 0) v /= p;
    }
  }
  return v == 1 ? s : 0;
}

// The geometry for N (E = 0 if the mixed-radix path does not take N): of the
// E values with the primes of N, the one with the fewest passes (then the
// largest), TPR = N/E within the workgroup bound.
MixedGeom mixed_geom(int64_t n) {
  MixedGeom best{};
  if (n < 2 || n > kMaxMixedN) return best;
  const int ps = prime_set(n);
  if (ps == 0 || ps == 2 || ps == 3 || ps == 5 || ps == 7) return best;  // not 7-smooth, or a prime power
  for (const int E : {
#define X(E) E,
         AFD_MIXED_E(X)
#undef X
       }) {
    if (n % E != 0 || prime_set(E) != ps) continue;
    const int tpr = int(n / E);
    if (tpr > mixed_max_threads(E)) continue;
    MixedGeom g{};
    g.E = E;
    g.tpr = tpr;
    g.threads = (tpr + 63) / 64 * 64;
    int rest = tpr, np = 0;
    bool ok = true;
    while (rest > 1 && ok) {
      const int r = gcd_int(rest, E);
      if (r == 1 || np + 1 >= kMaxMixedPasses) ok = false;
      else {
        g.radix[np++] = r;
        rest /= r;
      }
    }
    if (!ok) continue;
    g.radix[np++] = E;
    g.np = np;
    int ns = 1, off = 0;
    for (int s = 0; s < np; ++s) {
      g.ns[s] = ns;
      g.twoff[s] = off;
      if (s > 0) off += (g.radix[s] - 1) * ns;
      ns *= g.radix[s];
    }
    g.twsize = off;
    if (best.E == 0 || g.np < best.np || (g.np == best.np && g.E > best.E)) best = g;
  }
  return best;
}

// Stockham twiddles: pass s >= 1 (radix R, ns = the product of the earlier
// radices) holds e^{+2 pi i j r/(ns R)} at twoff(s) + (r - 1) ns + j.
void mixed_twiddles(const MixedGeom& g, double* tw) {
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int s = 1; s < g.np; ++s) {
    const int R = g.radix[s], ns = g.ns[s];
    for (int r = 1; r < R; ++r)
      for (int j = 0; j < ns; ++j) {
        const long double ang = two_pi * (long double)(j * r) / (long double)(ns * R);
        const size_t e = size_t(g.twoff[s]) + size_t(r - 1) * ns + j;
        tw[2 * e] = (double)cosl(ang);
        tw[2 * e + 1] = (double)sinl(ang);
      }
  }
}

// The device pass table: (radix, ns, twiddle offset) of each pass.
void mixed_pass_table(const MixedGeom& g, int* out) {
  for (int s = 0; s < g.np; ++s) {
    out[3 * s] = g.radix[s];
    out[3 * s + 1] = g.ns[s];
    out[3 * s + 2] = g.twoff[s];
  }
}

hipError_t setup_mixed_attributes() {
  hipError_t e = hipSuccess;
#define X(E)                                                                                                     \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius_mixed<double, E, true, false>)); \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius_mixed<double, E, false, false>)); \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius_mixed<float, E, false, true>)); \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_mixed<double, E, true>));        \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_mixed<double, E, false>));       \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_mixed<float, E, false>));
  AFD_MIXED_E(X)
#undef X
  return e;
}

hipError_t launch_fwd_mixed(const MixedGeom& geo, const int* passes, bool fp64, const void* sig, const void* tw,
                            void* c, int batch, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int n = geo.E * geo.tpr;
  const MixedArgs g{passes, geo.np, geo.tpr, geo.threads, geo.E};
  switch (g.E) {
#define X(E)                                                                                                     \
  case E:                                                                                                        \
    if (fp64 && mixed_split<double>(n))                                                                          \
      launch_ev(k_fwd_mixed<double, E, true>, dim3(1, batch), dim3(g.threads), uint32_t(mixed_region<double>(n)), \
                s, e0, e1, static_cast<const Cx<double>*>(sig), static_cast<const Cx<double>*>(tw),            \
                static_cast<Cx<double>*>(c), g);                                                         \
    else if (fp64)                                                                                               \
      launch_ev(k_fwd_mixed<double, E, false>, dim3(1, batch), dim3(g.threads),                                  \
                uint32_t(mixed_region<double>(n)), s, e0, e1, static_cast<const Cx<double>*>(sig),               \
                static_cast<const Cx<double>*>(tw), static_cast<Cx<double>*>(c), g);                             \
    else                                                                                                         \
      launch_ev(k_fwd_mixed<float, E, false>, dim3(1, batch), dim3(g.threads), uint32_t(mixed_region<float>(n)), \
                s, e0, e1, static_cast<const Cx<float>*>(sig), static_cast<const Cx<float>*>(tw),              \
                static_cast<Cx<float>*>(c), g);                                                          \
    break;
    AFD_MIXED_E(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_radius_mixed(const MixedGeom& geo, const int* passes, bool fp64, const RadiusParams& p, int batch,
                               hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (p.rpb != 1 || p.nrec != p.M || !p.tail || p.queue) return hipErrorInvalidValue;
  const int n = geo.E * geo.tpr;
  const MixedArgs g{passes, geo.np, geo.tpr, geo.threads, geo.E};
  switch (g.E) {
#define X(E)                                                                                                  \
  case E:                                                                                                     \
    if (fp64 && mixed_split<double>(n))                                                                       \
      launch_ev(k_radius_mixed<double, E, true, false>, dim3(p.M, batch), dim3(g.threads),                    \
                uint32_t(mixed_lds<double>(n)), s, e0, e1, p, g);                                             \
    else if (fp64)                                                                                            \
      launch_ev(k_radius_mixed<double, E, false, false>, dim3(p.M, batch), dim3(g.threads),                   \
                uint32_t(mixed_lds<double>(n)), s, e0, e1, p, g);                                             \
    else                                                                                                      \
      launch_ev(k_radius_mixed<float, E, false, true>, dim3(p.M, batch), dim3(g.threads),                     \
                uint32_t(mixed_lds<float>(n)), s, e0, e1, p, g);                                              \
    break;
    AFD_MIXED_E(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int mixed_lds_bytes(const MixedGeom& g, bool fp64) {
  const int n = g.E * g.tpr;
  return int(fp64 ? mixed_lds<double>(n) : mixed_lds<float>(n));
}

}  // namespace afd
