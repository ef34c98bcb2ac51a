// The decomposition for N = 3^K samples (K = 1..8): forward DFT of the
// remainder and the fused per-radius kernel on the radix-3 transforms of
// afd_tern.h.  The paper's closing remark states that its fast algorithm
// holds for N = p^K; only the transforms depend on the factorisation of N.
// The records, the merge, the double re-check and the update are the
// power-of-two path's own kernels, which take N as a parameter.
//
// Per radius m the kernel forms f(l) = r_m^l c_l for l below the radius'
// significant spectrum length (r_m^l = r_m^t r_m^(TPR v) for l = t + TPR v,
// the same two double-built tables as the power-of-two path), runs the
// inverse transform, scales by sqrt(1 - r_m^2) / (N (1 - r_m^N)) and
// selects over its N points as the power-of-two radius kernel does: FP64
// keeps the best point and runner-up, FP32 the points within the re-check
// band; the last workgroup merges the records into the winner (FP64) or the
// short-list (FP32).  One radius per workgroup.
#include "afd_select.h"
#include "afd_tern.h"

namespace afd {

// The transforms exchange complex values through LDS, or, beyond 32 KiB,
// real and imaginary parts in turn.
template <typename T, int K>
__host__ __device__ constexpr bool tern_split() {
  return size_t(ipow3(K)) * 2 * sizeof(T) > 32768;
}
template <typename T, int K>
__host__ __device__ constexpr size_t tern_region() {
  return size_t(ipow3(K)) * (tern_split<T, K>() ? 1 : 2) * sizeof(T);
}
template <typename T, int K>
static size_t tern_lds() {
  const size_t need = tern_region<T, K>() + kListScratchBytes;
  return need > sizeof(MergeScratch) ? need : sizeof(MergeScratch);
}

// c_l = sum_n g_n e^{-2 pi i l n/N}, one workgroup per signal.
template <typename T, int K>
__global__ __launch_bounds__(threads3(K)) void k_fwd3(const Cx<T>* __restrict__ g, const Cx<T>* __restrict__ tw,
                                                      Cx<T>* __restrict__ c) {
  constexpr int E = pickE3(K);
  using S = Shape3<K, E>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  const bool act = t < S::TPR;
  g += size_t(S::N) * blockIdx.y;
  c += size_t(S::N) * blockIdx.y;
  Cx<T> v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = act ? g[t + S::TPR * i] : Cx<T>{T(0), T(0)};
  fft3_regs<T, K, E, -1, tern_split<T, K>()>(v, t, act, smem, tw);
  if (act) {
#pragma unroll
    for (int p = 0; p < E; ++p) c[t + S::TPR * digrev3(p, S::LE)] = v[p];
  }
}

// From 3^7 points the forward DFT is split as N = N1 N2 (N1 = 3^(K/2)):
// n = l1 + N1 l2, l = k2 + N2 k1.  The first pass transforms each column l1
// over l2 and applies e^{-2 pi i l1 k2/N}, storing X[k2][l1]; the second
// transforms each row k2 over l1 into c[k2 + N2 k1].  Both run several
// short transforms per 64-thread workgroup on many CUs, where one
// workgroup holding all N points would serialise the whole transform.
constexpr int kFwd3SplitK = 7;
template <int K>
struct Split3 {
  static constexpr int K1 = K / 2, K2 = K - K1;
  static constexpr int N1 = ipow3(K1), N2 = ipow3(K2);
};
// transforms of 3^KK points per 64-thread workgroup
template <int KK>
__host__ __device__ constexpr int per_wave3() {
  return 64 / Shape3<KK, pickE3(KK)>::TPR;
}

template <typename T, int K>
__global__ __launch_bounds__(64) void k_fwd3_cols(const Cx<T>* __restrict__ g, const Cx<T>* __restrict__ tw2,
                                                  const double* __restrict__ omega, Cx<T>* __restrict__ xt) {
  using P = Split3<K>;
  constexpr int E2 = pickE3(P::K2);
  using S2 = Shape3<P::K2, E2>;
  constexpr int CPB = per_wave3<P::K2>();
  constexpr int N = ipow3(K);
  extern __shared__ __align__(16) unsigned char smem[];
  // adjacent threads take adjacent columns (contiguous loads)
  const int ci = int(threadIdx.x) % CPB, t = int(threadIdx.x) / CPB;
  const int l1 = int(blockIdx.x) * CPB + ci;
  const bool act = t < S2::TPR && l1 < P::N1;
  g += size_t(N) * blockIdx.y;
  xt += size_t(N) * blockIdx.y;
  unsigned char* region = smem + size_t(ci) * P::N2 * sizeof(Cx<T>);
  Cx<T> v[E2];
#pragma unroll
  for (int i = 0; i < E2; ++i) v[i] = act ? g[l1 + P::N1 * (t + S2::TPR * i)] : Cx<T>{T(0), T(0)};
  fft3_regs<T, P::K2, E2, -1, false>(v, t, act, region, tw2);
  if (act) {
#pragma unroll
    for (int p = 0; p < E2; ++p) {
      const int k2 = t + S2::TPR * digrev3(p, S2::LE);
      const int e = l1 * k2;  // < N
      const Cx<T> w{T(omega[2 * e]), T(-omega[2 * e + 1])};
      xt[size_t(k2) * P::N1 + l1] = cmul(v[p], w);
    }
  }
}

template <typename T, int K>
__global__ __launch_bounds__(64) void k_fwd3_rows(const Cx<T>* __restrict__ xt, const Cx<T>* __restrict__ tw1,
                                                  Cx<T>* __restrict__ c) {
  using P = Split3<K>;
  constexpr int E1 = pickE3(P::K1);
  using S1 = Shape3<P::K1, E1>;
  constexpr int RPB = per_wave3<P::K1>();
  constexpr int N = ipow3(K);
  extern __shared__ __align__(16) unsigned char smem[];
  // the threads of a row are adjacent (contiguous loads)
  const int ri = int(threadIdx.x) / S1::TPR, t = int(threadIdx.x) % S1::TPR;
  const int k2 = int(blockIdx.x) * RPB + ri;
  const bool act = ri < RPB && k2 < P::N2;
  xt += size_t(N) * blockIdx.y;
  c += size_t(N) * blockIdx.y;
  unsigned char* region = smem + size_t(ri < RPB ? ri : RPB - 1) * P::N1 * sizeof(Cx<T>);
  Cx<T> v[E1];
#pragma unroll
  for (int i = 0; i < E1; ++i) v[i] = act ? xt[size_t(k2) * P::N1 + t + S1::TPR * i] : Cx<T>{T(0), T(0)};
  fft3_regs<T, P::K1, E1, -1, false>(v, t, act, region, tw1);
  if (act) {
#pragma unroll
    for (int p = 0; p < E1; ++p) c[k2 + P::N2 * (t + S1::TPR * digrev3(p, S1::LE))] = v[p];
  }
}

template <typename T, int K, bool LIST>
__global__ __launch_bounds__(threads3(K)) void k_radius3(RadiusParams prm) {
  constexpr int E = pickE3(K);
  using S = Shape3<K, E>;
  constexpr int N = S::N, TPR = S::TPR;
  using Ord = DigrevOrder<S::LE>;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  const int b = blockIdx.y, slot = blockIdx.x;
  const int t = threadIdx.x;
  const bool act = t < TPR;
  // (radius, significant length) of this workgroup, longest spectra first
  const int2 wi = reinterpret_cast<const int2*>(prm.order)[slot];
  const int m = __builtin_amdgcn_readfirstlane(wi.x);
  const int L = __builtin_amdgcn_readfirstlane(wi.y);
  const Cx<T>* __restrict__ c = reinterpret_cast<const Cx<T>*>(prm.c) + size_t(N) * b;
  const T* __restrict__ pw = reinterpret_cast<const T*>(prm.pw) + size_t(m) * TPR;
  const T* __restrict__ pv = reinterpret_cast<const T*>(prm.pv) + size_t(m) * E;
  const Cx<T>* __restrict__ tw = reinterpret_cast<const Cx<T>*>(prm.tw);
  const T sc = reinterpret_cast<const T*>(prm.scale)[m];

  // Short spectra skip passes (uniform over the workgroup: one radius).  A
  // pass whose inputs x[job + r N/R] are zero for r > 0 only replicates
  // x[job], so with at most N/ns(P) terms the inputs of pass P are
  // x_P[i] = x[i / ns(P)]: register i of thread t holds x[a + D i] with
  // a = t / ns(P), D = TPR / ns(P) (TPR is a multiple of ns(P)).  From pass 1:
  // r^l = r^a (r^t table) times r^(D i) (the [M][E] table of r^((TPR/R0) i));
  // from pass 2 (three passes): ns(2) = TPR, so register i holds x[i], with
  // weight r^i from the r^t table (E <= TPR there).
  constexpr int NP = S::NP;
  int skip = 0;
  if constexpr (NP >= 2) skip = L <= N / S::ns(1) ? 1 : 0;
  if constexpr (NP >= 3) skip = L <= N / S::ns(2) ? 2 : skip;
  Cx<T> v[E];
  if (skip == 2) {
    if constexpr (NP >= 3) {
      static_assert(S::ns(2) == TPR && E <= TPR, "from pass 2 every thread holds x[0..E)");
#pragma unroll
      for (int i = 0; i < E; ++i) {
        v[i] = {T(0), T(0)};
        if (act && i < L) {
          const Cx<T> x = c[i];
          const T w = pw[i];
          v[i] = {x.x * w, x.y * w};
        }
      }
      fft3_regs<T, K, E, +1, tern_split<T, K>(), 2, 2>(v, t, act, smem, tw);
    }
  } else if (skip == 1) {
    if constexpr (NP >= 2) {
      constexpr int R0 = S::ns(1), D = TPR / R0;
      static_assert(TPR % R0 == 0, "TPR is a multiple of the first radix");
      const T* __restrict__ pq = reinterpret_cast<const T*>(prm.pq) + size_t(m) * E;
      const int a = t / R0;
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
      fft3_regs<T, K, E, +1, tern_split<T, K>(), 1, 1>(v, t, act, smem, tw);
    }
  } else {
    const T rt = act ? pw[t] : T(0);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int l = t + TPR * i;
      v[i] = {T(0), T(0)};
      if (act && l < L) {
        const Cx<T> x = c[l];
        const T w = rt * pv[i];
        v[i] = {x.x * w, x.y * w};
      }
    }
    fft3_regs<T, K, E, +1, tern_split<T, K>()>(v, t, act, smem, tw);
  }

  unsigned char* scratch = smem + tern_region<T, K>();
  const uint32_t fbase = uint32_t(m) * uint32_t(N);
  if constexpr (LIST) {
    const FlatOrder ord{fbase, uint32_t(N), 0u, uint32_t(N)};
    BlockList32* lists = reinterpret_cast<BlockList32*>(prm.out) + size_t(prm.nrec) * b;
    uint64_t* heads = prm.heads + size_t(prm.nrec) * b;
    uint64_t* seconds = prm.seconds + size_t(prm.nrec) * b;
    select_list_o<E, TPR, Ord>(v, act, sc, fbase, 1u, t, scratch, prm.tau_band, ord, lists + slot, heads + slot,
                               seconds + slot, prm.flagword + b);
  } else {
    if (prm.probe) {
      // a replayed step: the grid value at the forced point, scaled as the
      // selection scales its best value
      const int32_t* pr = prm.probe + size_t(prm.probe_stride) * b;
      const int pm = pr[0], pj = pr[1];
      if (act && m == pm && t == pj % TPR) {
        const int q = pj / TPR;
#pragma unroll
        for (int p = 0; p < E; ++p) {
          if (Ord::bin(p) == q) {
            prm.probe_out[2 * b] = double(v[p].x * sc);
            prm.probe_out[2 * b + 1] = double(v[p].y * sc);
          }
        }
      }
    }
    select_best_o<T, E, TPR, Ord>(v, act, sc, fbase, 1u, t, reinterpret_cast<Best*>(scratch),
                                  reinterpret_cast<BlockBest64*>(prm.out) + size_t(prm.nrec) * b + slot);
  }
  if (!last_arrival(prm.counter + b, gridDim.x, &s_last)) return;
  MergeScratch* Sm = reinterpret_cast<MergeScratch*>(smem);
  if constexpr (LIST) {
    select32_tail(reinterpret_cast<const BlockList32*>(prm.out) + size_t(prm.nrec) * b,
                  prm.heads + size_t(prm.nrec) * b, prm.seconds + size_t(prm.nrec) * b, prm.nrec, prm.recheck_k,
                  prm.tau_band, prm.flagword + b, prm.cand + b, Sm);
  } else {
    merge64_tail(reinterpret_cast<const BlockBest64*>(prm.out) + size_t(prm.nrec) * b, prm.nrec, N, prm.winner + b,
                 Sm);
  }
}

#define AFD_TERN_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

TernGeom tern_geom(int k) {
  TernGeom g{};
  if (k < 1 || k > kMaxTernK) return g;
  g.k = k;
  g.E = pickE3(k);
  g.tpr = ipow3(k) / g.E;
  g.threads = threads3(k);
  switch (k) {
#define X(K)                                                                          \
  case K:                                                                             \
    g.twsize = Shape3<K, pickE3(K)>::twsize();                                        \
    break;
    AFD_TERN_CASES(X)
#undef X
    default:
      break;
  }
  return g;
}

// Stockham twiddles of the length-3^k transforms: pass p >= 1 (radix R,
// ns = the product of the earlier radices) holds e^{+2 pi i k r/(ns R)} at
// (r - 1) ns + k, after the entries of the earlier passes.
void tern_twiddles(int k, double* tw) {
  const int E = pickE3(k), LE = ilog3c(E), q0 = k % LE, np = k / LE + (q0 ? 1 : 0);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  size_t off = 0;
  int ns = 1;
  for (int p = 0; p < np; ++p) {
    const int R = (p == 0 && q0) ? ipow3(q0) : E;
    if (p > 0) {
      for (int r = 1; r < R; ++r)
        for (int j = 0; j < ns; ++j) {
          const long double ang = two_pi * (long double)(j * r) / (long double)(ns * R);
          tw[2 * (off + size_t(r - 1) * ns + j)] = (double)cosl(ang);
          tw[2 * (off + size_t(r - 1) * ns + j) + 1] = (double)sinl(ang);
        }
      off += size_t(R - 1) * ns;
    }
    ns *= R;
  }
}

hipError_t setup_tern_attributes() {
  hipError_t e = hipSuccess;
#define X(K)                                                                                               \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius3<double, K, false>)); \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius3<float, K, true>));   \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd3<double, K>));           \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd3<float, K>));
  AFD_TERN_CASES(X)
#undef X
  return e;
}

// Forward DFT tables: the split's row (3^(K/2)) and column (3^(K - K/2))
// twiddle entries, 0 below the split.
int tern_fwd_twsize(int k, bool rows) {
  if (k < kFwd3SplitK) return 0;
  return tern_geom(rows ? k / 2 : k - k / 2).twsize;
}

hipError_t launch_fwd3(int k, bool fp64, const void* g, const void* tw, const void* tw1, const void* tw2,
                       const double* omega, void* xt, void* c, int batch, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (k >= kFwd3SplitK) {
    switch (k) {
#define X(K)                                                                                                      \
  case K: {                                                                                                       \
    using P = Split3<K>;                                                                                          \
    const dim3 gc((P::N1 + per_wave3<P::K2>() - 1) / per_wave3<P::K2>(), batch);                                  \
    const dim3 gr((P::N2 + per_wave3<P::K1>() - 1) / per_wave3<P::K1>(), batch);                                  \
    if (fp64) {                                                                                                   \
      launch_ev(k_fwd3_cols<double, K>, gc, dim3(64), uint32_t(per_wave3<P::K2>() * P::N2 * 16), s, e0, nullptr,  \
                static_cast<const Cx<double>*>(g), static_cast<const Cx<double>*>(tw2), omega,                   \
                static_cast<Cx<double>*>(xt));                                                                   \
      launch_ev(k_fwd3_rows<double, K>, gr, dim3(64), uint32_t(per_wave3<P::K1>() * P::N1 * 16), s, nullptr, e1,  \
                static_cast<const Cx<double>*>(xt), static_cast<const Cx<double>*>(tw1),                         \
                static_cast<Cx<double>*>(c));                                                                    \
    } else {                                                                                                      \
      launch_ev(k_fwd3_cols<float, K>, gc, dim3(64), uint32_t(per_wave3<P::K2>() * P::N2 * 8), s, e0, nullptr,    \
                static_cast<const Cx<float>*>(g), static_cast<const Cx<float>*>(tw2), omega,                     \
                static_cast<Cx<float>*>(xt));                                                                    \
      launch_ev(k_fwd3_rows<float, K>, gr, dim3(64), uint32_t(per_wave3<P::K1>() * P::N1 * 8), s, nullptr, e1,    \
                static_cast<const Cx<float>*>(xt), static_cast<const Cx<float>*>(tw1), static_cast<Cx<float>*>(c)); \
    }                                                                                                             \
    break;                                                                                                        \
  }
      X(7) X(8)
#undef X
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (k) {
#define X(K)                                                                                                     \
  case K:                                                                                                        \
    if (fp64)                                                                                                    \
      launch_ev(k_fwd3<double, K>, dim3(1, batch), dim3(threads3(K)), uint32_t(tern_region<double, K>()), s, e0, \
                e1, static_cast<const Cx<double>*>(g), static_cast<const Cx<double>*>(tw),                      \
                static_cast<Cx<double>*>(c));                                                                    \
    else                                                                                                         \
      launch_ev(k_fwd3<float, K>, dim3(1, batch), dim3(threads3(K)), uint32_t(tern_region<float, K>()), s, e0,   \
                e1, static_cast<const Cx<float>*>(g), static_cast<const Cx<float>*>(tw),                        \
                static_cast<Cx<float>*>(c));                                                                     \
    break;
    AFD_TERN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_radius3(int k, bool fp64, const RadiusParams& p, int batch, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
  if (p.rpb != 1 || p.nrec != p.M || !p.tail || p.queue) return hipErrorInvalidValue;
  switch (k) {
#define X(K)                                                                                                    \
  case K:                                                                                                       \
    if (fp64)                                                                                                   \
      launch_ev(k_radius3<double, K, false>, dim3(p.M, batch), dim3(threads3(K)),                               \
                uint32_t(tern_lds<double, K>()), s, e0, e1, p);                                                 \
    else                                                                                                        \
      launch_ev(k_radius3<float, K, true>, dim3(p.M, batch), dim3(threads3(K)), uint32_t(tern_lds<float, K>()), \
                s, e0, e1, p);                                                                                  \
    break;
    AFD_TERN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Radix of the first pass of the length-3^k transforms (ns(1)): the step of
// the pruned start's r^((TPR/R0) i) table.
int tern_first_radix(int k) {
  switch (k) {
#define X(K) \
  case K:    \
    return Shape3<K, pickE3(K)>::NP >= 2 ? Shape3<K, pickE3(K)>::ns(1) : 1;
    AFD_TERN_CASES(X)
#undef X
    default:
      return 1;
  }
}

int tern_lds_bytes(int k, bool fp64) {
  switch (k) {
#define X(K) \
  case K:    \
    return int(fp64 ? tern_lds<double, K>() : tern_lds<float, K>());
    AFD_TERN_CASES(X)
#undef X
    default:
      return 0;
  }
}

}  // namespace afd
