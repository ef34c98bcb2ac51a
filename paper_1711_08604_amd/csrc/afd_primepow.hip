// The decomposition for N = P^K samples (P = 3, K = 1..8; P = 5, K = 1..6;
// P = 7, K = 1..4): forward DFT of the remainder and the fused per-radius
// kernel on the radix-P transforms of afd_primepow.h.  The paper's closing
// remark states that its fast algorithm holds for N = p^K; only the
// transforms depend on the factorisation of N.  The records, the merge, the
// double re-check and the update are the power-of-two path's own kernels,
// which take N as a parameter.
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
#include "afd_primepow.h"

namespace afd {

// The transforms exchange complex values through LDS.  Double precision
// beyond 32 KiB exchanges real and imaginary parts in turn, which keeps two
// or three of the 3^8-point workgroups on a CU (non-split: 1.5x slower) and
// lets 5^6 points fit at all; single precision (at most 125 KB) always
// exchanges whole complex values, half the barriers and LDS instructions of
// the split form (measured 1.16x at 3^8 and 1.24x at 5^6, where its
// registers already hold one workgroup per CU).
template <typename T, int P, int K>
__host__ __device__ constexpr bool pp_split() {
  return sizeof(T) == 8 && size_t(ipow(P, K)) * 2 * sizeof(T) > 32768;
}
template <typename T, int P, int K>
__host__ __device__ constexpr size_t pp_region() {
  return size_t(ipow(P, K)) * (pp_split<T, P, K>() ? 1 : 2) * sizeof(T);
}
template <typename T, int P, int K>
static size_t pp_lds() {
  const size_t need = pp_region<T, P, K>() + kListScratchBytes;
  return need > sizeof(MergeScratch) ? need : sizeof(MergeScratch);
}

// c_l = sum_n g_n e^{-2 pi i l n/N}, one workgroup per signal.
template <typename T, int P, int K>
__global__ __launch_bounds__(threadsp(P, K)) void k_fwd_pp(const Cx<T>* __restrict__ g, const Cx<T>* __restrict__ tw,
                                                           Cx<T>* __restrict__ c) {
  constexpr int E = pickEp(P, K);
  using S = ShapeP<P, K, E>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  const bool act = t < S::TPR;
  g += size_t(S::N) * blockIdx.y;
  c += size_t(S::N) * blockIdx.y;
  Cx<T> v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = act ? g[t + S::TPR * i] : Cx<T>{T(0), T(0)};
  fftp_regs<T, P, K, E, -1, pp_split<T, P, K>()>(v, t, act, smem, tw);
  if (act) {
#pragma unroll
    for (int p = 0; p < E; ++p) c[t + S::TPR * digrev(P, p, S::LE)] = v[p];
  }
}

// From 2048 points the forward DFT is split as N = N1 N2 (N1 = P^(K/2)):
// n = l1 + N1 l2, l = k2 + N2 k1.  The first pass transforms each column l1
// over l2 and applies e^{-2 pi i l1 k2/N}, storing X[k2][l1]; the second
// transforms each row k2 over l1 into c[k2 + N2 k1].  Both run several
// short transforms per 64-thread workgroup on many CUs, where one
// workgroup holding all N points would serialise the whole transform.
constexpr int kFwdSplitN = 2048;
template <int P, int K>
struct SplitP {
  static constexpr int K1 = K / 2, K2 = K - K1;
  static constexpr int N1 = ipow(P, K1), N2 = ipow(P, K2);
};
// transforms of P^KK points per 64-thread workgroup
template <int P, int KK>
__host__ __device__ constexpr int per_wave_pp() {
  return 64 / ShapeP<P, KK, pickEp(P, KK)>::TPR;
}

template <typename T, int P, int K>
__global__ __launch_bounds__(64) void k_fwd_pp_cols(const Cx<T>* __restrict__ g, const Cx<T>* __restrict__ tw2,
                                                    const double* __restrict__ omega, Cx<T>* __restrict__ xt) {
  using Sp = SplitP<P, K>;
  constexpr int E2 = pickEp(P, Sp::K2);
  using S2 = ShapeP<P, Sp::K2, E2>;
  constexpr int CPB = per_wave_pp<P, Sp::K2>();
  constexpr int N = ipow(P, K);
  extern __shared__ __align__(16) unsigned char smem[];
  // adjacent threads take adjacent columns (contiguous loads)
  const int ci = int(threadIdx.x) % CPB, t = int(threadIdx.x) / CPB;
  const int l1 = int(blockIdx.x) * CPB + ci;
  const bool act = t < S2::TPR && l1 < Sp::N1;
  g += size_t(N) * blockIdx.y;
  xt += size_t(N) * blockIdx.y;
  unsigned char* region = smem + size_t(ci) * Sp::N2 * sizeof(Cx<T>);
  Cx<T> v[E2];
#pragma unroll
  for (int i = 0; i < E2; ++i) v[i] = act ? g[l1 + Sp::N1 * (t + S2::TPR * i)] : Cx<T>{T(0), T(0)};
  fftp_regs<T, P, Sp::K2, E2, -1, false>(v, t, act, region, tw2);
  if (act) {
#pragma unroll
    for (int p = 0; p < E2; ++p) {
      const int k2 = t + S2::TPR * digrev(P, p, S2::LE);
      const int e = l1 * k2;  // < N
      const Cx<T> w{T(omega[2 * e]), T(-omega[2 * e + 1])};
      xt[size_t(k2) * Sp::N1 + l1] = cmul(v[p], w);
    }
  }
}

template <typename T, int P, int K>
__global__ __launch_bounds__(64) void k_fwd_pp_rows(const Cx<T>* __restrict__ xt, const Cx<T>* __restrict__ tw1,
                                                    Cx<T>* __restrict__ c) {
  using Sp = SplitP<P, K>;
  constexpr int E1 = pickEp(P, Sp::K1);
  using S1 = ShapeP<P, Sp::K1, E1>;
  constexpr int RPB = per_wave_pp<P, Sp::K1>();
  constexpr int N = ipow(P, K);
  extern __shared__ __align__(16) unsigned char smem[];
  // the threads of a row are adjacent (contiguous loads)
  const int ri = int(threadIdx.x) / S1::TPR, t = int(threadIdx.x) % S1::TPR;
  const int k2 = int(blockIdx.x) * RPB + ri;
  const bool act = ri < RPB && k2 < Sp::N2;
  xt += size_t(N) * blockIdx.y;
  c += size_t(N) * blockIdx.y;
  unsigned char* region = smem + size_t(ri < RPB ? ri : RPB - 1) * Sp::N1 * sizeof(Cx<T>);
  Cx<T> v[E1];
#pragma unroll
  for (int i = 0; i < E1; ++i) v[i] = act ? xt[size_t(k2) * Sp::N1 + t + S1::TPR * i] : Cx<T>{T(0), T(0)};
  fftp_regs<T, P, Sp::K1, E1, -1, false>(v, t, act, region, tw1);
  if (act) {
#pragma unroll
    for (int p = 0; p < E1; ++p) c[k2 + Sp::N2 * (t + S1::TPR * digrev(P, p, S1::LE))] = v[p];
  }
}

template <typename T, int P, int K, bool LIST>
__global__ __launch_bounds__(threadsp(P, K)) void k_radius_pp(RadiusParams prm) {
  constexpr int E = pickEp(P, K);
  using S = ShapeP<P, K, E>;
  constexpr int N = S::N, TPR = S::TPR;
  using Ord = DigrevOrder<P, S::LE>;
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
  // x[job], so with at most N/ns(s) terms the inputs of pass s are
  // x_s[i] = x[i / ns(s)]: register i of thread t holds x[a + D i] with
  // a = t / ns(s), D = TPR / ns(s) (TPR is a multiple of ns(s)).  From pass 1:
  // r^l = r^a (r^t table) times r^(D i) (the [M][E] table of r^((TPR/R0) i));
  // from pass 2 where ns(2) = TPR (three passes of radix 3^e, or the shapes
  // whose first two passes span TPR): register i holds x[i], with weight r^i
  // from the r^t table (E <= TPR there).
  constexpr int NP = S::NP;
  constexpr bool kSkip2 = NP >= 3 && S::ns(NP >= 3 ? 2 : 0) == TPR && E <= TPR;
  int skip = 0;
  if constexpr (NP >= 2) skip = L <= N / S::ns(1) ? 1 : 0;
  if constexpr (kSkip2) skip = L <= N / S::ns(2) ? 2 : skip;
  Cx<T> v[E];
  if (skip == 2) {
    if constexpr (kSkip2) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        v[i] = {T(0), T(0)};
        if (act && i < L) {
          const Cx<T> x = c[i];
          const T w = pw[i];
          v[i] = {x.x * w, x.y * w};
        }
      }
      fftp_regs<T, P, K, E, +1, pp_split<T, P, K>(), 2, 2>(v, t, act, smem, tw);
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
      fftp_regs<T, P, K, E, +1, pp_split<T, P, K>(), 1, 1>(v, t, act, smem, tw);
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
    fftp_regs<T, P, K, E, +1, pp_split<T, P, K>()>(v, t, act, smem, tw);
  }

  unsigned char* scratch = smem + pp_region<T, P, K>();
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
    select32_tail<2, 8>(reinterpret_cast<const BlockList32*>(prm.out) + size_t(prm.nrec) * b,
                  prm.heads + size_t(prm.nrec) * b, prm.seconds + size_t(prm.nrec) * b, prm.nrec, prm.recheck_k,
                  prm.tau_band, prm.flagword + b, prm.cand + b, Sm);
  } else {
    merge64_tail<2, 8>(reinterpret_cast<const BlockBest64*>(prm.out) + size_t(prm.nrec) * b, prm.nrec, N, prm.winner + b,
                 Sm);
  }
}

// (P, K) of every supported N = P^K; the forward DFT runs in one workgroup
// below kFwdSplitN points (ONE) and split in two passes from there (TWO).
#define AFD_PP_ONE(X) X(3, 1) X(3, 2) X(3, 3) X(3, 4) X(3, 5) X(3, 6) X(5, 1) X(5, 2) X(5, 3) X(5, 4) \
  X(7, 1) X(7, 2) X(7, 3)
#define AFD_PP_TWO(X) X(3, 7) X(3, 8) X(5, 5) X(5, 6) X(7, 4)
#define AFD_PP_CASES(X) AFD_PP_ONE(X) AFD_PP_TWO(X)
#define AFD_PP_KEY(P, K) ((P) * 16 + (K))

static_assert(ipow(3, 6) < kFwdSplitN && ipow(3, 7) >= kFwdSplitN && ipow(5, 4) < kFwdSplitN &&
                  ipow(5, 5) >= kFwdSplitN && ipow(7, 3) < kFwdSplitN && ipow(7, 4) >= kFwdSplitN,
              "the case lists follow the split size");

bool pp_supported(int prime, int k) {
  switch (AFD_PP_KEY(prime, k)) {
#define X(P, K) case AFD_PP_KEY(P, K):
    AFD_PP_CASES(X)
#undef X
    return true;
    default:
      return false;
  }
}

PpGeom pp_geom(int prime, int k) {
  PpGeom g{};
  switch (AFD_PP_KEY(prime, k)) {
#define X(P, K)                                     \
  case AFD_PP_KEY(P, K):                            \
    g.prime = P;                                    \
    g.k = K;                                        \
    g.E = pickEp(P, K);                             \
    g.tpr = ipow(P, K) / pickEp(P, K);              \
    g.threads = threadsp(P, K);                     \
    g.twsize = ShapeP<P, K, pickEp(P, K)>::twsize(); \
    break;
    AFD_PP_CASES(X)
#undef X
    default:
      break;
  }
  return g;
}

// Stockham twiddles of the length-prime^k transforms: pass s >= 1 (radix R,
// ns = the product of the earlier radices) holds e^{+2 pi i j r/(ns R)} at
// (r - 1) ns + j, after the entries of the earlier passes.
void pp_twiddles(int prime, int k, double* tw) {
  const int E = pickEp(prime, k), LE = ilogc(prime, E), q0 = k % LE, np = k / LE + (q0 ? 1 : 0);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  size_t off = 0;
  int ns = 1;
  for (int s = 0; s < np; ++s) {
    const int R = (s == 0 && q0) ? ipow(prime, q0) : E;
    if (s > 0) {
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

hipError_t setup_pp_attributes() {
  hipError_t e = hipSuccess;
#define X(P, K)                                                                                                  \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius_pp<double, P, K, false>)); \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius_pp<float, P, K, true>));
  AFD_PP_CASES(X)
#undef X
#define X(P, K)                                                                                      \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_pp<double, P, K>)); \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_pp<float, P, K>));
  AFD_PP_ONE(X)
#undef X
  return e;
}

// Forward DFT tables: the split's row (prime^(k/2)) and column
// (prime^(k - k/2)) twiddle entries, 0 below the split.
int pp_fwd_twsize(int prime, int k, bool rows) {
  if (!pp_supported(prime, k) || ipow(prime, k) < kFwdSplitN) return 0;
  return pp_geom(prime, rows ? k / 2 : k - k / 2).twsize;
}

hipError_t launch_fwd_pp(int prime, int k, bool fp64, const void* g, const void* tw, const void* tw1,
                         const void* tw2, const double* omega, void* xt, void* c, int batch, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1) {
  switch (AFD_PP_KEY(prime, k)) {
#define X(P, K)                                                                                                   \
  case AFD_PP_KEY(P, K): {                                                                                        \
    using Sp = SplitP<P, K>;                                                                                      \
    constexpr int CPB = per_wave_pp<P, Sp::K2>(), RPB = per_wave_pp<P, Sp::K1>();                                 \
    const dim3 gc((Sp::N1 + CPB - 1) / CPB, batch), gr((Sp::N2 + RPB - 1) / RPB, batch);                          \
    if (fp64) {                                                                                                   \
      launch_ev(k_fwd_pp_cols<double, P, K>, gc, dim3(64), uint32_t(CPB * Sp::N2 * 16), s, e0, nullptr,           \
                static_cast<const Cx<double>*>(g), static_cast<const Cx<double>*>(tw2), omega,                   \
                static_cast<Cx<double>*>(xt));                                                                   \
      launch_ev(k_fwd_pp_rows<double, P, K>, gr, dim3(64), uint32_t(RPB * Sp::N1 * 16), s, nullptr, e1,           \
                static_cast<const Cx<double>*>(xt), static_cast<const Cx<double>*>(tw1),                         \
                static_cast<Cx<double>*>(c));                                                                    \
    } else {                                                                                                      \
      launch_ev(k_fwd_pp_cols<float, P, K>, gc, dim3(64), uint32_t(CPB * Sp::N2 * 8), s, e0, nullptr,             \
                static_cast<const Cx<float>*>(g), static_cast<const Cx<float>*>(tw2), omega,                     \
                static_cast<Cx<float>*>(xt));                                                                    \
      launch_ev(k_fwd_pp_rows<float, P, K>, gr, dim3(64), uint32_t(RPB * Sp::N1 * 8), s, nullptr, e1,             \
                static_cast<const Cx<float>*>(xt), static_cast<const Cx<float>*>(tw1), static_cast<Cx<float>*>(c)); \
    }                                                                                                             \
    break;                                                                                                        \
  }
    AFD_PP_TWO(X)
#undef X
#define X(P, K)                                                                                                  \
  case AFD_PP_KEY(P, K):                                                                                         \
    if (fp64)                                                                                                    \
      launch_ev(k_fwd_pp<double, P, K>, dim3(1, batch), dim3(threadsp(P, K)), uint32_t(pp_region<double, P, K>()), \
                s, e0, e1, static_cast<const Cx<double>*>(g), static_cast<const Cx<double>*>(tw),                 \
                static_cast<Cx<double>*>(c));                                                                    \
    else                                                                                                         \
      launch_ev(k_fwd_pp<float, P, K>, dim3(1, batch), dim3(threadsp(P, K)), uint32_t(pp_region<float, P, K>()),   \
                s, e0, e1, static_cast<const Cx<float>*>(g), static_cast<const Cx<float>*>(tw),                   \
                static_cast<Cx<float>*>(c));                                                                     \
    break;
    AFD_PP_ONE(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_radius_pp(int prime, int k, bool fp64, const RadiusParams& p, int batch, hipStream_t s,
                            hipEvent_t e0, hipEvent_t e1) {
  if (p.rpb != 1 || p.nrec != p.M || !p.tail || p.queue) return hipErrorInvalidValue;
  switch (AFD_PP_KEY(prime, k)) {
#define X(P, K)                                                                                         \
  case AFD_PP_KEY(P, K):                                                                                \
    if (fp64)                                                                                           \
      launch_ev(k_radius_pp<double, P, K, false>, dim3(p.M, batch), dim3(threadsp(P, K)),               \
                uint32_t(pp_lds<double, P, K>()), s, e0, e1, p);                                        \
    else                                                                                                \
      launch_ev(k_radius_pp<float, P, K, true>, dim3(p.M, batch), dim3(threadsp(P, K)),                 \
                uint32_t(pp_lds<float, P, K>()), s, e0, e1, p);                                         \
    break;
    AFD_PP_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Radix of the first pass of the length-prime^k transforms (ns(1)): the
// step of the pruned start's r^((TPR/R0) i) table.
int pp_first_radix(int prime, int k) {
  switch (AFD_PP_KEY(prime, k)) {
#define X(P, K)          \
  case AFD_PP_KEY(P, K): \
    return ShapeP<P, K, pickEp(P, K)>::NP >= 2 ? ShapeP<P, K, pickEp(P, K)>::ns(1) : 1;
    AFD_PP_CASES(X)
#undef X
    default:
      return 1;
  }
}

int pp_lds_bytes(int prime, int k, bool fp64) {
  switch (AFD_PP_KEY(prime, k)) {
#define X(P, K)          \
  case AFD_PP_KEY(P, K): \
    return int(fp64 ? pp_lds<double, P, K>() : pp_lds<float, P, K>());
    AFD_PP_CASES(X)
#undef X
    default:
      return 0;
  }
}

}  // namespace afd
