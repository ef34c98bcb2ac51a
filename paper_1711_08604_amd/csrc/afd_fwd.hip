// Forward DFT of the remainder samples, c_l = sum_n G(z_n) e^{-2 pi i l n/N}
// (Sec. 3.1, eq. term4; the paper's radix-2 split is eq. term3).
//
// Up to 2^11 points one workgroup runs the whole Stockham transform.  From
// 2^12 points the transform is split as N = N1 N2 (n = l1 + N1 l2,
// l = k2 + N2 k1): workgroups of the first pass each take 8 columns l1, run
// the length-N2 DFTs over l2, apply e^{-2 pi i l1 k2/N} and store the
// intermediate as X[k2][l1]; workgroups of the second pass each take 8 rows
// k2 and run the length-N1 DFTs over l1, writing c[k2 + N2 k1] -- or, for
// the radius transforms beyond the LDS, the same values in column order
// (row k2 contiguous: the column l2 = k2 of those transforms).  Both passes
// spread the work over many CUs instead of serialising it on one.
#include "afd_device.h"
#include "afd_internal.h"

namespace afd {

constexpr int kFwdTwoPassMin = 12;
constexpr int kColsPerBlock = 8;

template <typename T, int LOGN>
__host__ __device__ constexpr int fwd_threads() {
  return Shape<LOGN, pickE<T, LOGN>()>::TPR;
}

template <typename T, int LOGN>
__global__ __launch_bounds__((fwd_threads<T, LOGN>())) void k_fft_fwd(const Cx<T>* __restrict__ g,
                                                                       const Cx<T>* __restrict__ tw,
                                                                       Cx<T>* __restrict__ c) {
  constexpr int E = pickE<T, LOGN>();
  using S = Shape<LOGN, E>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  g += size_t(S::N) * blockIdx.y;  // signal of a batch
  c += size_t(S::N) * blockIdx.y;
  Cx<T> v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = g[t + S::TPR * i];
  fft_regs<T, LOGN, E, -1, pickSplit<T, LOGN>()>(v, t, smem, tw);
#pragma unroll
  for (int p = 0; p < E; ++p) c[out_bin<LOGN, E>(t, p)] = v[p];
}

template <int LOGN>
struct Split2 {
  static constexpr int L1 = LOGN / 2;
  static constexpr int L2 = LOGN - L1;
  static constexpr int N1 = 1 << L1;
  static constexpr int N2 = 1 << L2;
};

template <typename T, int LOGN>
__host__ __device__ constexpr int cols_threads() {
  return kColsPerBlock * Shape<Split2<LOGN>::L2, pickE<T, Split2<LOGN>::L2>()>::TPR;
}
template <typename T, int LOGN>
__host__ __device__ constexpr int rows_threads() {
  return kColsPerBlock * Shape<Split2<LOGN>::L1, pickE<T, Split2<LOGN>::L1>()>::TPR;
}

// First pass: X[k2][l1] = e^{-2 pi i l1 k2/N} sum_l2 x[l1 + N1 l2] e^{-2 pi i l2 k2/N2}
template <typename T, int LOGN>
__global__ __launch_bounds__((cols_threads<T, LOGN>())) void k_fwd_cols(const Cx<T>* __restrict__ x,
                                                                         const Cx<T>* __restrict__ tw2,
                                                                         const double* __restrict__ omega,
                                                                         Cx<T>* __restrict__ xt) {
  using P = Split2<LOGN>;
  constexpr int E2 = pickE<T, P::L2>();
  using S2 = Shape<P::L2, E2>;
  constexpr int N = 1 << LOGN;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ci = threadIdx.x % kColsPerBlock, t = threadIdx.x / kColsPerBlock;
  const int l1 = blockIdx.x * kColsPerBlock + ci;
  x += size_t(N) * blockIdx.y;  // signal of a batch
  xt += size_t(N) * blockIdx.y;
  unsigned char* region = smem + size_t(ci) * fft_region_bytes<T, P::L2, false>();
  Cx<T> v[E2];
#pragma unroll
  for (int i = 0; i < E2; ++i) v[i] = x[l1 + P::N1 * (t + S2::TPR * i)];
  fft_regs<T, P::L2, E2, -1, false>(v, t, region, tw2);
#pragma unroll
  for (int p = 0; p < E2; ++p) {
    const int k2 = out_bin<P::L2, E2>(t, p);
    const int e = (l1 * k2) & (N - 1);
    const Cx<T> w{T(omega[2 * e]), T(-omega[2 * e + 1])};
    xt[size_t(k2) * P::N1 + l1] = cmul(v[p], w);
  }
}

// Second pass: c[k2 + N2 k1] = sum_l1 X[k2][l1] e^{-2 pi i l1 k1/N1}, stored at
// c[k2 + N2 k1] or, with COLS, at c[k2 N1 + k1].
template <typename T, int LOGN, bool COLS>
__global__ __launch_bounds__((rows_threads<T, LOGN>())) void k_fwd_rows(const Cx<T>* __restrict__ xt,
                                                                         const Cx<T>* __restrict__ tw1,
                                                                         Cx<T>* __restrict__ c,
                                                                         Cx<T>* __restrict__ c0) {
  using P = Split2<LOGN>;
  constexpr int E1 = pickE<T, P::L1>();
  using S1 = Shape<P::L1, E1>;
  extern __shared__ __align__(16) unsigned char smem[];
  // COLS: the threads of a row are adjacent (contiguous loads and stores);
  // otherwise the rows are interleaved (stores of kColsPerBlock adjacent bins)
  const int ri = COLS ? int(threadIdx.x) / S1::TPR : int(threadIdx.x) % kColsPerBlock;
  const int t = COLS ? int(threadIdx.x) % S1::TPR : int(threadIdx.x) / kColsPerBlock;
  const int k2 = blockIdx.x * kColsPerBlock + ri;
  xt += (size_t(1) << LOGN) * blockIdx.y;  // signal of a batch
  c += (size_t(1) << LOGN) * blockIdx.y;
  unsigned char* region = smem + size_t(ri) * fft_region_bytes<T, P::L1, false>();
  Cx<T> v[E1];
#pragma unroll
  for (int i = 0; i < E1; ++i) v[i] = xt[size_t(k2) * P::N1 + t + S1::TPR * i];
  fft_regs<T, P::L1, E1, -1, false>(v, t, region, tw1);
#pragma unroll
  for (int p = 0; p < E1; ++p) {
    const int k1 = out_bin<P::L1, E1>(t, p);
    if constexpr (COLS) {
      c[size_t(k2) * P::N1 + k1] = v[p];
      // with c0, the bins below N2 2^kBigMedShift2 also in natural order
      // (c_{k2 + N2 k1}: k1 < 2^kBigMedShift2)
      if (c0 != nullptr && k1 < (1 << kBigMedShift2))
        c0[(size_t(P::N2) << kBigMedShift2) * blockIdx.y + size_t(k1) * P::N2 + k2] = v[p];
    } else
      c[k2 + P::N2 * k1] = v[p];
  }
}

// ---------------------------------------------------------------- host side
template <typename T, int LOGN>
static FftGeom geom_of() {
  constexpr int E = pickE<T, LOGN>();
  using S = Shape<LOGN, E>;
  FftGeom g;
  g.E = E;
  g.tpr = S::TPR;
  g.twsize = S::twsize();
  g.split = pickSplit<T, LOGN>();
  g.lds_elems = S::LDS_ELEMS;
  return g;
}

template <typename T, int LOGN>
static void twiddles_of(double* out) {
  constexpr int E = pickE<T, LOGN>();
  using S = Shape<LOGN, E>;
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int p = 1; p < S::NP; ++p) {
    const int ns = S::ns(p), R = S::radix(p), off = S::twoff(p);
    const long long L = (long long)ns * R;
    for (int r = 1; r < R; ++r) {
      for (int k = 0; k < ns; ++k) {
        const long long e = ((long long)k * r) % L;  // reduce the angle exactly before rounding
        const long double ang = two_pi * (long double)e / (long double)L;
        const int i = off + (r - 1) * ns + k;
        out[2 * i] = (double)cosl(ang);
        out[2 * i + 1] = (double)sinl(ang);
      }
    }
  }
}

#define AFD_FWD_LOGN_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)
#define AFD_FWD2_LOGN_CASES(X) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)
#define AFD_FWD_ALL_LOGN_CASES(X) AFD_FWD_LOGN_CASES(X) X(15) X(16) X(17) X(18) X(19) X(20)

// the spectrum goes out in column order when the radius transforms run as
// two passes through HBM
template <int LOGN>
constexpr bool fwd_cols_out() {
  return LOGN > kMaxLdsLogN;
}

FftGeom fft_geom(int logn, bool fp64) {
  switch (logn) {
#define X(L) \
  case L:    \
    return fp64 ? geom_of<double, L>() : geom_of<float, L>();
    AFD_FWD_LOGN_CASES(X)
#undef X
    default:
      return FftGeom{0, 0, 0, false, 0};
  }
}

void fft_twiddles(int logn, bool fp64, double* out) {
  switch (logn) {
#define X(L)                      \
  case L:                         \
    if (fp64)                     \
      twiddles_of<double, L>(out); \
    else                          \
      twiddles_of<float, L>(out);  \
    break;
    AFD_FWD_LOGN_CASES(X)
#undef X
    default:
      break;
  }
}

FwdPlan fwd_plan(int logn, bool fp64) {
  FwdPlan f{};
  f.two_pass = logn >= kFwdTwoPassMin;
  if (f.two_pass) {
    f.l1 = logn / 2;
    f.l2 = logn - f.l1;
    f.tw1_size = fft_geom(f.l1, fp64).twsize;
    f.tw2_size = fft_geom(f.l2, fp64).twsize;
  } else {
    f.l1 = f.l2 = 0;
    f.tw1_size = fft_geom(logn, fp64).twsize;
    f.tw2_size = 0;
  }
  return f;
}

hipError_t setup_fwd_attributes() {
  hipError_t e = hipSuccess;
#define X(L)                                                                                              \
  if (e == hipSuccess)                                                                                    \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fft_fwd<double, L>));                             \
  if (e == hipSuccess)                                                                                    \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fft_fwd<float, L>));
  AFD_FWD_LOGN_CASES(X)
#undef X
#define X(L)                                                                                              \
  if (e == hipSuccess)                                                                                    \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_cols<double, L>));                             \
  if (e == hipSuccess)                                                                                    \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_cols<float, L>));                             \
  if (e == hipSuccess)                                                                                    \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_rows<double, L, fwd_cols_out<L>()>));         \
  if (e == hipSuccess)                                                                                    \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_fwd_rows<float, L, fwd_cols_out<L>()>));
  AFD_FWD2_LOGN_CASES(X)
#undef X
  return e;
}

template <typename T, int LOGN>
static hipError_t launch_fwd_t(const void* g, const void* tw1, const void* tw2, const double* omega, void* xt,
                               void* c, void* c0, int batch, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (LOGN < kFwdTwoPassMin) {
    constexpr int thr = fwd_threads<T, LOGN>();
    constexpr size_t lds = fft_region_bytes<T, LOGN, pickSplit<T, LOGN>()>();
    launch_ev(k_fft_fwd<T, LOGN>, dim3(1, batch), dim3(thr), uint32_t(lds), s, e0, e1, reinterpret_cast<const Cx<T>*>(g),
              reinterpret_cast<const Cx<T>*>(tw1), reinterpret_cast<Cx<T>*>(c));
  } else {
    using P = Split2<LOGN>;
    constexpr int thr_c = cols_threads<T, LOGN>();
    constexpr int thr_r = rows_threads<T, LOGN>();
    constexpr size_t lds_c = kColsPerBlock * fft_region_bytes<T, P::L2, false>();
    constexpr size_t lds_r = kColsPerBlock * fft_region_bytes<T, P::L1, false>();
    launch_ev(k_fwd_cols<T, LOGN>, dim3(P::N1 / kColsPerBlock, batch), dim3(thr_c), uint32_t(lds_c), s, e0, nullptr,
              reinterpret_cast<const Cx<T>*>(g), reinterpret_cast<const Cx<T>*>(tw2), omega,
              reinterpret_cast<Cx<T>*>(xt));
    launch_ev(k_fwd_rows<T, LOGN, fwd_cols_out<LOGN>()>, dim3(P::N2 / kColsPerBlock, batch), dim3(thr_r),
              uint32_t(lds_r), s,
              nullptr, e1, reinterpret_cast<const Cx<T>*>(xt), reinterpret_cast<const Cx<T>*>(tw1),
              reinterpret_cast<Cx<T>*>(c), reinterpret_cast<Cx<T>*>(c0));
  }
  return hipGetLastError();
}

hipError_t launch_fwd(int logn, bool fp64, const void* g, const void* tw1, const void* tw2, const double* omega,
                      void* xt, void* c, int batch, hipStream_t s, hipEvent_t e0, hipEvent_t e1, void* c0) {
  switch (logn) {
#define X(L)                                                                                  \
  case L:                                                                                     \
    return fp64 ? launch_fwd_t<double, L>(g, tw1, tw2, omega, xt, c, c0, batch, s, e0, e1)    \
                : launch_fwd_t<float, L>(g, tw1, tw2, omega, xt, c, c0, batch, s, e0, e1);
    AFD_FWD_ALL_LOGN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace afd
