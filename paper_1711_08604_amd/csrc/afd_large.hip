// Per-radius inverse DFTs beyond the LDS, N = 2^15 .. 2^20 (Sec. 3.1, eq. rcl;
// Sec. 3.2, Steps 1-2).
//
// A radius' transform y_m[j] = sum_l r_m^l c_l e^{2 pi i j l/N} no longer fits
// one workgroup, so it is split as N = N1 N2 with l = N2 l1 + l2 and
// j = j1 + N1 j2:
//
//   y_m[j1 + N1 j2] = sum_l2 e^{2 pi i j2 l2/N2} Z_m[j1][l2],
//   Z_m[j1][l2]     = r_m^l2 e^{2 pi i j1 l2/N} sum_l1 r_m^(N2 l1) c_{N2 l1 + l2} e^{2 pi i j1 l1/N1}.
//
// The column pass (k_big_cols) runs the length-N1 transforms of CA columns
// l2 per workgroup, reading the spectrum in column order (the forward DFT
// writes it that way), applies r_m^l2 e^{2 pi i j1 l2/N}, transposes through
// LDS and stores Z_m with the columns contiguous.  The row pass (k_big_rows)
// runs the length-N2 transforms of RB x RPT rows j1 per workgroup, scales by
// s_m, forms |.|^2 and selects as the LDS-resident kernel does (flat index
// m N + j1 + N1 j2), one record per workgroup.  Radii are processed in
// chunks so the intermediate stays within a fixed budget.  After the last
// chunk of a step, k_big_merge merges each radius' workgroup records into a
// per-radius record and those into the winner (FP64) or the short-list
// (FP32): a launch of its own, because a last-workgroup merge inside the row
// pass held every row workgroup through a store-and-count round trip at its
// end (measured: 26% of the row pass at N = 2^20 in double precision).
//
// Short spectra need no intermediate.  A radius whose significant length L
// (the terms r_m^l c_l beyond it are dropped, as in the LDS-resident kernel)
// is at most N2 has only l1 = 0 in every column, whose transform is then the
// constant c_{l2}, so Z_m[j1][l2] = r_m^l2 e^{2 pi i j1 l2/N} c_{l2} for
// l2 < L and 0 beyond.  The column pass skips such a radius and the row pass
// forms its rows from the spectrum itself, starting at a later Stockham pass
// when L is short enough (see deep_row_inputs); at N = 2^20 that is every
// radius below about 0.97.
#include "afd_select.h"

namespace afd {

// DL > 0: the split N1 = 2^(LOGN/2 - DL), N2 = 2^(LOGN - LOGN/2 + DL) of the
// row-only pass for radii of medium spectrum length (see k_big_rows).
template <typename T, int LOGN, int DL = 0>
struct Big {
  static constexpr int L1 = LOGN / 2 - DL, L2 = LOGN - L1;
  static constexpr int N = 1 << LOGN, N1 = 1 << L1, N2 = 1 << L2;
  static constexpr int E1 = pickE<T, L1>(), E2 = pickE<T, L2>();
  static constexpr int TPR1 = N1 / E1, TPR2 = N2 / E2;
  // columns per workgroup: 64-byte runs of the intermediate, >= 256 threads
  static constexpr int CA0 = sizeof(T) == 4 ? 8 : 4;
  static constexpr int CA = 256 / TPR1 > CA0 ? 256 / TPR1 : CA0;
  static constexpr int THR_A = CA * TPR1;
  // Row pass: RB row transforms side by side per workgroup of 256 threads
  // (a longer row takes a workgroup of its own), each over RPT rows one
  // after another.  Measured on the whole N = 2^20 decomposition: in single
  // precision 512-thread workgroups were 7% slower in the base split (0.5%
  // in the split shifted by 4) and 1024 threads 31%, because a workgroup's
  // band list grows with its rows; in double precision 128 threads were
  // 0.4% slower and 512 threads 3%.  Double precision, where a row transform
  // is one wave, takes 16, 8 or 4 rows in turn, the most that leave a radius
  // at least 16 workgroups, so that each workgroup's fixed latencies (its
  // first loads, the record of its best point) are paid once per 64 rows at
  // N = 2^20 (16 rows per workgroup: 3% slower; 32 rows: 0.8% slower).
  static constexpr int THR_B0 = 256;
  static constexpr int RB = THR_B0 / TPR2 > 1 ? THR_B0 / TPR2 : 1;
  static constexpr int THR_B = RB * TPR2;
  static constexpr int RPT = (sizeof(T) != 8 || TPR2 != 64) ? 1
                             : N1 / (RB * 16) >= 16        ? 16
                             : N1 / (RB * 8) >= 16         ? 8
                             : N1 / (RB * 4) >= 16         ? 4
                                                           : 1;
  // waves per SIMD the row pass's register budget allows (single precision,
  // and double precision over several rows: at most 128 VGPRs)
  // (the 16 N2-point rows of the largest shift hold one 512-thread workgroup
  // per CU: two waves per SIMD)
  static constexpr int WPE_B = (sizeof(T) == 4 || RPT > 1) ? (DL >= 4 ? 2 : 4) : 1;
  static constexpr int G = N1 / (RB * RPT);  // row workgroups (records) per radius
  static constexpr int SW = (LOGN + 1) / 2;
  static constexpr int LDT = CA + 1;  // row pitch of the LDS transpose (reals)
  static_assert(N2 % CA == 0 && N1 % (RB * RPT) == 0, "tiles must divide the transform");
  static_assert(G <= 256, "the radius merge holds one workgroup record per thread");
  static_assert(sizeof(T) == 8 || RPT == 1, "a single-precision row workgroup lists the band of its own rows");
  // LDS per workgroup, sized for occupancy: the column transforms and the
  // transpose move real and imaginary parts in turn through half the space;
  // the row transforms do so in double precision, and the row selection's
  // scratch reuses the transform regions once every row is done with them.
  static constexpr size_t region_a = fft_region_bytes<T, L1, true>();
  static constexpr size_t region_b = fft_region_bytes<T, L2, sizeof(T) == 8>();
  static constexpr size_t lds_a = (size_t(CA) * region_a > size_t(N1) * LDT * sizeof(T))
                                      ? size_t(CA) * region_a
                                      : size_t(N1) * LDT * sizeof(T);
  static constexpr size_t sel_b = sizeof(T) == 4 ? kListScratchBytes : 16 * sizeof(Best);
  static constexpr size_t lds_b = size_t(RB) * region_b > sel_b ? size_t(RB) * region_b : sel_b;
};

template <typename T, int LOGN>
__global__ __launch_bounds__((Big<T, LOGN>::THR_A)) void k_big_cols(BigParams p) {
  using B = Big<T, LOGN>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ci = threadIdx.x / B::TPR1, t = threadIdx.x - ci * B::TPR1;
  const int l2 = blockIdx.x * B::CA + ci;
  const int ml = blockIdx.y, m = p.border[p.m0 + ml];
  if (p.lsig[m] <= B::N2) return;  // formed by the row pass (uniform)

  // weighted column x[l1] = r^(N2 l1) c_{N2 l1 + l2} (the factor r^l2 is applied after the transform)
  const Cx<T>* __restrict__ col = reinterpret_cast<const Cx<T>*>(p.c) + size_t(l2) * B::N1;
  const T* __restrict__ pa = reinterpret_cast<const T*>(p.pa) + size_t(m) * B::N1;
  Cx<T> v[B::E1];
#pragma unroll
  for (int i = 0; i < B::E1; ++i) {
    const int l1 = t + B::TPR1 * i;
    const Cx<T> x = col[l1];
    const T w = pa[l1];
    v[i] = {x.x * w, x.y * w};
  }
  fft_regs<T, B::L1, B::E1, +1, true, 0, 0, true>(v, t, smem + size_t(ci) * B::region_a,
                                                  reinterpret_cast<const Cx<T>*>(p.tw1));
  __syncthreads();  // the transpose below overlays every column's region

  // transpose through LDS, real parts then imaginary parts
  T* tr = reinterpret_cast<T*>(smem);
  const int cj = threadIdx.x % B::CA, jr = threadIdx.x / B::CA;
  constexpr int JS = B::THR_A / B::CA;
  constexpr int NJ = B::N1 / JS;
#pragma unroll
  for (int q = 0; q < B::E1; ++q) tr[out_bin<B::L1, B::E1>(t, q) * B::LDT + ci] = v[q].x;
  __syncthreads();
  T xr[NJ];
#pragma unroll
  for (int k = 0; k < NJ; ++k) xr[k] = tr[(jr + JS * k) * B::LDT + cj];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < B::E1; ++q) tr[out_bin<B::L1, B::E1>(t, q) * B::LDT + ci] = v[q].y;
  __syncthreads();

  const int l2o = blockIdx.x * B::CA + cj;
  const T rl = reinterpret_cast<const T*>(p.pb)[size_t(m) * B::N2 + l2o];
  const Cx<T>* __restrict__ wl = reinterpret_cast<const Cx<T>*>(p.wl);
  const Cx<T>* __restrict__ wh = reinterpret_cast<const Cx<T>*>(p.wh);
  Cx<T>* __restrict__ z = reinterpret_cast<Cx<T>*>(p.z) + size_t(ml) * B::N + l2o;
#pragma unroll
  for (int k = 0; k < NJ; ++k) {
    const int j1 = jr + JS * k;
    const uint32_t e = (uint32_t(j1) * uint32_t(l2o)) & uint32_t(B::N - 1);
    Cx<T> w = cmul(wh[e >> B::SW], wl[e & ((1u << B::SW) - 1u)]);
    w = {w.x * rl, w.y * rl};
    z[size_t(j1) * B::N2] = cmul(Cx<T>{xr[k], tr[j1 * B::LDT + cj]}, w);
  }
}

// e^{2 pi i e/N} = wh[e >> SW] wl[e mod 2^SW] (e mod N)
template <typename T, int LOGN>
__device__ __forceinline__ Cx<T> big_twiddle(const BigParams& p, uint32_t e) {
  using B = Big<T, LOGN>;
  e &= uint32_t(B::N - 1);
  return cmul(reinterpret_cast<const Cx<T>*>(p.wh)[e >> B::SW],
              reinterpret_cast<const Cx<T>*>(p.wl)[e & ((1u << B::SW) - 1u)]);
}

// Inputs of Stockham pass P of the row transform for the row j1 of a short
// radius: job u of thread t takes Z[j1][l2] with l2 = (t + TPR2 u) / ns(P) +
// r N2 / (R_P ns(P)) (passes 0..P-1 of a spectrum with at most N2 / ns(P)
// terms only copy their inputs; P = 0 is the plain load order), Z[j1][l2] =
// c_{l2} e^{2 pi i j1 l2/N} r^l2.  With ns(P) dividing TPR2, l2 = t / ns(P) +
// o(u, r), so the twiddle is the thread's e^{2 pi i j1 (t / ns(P))/N} times a
// wave-uniform e^{2 pi i j1 o/N}, and the spectrum comes from its
// natural-order copy: every load is contiguous or uniform across the wave.
template <typename T, int LOGN, int P, int E, int DL = 0>
__device__ __forceinline__ void deep_row_inputs(Cx<T> (&v)[E], int t, int j1, int L, const BigParams& p, int m) {
  using B = Big<T, LOGN, DL>;
  using B0 = Big<T, LOGN>;
  using S = Shape<B::L2, B::E2>;
  static_assert(E == B::E2, "row transform values per thread");
  constexpr int R = S::radix(P), NS = S::ns(P), J = B::E2 / R, D = B::N2 / (R * NS);
  static_assert(S::TPR % NS == 0, "the lane part of l2 separates");
  const Cx<T>* __restrict__ c0 = reinterpret_cast<const Cx<T>*>(p.c0);
  // r^l2 from the tables of the base split: r^(l2 mod N2) r^(N2 (l2 / N2))
  const T* __restrict__ pb = reinterpret_cast<const T*>(p.pb) + size_t(m) * B0::N2;
  const T* __restrict__ pa = reinterpret_cast<const T*>(p.pa) + size_t(m) * B0::N1;
  const int base = t / NS;
  const Cx<T> wa = big_twiddle<T, LOGN>(p, uint32_t(j1) * uint32_t(base));
#pragma unroll
  for (int u = 0; u < J; ++u) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int o = (S::TPR / NS) * u + D * r;
      const int l2 = base + o;
      v[u + r * J] = {T(0), T(0)};
      if (l2 < L) {
        Cx<T> w = cmul(wa, big_twiddle<T, LOGN>(p, uint32_t(j1) * uint32_t(o)));
        T rl;
        if constexpr (DL == 0)
          rl = pb[l2];
        else
          rl = pb[l2 & (B0::N2 - 1)] * pa[l2 >> B0::L2];
        w = {w.x * rl, w.y * rl};
        v[u + r * J] = cmul(c0[l2], w);
      }
    }
  }
}

// DL > 0: the row-only pass of the radii of medium spectrum length
// (L <= N2 2^DL of the base split): with the split shifted by DL their
// spectrum fits the longer rows, which are formed from the spectrum itself
// as the short radii's are, and no column pass or intermediate is needed.
template <typename T, int LOGN, bool LIST, int DL = 0>
__global__ __launch_bounds__((Big<T, LOGN, DL>::THR_B))
__attribute__((amdgpu_waves_per_eu(Big<T, LOGN, DL>::WPE_B))) void k_big_rows(BigParams p) {
  using B = Big<T, LOGN, DL>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ri = threadIdx.x / B::TPR2, t0 = threadIdx.x - ri * B::TPR2;
  const int ml = blockIdx.y, m = p.border[p.m0 + ml];

  using S2 = Shape<B::L2, B::E2>;
  constexpr bool SPLIT = sizeof(T) == 8;
  unsigned char* region = smem + size_t(ri) * B::region_b;
  const Cx<T>* tw2 = reinterpret_cast<const Cx<T>*>(DL == 0 ? p.tw2 : p.tw2m[DL == kBigMedShift ? 0 : 1]);
  const int L = p.lsig[m];
  const T sc = reinterpret_cast<const T*>(p.scale)[m];  // loaded before the transform's barriers
  const int rec = m * p.gstride + int(blockIdx.x);
  Best run{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};  // double precision: this thread's best over its rows
#pragma unroll 1
  for (int k = 0; k < B::RPT; ++k) {
    // the thread index goes through an opaque zero in every row, so that the
    // transform's per-thread twiddle loads are not hoisted out of the row
    // loop and kept live across it (which would exceed the register budget)
    int zero = 0;
    if constexpr (B::RPT > 1) asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
    const int t = t0 + zero;
    int j1 = (int(blockIdx.x) * B::RB + ri) * B::RPT + k;
    // a row of at least 64 threads spans whole waves: j1 is wave-uniform, so
    // the row's uniform twiddles come through scalar loads
    if constexpr (B::TPR2 % 64 == 0) j1 = __builtin_amdgcn_readfirstlane(j1);
    Cx<T> v[B::E2];
    if constexpr (DL == 0) {
      if (L > B::N2) {
        const Cx<T>* __restrict__ row = reinterpret_cast<const Cx<T>*>(p.z) + size_t(ml) * B::N + size_t(j1) * B::N2;
#pragma unroll
        for (int i = 0; i < B::E2; ++i) v[i] = row[t + B::TPR2 * i];
        fft_regs<T, B::L2, B::E2, +1, SPLIT, 0, 0, true>(v, t, region, tw2);
      } else if (S2::NP >= 3 && L <= B::N2 / S2::ns(2)) {  // uniform: one radius per workgroup
        if constexpr (S2::NP >= 3) {
          deep_row_inputs<T, LOGN, 2>(v, t, j1, L, p, m);
          fft_regs<T, B::L2, B::E2, +1, SPLIT, 2, 2, true>(v, t, region, tw2);
        }
      } else if (S2::NP >= 2 && L <= B::N2 / S2::radix(0)) {
        if constexpr (S2::NP >= 2) {
          deep_row_inputs<T, LOGN, 1>(v, t, j1, L, p, m);
          fft_regs<T, B::L2, B::E2, +1, SPLIT, 1, 1, true>(v, t, region, tw2);
        }
      } else {
        deep_row_inputs<T, LOGN, 0>(v, t, j1, L, p, m);
        fft_regs<T, B::L2, B::E2, +1, SPLIT, 0, 0, true>(v, t, region, tw2);
      }
    } else {
      // L <= N2 (the launch holds medium radii only); rows longer than a
      // wave synchronise the workgroup
      constexpr bool WAVE = 64 % B::TPR2 == 0;
      const TwLate<T> twl{tw2};
      if (S2::NP >= 2 && L <= B::N2 / S2::radix(0)) {
        if constexpr (S2::NP >= 2) {
          deep_row_inputs<T, LOGN, 1, B::E2, DL>(v, t, j1, L, p, m);
          fft_regs<T, B::L2, B::E2, +1, SPLIT, 1, 1, WAVE>(v, t, region, twl);
        }
      } else {
        deep_row_inputs<T, LOGN, 0, B::E2, DL>(v, t, j1, L, p, m);
        fft_regs<T, B::L2, B::E2, +1, SPLIT, 0, 0, WAVE>(v, t, region, twl);
      }
    }

    // register q of thread t holds j2 = t + TPR2 bitrev(q): flat index m N + j1 + N1 j2
    const uint32_t fbase = uint32_t(m) * uint32_t(B::N) + uint32_t(j1);
    if constexpr (LIST) {
      __syncthreads();  // every row is done with its region: the selection reuses them
      const FlatOrder ord{uint32_t(m) * uint32_t(B::N) + uint32_t(blockIdx.x) * uint32_t(B::RB), uint32_t(B::RB),
                          uint32_t(B::N1), uint32_t(B::RB) * uint32_t(B::N2)};
      select_list<B::L2>(v, true, sc, fbase, uint32_t(B::N1), t, smem, p.tau_band, ord,
                         reinterpret_cast<BlockList32*>(p.blocks) + rec, nullptr, nullptr, p.flagword);
    } else {
      if (p.probe) {
        // a replayed step: the grid value at the forced point j = j1 + N1 j2,
        // scaled as the selection scales its best value
        const int pm = p.probe[0], pj = p.probe[1];
        const int pj2 = pj >> B::L1;
        if (m == pm && j1 == (pj & (B::N1 - 1)) && t == (pj2 & (B::TPR2 - 1))) {
          const int u = pj2 / B::TPR2;
#pragma unroll
          for (int q = 0; q < B::E2; ++q) {
            if (bitrev(q, ilog2c(B::E2)) == u) {
              p.probe_out[0] = double(v[q].x * sc);
              p.probe_out[1] = double(v[q].y * sc);
            }
          }
        }
      }
      best_merge(run, thread_best<B::L2, T>(v, sc, fbase, uint32_t(B::N1), t));
    }
  }
  if constexpr (!LIST) {
    __syncthreads();  // every row is done with its region: the reduction's scratch reuses them
    store_block_best(run, reinterpret_cast<Best*>(smem), reinterpret_cast<BlockBest64*>(p.blocks) + rec);
  }
}

// After the row passes of every chunk of a step: workgroup m merges radius
// m's G workgroup records into its per-radius record (and, in single
// precision, its head key), and the last workgroup to finish merges the M
// per-radius records into the winner (FP64) or the short-list (FP32).
template <typename T, int LOGN, bool LIST>
__global__ __launch_bounds__(256) void k_big_merge(BigParams p) {
  using B = Big<T, LOGN>;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  MergeScratch* Sm = reinterpret_cast<MergeScratch*>(smem);
  const int m = blockIdx.x;
  // a radius of medium spectrum length ran in the shifted split's row pass
  const int L = p.lsig[m];
  const int g = !p.med || L <= B::N2               ? B::G
                : L <= (B::N2 << kBigMedShift)  ? Big<T, LOGN, kBigMedShift>::G
                : L <= (B::N2 << kBigMedShift2) ? Big<T, LOGN, kBigMedShift2>::G
                                                : B::G;
  if constexpr (LIST) {
    merge_list_group(reinterpret_cast<const BlockList32*>(p.blocks) + size_t(m) * p.gstride, g, p.tau_band,
                     reinterpret_cast<BlockList32*>(p.rrec) + m, p.heads + m, Sm);
  } else {
    merge_best_group(reinterpret_cast<const BlockBest64*>(p.blocks) + size_t(m) * p.gstride, g,
                     reinterpret_cast<BlockBest64*>(p.rrec) + m, Sm);
  }
  if (!last_arrival(p.counter_g, gridDim.x, &s_last)) return;
  if constexpr (LIST) {
    select32_tail<2, 8>(reinterpret_cast<const BlockList32*>(p.rrec), p.heads, nullptr, p.M, p.recheck_k, p.tau_band,
                  p.flagword, p.cand, Sm);
  } else {
    merge64_tail<2, 8>(reinterpret_cast<const BlockBest64*>(p.rrec), p.M, B::N, p.winner, Sm);
  }
}

// ---------------------------------------------------------------- host side
#define AFD_BIG_LOGN_CASES(X) X(15) X(16) X(17) X(18) X(19) X(20)

template <typename T, int LOGN>
static BigGeom big_geom_of() {
  using B = Big<T, LOGN>;
  BigGeom g;
  g.l1 = B::L1;
  g.l2 = B::L2;
  g.sw = B::SW;
  g.ca = B::CA;
  g.thr_a = B::THR_A;
  g.rb = B::RB;
  g.thr_b = B::THR_B;
  g.g = B::G;
  using BM = Big<T, LOGN, kBigMedShift>;
  using BM2 = Big<T, LOGN, kBigMedShift2>;
  g.g_med[0] = BM::G;
  g.thr_b_med[0] = BM::THR_B;
  g.lds_b_med[0] = BM::lds_b;
  g.g_med[1] = BM2::G;
  g.thr_b_med[1] = BM2::THR_B;
  g.lds_b_med[1] = BM2::lds_b;
  g.gstride = B::G;
  if (BM::G > g.gstride) g.gstride = BM::G;
  if (BM2::G > g.gstride) g.gstride = BM2::G;
  g.lds_a = B::lds_a;
  g.lds_b = B::lds_b;
  g.rec_bytes = sizeof(T) == 4 ? sizeof(BlockList32) : sizeof(BlockBest64);
  return g;
}

BigGeom big_geom(int logn, bool fp64) {
  switch (logn) {
#define X(L) \
  case L:    \
    return fp64 ? big_geom_of<double, L>() : big_geom_of<float, L>();
    AFD_BIG_LOGN_CASES(X)
#undef X
    default:
      return BigGeom{};
  }
}

hipError_t setup_big_attributes() {
  hipError_t e = hipSuccess;
#define X(L)                                                                                        \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_cols<float, L>));        \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_cols<double, L>));       \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_rows<float, L, true>));  \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_rows<double, L, false>));      \
  if (e == hipSuccess)                                                                                      \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_rows<float, L, true, kBigMedShift>));       \
  if (e == hipSuccess)                                                                                      \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_rows<double, L, false, kBigMedShift>));     \
  if (e == hipSuccess)                                                                                      \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_rows<float, L, true, kBigMedShift2>));      \
  if (e == hipSuccess)                                                                                      \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_rows<double, L, false, kBigMedShift2>));    \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_merge<float, L, true>));      \
  if (e == hipSuccess) e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_big_merge<double, L, false>));
  AFD_BIG_LOGN_CASES(X)
#undef X
  return e;
}

template <typename T, int LOGN>
static hipError_t launch_big_t(const BigParams& p, int nr, bool cols, int med, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1, hipEvent_t r0, hipEvent_t r1) {
  using B = Big<T, LOGN>;
  if (nr < 1 || p.m0 < 0 || p.m0 + nr > p.M || (cols && med) || med < 0 || med > 2) return hipErrorInvalidValue;
  if (med == 1) {
    using BM = Big<T, LOGN, kBigMedShift>;
    launch_ev(k_big_rows<T, LOGN, sizeof(T) == 4, kBigMedShift>, dim3(BM::G, nr), dim3(BM::THR_B),
              uint32_t(BM::lds_b), s, r0 ? r0 : e0, r1 ? r1 : e1, p);
    return hipGetLastError();
  }
  if (med == 2) {
    using BM = Big<T, LOGN, kBigMedShift2>;
    launch_ev(k_big_rows<T, LOGN, sizeof(T) == 4, kBigMedShift2>, dim3(BM::G, nr), dim3(BM::THR_B),
              uint32_t(BM::lds_b), s, r0 ? r0 : e0, r1 ? r1 : e1, p);
    return hipGetLastError();
  }
  if (cols) {
    launch_ev(k_big_cols<T, LOGN>, dim3(B::N2 / B::CA, nr), dim3(B::THR_A), uint32_t(B::lds_a), s, e0, nullptr, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e0 = nullptr;
  }
  launch_ev(k_big_rows<T, LOGN, sizeof(T) == 4>, dim3(B::G, nr), dim3(B::THR_B), uint32_t(B::lds_b), s,
            r0 ? r0 : e0, r1 ? r1 : e1, p);
  return hipGetLastError();
}

template <typename T, int LOGN>
static hipError_t launch_big_merge_t(const BigParams& p, hipStream_t s, hipEvent_t e1) {
  launch_ev(k_big_merge<T, LOGN, sizeof(T) == 4>, dim3(p.M), dim3(256), uint32_t(sizeof(MergeScratch)), s, nullptr, e1,
            p);
  return hipGetLastError();
}

hipError_t launch_big_merge(int logn, bool fp64, const BigParams& p, hipStream_t s, hipEvent_t e1) {
  switch (logn) {
#define X(L) \
  case L:    \
    return fp64 ? launch_big_merge_t<double, L>(p, s, e1) : launch_big_merge_t<float, L>(p, s, e1);
    AFD_BIG_LOGN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_big(int logn, bool fp64, const BigParams& p, int nr, bool cols, int med, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1, hipEvent_t r0, hipEvent_t r1) {
  switch (logn) {
#define X(L) \
  case L:    \
    return fp64 ? launch_big_t<double, L>(p, nr, cols, med, s, e0, e1, r0, r1)                    \
                : launch_big_t<float, L>(p, nr, cols, med, s, e0, e1, r0, r1);
    AFD_BIG_LOGN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace afd
