// The tail of a Core-AFD step for 2^10 <= N <= 2^14 points, after the
// radius kernel: the double-precision re-check of the short-list by the
// direct rule (Sec. 3.1, eq. term81), the winner, the remainder update of
// Sec. 2, eq. (7), and the forward DFT of the new remainder (Sec. 3.1,
// eq. term4) that the next step's radius kernel reads.
//
// Three phases over the samples of one signal:
//   A  re-check: one wave per (candidate, chunk of 1024 samples) task sums
//      G[n] / (1 - r e^{2 pi i (j - n)/N}) over its chunk (N/256 workgroups);
//   B  every transform workgroup picks the winner from the partial sums,
//      updates its columns n = l1 + N1 l2 of the samples in double, and runs
//      the length-N2 column DFTs of the four-step split N = N1 N2, storing
//      X[k2][l1] = e^{-2 pi i l1 k2/N} sum_l2 G'[l1 + N1 l2] e^{-2 pi i l2 k2/N2};
//   C  the length-N1 row DFTs give c[k2 + N2 k1]; workgroup 0 sums the
//      energy of the new remainder and records the step.
// A single signal runs all three in one launch of at most 64 workgroups,
// separated by grid barriers (every workgroup is resident: a few dozen
// 256-thread workgroups on a 256-CU device); a batch runs one launch per
// phase with the signal in grid dimension y.  Both forms execute the same
// arithmetic in the same order, so a signal's results do not depend on the
// form.  Without an update (update = 0) phases B and C transform the samples
// as they are: the spectrum of the first step.
#include "afd_update.h"

namespace afd {

constexpr int kAdvThreads = 256;
constexpr int kAdvE = 4;                  // values per thread in the column and row DFTs
constexpr int kAdvPts = 16;               // samples per lane of a re-check task
constexpr int kAdvChunk = 64 * kAdvPts;   // samples per re-check task
// Spin limit of a grid barrier wait (seconds): a wait that runs out reports
// an error instead of hanging.
constexpr unsigned int kAdvSpinLimit = 1u << 22;
constexpr int kBarStride = 16;  // barrier counters 128 bytes apart

template <int LOGN>
struct AdvShape {
  static constexpr int N = 1 << LOGN;
  static constexpr int L1 = LOGN / 2, L2 = LOGN - L1;
  static constexpr int N1 = 1 << L1, N2 = 1 << L2;
  static constexpr int TPC = N2 / kAdvE;         // threads per column DFT
  static constexpr int CPB = kAdvThreads / TPC;  // columns per workgroup
  static constexpr int TPR = N1 / kAdvE;         // threads per row DFT
  static constexpr int RPB = kAdvThreads / TPR;  // rows per workgroup
  static constexpr int NB = N1 / CPB;            // transform workgroups
  static constexpr int NCH = N / kAdvChunk;      // re-check chunks
  static constexpr int GA = N / 256;             // re-check workgroups
  static_assert(N2 / RPB == NB, "column and row passes use the same workgroups");
  static_assert(GA >= NB && NCH >= 1, "geometry");
  // the transforms' exchange regions, or (before them) the scratch of the merge
  template <typename T>
  static constexpr size_t lds_bytes() {
    constexpr size_t a = CPB * align16(size_t(Shape<L2, kAdvE>::LDS_ELEMS) * sizeof(Cx<T>));
    constexpr size_t b = RPB * align16(size_t(Shape<L1, kAdvE>::LDS_ELEMS) * sizeof(Cx<T>));
    constexpr size_t t = a > b ? a : b;
    return t > sizeof(MergeScratch) ? t : sizeof(MergeScratch);
  }
};

// Coherent (agent-scope) transfer of a complex value between workgroups of
// one launch.
__device__ __forceinline__ void st_agent(Cx<float>* p, Cx<float> v) {
  st_agent(reinterpret_cast<uint64_t*>(p),
           (uint64_t(__float_as_uint(v.y)) << 32) | uint64_t(__float_as_uint(v.x)));
}
__device__ __forceinline__ void st_agent(Cx<double>* p, Cx<double> v) {
  st_agent(&p->x, v.x);
  st_agent(&p->y, v.y);
}
__device__ __forceinline__ Cx<float> ld_agent(const Cx<float>* p) {
  const uint64_t u = ld_agent(reinterpret_cast<const uint64_t*>(p));
  return {__uint_as_float(uint32_t(u)), __uint_as_float(uint32_t(u >> 32))};
}
__device__ __forceinline__ Cx<double> ld_agent(const Cx<double>* p) { return {ld_agent(&p->x), ld_agent(&p->y)}; }

// Grid barrier on counters that only grow during a call.  Workgroup w
// arrives on counter w mod 8 (eight counters on separate cache lines, so
// that arrivals do not queue on one address), and a barrier is passed when
// every counter has reached the arrivals of the call's earlier barriers plus
// this one's.  Each wave waits for its stores to complete before its
// workgroup counts the arrival, so the agent-scope loads after the wait see
// them.
__device__ __forceinline__ void grid_arrive(unsigned long long* ctr) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(ctr + (blockIdx.x % kBarGroups) * kBarStride, 1ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
// Lanes 0..7 of wave 0 poll one counter each against target[lane].
__device__ __forceinline__ void grid_wait(unsigned long long* ctr, const unsigned long long (&target)[kBarGroups],
                                          int* status) {
  if (threadIdx.x < 64) {
    const int g = int(threadIdx.x);
    unsigned long long tg = 0;
#pragma unroll
    for (int k = 0; k < kBarGroups; ++k)
      if (g == k) tg = target[k];
    unsigned int spins = 0;
    for (;;) {
      const unsigned long long v =
          g < kBarGroups ? __hip_atomic_load(ctr + g * kBarStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : ~0ull;
      if (__ballot(v >= tg) == ~0ull) break;
      __builtin_amdgcn_s_sleep(2);
      ++spins;
      // after one wait of the call has run out, the others stop early
      if (spins >= kAdvSpinLimit ||
          ((spins & 1023u) == 0 && (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2))) {
        if (g == 0) atomicOr(status, 2);
        break;
      }
    }
  }
  __syncthreads();
}

// Winner of the short-list in one wave: lane l holds candidates l + 64 q
// (q < 4, count <= kKMax), each with its key, radius and the chunk partial
// sums of the direct rule in partials[i][0..nch).  P = |sqrt(1-r^2)/N sum|^2;
// the largest P wins, ties to the lowest flat index; the runner-up is the
// largest P of the others.  Every lane returns the result.
template <int NCH>
__device__ __forceinline__ Winner winner_wave(int count, int cflags, const uint64_t (&key)[4], const double (&rr)[4],
                                              const double* __restrict__ partials, int N, int logn) {
  const int lane = int(threadIdx.x) & 63;
  double pl = -1.0, p2l = -1.0, vxl = 0.0, vyl = 0.0, err = 0.0;
  uint32_t fl = 0xffffffffu;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (64 * q < count) {  // the same for the whole wave
      const int i = lane + 64 * q;
      double pv[2 * NCH];  // every partial sum of the slot in flight at once
#pragma unroll
      for (int k = 0; k < 2 * NCH; ++k) pv[k] = ld_agent(partials + 2 * size_t(i) * NCH + k);
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        ax += pv[2 * ch];
        ay += pv[2 * ch + 1];
      }
      const double sc = sqrt((1.0 - rr[q]) * (1.0 + rr[q])) / double(N);
      const double vx = ax * sc, vy = ay * sc;
      const double P = vx * vx + vy * vy;
      const uint32_t f = key_f(key[q]);
      if (i < count) {
        err = fmax(err, fabs(double(key_p(key[q])) - P));
        if (better64(P, f, pl, fl)) {
          p2l = fmax(pl, p2l);
          pl = P;
          fl = f;
          vxl = vx;
          vyl = vy;
        } else {
          p2l = fmax(p2l, P);
        }
      }
    }
  }
  // P >= 0, so the bits of P + 1 order the lanes (0: no candidate)
  const uint64_t kp = pl >= 0.0 ? uint64_t(__double_as_longlong(pl)) + 1u : 0u;
  const uint64_t kmax = wave_max_u64(kp);
  const uint32_t fwin = wave_reduce_bits<MinU32>(kp == kmax ? fl : 0xffffffffu);
  const bool mine = kmax != 0 && kp == kmax && fl == fwin;
  const uint64_t who = __ballot(mine);
  const int src = who ? __ffsll((long long)who) - 1 : 0;
  const double p1 = lane_f64(pl, src);
  const double p2 = wave_max_f64(mine ? p2l : pl);
  err = wave_max_f64(err);
  const bool forced = (cflags & kFlagForced) != 0;
  const bool valid = kmax != 0;
  Winner o;
  o.m = valid ? int32_t(fwin >> logn) : 0;
  o.j = valid ? int32_t(fwin & uint32_t(N - 1)) : 0;
  o.cx = valid ? lane_f64(vxl, src) : 0.0;
  o.cy = valid ? lane_f64(vyl, src) : 0.0;
  if (forced || count < 2 || !valid) o.margin = __builtin_nan("");
  else o.margin = p1 > 0.0 ? (p1 - p2) / p1 : 0.0;
  o.kcount = forced ? 1 : count;
  o.flags = cflags & 7;
  o.ax = o.ay = 0.0;
  o.fp32err = (forced || !valid || !(p1 > 0.0)) ? 0.0 : err / p1;
  return o;
}

// Step record (as write_record) from the winner and its angle in registers.
__device__ __forceinline__ void record_step(const RecordArgs& R, int step, const Winner& W, const Blaschke& B,
                                            double E) {
  R.idx[2 * step] = min(max(W.m, 0), R.M - 1);
  R.idx[2 * step + 1] = B.j;
  R.a[2 * step] = B.r * B.wjx;
  R.a[2 * step + 1] = -(B.r * B.wjy);
  R.coef[2 * step] = W.cx;
  R.coef[2 * step + 1] = W.cy;
  R.energy[step + 1] = E;
  R.margin[step] = W.margin;
  R.kcount[step] = W.kcount;
  R.flags[step] = W.flags;
  R.fp32err[step] = W.fp32err;
}

// At most a few dozen workgroups per launch: one wave per SIMD is all the
// occupancy there is, so the compiler may keep every load in flight.
template <typename T, int LOGN>
__global__ __launch_bounds__(kAdvThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_advance(AdvanceArgs a) {
  using S = AdvShape<LOGN>;
  constexpr int N = S::N;
  constexpr int WPB = kAdvThreads / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double wd[16];
  __shared__ Winner s_win;
  __shared__ CandList s_cand;
  const int tid = int(threadIdx.x), w = int(blockIdx.x), b = int(blockIdx.y);
  const int lane = tid & 63, wave = tid >> 6;
  const bool fused = a.phase < 0;
  const bool recheck = a.update && a.recheck;
  const bool runA = recheck && (fused || a.phase == 0);
  const bool runB = w < S::NB && (fused || a.phase == 1);
  const bool runC = w < S::NB && (fused || a.phase == 2);

  // the radius kernel's records are merged here (by every workgroup that
  // needs the short-list or the winner; all reach the same result)
  const bool merge = a.update && a.nrec > 0 && (fused || a.phase <= 1);
  MergeScratch* Sm = reinterpret_cast<MergeScratch*>(smem);
  const CandList* cand = a.cand + b;
  Winner* __restrict__ winner = a.winner + b;
  double* __restrict__ g64 = a.g64 + 2 * size_t(N) * b;
  Cx<T>* __restrict__ xt = reinterpret_cast<Cx<T>*>(a.xt) + size_t(N) * b;
  Cx<T>* __restrict__ c = reinterpret_cast<Cx<T>*>(a.c) + size_t(N) * b;
  double* __restrict__ partials = a.partials + 2 * size_t(kKMax) * S::NCH * b;
  double* __restrict__ epart = a.epart + size_t(S::NB) * b;

  // ---- everything that does not depend on the winner is loaded first
  const int ci = tid % S::CPB, tt = tid / S::CPB;  // phase B: column l1, thread of its DFT
  const int l1 = w * S::CPB + ci;
  const int tr = tid % S::TPR, ri = tid / S::TPR;  // phase C: thread of the DFT of row k2
  const int k2r = w * S::RPB + ri;
  double gx[kAdvE], gy[kAdvE];
  Cx<T> xtw[kAdvE];
  TwRegs<T, S::L2, kAdvE> twc;
  TwRegs<T, S::L1, kAdvE> twr;
  if (runB) {
#pragma unroll
    for (int i = 0; i < kAdvE; ++i) {
      const int n = l1 + S::N1 * (tt + S::TPC * i);
      gx[i] = g64[2 * n];
      gy[i] = g64[2 * n + 1];
    }
    if (a.fft) {
      tw_regs_load(twc, tt, reinterpret_cast<const Cx<T>*>(a.tw2));
#pragma unroll
      for (int p = 0; p < kAdvE; ++p)
        xtw[p] = reinterpret_cast<const Cx<T>*>(a.omega_t)[(l1 * out_bin<S::L2, kAdvE>(tt, p)) & (N - 1)];
    }
  }
  if (runC && a.fft) tw_regs_load(twr, tr, reinterpret_cast<const Cx<T>*>(a.tw1));
  if (merge && recheck) {
    select32_tail<4>(reinterpret_cast<const BlockList32*>(a.recs) + size_t(a.nrec) * b, a.heads + size_t(a.nrec) * b,
                  a.seconds + size_t(a.nrec) * b, a.nrec, a.recheck_k, a.tau_band, a.flagword + b, &s_cand, Sm,
                  false);
    __syncthreads();
    cand = &s_cand;
  }
  int count = 0, cflags = 0;
  if (recheck) {
    count = min(max(cand->count, 0), kKMax);
    cflags = cand->flags;
  }
  // the winner's inputs (wave 0 of the transform workgroups)
  uint64_t ckey[4] = {0, 0, 0, 0};
  double crad[4] = {0.0, 0.0, 0.0, 0.0};
  if (runB && recheck && wave == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) ckey[q] = cand->keys[lane + 64 * q];
  }

  // the radii of the candidates, in the same round trip as the re-check
  // inputs (unused slots read a clamped radius: keys has kKMax entries)
  if (runB && recheck && wave == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) crad[q] = a.radii[min(int(key_f(ckey[q]) >> LOGN), a.M - 1)];
  }

  // ---- A: partial sums of the direct rule, one wave per (candidate, chunk)
  if (runA) {
    const int tasks = count * S::NCH;
    const int stride = int(gridDim.x) * WPB;
    // the re-check-only workgroups take the first tasks: the transform
    // workgroups have their own loads in flight
    int task = w >= S::NB ? (w - S::NB) * WPB + wave : (int(gridDim.x) - S::NB + w) * WPB + wave;
    // the key of a task is read before the count is known (keys has kKMax entries)
    uint64_t knext = cand->keys[min(task / S::NCH, kKMax - 1)];
    for (; task < tasks; task += stride) {
      const int i = task / S::NCH, ch = task % S::NCH;
      const uint32_t f = key_f(knext);
      knext = cand->keys[min((task + stride) / S::NCH, kKMax - 1)];
      const int j = int(f & uint32_t(N - 1));
      const double r = a.radii[f >> LOGN];
      // all samples and unit roots of the chunk in flight at once, then the sums
      Cx<double> om[kAdvPts], gs[kAdvPts];
#pragma unroll
      for (int q = 0; q < kAdvPts; ++q) {
        const int n = ch * kAdvChunk + lane + 64 * q;
        om[q] = reinterpret_cast<const Cx<double>*>(a.omega)[(j - n) & (N - 1)];
        gs[q] = reinterpret_cast<const Cx<double>*>(g64)[n];
      }
      __builtin_amdgcn_sched_barrier(0);
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int q = 0; q < kAdvPts; ++q) {
        const double dx = fma(-r, om[q].x, 1.0), dy = -r * om[q].y;
        const double inv = 1.0 / fma(dx, dx, dy * dy);
        ax += fma(gs[q].x, dx, gs[q].y * dy) * inv;
        ay += fma(gs[q].y, dx, -gs[q].x * dy) * inv;
      }
      ax = wave_sum_f64(ax);
      ay = wave_sum_f64(ay);
      if (lane == 0) {
        st_agent(partials + 2 * (size_t(i) * S::NCH + ch), ax);
        st_agent(partials + 2 * (size_t(i) * S::NCH + ch) + 1, ay);
      }
    }
  }
  unsigned long long target[kBarGroups];
#pragma unroll
  for (int k = 0; k < kBarGroups; ++k) target[k] = a.bar_base[k];
  if (fused && recheck) {
    grid_arrive(a.bar);
#pragma unroll
    for (int k = 0; k < kBarGroups; ++k) target[k] += bar_group_count(int(gridDim.x), k);
    if (!runB) return;  // re-check only
    grid_wait(a.bar, target, a.status);
    // every merge has read the step's fallback flag
    if (merge && w == 0 && tid == 0) st_agent(a.flagword + b, 0u);
  }
  if (!runB && !runC) return;

  // ---- B: winner, update of this workgroup's columns, column DFTs
  Cx<T> v[kAdvE];
  Blaschke B{};
  double acc = 0.0;
  if (runB) {
    if (a.update) {
      if (recheck) {
        if (wave == 0) {
          const Winner o = winner_wave<S::NCH>(count, cflags, ckey, crad, partials, N, LOGN);
          if (lane == 0) {
            s_win = o;
            if (w == 0) *winner = o;
          }
        }
      } else if (merge) {
        // the FP64 grid maximum from the radius kernel's records
        merge64_tail<4>(reinterpret_cast<const BlockBest64*>(a.recs) + size_t(a.nrec) * b, a.nrec, N, &s_win,
                     Sm);
        __syncthreads();
        if (w == 0 && tid == 0) *winner = s_win;
      } else if (tid == 0) {
        s_win = *winner;  // written by the radius kernel
      }
      __syncthreads();
      B = blaschke_of(s_win, a.radii, a.omega, N, a.M);
#pragma unroll
      for (int i = 0; i < kAdvE; ++i) {
        const int n = l1 + S::N1 * (tt + S::TPC * i);
        double hx, hy;
        blaschke_apply(B, a.omega, N, n, gx[i], gy[i], hx, hy);
        g64[2 * n] = hx;
        g64[2 * n + 1] = hy;
        acc += fma(hx, hx, hy * hy);
        v[i] = {T(hx), T(hy)};
      }
    } else {
#pragma unroll
      for (int i = 0; i < kAdvE; ++i) v[i] = {T(gx[i]), T(gy[i])};
    }
    if (a.fft) {
      unsigned char* region = smem + size_t(ci) * align16(size_t(Shape<S::L2, kAdvE>::LDS_ELEMS) * sizeof(Cx<T>));
      fft_regs<T, S::L2, kAdvE, -1, false>(v, tt, region, twc);
#pragma unroll
      for (int p = 0; p < kAdvE; ++p) {
        const Cx<T> tw{xtw[p].x, -xtw[p].y};
        st_agent(xt + size_t(out_bin<S::L2, kAdvE>(tt, p)) * S::N1 + l1, cmul(v[p], tw));
      }
    }
    // the energy partial sum goes out while the intermediate is in flight
    if (a.update) {
      const double tot = block_sum_f64(acc, wd);
      if (tid == 0) st_agent(epart + w, tot);
    }
  }
  if (fused) {
    grid_arrive(a.bar);
#pragma unroll
    for (int k = 0; k < kBarGroups; ++k) target[k] += bar_group_count(S::NB, k);
    if (!a.fft && w != 0) return;
    grid_wait(a.bar, target, a.status);
  }

  // ---- C: row DFTs, record of the step
  if (runC) {
    const bool rec = a.update && w == 0;
    // a batch's record launch: every merge of the step has read the fallback flag
    if (!fused && rec && recheck && a.nrec > 0 && tid == 0) st_agent(a.flagword + b, 0u);
    const double ep = (rec && tid < S::NB) ? ld_agent(epart + tid) : 0.0;
    if (a.fft) {
#pragma unroll
      for (int i = 0; i < kAdvE; ++i) v[i] = ld_agent(xt + size_t(k2r) * S::N1 + tr + S::TPR * i);
      unsigned char* region = smem + size_t(ri) * align16(size_t(Shape<S::L1, kAdvE>::LDS_ELEMS) * sizeof(Cx<T>));
      fft_regs<T, S::L1, kAdvE, -1, false>(v, tr, region, twr);
#pragma unroll
      for (int p = 0; p < kAdvE; ++p) c[k2r + S::N2 * out_bin<S::L1, kAdvE>(tr, p)] = v[p];
    }
    if (rec) {
      const double E = block_sum_f64(ep, wd) / double(N);
      if (tid == 0) {
        Winner W;
        if (!fused) {  // a separate launch: the winner and its angle from memory
          W = *winner;
          B = blaschke_of(W, a.radii, a.omega, N, a.M);
        } else {
          W = s_win;
        }
        record_step(record_of(a.R, b), a.step, W, B, E);
      }
    }
  }
}

// ---------------------------------------------------------------- host side
template <int LOGN, int E>
static void stockham_twiddles(double* out) {
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

bool advance_supported(int logn) { return logn >= 10 && logn <= kMaxLdsLogN; }

AdvGeom advance_geom(int logn) {
  AdvGeom g{};
  switch (logn) {
#define X(L)                                        \
  case L:                                           \
    g.l1 = AdvShape<L>::L1;                         \
    g.l2 = AdvShape<L>::L2;                         \
    g.nb = AdvShape<L>::NB;                         \
    g.ga = AdvShape<L>::GA;                         \
    g.nch = AdvShape<L>::NCH;                       \
    g.tw1_size = Shape<AdvShape<L>::L1, kAdvE>::twsize(); \
    g.tw2_size = Shape<AdvShape<L>::L2, kAdvE>::twsize(); \
    break;
    X(10) X(11) X(12) X(13) X(14)
#undef X
    default:
      break;
  }
  return g;
}

void advance_twiddles(int l, double* out) {
  switch (l) {
    case 5: stockham_twiddles<5, kAdvE>(out); break;
    case 6: stockham_twiddles<6, kAdvE>(out); break;
    case 7: stockham_twiddles<7, kAdvE>(out); break;
    default: break;
  }
}

template <typename T, int LOGN>
static hipError_t launch_advance_t(const AdvanceArgs& a0, int batch, bool fused, hipStream_t s, hipEvent_t e0,
                                   hipEvent_t e1) {
  using S = AdvShape<LOGN>;
  constexpr uint32_t lds = uint32_t(S::template lds_bytes<T>());
  AdvanceArgs a = a0;
  const bool recheck = a.update && a.recheck;
  if (batch == 1 && fused) {
    a.phase = -1;
    launch_ev(k_advance<T, LOGN>, dim3(recheck ? S::GA : S::NB, 1), dim3(kAdvThreads), lds, s, e0, e1, a);
    return hipGetLastError();
  }
  if (recheck) {
    a.phase = 0;
    launch_ev(k_advance<T, LOGN>, dim3(S::GA, batch), dim3(kAdvThreads), lds, s, e0, nullptr, a);
    e0 = nullptr;
  }
  a.phase = 1;
  launch_ev(k_advance<T, LOGN>, dim3(S::NB, batch), dim3(kAdvThreads), lds, s, e0, nullptr, a);
  a.phase = 2;
  launch_ev(k_advance<T, LOGN>, dim3(a.fft ? S::NB : 1, batch), dim3(kAdvThreads), lds, s, nullptr, e1, a);
  return hipGetLastError();
}

void advance_bar_advance(int logn, AdvanceArgs& a) {
  const AdvGeom g = advance_geom(logn);
  const bool recheck = a.update && a.recheck;
  for (int k = 0; k < kBarGroups; ++k)
    a.bar_base[k] += (recheck ? bar_group_count(g.ga, k) : 0ull) + bar_group_count(g.nb, k);
}

hipError_t launch_advance(int logn, bool fp64, const AdvanceArgs& a, int batch, bool fused, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1) {
  switch (logn) {
#define X(L) \
  case L:    \
    return fp64 ? launch_advance_t<double, L>(a, batch, fused, s, e0, e1)                              \
                : launch_advance_t<float, L>(a, batch, fused, s, e0, e1);
    X(10) X(11) X(12) X(13) X(14)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace afd
