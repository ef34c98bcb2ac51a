// Fused per-radius kernel of the maximal-selection loop (Sec. 3.1, eq. rcl
// and Theorem 2.1; Sec. 3.2, Steps 1-2).
//
// One workgroup handles rpb radii.  For radius m it forms the weighted
// spectrum f(l) = r_m^l c_l in registers (r_m^l = r_m^t * r_m^(TPR v) from two
// double-built tables), runs the inverse DFT with LDS-staged Stockham passes,
// scales by s_m = sqrt(1 - r_m^2) / (N (1 - r_m^N)) and reduces
// |<G_k, e_{a_{m,j}}>~|^2 over its points: FP64 keeps the best point, its grid
// value and the runner-up value; FP32 keeps every point within the re-check
// band of the workgroup maximum.  The grid values are never written to HBM.
// The last workgroup to finish merges the per-workgroup records: FP64 into
// the winner, FP32 into the short-list for the double re-check (or, for
// 2^10 <= N <= 2^14, every workgroup of the step tail merges them itself).
#include "afd_select.h"

namespace afd {


template <typename T, int LOGN>
__host__ __device__ constexpr int radius_threads() {
  return Shape<LOGN, pickE<T, LOGN>()>::TPR < 64 ? 64 : Shape<LOGN, pickE<T, LOGN>()>::TPR;
}

// Waves per SIMD the register budget must allow: single precision keeps at
// most 128 VGPRs (two 512-thread or four 256-thread workgroups per CU), no
// constraint for double precision.
template <typename T, int LOGN>
__host__ __device__ constexpr int radius_min_waves() {
  return sizeof(T) == 4 ? 4 : 1;
}

template <typename T, int LOGN>
static size_t radius_lds(int rpb) {
  const size_t need = size_t(rpb) * fft_region_bytes<T, LOGN, pickSplit<T, LOGN>()>() + kListScratchBytes;
  return need > sizeof(MergeScratch) ? need : sizeof(MergeScratch);
}

// Double precision takes its slots from a work queue when the grid cannot
// hold them all at once (measured: 68.0 -> 64.2 us at N = 2^14, M = 1000);
// in single precision the loop it needs costs more than it recovers.
template <typename T>
__host__ __device__ constexpr bool radius_queued() {
  return sizeof(T) == 8;
}

// Inputs of Stockham pass P (P >= 2) when the spectrum has at most
// N / ns(P) terms.  Pass p sends its job's inputs x_p[job + r N/R_p] through
// the twiddles and an R_p-point DFT to x_{p+1}[(job / ns_p) ns_{p+1} +
// (job mod ns_p) + q ns_p]; with only r = 0 nonzero that is a copy, so by
// induction x_P[i] = x[i / ns(P)] and the inputs of job u of thread t are
// x[(t + TPR u) / ns(P) + r N / (R_P ns(P))], loaded directly: passes 0..P-1
// and their exchanges are skipped, and the skipped butterflies would only
// have added zeros.  Every index is below N / ns(P) <= TPR, so the weight is
// one entry r_m^l of the [M][TPR] table.
template <typename T, int LOGN, int E, int P>
__device__ __forceinline__ void deep_inputs(Cx<T> (&v)[E], int t, int L, const Cx<T>* __restrict__ c,
                                            const T* __restrict__ pwm) {
  using S = Shape<LOGN, E>;
  constexpr int R = S::radix(P), NS = S::ns(P), J = E / R, D = S::N / (R * NS);
  static_assert(P >= 2 && S::N / NS <= S::TPR, "the weights come from the r^t table");
#pragma unroll
  for (int u = 0; u < J; ++u) {
    const int a = (t + u * S::TPR) / NS;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int l = a + D * r;
      v[u + r * J] = {T(0), T(0)};
      if (l < L) {
        const Cx<T> x = c[l];
        const T w = pwm[l];
        v[u + r * J] = {x.x * w, x.y * w};
      }
    }
  }
}

// Record slot `slot` of signal b: one radius (rpb = 1, the radii in the order
// of decreasing significant spectrum length, so the longest transforms come
// first; the radius and its length in one load) or rpb consecutive radii.
// With a work queue, thread 0 claims the next slot after the transform and
// the claim's round trip overlaps the selection; the returned ticket is
// meaningful in thread 0 only.  PROBE (double precision, replay): the grid
// value at the forced point is also stored; it is a separate instantiation
// so that the probe's code does not weigh on the decomposition's.
template <typename T, int LOGN, bool LIST, bool PROBE, bool FOLD>
__device__ __forceinline__ unsigned int radius_slot(const RadiusParams& prm, int slot, int b, unsigned char* smem) {
  constexpr int E = pickE<T, LOGN>();
  constexpr bool SPLIT = pickSplit<T, LOGN>();
  using S = Shape<LOGN, E>;
  constexpr int N = S::N, TPR = S::TPR;
  // in the queue loop, the thread index goes through an opaque zero so that
  // nothing derived from it is hoisted out of the slot and kept live across
  // the transform (which would exceed the register budget)
  int zero = 0;
  if constexpr (radius_queued<T>()) asm volatile("s_mov_b32 %0, 0" : "=s"(zero));
  const int tid = int(threadIdx.x) + zero;
  const int rl = tid / TPR, t = tid - rl * TPR;
  int m, L;
  // (a transform of at least 64 threads always has a workgroup of its own)
  if (S::TPR >= 64 || prm.rpb == 1) {
    const int2 wi = reinterpret_cast<const int2*>(prm.order)[slot];
    // one radius per workgroup: uniform, so its per-radius values sit in
    // scalar registers
    m = __builtin_amdgcn_readfirstlane(wi.x);
    L = __builtin_amdgcn_readfirstlane(wi.y);
  } else {
    m = slot * prm.rpb + rl;
    L = prm.lsig[m < prm.M ? m : prm.M - 1];
  }
  const bool active = m < prm.M;
  const int mm = active ? m : prm.M - 1;
  constexpr size_t region = fft_region_bytes<T, LOGN, SPLIT>();
  unsigned char* lds_r = smem + size_t(rl) * region;
  unsigned char* scratch = smem + size_t(prm.rpb) * region;

  // signal b of a batch: its spectrum and records
  const Cx<T>* __restrict__ c = reinterpret_cast<const Cx<T>*>(prm.c) + size_t(N) * b;
  if constexpr (FOLD) {
    // a radius whose series outlasts N terms has its own folded spectrum
    // (one radius per workgroup: a uniform choice, in scalar registers)
    int fs = prm.fslot[mm];
    if (S::TPR >= 64 || prm.rpb == 1) fs = __builtin_amdgcn_readfirstlane(fs);
    if (fs >= 0) c = reinterpret_cast<const Cx<T>*>(prm.cfold) + (size_t(b) * size_t(prm.nfold) + size_t(fs)) * N;
  }
  const T* __restrict__ pw = reinterpret_cast<const T*>(prm.pw);
  const T* __restrict__ pv = reinterpret_cast<const T*>(prm.pv);
  const Cx<T>* __restrict__ tw = reinterpret_cast<const Cx<T>*>(prm.tw);
  // the selection's scale is loaded now: after the transform's barriers its
  // load would be one more exposed round trip
  const T sc = reinterpret_cast<const T*>(prm.scale)[mm];

  // weighted spectrum f(l) = r_m^l c_l for l < L; the weights of the later
  // terms sum to less than 2^-40 (single) / 2^-60 (double precision) and they
  // are dropped
  constexpr int R0 = S::radix(0);
  Cx<T> v[E];
  // With L <= N/R0 the first pass (radix R0, inputs x[job + r N/R0]) only
  // replicates x[job]: thread t's inputs of the second pass are then
  // x[t/R0 + (TPR/R0) i], loaded directly, and the first pass and its
  // exchange are skipped.  Uniform over the workgroup (one radius).
  // Shorter spectra skip more passes (see deep_inputs): at most N / ns(2)
  // terms start at pass 2, at most N / ns(3) at pass 3.
  bool pruned = false;
  int deep = 0;
  if constexpr (S::NP >= 2 && R0 <= TPR) pruned = prm.rpb == 1 && L <= N / R0;
  if constexpr (S::NP >= 3) deep = pruned && L <= N / S::ns(2) ? 2 : 0;
  if constexpr (S::NP >= 4) deep = deep && L <= N / S::ns(3) ? 3 : deep;
  if (deep) {
    if constexpr (S::NP >= 3) {
      const T* __restrict__ pwm = pw + size_t(mm) * TPR;
      if constexpr (S::NP >= 4) {
        if (deep == 3) {
          deep_inputs<T, LOGN, E, 3>(v, t, L, c, pwm);
          fft_regs<T, LOGN, E, +1, SPLIT, 3, 3>(v, t, lds_r, tw);
        } else {
          deep_inputs<T, LOGN, E, 2>(v, t, L, c, pwm);
          fft_regs<T, LOGN, E, +1, SPLIT, 2, 2>(v, t, lds_r, tw);
        }
      } else {
        deep_inputs<T, LOGN, E, 2>(v, t, L, c, pwm);
        fft_regs<T, LOGN, E, +1, SPLIT, 2, 2>(v, t, lds_r, tw);
      }
    }
  } else if (pruned) {
    if constexpr (S::NP >= 2 && R0 <= TPR) {
      const int a = t / R0;  // r^l = r^a r^((TPR/R0) i)
      const T ra = pw[size_t(mm) * TPR + a];
      const T* __restrict__ pq = reinterpret_cast<const T*>(prm.pq) + size_t(mm) * E;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = a + (TPR / R0) * i;
        v[i] = {T(0), T(0)};
        if ((TPR / R0) * i < L && l < L) {
          const Cx<T> x = c[l];
          const T w = ra * pq[i];
          v[i] = {x.x * w, x.y * w};
        }
      }
      fft_regs<T, LOGN, E, +1, SPLIT, 1, 1>(v, t, lds_r, tw);
    }
  } else {
    const T rt = pw[size_t(mm) * TPR + t];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int l = t + TPR * i;
      v[i] = {T(0), T(0)};
      if (TPR * i < L && l < L) {
        const Cx<T> x = c[l];
        const T w = rt * pv[size_t(mm) * E + i];
        v[i] = {x.x * w, x.y * w};
      }
      // double precision: bound the loads in flight (128-register budget)
      if (sizeof(T) == 8 && (i % 4) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    fft_regs<T, LOGN, E, +1, SPLIT>(v, t, lds_r, tw);
  }

  const uint32_t fbase = uint32_t(mm) * uint32_t(N);
  unsigned int ticket = 0;
  if (radius_queued<T>() && prm.queue != nullptr && threadIdx.x == 0)
    ticket = __hip_atomic_fetch_add(prm.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if constexpr (LIST) {
    const uint32_t r0 = prm.rpb == 1 ? uint32_t(mm) : uint32_t(slot) * uint32_t(prm.rpb);
    const uint32_t ract = uint32_t(prm.M) - r0 < uint32_t(prm.rpb) ? uint32_t(prm.M) - r0 : uint32_t(prm.rpb);
    const FlatOrder ord{r0 * uint32_t(N), ract * uint32_t(N), 0u, ract * uint32_t(N)};
    BlockList32* lists = reinterpret_cast<BlockList32*>(prm.out) + size_t(prm.nrec) * b;
    uint64_t* heads = prm.heads + size_t(prm.nrec) * b;
    uint64_t* seconds = prm.seconds + size_t(prm.nrec) * b;
    select_list<LOGN>(v, active, sc, fbase, 1u, t, scratch, prm.tau_band, ord, lists + slot, heads + slot,
                      seconds + slot, prm.flagword + b);
  } else {
    if constexpr (PROBE) {
      // a replayed step: the grid value at the forced point, scaled exactly
      // as the selection scales its best value (register p holds bin
      // t + TPR bitrev(p))
      const int32_t* pr = prm.probe + size_t(prm.probe_stride) * b;
      const int pm = pr[0], pj = pr[1];
      if (active && m == pm && t == (pj & (TPR - 1))) {
        const int q = pj / TPR;
#pragma unroll
        for (int p = 0; p < E; ++p) {
          if (bitrev(p, ilog2c(E)) == q) {
            prm.probe_out[2 * b] = double(v[p].x * sc);
            prm.probe_out[2 * b + 1] = double(v[p].y * sc);
          }
        }
      }
    }
    select_best<LOGN, T>(v, active, sc, fbase, 1u, t, reinterpret_cast<Best*>(scratch),
                         reinterpret_cast<BlockBest64*>(prm.out) + size_t(prm.nrec) * b + slot);
  }
  return ticket;
}

// With prm.queue, a single signal's record slots come from a work queue: the
// grid holds only the workgroups that fit on the device at once, each takes
// its own slot first and then the next free one (longest transforms first),
// claimed once the current slot's transform is done.  Every processed slot
// claims one ticket, so a launch takes nrec tickets.  A slot's record does
// not depend on the workgroup that
// computes it.  Every workgroup leaves once the queue is exhausted; none
// waits on another.
template <typename T, int LOGN, bool LIST, bool PROBE = false, bool FOLD = false>
__global__ __launch_bounds__((radius_threads<T, LOGN>())) __attribute__((amdgpu_waves_per_eu(
    radius_min_waves<T, LOGN>()))) void k_radius(RadiusParams prm) {
  constexpr int N = 1 << LOGN;
  static_assert(radius_threads<T, LOGN>() % 64 == 0, "the wave reductions need whole waves");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  __shared__ int s_next;
  const int b = blockIdx.y;
  if constexpr (radius_queued<T>()) {
    // the first slot is the workgroup's own index; with a queue, the slots
    // from gridDim.x on are handed out one per fetch, until a fetch comes
    // back past the last slot
    int slot = int(blockIdx.x);
    while (slot < prm.nrec) {  // uniform
      const unsigned int ticket = radius_slot<T, LOGN, LIST, PROBE, FOLD>(prm, slot, b, smem);
      if (!prm.queue) break;
      __syncthreads();  // every thread is done with the LDS and with s_next
      if (threadIdx.x == 0) s_next = int(gridDim.x) + int(ticket - prm.qbase);
      __syncthreads();
      slot = __builtin_amdgcn_readfirstlane(s_next);  // uniform: a scalar register
    }
    if (prm.queue) return;  // the step tail merges the records
  } else {
    radius_slot<T, LOGN, LIST, PROBE, FOLD>(prm, int(blockIdx.x), b, smem);
  }
  if (!prm.tail) return;  // the step tail merges the records
  if (!last_arrival(prm.counter + b, gridDim.x, &s_last)) return;
  MergeScratch* Sm = reinterpret_cast<MergeScratch*>(smem);
  if constexpr (LIST) {
    select32_tail(reinterpret_cast<const BlockList32*>(prm.out) + size_t(prm.nrec) * b,
                  prm.heads + size_t(prm.nrec) * b, prm.seconds + size_t(prm.nrec) * b, prm.nrec, prm.recheck_k,
                  prm.tau_band, prm.flagword + b, prm.cand + b, Sm);
  } else {
    merge64_tail(reinterpret_cast<const BlockBest64*>(prm.out) + size_t(prm.nrec) * b, prm.nrec, N,
                 prm.winner + b, Sm);
  }
}

#define AFD_LDS_LOGN_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

int radius_lds_bytes(int logn, bool fp64, int rpb) {
  switch (logn) {
#define X(L) \
  case L:    \
    return int(fp64 ? radius_lds<double, L>(rpb) : radius_lds<float, L>(rpb));
    AFD_LDS_LOGN_CASES(X)
#undef X
    default:
      return 0;
  }
}

int radius_first_radix(int logn, bool fp64) {
  switch (logn) {
#define X(L) \
  case L:    \
    return fp64 ? Shape<L, pickE<double, L>()>::radix(0) : Shape<L, pickE<float, L>()>::radix(0);
    AFD_LDS_LOGN_CASES(X)
#undef X
    default:
      return 0;
  }
}

int significant_length(double r, int bits, int64_t n) {
  if (!(r > 0.0)) return 1;
  // r^L / (1 - r) <= 2^-bits  <=>  L >= (bits ln 2 + ln(1/(1 - r))) / (-ln r)
  const long double need = ((long double)bits * logl(2.0L) - logl(1.0L - (long double)r)) / -logl((long double)r);
  if (!(need < (long double)n)) return int(n);
  const long double L = ceill(need);
  return L < 1.0L ? 1 : int(L);
}

int radius_threads_of(int logn, bool fp64) {
  switch (logn) {
#define X(L) \
  case L:    \
    return fp64 ? radius_threads<double, L>() : radius_threads<float, L>();
    AFD_LDS_LOGN_CASES(X)
#undef X
    default:
      return 0;
  }
}

// Workgroups of the radius kernel that fit on the device at once (its
// occupancy times the CU count): the grid of a queued launch.
int radius_slots(int logn, bool fp64, int rpb) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = hipErrorInvalidValue;
  switch (logn) {
#define X(L)                                                                                                   \
  case L:                                                                                                      \
    e = fp64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_radius<double, L, false>,                  \
                                                            radius_threads<double, L>(), radius_lds<double, L>(rpb)) \
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_radius<float, L, true>,                    \
                                                            radius_threads<float, L>(), radius_lds<float, L>(rpb)); \
    break;
    AFD_LDS_LOGN_CASES(X)
#undef X
    default:
      break;
  }
  return e == hipSuccess ? per * cus : 0;
}

hipError_t setup_radius_attributes() {
  hipError_t e = hipSuccess;
#define X(L)                                                                                  \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<double, L, false>));                 \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<double, L, false, true>));           \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<float, L, true>));          \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<double, L, false, false, true>)); \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<double, L, false, true, true>)); \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<float, L, true, false, true>));
  AFD_LDS_LOGN_CASES(X)
#undef X
  return e;
}

hipError_t launch_radius(int logn, bool fp64, const RadiusParams& p, int blocks, int batch, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1) {
  switch (logn) {
#define X(L)                                                                                 \
  case L: {                                                                                  \
    if (fp64) {                                                                              \
      constexpr int thr = radius_threads<double, L>();                                       \
      const size_t lds = radius_lds<double, L>(p.rpb);                                       \
      if (p.fslot && p.probe)                                                                \
        launch_ev(k_radius<double, L, false, true, true>, dim3(blocks, batch), dim3(thr), uint32_t(lds), s, e0, e1, \
                  p);                                                                        \
      else if (p.fslot)                                                                      \
        launch_ev(k_radius<double, L, false, false, true>, dim3(blocks, batch), dim3(thr), uint32_t(lds), s, e0, \
                  e1, p);                                                                    \
      else if (p.probe)                                                                      \
        launch_ev(k_radius<double, L, false, true>, dim3(blocks, batch), dim3(thr), uint32_t(lds), s, e0, e1, p); \
      else                                                                                   \
        launch_ev(k_radius<double, L, false>, dim3(blocks, batch), dim3(thr), uint32_t(lds), s, e0, e1, p); \
    } else {                                                                                 \
      constexpr int thr = radius_threads<float, L>();                                        \
      const size_t lds = radius_lds<float, L>(p.rpb);                                        \
      if (p.fslot)                                                                           \
        launch_ev(k_radius<float, L, true, false, true>, dim3(blocks, batch), dim3(thr), uint32_t(lds), s, e0, e1, \
                  p);                                                                        \
      else                                                                                   \
        launch_ev(k_radius<float, L, true>, dim3(blocks, batch), dim3(thr), uint32_t(lds), s, e0, e1, p); \
    }                                                                                        \
    return hipGetLastError();                                                                \
  }
    AFD_LDS_LOGN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace afd
