// Selection on the polar grid (Sec. 2, eq. ak; Sec. 3.2, Step 2): block-level
// reductions of |<G_k, e_a>~|^2 and the grid-level merges that run in the
// last workgroup of a launch.  Every reduction is order-fixed (wave xor
// butterflies, then waves in index order), so results do not depend on
// scheduling.  Ties go to the lowest flat index m*N + j.
#pragma once

#include "afd_device.h"
#include "afd_internal.h"

namespace afd {

// ---------------------------------------------------------------- keys and bests
// FP64 selection state: best value, its flat index and grid value, runner-up value.
struct Best {
  double p1, p2, vx, vy;
  uint32_t f;
};

__device__ __forceinline__ void best_merge(Best& a, const Best& b) {
  if (better64(b.p1, b.f, a.p1, a.f)) {
    a.p2 = fmax(a.p1, b.p2);
    a.p1 = b.p1;
    a.f = b.f;
    a.vx = b.vx;
    a.vy = b.vy;
  } else {
    a.p2 = fmax(a.p2, b.p1);
  }
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  return __longlong_as_double((long long)dpp_u64<CTRL>(uint64_t(__double_as_longlong(v))));
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
  return __longlong_as_double((long long)lane_u64(uint64_t(__double_as_longlong(v)), lane));
}
template <int CTRL>
__device__ __forceinline__ Best best_dpp(const Best& a) {
  return Best{dpp_f64<CTRL>(a.p1), dpp_f64<CTRL>(a.p2), dpp_f64<CTRL>(a.vx), dpp_f64<CTRL>(a.vy), dpp_u32<CTRL>(a.f)};
}
__device__ __forceinline__ Best best_lane(const Best& a, int lane) {
  return Best{lane_f64(a.p1, lane), lane_f64(a.p2, lane), lane_f64(a.vx, lane), lane_f64(a.vy, lane),
              lane_u32(a.f, lane)};
}
// best and runner-up over the wave (every lane gets the result; all lanes active)
__device__ __forceinline__ Best wave_best(Best b) {
  best_merge(b, best_dpp<kDppXor1>(b));
  best_merge(b, best_dpp<kDppXor2>(b));
  best_merge(b, best_dpp<kDppHalfMirror>(b));
  best_merge(b, best_dpp<kDppMirror>(b));
  Best r = best_lane(b, 0);
  best_merge(r, best_lane(b, 16));
  best_merge(r, best_lane(b, 32));
  best_merge(r, best_lane(b, 48));
  return r;
}

__device__ __forceinline__ int nwaves() { return int((blockDim.x + 63) >> 6); }

// Block-wide best and runner-up, valid in wave 0 (the callers store it from
// thread 0): the wave results meet in LDS and wave 0 merges them.  `wb` is an
// LDS array of 16; it must not be rewritten before the next barrier.
__device__ __forceinline__ Best block_best(Best b, Best* wb) {
  b = wave_best(b);
  if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = b;
  __syncthreads();
  Best r{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  if (threadIdx.x < 64) {
    if (int(threadIdx.x) < nwaves()) r = wb[threadIdx.x];
    r = wave_best(r);
  }
  return r;
}

// Block-wide results, returned to every thread.  `w*` are LDS arrays of 16.

__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, uint64_t* wb) {
  v = wave_max_u64(v);
  if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t b = wb[0];
  for (int w = 1; w < nwaves(); ++w) b = wb[w] > b ? wb[w] : b;
  __syncthreads();
  return b;
}

__device__ __forceinline__ float block_max_f32(float v, float* wf) {
  v = wave_max_f32(v);
  if ((threadIdx.x & 63) == 0) wf[threadIdx.x >> 6] = v;
  __syncthreads();
  float b = wf[0];
  for (int w = 1; w < nwaves(); ++w) b = fmaxf(b, wf[w]);
  __syncthreads();
  return b;
}

// SUM: block sum, else block minimum; `w` is an LDS array of 16
template <bool SUM>
__device__ __forceinline__ uint32_t block_reduce_u32(uint32_t v, uint32_t* w) {
  if constexpr (SUM)
    v = wave_reduce_bits<SumU32>(v);
  else
    v = wave_reduce_bits<MinU32>(v);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = w[0];
  for (int i = 1; i < nwaves(); ++i) r = SUM ? r + w[i] : (w[i] < r ? w[i] : r);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_sum_f64(double v, double* wd) {
  v = wave_sum_f64(v);
  if ((threadIdx.x & 63) == 0) wd[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = wd[0];
  for (int w = 1; w < nwaves(); ++w) s += wd[w];
  __syncthreads();
  return s;
}

// Append key k of every lane with q set to buf (one LDS atomic per wave);
// entries past cap are counted but dropped.
__device__ __forceinline__ void wave_append(bool q, uint64_t k, uint32_t* cnt, uint64_t* buf, uint32_t cap) {
  const uint64_t mask = __ballot(q);
  if (mask == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll(static_cast<long long>(mask)) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(cnt, uint32_t(__popcll(mask)));
  base = lane_u32(base, leader);
  if (q) {
    const uint32_t pos = base + uint32_t(__popcll(mask & ((uint64_t(1) << lane) - 1)));
    if (pos < cap) buf[pos] = k;
  }
}

// The first ndst keys of buf[0..n) in descending order, written to dst (LDS or
// global).  Keys are distinct.  Rank counting for short lists, an LDS bitonic
// sort (in place in buf, capacity >= next power of two of n) otherwise.
__device__ __forceinline__ void top_desc(uint64_t* buf, uint32_t n, uint64_t* dst, uint32_t ndst) {
  if (n <= 256) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint64_t ki = buf[i];
      uint32_t rank = 0;
      for (uint32_t j = 0; j < n; ++j) rank += buf[j] > ki ? 1u : 0u;
      if (rank < ndst) dst[rank] = ki;
    }
    __syncthreads();
    return;
  }
  uint32_t p2 = 1;
  while (p2 < n) p2 <<= 1;
  for (uint32_t i = n + threadIdx.x; i < p2; i += blockDim.x) buf[i] = 0;
  __syncthreads();
  for (uint32_t k = 2; k <= p2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = buf[i], c = buf[ixj];
          if ((i & k) == 0 ? (a < c) : (a > c)) {
            buf[i] = c;
            buf[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  const uint32_t m = n < ndst ? n : ndst;
  for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) dst[i] = buf[i];
  __syncthreads();
}

// Copy n (<= 64) keys from LDS to global memory with wave 0.
__device__ __forceinline__ void wave0_copy_keys(const uint64_t* src, uint64_t* dst, uint32_t n);

// ---------------------------------------------------------------- cross-workgroup records
// Records that the last workgroup of a launch reads are stored and loaded
// with agent-scope atomics (coherent across the XCDs' L2 caches without a
// cache write-back or invalidation, so the inputs other workgroups keep in L2
// stay there).
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  st_agent(reinterpret_cast<uint64_t*>(p), uint64_t(__double_as_longlong(v)));
}
__device__ __forceinline__ void st_agent(float* p, float v) {
  st_agent(reinterpret_cast<uint32_t*>(p), __float_as_uint(v));
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __longlong_as_double(static_cast<long long>(ld_agent(reinterpret_cast<const uint64_t*>(p))));
}
__device__ __forceinline__ float ld_agent(const float* p) {
  return __uint_as_float(ld_agent(reinterpret_cast<const uint32_t*>(p)));
}

// ---------------------------------------------------------------- last workgroup
// Every workgroup calls this once its records are stored; it returns true in
// exactly one workgroup (the last to arrive).  Contract: the records the last
// workgroup reads are stored by wave 0 with st_agent and read with ld_agent.
// Wave 0 waits for its stores to complete before thread 0 counts the
// arrival, so the last workgroup's later loads see every record.  The counter
// is reset for the next launch.  `flag` is an LDS int.
// last_arrival counts `total` arrivals instead (a group of workgroups, or
// arrivals spread over several launches).
__device__ __forceinline__ bool last_arrival(unsigned int* counter, unsigned int total, int* flag) {
  __syncthreads();
  if (threadIdx.x < 64) {
    __builtin_amdgcn_s_waitcnt(0);
    if (threadIdx.x == 0) {
      const unsigned int prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int last = prev == total - 1;
      if (last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *flag = last;
    }
  }
  __syncthreads();
  return *flag != 0;
}

__device__ __forceinline__ bool last_workgroup(unsigned int* counter, int* flag) {
  return last_arrival(counter, gridDim.x * gridDim.y * gridDim.z, flag);
}

__device__ __forceinline__ void wave0_copy_keys(const uint64_t* src, uint64_t* dst, uint32_t n) {
  if (threadIdx.x < n) st_agent(dst + threadIdx.x, src[threadIdx.x]);
}

// LDS layout used by the grid-level merges (placed in a kernel's dynamic LDS).
constexpr int kHeadCap = 2048;    // head keys the FP32 grid merge holds in LDS
constexpr int kSecondCap = 1024;  // second keys it holds (more blocks: every band list is read)
// Records per thread a grid merge loads in its first round trip (a template
// parameter PRE of the merges: 2 where a 512-thread workgroup merges inside a
// register-bound transform kernel, 4 in the 256-thread step tail).

struct MergeScratch {
  uint64_t heads[kHeadCap];
  uint64_t seconds[kSecondCap];
  uint64_t buf[kSelCap];
  uint32_t cblk[kSelCap];
  uint64_t sorted[kListC];
  uint64_t hcut;
  uint64_t wb[16];
  Best bb[16];
  float wf[16];
  double wd[16];
  uint32_t scount, sblocks, sflags, stotal, sband;
  int last;
};

// FP64: best and runner-up over a group of workgroup records (the workgroups
// of one radius) into one record of the same form.
__device__ __forceinline__ void merge_best_group(const BlockBest64* __restrict__ recs, int n,
                                                 BlockBest64* __restrict__ out, MergeScratch* S) {
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const BlockBest64* o = recs + i;
    const Best x{ld_agent(&o->p1), ld_agent(&o->p2), ld_agent(&o->vx), ld_agent(&o->vy), ld_agent(&o->f)};
    best_merge(b, x);
  }
  const Best r = block_best(b, S->bb);
  if (threadIdx.x == 0) {
    st_agent(&out->p1, r.p1);
    st_agent(&out->p2, r.p2);
    st_agent(&out->vx, r.vx);
    st_agent(&out->vy, r.vy);
    st_agent(&out->f, r.f);
  }
}

// FP32: the lists of a group of workgroups (the workgroups of one radius)
// merged into one list of the same form: every listed point within tau_band
// of the group maximum, the top kListC by key.  Each member list holds its own
// top keys in descending order, so the top kListC of the union are exact, and
// none of them is below the kListC-th largest member head (those heads alone
// are kListC keys): only keys at or above it are gathered.  More than kSelCap
// such keys are merged by popping the member lists, one list per thread
// (n <= blockDim.x).
__device__ __forceinline__ void merge_list_group(const BlockList32* __restrict__ L, int n, float tau_band,
                                                 BlockList32* __restrict__ out, uint64_t* head, MergeScratch* S) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = nwaves();
  // every member's header and head key in one round trip (n <= blockDim.x)
  uint32_t cm = 0, fl = 0;
  float pmm = -1.f;
  uint64_t hm = 0;
  if (tid < n) {
    const BlockList32* B = L + tid;
    cm = ld_agent(&B->count);
    fl = ld_agent(&B->flags);
    pmm = ld_agent(&B->pmax);
    hm = ld_agent(&B->keys[0]);
  }
  if (tid == 0) {
    S->sflags = 0;
    S->scount = 0;
    S->stotal = 0;
    S->sband = 0;
    S->hcut = 0;
  }
  const float pg = block_max_f32(cm > 0 ? pmm : -1.f, S->wf);  // its barriers order the initialisation above
  if (fl) atomicOr(&S->sflags, fl);
  const float theta = pg - pg * tau_band;
  // the kListC-th largest head among the members that reach the band (0 if
  // fewer), and the list length of each member that reaches it (0: skipped)
  const uint64_t hd = cm > 0 && key_p(hm) >= theta ? hm : 0;
  if (tid < n) {
    S->buf[tid] = hd;
    S->cblk[tid] = cm > 0 && pmm >= theta ? cm : 0u;
  }
  __syncthreads();
  if (hd) {
    uint32_t rank = 0;
    for (int i = 0; i < n; ++i) rank += S->buf[i] > hd ? 1u : 0u;
    if (rank == uint32_t(kListC) - 1) S->hcut = hd;  // keys are distinct: one thread at most
  }
  __syncthreads();
  const uint64_t hcut = S->hcut;
  // one wave per member list that reaches the band, the keys (and totals)
  // of kGroupBatch consecutive lists per round trip: where most members reach
  // the band (a flat radius) one list per round trip held every wave for n/nw
  // dependent loads
  constexpr int kGroupBatch = 8;
  for (int i0 = wave * kGroupBatch; i0 < n; i0 += nw * kGroupBatch) {
    uint64_t k[kGroupBatch];
    uint32_t tot[kGroupBatch];
#pragma unroll
    for (int q = 0; q < kGroupBatch; ++q) {
      const int i = i0 + q;
      const uint32_t cnt = i < n ? S->cblk[i] : 0u;
      k[q] = cnt > 0 && lane < int(cnt) ? ld_agent(&L[i].keys[lane]) : 0;
      tot[q] = cnt > 0 && lane == 0 ? ld_agent(&L[i].total) : 0u;
    }
#pragma unroll
    for (int q = 0; q < kGroupBatch; ++q) {
      const int i = i0 + q;
      const uint32_t cnt = i < n ? S->cblk[i] : 0u;
      if (cnt == 0) continue;  // uniform over the wave
      const bool inband = lane < int(cnt) && key_p(k[q]) >= theta;
      const uint64_t bm = __ballot(inband);
      if (lane == 0 && bm) atomicAdd(&S->sband, uint32_t(__popcll(bm)));
      wave_append(inband && k[q] >= hcut, k[q], &S->scount, S->buf, uint32_t(kSelCap));
      // a member list cut inside the band: count the points it could not hold
      const uint64_t last = lane_u64(k[q], __builtin_amdgcn_readfirstlane(int(cnt) - 1));
      if (lane == 0 && key_p(last) >= theta && tot[q] > cnt) atomicAdd(&S->stotal, tot[q] - cnt);
    }
  }
  __syncthreads();
  const uint32_t nb = S->scount;
  uint32_t cnt_out = 0;
  if (nb <= uint32_t(kSelCap)) {
    top_desc(S->buf, nb, S->sorted, uint32_t(kListC));
    cnt_out = nb < uint32_t(kListC) ? nb : uint32_t(kListC);
  } else {
    uint32_t hp = 0, hc = 0;
    uint64_t hk = 0;
    if (tid < n) {
      hc = ld_agent(&L[tid].count);
      hk = hc > 0 ? ld_agent(&L[tid].keys[0]) : 0;
      if (!(key_p(hk) >= theta)) hk = 0;
    }
    for (; cnt_out < uint32_t(kListC); ++cnt_out) {
      const uint64_t g = block_max_u64(hk, S->wb);
      if (g == 0) break;
      if (tid == 0) S->sorted[cnt_out] = g;
      if (hk == g) {  // keys are distinct: exactly one thread owns g
        ++hp;
        hk = hp < hc ? ld_agent(&L[tid].keys[hp]) : 0;
        if (!(key_p(hk) >= theta)) hk = 0;
      }
    }
    if (tid == 0) atomicOr(&S->sflags, uint32_t(kFlagFallback));
    __syncthreads();
  }
  wave0_copy_keys(S->sorted, out->keys, cnt_out);
  if (tid == 0) {
    const uint32_t tot = S->sband + S->stotal;  // points in the band (cut members' extra as an upper bound)
    st_agent(&out->pmax, pg);
    st_agent(&out->count, cnt_out);
    st_agent(&out->total, tot);
    st_agent(&out->flags, S->sflags);
    if (head) st_agent(head, cnt_out > 0 ? S->sorted[0] : uint64_t(0));
  }
}

// FP64: global best of the per-block records -> winner (coefficient = the
// grid value of the FFT form).  Each thread loads its first PRE records in
// one round trip, then BATCH records per round trip (workgroups with few
// threads and many records: the loop's loads would otherwise wait one by
// one).
template <int PRE = 2, int BATCH = 1>
__device__ __forceinline__ void merge64_tail(const BlockBest64* __restrict__ blocks, int nb, int N,
                                             Winner* __restrict__ w, MergeScratch* S) {
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  {
    // the first PRE records of each thread in one round trip
    Best x[PRE];
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int i = int(threadIdx.x) + q * int(blockDim.x);
      const BlockBest64* o = blocks + (i < nb ? i : nb - 1);
      x[q] = Best{ld_agent(&o->p1), ld_agent(&o->p2), ld_agent(&o->vx), ld_agent(&o->vy), ld_agent(&o->f)};
    }
#pragma unroll
    for (int q = 0; q < PRE; ++q)
      if (int(threadIdx.x) + q * int(blockDim.x) < nb) best_merge(b, x[q]);
  }
  if constexpr (BATCH == 1) {
    for (int i = int(threadIdx.x) + PRE * int(blockDim.x); i < nb; i += blockDim.x) {
      const BlockBest64* o = blocks + i;
      const Best x{ld_agent(&o->p1), ld_agent(&o->p2), ld_agent(&o->vx), ld_agent(&o->vy), ld_agent(&o->f)};
      best_merge(b, x);
    }
  } else {
    for (int i0 = int(threadIdx.x) + PRE * int(blockDim.x); i0 < nb; i0 += BATCH * int(blockDim.x)) {
      Best x[BATCH];
#pragma unroll
      for (int q = 0; q < BATCH; ++q) {
        const int i = i0 + q * int(blockDim.x);
        const BlockBest64* o = blocks + (i < nb ? i : nb - 1);
        x[q] = Best{ld_agent(&o->p1), ld_agent(&o->p2), ld_agent(&o->vx), ld_agent(&o->vy), ld_agent(&o->f)};
      }
#pragma unroll
      for (int q = 0; q < BATCH; ++q)
        if (i0 + q * int(blockDim.x) < nb) best_merge(b, x[q]);
    }
  }
  const Best r = block_best(b, S->bb);
  if (threadIdx.x == 0) {
    Winner o;
    const bool valid = r.f != 0xffffffffu;  // false only if every value was NaN
    o.m = valid ? int32_t(r.f / uint32_t(N)) : 0;
    o.j = valid ? int32_t(r.f % uint32_t(N)) : 0;
    o.kcount = 0;
    o.flags = 0;
    o.ax = o.ay = 0.0;
    o.cx = valid ? r.vx : 0.0;
    o.cy = valid ? r.vy : 0.0;
    o.margin = !valid ? __builtin_nan("") : r.p1 > 0.0 ? (r.p1 - r.p2) / r.p1 : 0.0;
    o.fp32err = 0.0;
    *w = o;
  }
}

// FP32: short-list for the double re-check.  Every listed point within
// tau_band of the FP32 maximum, sorted by key and cut at kKMax; if that is
// fewer than recheck_k points, the head keys (best points) of the best blocks
// below the band are appended until it is not.  Each block's head key is in
// the dense array `heads` (0: no finite point), so one coalesced pass finds
// the maximum, the band blocks and the top-up candidates.  A flat grid (more
// band points or band blocks than the gather holds) falls back to an exact
// pop-merge of the sorted per-block lists.  `flagword` collects the blocks'
// fallback flag for the step; it is read here, and cleared unless several
// workgroups merge the same records (then the caller clears it once all
// have read it).  The result depends only on the records, not on the
// workgroup size or on scheduling.  BATCH: head keys per thread, and band
// lists per wave, fetched per round trip after the first.
template <int PRE = 2, int BATCH = 1>
__device__ __forceinline__ void select32_tail(const BlockList32* __restrict__ lists,
                                              const uint64_t* __restrict__ heads,
                                              const uint64_t* __restrict__ seconds, int nb, int recheck_k,
                                              float tau_band, unsigned int* flagword, CandList* __restrict__ cand,
                                              MergeScratch* S, bool clear_flag = true) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = nwaves();
  // the head keys, staged in LDS when they fit (otherwise re-read from
  // memory), and in the same round trip the second keys
  const bool fits = nb <= kHeadCap;
  const bool use2 = seconds != nullptr && nb <= kSecondCap;
  uint64_t mx = 0;
  {
    // the first PRE keys of each thread in one round trip (clamped
    // addresses, no branches between the loads)
    uint64_t hk[PRE], sk[PRE];
#pragma unroll
    for (int i = 0; i < PRE; ++i) {
      const int b = tid + i * int(blockDim.x);
      const int bc = b < nb ? b : nb - 1;
      hk[i] = ld_agent(heads + bc);
      sk[i] = use2 ? ld_agent(seconds + bc) : 0;
    }
#pragma unroll
    for (int i = 0; i < PRE; ++i) {
      const int b = tid + i * int(blockDim.x);
      if (b < nb) {
        if (use2) S->seconds[b] = sk[i];
        if (fits) S->heads[b] = hk[i];
        mx = hk[i] > mx ? hk[i] : mx;
      }
    }
  }
  if constexpr (BATCH == 1) {
    for (int b = tid + PRE * int(blockDim.x); b < nb; b += blockDim.x) {
      const uint64_t k = ld_agent(heads + b);
      if (use2) S->seconds[b] = ld_agent(seconds + b);
      if (fits) S->heads[b] = k;
      mx = k > mx ? k : mx;
    }
  } else {
    for (int b0 = tid + PRE * int(blockDim.x); b0 < nb; b0 += BATCH * int(blockDim.x)) {
      uint64_t hk[BATCH], sk[BATCH];
#pragma unroll
      for (int i = 0; i < BATCH; ++i) {
        const int b = b0 + i * int(blockDim.x);
        const int bc = b < nb ? b : nb - 1;
        hk[i] = ld_agent(heads + bc);
        sk[i] = use2 ? ld_agent(seconds + bc) : 0;
      }
#pragma unroll
      for (int i = 0; i < BATCH; ++i) {
        const int b = b0 + i * int(blockDim.x);
        if (b < nb) {
          if (use2) S->seconds[b] = sk[i];
          if (fits) S->heads[b] = hk[i];
          mx = hk[i] > mx ? hk[i] : mx;
        }
      }
    }
  }
  if (tid == 0) {
    S->sflags = ld_agent(flagword) & uint32_t(kFlagFallback);
    if (clear_flag) st_agent(flagword, 0u);
    S->scount = 0;
    S->sblocks = 0;
  }
  const uint64_t gk = block_max_u64(mx, S->wb);  // its barriers order the stores above
  const float pg = gk ? key_p(gk) : -1.f;
  const float theta = pg - pg * tau_band;
  auto head_of = [&](int b) { return fits ? S->heads[b] : ld_agent(heads + b); };
  // blocks whose head reaches the band: a block whose second key is below
  // the band contributes its head alone (its list is not read)
  for (int b0 = 0; b0 < nb; b0 += blockDim.x) {
    const int b = b0 + tid;
    const uint64_t k = b < nb ? head_of(b) : 0;
    const bool inb = k != 0 && key_p(k) >= theta;
    const bool alone = inb && use2 && key_p(S->seconds[b]) < theta;
    wave_append(alone, k, &S->scount, S->buf, uint32_t(kSelCap));
    const bool q = inb && !alone;
    const uint64_t mask = __ballot(q);
    if (mask) {
      const int leader = __ffsll(static_cast<long long>(mask)) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&S->sblocks, uint32_t(__popcll(mask)));
      base = lane_u32(base, leader);
      if (q) {
        const uint32_t pos = base + uint32_t(__popcll(mask & ((uint64_t(1) << lane) - 1)));
        if (pos < uint32_t(kSelCap)) S->cblk[pos] = uint32_t(b);
      }
    }
  }
  __syncthreads();
  const uint32_t nbb = S->sblocks;
  const uint32_t ncb = nbb < uint32_t(kSelCap) ? nbb : uint32_t(kSelCap);
  // one wave per band block: its count, total and all kListC key slots in
  // one round trip (slots at or beyond the count are masked); BATCH blocks
  // per wave and round trip
  auto band_list = [&](uint32_t cnt, uint32_t tot, uint64_t k) {
    const bool q = lane < int(cnt) && key_p(k) >= theta;
    wave_append(q, k, &S->scount, S->buf, uint32_t(kSelCap));
    // the list was cut inside the band: its last listed key is still in it
    if (cnt > 0 && cnt <= uint32_t(kListC) && tot > cnt) {
      const uint64_t klast = lane_u64(k, int(cnt) - 1);
      if (lane == 0 && key_p(klast) >= theta) atomicOr(&S->sflags, uint32_t(kFlagListTruncated));
    }
  };
  if constexpr (BATCH == 1) {
    for (uint32_t i = wave; i < ncb; i += nw) {
      const BlockList32* L = lists + S->cblk[i];
      const uint32_t cnt = uint32_t(__builtin_amdgcn_readfirstlane(int(ld_agent(&L->count))));
      const uint32_t tot = uint32_t(__builtin_amdgcn_readfirstlane(int(ld_agent(&L->total))));
      band_list(cnt, tot, ld_agent(&L->keys[lane]));
    }
  } else {
    for (uint32_t i0 = wave; i0 < ncb; i0 += uint32_t(nw) * BATCH) {
      uint32_t cnt[BATCH], tot[BATCH];
      uint64_t k[BATCH];
#pragma unroll
      for (int q = 0; q < BATCH; ++q) {
        const uint32_t i = i0 + uint32_t(q * nw);
        const BlockList32* L = lists + S->cblk[i < ncb ? i : i0];
        cnt[q] = uint32_t(__builtin_amdgcn_readfirstlane(int(ld_agent(&L->count))));
        tot[q] = uint32_t(__builtin_amdgcn_readfirstlane(int(ld_agent(&L->total))));
        k[q] = ld_agent(&L->keys[lane]);
      }
#pragma unroll
      for (int q = 0; q < BATCH; ++q)
        if (i0 + uint32_t(q * nw) < ncb) band_list(cnt[q], tot[q], k[q]);
    }
  }
  __syncthreads();
  const uint32_t band = S->scount;

  if (band <= uint32_t(kSelCap) && nbb <= uint32_t(kSelCap)) {
    top_desc(S->buf, band, cand->keys, uint32_t(kKMax));
    uint32_t keff = band < uint32_t(kKMax) ? band : uint32_t(kKMax);
    if (band > uint32_t(kKMax) && tid == 0) atomicOr(&S->sflags, uint32_t(kFlagBandTruncated));
    if (keff < uint32_t(recheck_k)) {
      const uint32_t need = uint32_t(recheck_k) - keff;  // <= 63
      if (fits) {
        // each wave: the top `need` heads below the band among its lanes'
        // heads (b = tid + i blockDim), by rounds of a wave maximum (no
        // workgroup barrier); the first HR heads of a lane stay in registers
        constexpr int HR = 4;
        uint64_t h[HR];
#pragma unroll
        for (int i = 0; i < HR; ++i) {
          const int b = tid + i * int(blockDim.x);
          h[i] = b < nb ? S->heads[b] : 0;
          if (h[i] != 0 && key_p(h[i]) >= theta) h[i] = 0;
        }
        const bool more = nb > HR * int(blockDim.x);
        uint64_t* wl = S->buf;  // free after top_desc: [nw][need]
        for (uint32_t r = 0; r < need; ++r) {
          uint64_t lm = 0;
#pragma unroll
          for (int i = 0; i < HR; ++i) lm = h[i] > lm ? h[i] : lm;
          if (more) {
            for (int b = tid + HR * int(blockDim.x); b < nb; b += blockDim.x) {
              const uint64_t k = S->heads[b];
              if (k != 0 && key_p(k) < theta && k > lm) lm = k;
            }
          }
          const uint64_t w = wave_max_u64(lm);
          if (lane == 0) wl[uint32_t(wave) * need + r] = w;
          // keys are distinct: one lane owns w
#pragma unroll
          for (int i = 0; i < HR; ++i)
            if (h[i] == w) h[i] = 0;
          if (more && lm == w && w != 0) {
            for (int b = tid + HR * int(blockDim.x); b < nb; b += blockDim.x)
              if (S->heads[b] == w) S->heads[b] = 0;
          }
        }
        __syncthreads();
        // ... then the top `need` of the waves' candidates by rank
        const uint32_t nc = uint32_t(nw) * need;
        uint32_t nz = 0;
        if (PRE >= 4 && nc <= 64) {
          // wave 0, one candidate per lane, ranked against the others in
          // registers (kept out of the 128-register transform kernels)
          if (wave == 0) {
            const uint64_t k = uint32_t(lane) < nc ? wl[lane] : 0;
            uint32_t rank = 0;
            for (uint32_t j = 0; j < nc; ++j) rank += lane_u64(k, int(j)) > k ? 1u : 0u;
            if (k && rank < need) cand->keys[keff + rank] = k;
            // (the band count in scount was read by every thread before the rounds)
            const uint32_t cnt = uint32_t(__popcll(__ballot(k != 0)));
            if (lane == 0) S->scount = cnt;
          }
          __syncthreads();
          nz = S->scount;
        } else {
          for (uint32_t i = tid; i < nc; i += blockDim.x) {
            const uint64_t k = wl[i];
            if (k) {
              uint32_t rank = 0;
              for (uint32_t j = 0; j < nc; ++j) rank += wl[j] > k ? 1u : 0u;
              if (rank < need) cand->keys[keff + rank] = k;
            }
          }
          for (uint32_t j = tid; j < nc; j += blockDim.x) nz += wl[j] ? 1u : 0u;
          nz = block_reduce_u32<true>(nz, reinterpret_cast<uint32_t*>(S->wf));
        }
        keff += nz < need ? nz : need;
      } else {
        // many blocks: rounds of a workgroup maximum over all heads below the band
        uint64_t last_taken = ~uint64_t(0);
        for (uint32_t r = 0; r < need; ++r) {
          uint64_t tb = 0;
          for (int b = tid; b < nb; b += blockDim.x) {
            const uint64_t k = ld_agent(heads + b);
            if (k != 0 && key_p(k) < theta && k < last_taken && k > tb) tb = k;
          }
          const uint64_t g = block_max_u64(tb, S->wb);
          if (g == 0) break;
          if (tid == 0) cand->keys[keff] = g;
          ++keff;
          last_taken = g;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      cand->count = int32_t(keff);
      cand->flags = int32_t(S->sflags);
      cand->pmax32 = pg;
    }
    return;
  }

  {
    // Exact fallback (flat grids only): pop-merge of the sorted per-block
    // lists.  Each thread keeps the head key and position of up to HC of its
    // lists in registers; lists beyond that are rescanned each round.
    constexpr int HC = 16;
    uint64_t hk[HC];
    uint32_t hp[HC];
#pragma unroll
    for (int i = 0; i < HC; ++i) {
      const int b = tid + i * int(blockDim.x);
      hp[i] = 0;
      hk[i] = (b < nb && ld_agent(&lists[b].count) > 0) ? ld_agent(&lists[b].keys[0]) : 0;
    }
    const bool spill = nb > HC * int(blockDim.x);
    const int want = recheck_k > kListC ? recheck_k : kListC;
    uint64_t last_taken = ~uint64_t(0);
    int r = 0;
    for (; r < want; ++r) {
      uint64_t tb = 0;
#pragma unroll
      for (int i = 0; i < HC; ++i) tb = hk[i] > tb ? hk[i] : tb;
      if (spill) {
        for (int b = tid + HC * int(blockDim.x); b < nb; b += blockDim.x) {
          const uint32_t cnt = ld_agent(&lists[b].count);
          for (uint32_t q = 0; q < cnt; ++q) {
            const uint64_t k = ld_agent(&lists[b].keys[q]);
            if (k < last_taken) {
              if (k > tb) tb = k;
              break;
            }
          }
        }
      }
      const uint64_t g = block_max_u64(tb, S->wb);
      if (g == 0) break;
      if (tid == 0) cand->keys[r] = g;
#pragma unroll
      for (int i = 0; i < HC; ++i) {
        if (hk[i] == g) {
          const int b = tid + i * int(blockDim.x);
          const uint32_t cnt = ld_agent(&lists[b].count);
          ++hp[i];
          hk[i] = hp[i] < cnt ? ld_agent(&lists[b].keys[hp[i]]) : 0;
          if (hp[i] >= cnt && ld_agent(&lists[b].total) > cnt) atomicOr(&S->sflags, uint32_t(kFlagListTruncated));
        }
      }
      last_taken = g;
    }
    __syncthreads();
    if (tid == 0) {
      cand->count = r;
      cand->flags = int32_t(S->sflags | uint32_t(kFlagFallback) | uint32_t(kFlagBandTruncated));
      cand->pmax32 = pg;
    }
  }
}

// ---------------------------------------------------------------- workgroup selection
// LDS scratch of select_list: 512 bytes of counters, then kListCap gathered
// keys and kListC sorted keys.
constexpr size_t kListScratchBytes = 512 + sizeof(uint64_t) * (kListCap + kListC);

// Header of a workgroup list (thread 0; wave 0 stores the keys): also the
// workgroup's head key and second key in the dense arrays read by the grid
// merge (0: none; the second key may exceed the true second, never fall
// below it), and the fallback flag of the step.
__device__ __forceinline__ void list_header(BlockList32* o, uint64_t* head, uint64_t* second, unsigned int* flagword,
                                            float pb, uint32_t count, uint32_t total, uint32_t flags, uint64_t first,
                                            uint64_t next) {
  st_agent(&o->pmax, pb);
  st_agent(&o->count, count);
  st_agent(&o->total, total);
  st_agent(&o->flags, flags);
  if (head) st_agent(head, count > 0 ? first : uint64_t(0));
  if (second) st_agent(second, count > 1 ? next : uint64_t(0));
  if (flags && flagword) __hip_atomic_fetch_or(flagword, flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The flat indices of a workgroup's points in increasing order: rank i is
// first + (i mod na) + (i / na) * step (na consecutive indices, then a jump).
// Used to list the lowest indices of a workgroup whose values all tie.
struct FlatOrder {
  uint32_t first, na, step, count;
  __device__ __forceinline__ uint32_t rank(uint32_t i) const { return first + (i % na) + (i / na) * step; }
};

// Register order of a transform's output: register p of thread t holds bin
// t + TPR * O::bin(p), and O::reg(q) is the register holding bin t + TPR q.
// The power-of-two transforms leave their bins in bit-reversed order.
template <int LE>
struct BitrevOrder {
  static __host__ __device__ constexpr int bin(int p) { return bitrev(p, LE); }
  static __host__ __device__ constexpr int reg(int q) { return bitrev(q, LE); }
};

// FP64 workgroup selection: best point (value, flat index, grid value) and the
// runner-up value.  Within a thread the bins are visited in increasing index
// order, so a strict comparison keeps the lowest index among equal values.
// E values per thread, TPR threads per transform (0: the run-time count
// tpr_rt), output order O.
template <typename T, int E, int TPR, class O>
__device__ __forceinline__ void select_best_o(const Cx<T> (&v)[E], bool active, T sc, uint32_t fbase,
                                              uint32_t fstride, int t, Best* wb, BlockBest64* o, int tpr_rt = TPR) {
  const int tpr = TPR > 0 ? TPR : tpr_rt;
  double y1 = -1.0, y2 = -1.0;
  int i1 = 0;
  T bx = T(0), by = T(0);
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int p = O::reg(q);  // register holding bin t + TPR*q
    const double y = double(fma(v[p].x, v[p].x, v[p].y * v[p].y));
    if (y > y1) {
      y2 = y1;
      y1 = y;
      i1 = p;
      bx = v[p].x;
      by = v[p].y;
    } else {
      y2 = fmax(y2, y);
    }
  }
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  if (active) {
    const double s2 = double(sc) * double(sc);
    b.vx = double(bx * sc);
    b.vy = double(by * sc);
    b.f = fbase + fstride * uint32_t(t + tpr * O::bin(i1));
    // exact |.|^2 of the scaled grid value, as compared across radii
    b.p1 = b.vx * b.vx + b.vy * b.vy;
    b.p2 = fmin(y2 * s2, b.p1);
  }
  const Best r = block_best(b, wb);
  if (threadIdx.x == 0) {
    st_agent(&o->p1, r.p1);
    st_agent(&o->p2, r.p2);
    st_agent(&o->vx, r.vx);
    st_agent(&o->vy, r.vy);
    st_agent(&o->f, r.f);
  }
}

// The same for the power-of-two transforms.  (A copy of the loop rather
// than a call of select_best_o: through the extra inlining level the 2^14-point
// double-precision radius kernel needs 59 more VGPRs.)
template <int LOGN, typename T>
__device__ __forceinline__ void select_best(const Cx<T> (&v)[pickE<T, LOGN>()], bool active, T sc, uint32_t fbase,
                                            uint32_t fstride, int t, Best* wb, BlockBest64* o) {
  constexpr int E = pickE<T, LOGN>();
  constexpr int LE = ilog2c(E);
  double y1 = -1.0, y2 = -1.0;
  int i1 = 0;
  T bx = T(0), by = T(0);
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int p = bitrev(q, LE);  // register holding bin t + TPR*q
    const double y = double(fma(v[p].x, v[p].x, v[p].y * v[p].y));
    if (y > y1) {
      y2 = y1;
      y1 = y;
      i1 = p;
      bx = v[p].x;
      by = v[p].y;
    } else {
      y2 = fmax(y2, y);
    }
  }
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  if (active) {
    const double s2 = double(sc) * double(sc);
    b.vx = double(bx * sc);
    b.vy = double(by * sc);
    b.f = fbase + fstride * uint32_t(t + Shape<LOGN, E>::TPR * bitrev(i1, LE));
    // exact |.|^2 of the scaled grid value, as compared across radii
    b.p1 = b.vx * b.vx + b.vy * b.vy;
    b.p2 = fmin(y2 * s2, b.p1);
  }
  const Best r = block_best(b, wb);
  if (threadIdx.x == 0) {
    st_agent(&o->p1, r.p1);
    st_agent(&o->p2, r.p2);
    st_agent(&o->vx, r.vx);
    st_agent(&o->vy, r.vy);
    st_agent(&o->f, r.f);
  }
}

// The per-thread part of select_best, returned instead of reduced: for a
// thread that selects over several transforms (rows) in turn and merges
// them (best_merge) before the workgroup reduction.  (select_best keeps its
// own copy of the loop: written through this function it needs 13 more
// VGPRs in the 2^14-point double-precision radius kernel.)
template <int LOGN, typename T>
__device__ __forceinline__ Best thread_best(const Cx<T> (&v)[pickE<T, LOGN>()], T sc, uint32_t fbase,
                                            uint32_t fstride, int t) {
  constexpr int E = pickE<T, LOGN>();
  constexpr int LE = ilog2c(E);
  double y1 = -1.0, y2 = -1.0;
  int i1 = 0;
  T bx = T(0), by = T(0);
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int p = bitrev(q, LE);  // register holding bin t + TPR*q
    const double y = double(fma(v[p].x, v[p].x, v[p].y * v[p].y));
    if (y > y1) {
      y2 = y1;
      y1 = y;
      i1 = p;
      bx = v[p].x;
      by = v[p].y;
    } else {
      y2 = fmax(y2, y);
    }
  }
  Best b;
  const double s2 = double(sc) * double(sc);
  b.vx = double(bx * sc);
  b.vy = double(by * sc);
  b.f = fbase + fstride * uint32_t(t + Shape<LOGN, E>::TPR * bitrev(i1, LE));
  b.p1 = b.vx * b.vx + b.vy * b.vy;
  b.p2 = fmin(y2 * s2, b.p1);
  return b;
}

// Thread 0 stores the workgroup's best and runner-up of the threads' b.
__device__ __forceinline__ void store_block_best(const Best& b, Best* wb, BlockBest64* o) {
  const Best r = block_best(b, wb);
  if (threadIdx.x == 0) {
    st_agent(&o->p1, r.p1);
    st_agent(&o->p2, r.p2);
    st_agent(&o->vx, r.vx);
    st_agent(&o->vy, r.vy);
    st_agent(&o->f, r.f);
  }
}

// FP32 workgroup list: the workgroup's points within tau_band of its
// maximum, best first, at most kListC of them (exact top by key).  Points
// are compared unscaled (|y|^2 against the threshold divided by s_m^2) and
// keys are formed only for points that pass.
template <int E, int TPR, class O>
__device__ __forceinline__ void select_list_o(const Cx<float> (&v)[E], bool active, float sc, uint32_t fbase,
                                              uint32_t fstride, int t, unsigned char* scratch, float tau_band,
                                              const FlatOrder& ord, BlockList32* o, uint64_t* head,
                                              uint64_t* second, unsigned int* flagword, int tpr_rt = TPR) {
  static_assert(E <= 32, "the taken mask holds one bit per register");
  const int tpr = TPR > 0 ? TPR : tpr_rt;
  const float s2 = sc * sc;
  float Y[E];
  float ym = 0.f;
#pragma unroll
  for (int p = 0; p < E; ++p) {
    Y[p] = fmaf(v[p].x, v[p].x, v[p].y * v[p].y);
    ym = fmaxf(ym, Y[p]);
  }
  float pm = active ? ym * s2 : -1.f;
  pm = wave_max_f32(pm);
  float* wmax = reinterpret_cast<float*>(scratch);               // [16]
  float* wmin = reinterpret_cast<float*>(scratch + 64);          // [16]
  uint32_t* cnt = reinterpret_cast<uint32_t*>(scratch + 128);    // [1]
  uint64_t* wbest = reinterpret_cast<uint64_t*>(scratch + 256);  // [16]
  uint64_t* keys = reinterpret_cast<uint64_t*>(scratch + 512);   // [kListCap]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = nwaves();
  if (lane == 0) wmax[wave] = pm;
  if (tid == 0) *cnt = 0;
  __syncthreads();
  float pb = wmax[0];
  for (int w = 1; w < nw; ++w) pb = fmaxf(pb, wmax[w]);

  const float theta = pb - pb * tau_band;
  // per-thread unscaled threshold; inactive threads never pass
  const float ty = active ? (s2 > 0.f ? theta / s2 : 3.4e38f) : 3.4e38f;
#pragma unroll
  for (int p = 0; p < E; ++p) {
    const bool q = Y[p] >= ty;
    const uint64_t mask = __ballot(q);
    if (mask) {
      const int leader = __ffsll(static_cast<long long>(mask)) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(cnt, uint32_t(__popcll(mask)));
      base = lane_u32(base, leader);
      if (q) {
        const uint32_t pos = base + uint32_t(__popcll(mask & ((uint64_t(1) << lane) - 1)));
        if (pos < uint32_t(kListCap)) keys[pos] = key32(Y[p] * s2, fbase + fstride * uint32_t(t + tpr * O::bin(p)));
      }
    }
  }
  __syncthreads();
  const uint32_t n = *cnt;

  if (n <= uint32_t(kListCap)) {
    // the sorted top keys are staged in LDS and stored by wave 0
    uint64_t* sorted = reinterpret_cast<uint64_t*>(scratch + 512 + sizeof(uint64_t) * kListCap);
    top_desc(keys, n, sorted, uint32_t(kListC));
    wave0_copy_keys(sorted, o->keys, n < uint32_t(kListC) ? n : uint32_t(kListC));
    if (tid == 0)
      list_header(o, head, second, flagword, pb, n < uint32_t(kListC) ? n : uint32_t(kListC), n, 0u, sorted[0],
                  sorted[1]);
    return;
  }

  // More than kListCap points in the band.  If every value is exactly equal
  // (e.g. the r = 0 ring) the best keys are the lowest flat indices.
  // Otherwise the top kListC keys are the top keys among the points whose P
  // reaches t, the largest P with at least kListC band points at or above it
  // (bisection on the bits of P >= 0); only if exact ties at t still leave
  // more than kListCap such points, kListC rounds of exact workgroup argmax.
  float pn = 3.4e38f;
  if (active) {
#pragma unroll
    for (int p = 0; p < E; ++p) pn = fminf(pn, Y[p] * s2);
  }
  pn = wave_min_f32(pn);
  if (lane == 0) wmin[wave] = pn;
  __syncthreads();
  float pbn = wmin[0];
  for (int w = 1; w < nw; ++w) pbn = fminf(pbn, wmin[w]);
  if (pb == pbn) {
    const uint32_t c = ord.count < uint32_t(kListC) ? ord.count : uint32_t(kListC);
    if (uint32_t(tid) < c) st_agent(&o->keys[tid], key32(pb, ord.rank(uint32_t(tid))));  // wave 0 (c <= 64)
    if (tid == 0)
      list_header(o, head, second, flagword, pb, c, ord.count, uint32_t(kFlagFallback), key32(pb, ord.rank(0)),
                  key32(pb, ord.rank(1)));
    return;
  }
  {
    // Y becomes P = Y s2 for the band points and 0 elsewhere (P >= 0: the
    // order of P is the order of its bits)
    uint32_t pmin = 0xffffffffu;
#pragma unroll
    for (int p = 0; p < E; ++p) {
      const bool in = active && Y[p] >= ty;
      Y[p] = in ? Y[p] * s2 : 0.f;
      if (in) pmin = min(pmin, __float_as_uint(Y[p]));
    }
    uint32_t* wred = reinterpret_cast<uint32_t*>(wmin);
    __syncthreads();  // every thread has read wmin above
    uint32_t lo = block_reduce_u32<false>(pmin, wred);
    uint32_t hi = __float_as_uint(pb);
    while (lo < hi) {  // uniform: lo and hi come from block reductions
      const uint32_t mid = lo + (hi - lo + 1) / 2;
      const float fm = __uint_as_float(mid);
      uint32_t c = 0;
#pragma unroll
      for (int p = 0; p < E; ++p) c += Y[p] >= fm ? 1u : 0u;
      if (block_reduce_u32<true>(c, wred) >= uint32_t(kListC))
        lo = mid;
      else
        hi = mid - 1;
    }
    const float fl = __uint_as_float(lo);  // > 0: excludes the points outside the band
    if (tid == 0) *cnt = 0;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < E; ++p) {
      const bool q = Y[p] >= fl;
      const uint64_t k = q ? key32(Y[p], fbase + fstride * uint32_t(t + tpr * O::bin(p))) : 0;
      wave_append(q, k, cnt, keys, uint32_t(kListCap));
    }
    __syncthreads();
    const uint32_t n2 = *cnt;
    if (n2 <= uint32_t(kListCap)) {
      uint64_t* sorted = reinterpret_cast<uint64_t*>(scratch + 512 + sizeof(uint64_t) * kListCap);
      top_desc(keys, n2, sorted, uint32_t(kListC));
      const uint32_t c = n2 < uint32_t(kListC) ? n2 : uint32_t(kListC);
      wave0_copy_keys(sorted, o->keys, c);
      if (tid == 0) list_header(o, head, second, flagword, pb, c, n, uint32_t(kFlagFallback), sorted[0], sorted[1]);
      return;
    }
  }
  uint32_t taken = 0;
  uint32_t rounds = 0;
  uint64_t first = 0, next = 0;
  for (; rounds < uint32_t(kListC); ++rounds) {
    uint64_t tb = 0;
#pragma unroll
    for (int p = 0; p < E; ++p) {
      if (!((taken >> p) & 1u) && Y[p] > 0.f) {
        const uint64_t k = key32(Y[p], fbase + fstride * uint32_t(t + tpr * O::bin(p)));
        tb = k > tb ? k : tb;
      }
    }
    const uint64_t b = block_max_u64(tb, wbest);
    if (b == 0) break;
    if (rounds == 0) first = b;
    if (rounds == 1) next = b;
    if (tid == 0) st_agent(&o->keys[rounds], b);
#pragma unroll
    for (int p = 0; p < E; ++p) {
      if (Y[p] > 0.f && key32(Y[p], fbase + fstride * uint32_t(t + tpr * O::bin(p))) == b) taken |= 1u << p;
    }
  }
  if (tid == 0) list_header(o, head, second, flagword, pb, rounds, n, uint32_t(kFlagFallback), first, next);
}

template <int LOGN>
__device__ __forceinline__ void select_list(const Cx<float> (&v)[pickE<float, LOGN>()], bool active, float sc,
                                            uint32_t fbase, uint32_t fstride, int t, unsigned char* scratch,
                                            float tau_band, const FlatOrder& ord, BlockList32* o, uint64_t* head,
                                            uint64_t* second, unsigned int* flagword) {
  constexpr int E = pickE<float, LOGN>();
  select_list_o<E, Shape<LOGN, E>::TPR, BitrevOrder<ilog2c(E)>>(v, active, sc, fbase, fstride, t, scratch, tau_band,
                                                                ord, o, head, second, flagword);
}

}  // namespace afd
