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

__device__ __forceinline__ Best best_shfl(const Best& a, int m) {
  Best o;
  o.p1 = __shfl_xor(a.p1, m);
  o.p2 = __shfl_xor(a.p2, m);
  o.vx = __shfl_xor(a.vx, m);
  o.vy = __shfl_xor(a.vy, m);
  o.f = __shfl_xor(a.f, m);
  return o;
}

__device__ __forceinline__ int nwaves() { return int((blockDim.x + 63) >> 6); }

// Block-wide results, returned to every thread.  `w*` are LDS arrays of 16.
__device__ __forceinline__ Best block_best(Best b, Best* wb) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) best_merge(b, best_shfl(b, m));
  if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = b;
  __syncthreads();
  Best r = wb[0];
  for (int w = 1; w < nwaves(); ++w) best_merge(r, wb[w]);
  __syncthreads();
  return r;
}

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

__device__ __forceinline__ double block_sum_f64(double v, double* wd) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
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
  base = __shfl(base, leader);
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
__device__ __forceinline__ bool last_workgroup(unsigned int* counter, int* flag) {
  __syncthreads();
  if (threadIdx.x < 64) {
    __builtin_amdgcn_s_waitcnt(0);
    if (threadIdx.x == 0) {
      const unsigned int total = gridDim.x * gridDim.y * gridDim.z;
      const unsigned int prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int last = prev == total - 1;
      if (last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *flag = last;
    }
  }
  __syncthreads();
  return *flag != 0;
}

__device__ __forceinline__ void wave0_copy_keys(const uint64_t* src, uint64_t* dst, uint32_t n) {
  if (threadIdx.x < n) st_agent(dst + threadIdx.x, src[threadIdx.x]);
}

// LDS layout used by the grid-level merges (placed in a kernel's dynamic LDS).
struct MergeScratch {
  uint64_t buf[kSelCap];
  uint32_t cblk[kSelCap];
  uint64_t wb[16];
  Best bb[16];
  float wf[16];
  double wd[16];
  uint32_t scount, sblocks, sflags;
  int last;
};

// FP64: global best of the per-block records -> winner (coefficient = the
// grid value of the FFT form).
__device__ __forceinline__ void merge64_tail(const BlockBest64* __restrict__ blocks, int nb, int N, int logn,
                                             Winner* __restrict__ w, MergeScratch* S) {
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const BlockBest64* o = blocks + i;
    const Best x{ld_agent(&o->p1), ld_agent(&o->p2), ld_agent(&o->vx), ld_agent(&o->vy), ld_agent(&o->f)};
    best_merge(b, x);
  }
  const Best r = block_best(b, S->bb);
  if (threadIdx.x == 0) {
    Winner o;
    const bool valid = r.f != 0xffffffffu;  // false only if every value was NaN
    o.m = valid ? int32_t(r.f >> logn) : 0;
    o.j = valid ? int32_t(r.f & uint32_t(N - 1)) : 0;
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
// fewer than recheck_k points, the best points of the next-best blocks
// (maxima below the band) are appended until it is not.  A flat grid (more
// band points or band blocks than the gather holds) falls back to an exact
// pop-merge of the sorted per-block lists.
__device__ __forceinline__ void select32_tail(const BlockList32* __restrict__ lists, int nb, int recheck_k,
                                              float tau_band, CandList* __restrict__ cand, MergeScratch* S) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = nwaves();
  float pm = -1.f;
  uint32_t fl = 0;
  for (int b = tid; b < nb; b += blockDim.x) {
    fl |= ld_agent(&lists[b].flags);
    if (ld_agent(&lists[b].count) > 0) pm = fmaxf(pm, ld_agent(&lists[b].pmax));
  }
  if (tid == 0) {
    S->sflags = 0;
    S->scount = 0;
    S->sblocks = 0;
  }
  const float pg = block_max_f32(pm, S->wf);  // its barriers order the initialisation above
  if (fl) atomicOr(&S->sflags, fl & uint32_t(kFlagFallback));
  const float theta = pg - pg * tau_band;
  // blocks whose maximum reaches the band
  for (int b0 = 0; b0 < nb; b0 += blockDim.x) {
    const int b = b0 + tid;
    const bool q = b < nb && ld_agent(&lists[b].count) > 0 && ld_agent(&lists[b].pmax) >= theta;
    const uint64_t mask = __ballot(q);
    if (mask) {
      const int leader = __ffsll(static_cast<long long>(mask)) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&S->sblocks, uint32_t(__popcll(mask)));
      base = __shfl(base, leader);
      if (q) {
        const uint32_t pos = base + uint32_t(__popcll(mask & ((uint64_t(1) << lane) - 1)));
        if (pos < uint32_t(kSelCap)) S->cblk[pos] = uint32_t(b);
      }
    }
  }
  __syncthreads();
  const uint32_t nbb = S->sblocks;
  const uint32_t ncb = nbb < uint32_t(kSelCap) ? nbb : uint32_t(kSelCap);
  // one wave per band block: one coalesced load of its (at most 64) keys
  for (uint32_t i = wave; i < ncb; i += nw) {
    const BlockList32* L = lists + S->cblk[i];
    const uint32_t cnt = ld_agent(&L->count);
    const uint64_t k = lane < int(cnt) ? ld_agent(&L->keys[lane]) : 0;
    const bool q = lane < int(cnt) && key_p(k) >= theta;
    wave_append(q, k, &S->scount, S->buf, uint32_t(kSelCap));
    if (lane == 0 && cnt > 0 && ld_agent(&L->total) > cnt && key_p(ld_agent(&L->keys[cnt - 1])) >= theta)
      atomicOr(&S->sflags, uint32_t(kFlagListTruncated));
  }
  __syncthreads();
  const uint32_t band = S->scount;

  if (band <= uint32_t(kSelCap) && nbb <= uint32_t(kSelCap)) {
    top_desc(S->buf, band, cand->keys, uint32_t(kKMax));
    uint32_t keff = band < uint32_t(kKMax) ? band : uint32_t(kKMax);
    if (band > uint32_t(kKMax) && tid == 0) atomicOr(&S->sflags, uint32_t(kFlagBandTruncated));
    if (keff < uint32_t(recheck_k)) {
      // top up with the maxima of the blocks below the band; each thread keeps
      // the heads of its blocks in registers (re-read for more than 16 blocks)
      constexpr int HC = 16;
      uint64_t head[HC];
      uint32_t popped = 0;
#pragma unroll
      for (int i = 0; i < HC; ++i) {
        const int b = tid + i * int(blockDim.x);
        head[i] = (b < nb && ld_agent(&lists[b].count) > 0 && ld_agent(&lists[b].pmax) < theta) ? ld_agent(&lists[b].keys[0]) : 0;
      }
      const bool spill = nb > HC * int(blockDim.x);
      uint32_t need = uint32_t(recheck_k) - keff;
      uint64_t last_taken = ~uint64_t(0);
      for (uint32_t r = 0; r < need; ++r) {
        uint64_t tb = 0;
#pragma unroll
        for (int i = 0; i < HC; ++i)
          if (!((popped >> i) & 1u) && head[i] > tb) tb = head[i];
        if (spill) {
          for (int b = tid + HC * int(blockDim.x); b < nb; b += blockDim.x) {
            if (ld_agent(&lists[b].count) > 0 && ld_agent(&lists[b].pmax) < theta) {
              const uint64_t k = ld_agent(&lists[b].keys[0]);
              if (k < last_taken && k > tb) tb = k;
            }
          }
        }
        const uint64_t g = block_max_u64(tb, S->wb);
        if (g == 0) break;
        if (tid == 0) cand->keys[keff] = g;
        ++keff;
#pragma unroll
        for (int i = 0; i < HC; ++i)
          if (head[i] == g) popped |= 1u << i;
        last_taken = g;  // keys are distinct: later rounds take strictly smaller keys
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

}  // namespace afd
