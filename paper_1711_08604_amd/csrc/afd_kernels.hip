// Kernels of the FFT-based Core-AFD maximal-selection loop for gfx950.
//
// Per step k (Sec. 3.2, Steps 1-2, and Sec. 2, eqs. (3), (7)):
//   k_fft_fwd   c = DFT(G_k)                                  (Sec. 3.1, eq. term4)
//   k_radius    per radius m: y = IDFT+(c_l r_m^l), V = s_m y, |V|^2,
//               block-level selection                         (Sec. 3.1, eq. rcl; Thm 2.1)
//   k_merge64   FP64: global maximum, lowest flat index on ties (eq. ak; Step 2)
//   k_select32  FP32: short-list of the best candidates over all radii
//   k_recheck   FP64 direct rule for each short-listed point     (Sec. 3.1, eq. term81)
//   k_finalize  winner, coefficient and margin from the FP64 values
//   k_update    G_{k+1} = (G_k - c_k e_{a_k}) (1 - conj(a_k) z)/(z - a_k) (eq. (7))
//   k_record    E_k = (1/N) sum |G_{k+1}|^2 and the step's outputs
#include "afd_device.h"
#include "afd_internal.h"

#include <math.h>

namespace afd {

// ---------------------------------------------------------------- geometry
template <int LOGN>
__host__ __device__ constexpr int pickE() {
  return (1 << LOGN) < 16 ? (1 << LOGN) : 16;
}
template <int LOGN>
__host__ __device__ constexpr bool pickSplit() {
  return LOGN >= 14;
}

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

template <typename T, int LOGN>
__host__ __device__ constexpr size_t fft_region_bytes() {
  using S = Shape<LOGN, pickE<LOGN>()>;
  return align16(size_t(S::LDS_ELEMS) * (pickSplit<LOGN>() ? sizeof(T) : sizeof(Cx<T>)));
}

constexpr size_t kScratchBytes = 512 + sizeof(uint64_t) * kListCap;

// ---------------------------------------------------------------- forward DFT (one workgroup)
template <int LOGN>
__host__ __device__ constexpr int fwd_threads() {
  return Shape<LOGN, pickE<LOGN>()>::TPR;
}
template <int LOGN>
__host__ __device__ constexpr int radius_threads() {
  return Shape<LOGN, pickE<LOGN>()>::TPR < 64 ? 64 : Shape<LOGN, pickE<LOGN>()>::TPR;
}

template <typename T, int LOGN>
__global__ __launch_bounds__(fwd_threads<LOGN>()) void k_fft_fwd(const Cx<T>* __restrict__ g, const Cx<T>* __restrict__ tw,
                                                  Cx<T>* __restrict__ c) {
  constexpr int E = pickE<LOGN>();
  using S = Shape<LOGN, E>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  Cx<T> v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = g[t + S::TPR * i];
  fft_regs<T, LOGN, E, -1, pickSplit<LOGN>()>(v, t, smem, tw);
#pragma unroll
  for (int p = 0; p < E; ++p) c[out_bin<LOGN, E>(t, p)] = v[p];
}

// ---------------------------------------------------------------- radius kernel
// FP64 selection inside a block: best (value, flat index, grid value) and the
// runner-up value.
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

template <int LOGN, typename T>
__device__ __forceinline__ void select_best(const Cx<T> (&v)[pickE<LOGN>()], bool active, T sc, uint32_t fbase,
                                            int t, unsigned char* scratch, BlockBest64* out) {
  constexpr int E = pickE<LOGN>();
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  if (active) {
#pragma unroll
    for (int p = 0; p < E; ++p) {
      const double vx = double(v[p].x * sc), vy = double(v[p].y * sc);
      const double P = vx * vx + vy * vy;
      const uint32_t f = fbase + uint32_t(out_bin<LOGN, E>(t, p));
      if (better64(P, f, b.p1, b.f)) {
        b.p2 = fmax(b.p2, b.p1);
        b.p1 = P;
        b.f = f;
        b.vx = vx;
        b.vy = vy;
      } else {
        b.p2 = fmax(b.p2, P);
      }
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) best_merge(b, best_shfl(b, m));
  Best* wb = reinterpret_cast<Best*>(scratch);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wb[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    Best r = wb[0];
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 1; w < nw; ++w) best_merge(r, wb[w]);
    BlockBest64 o;
    o.p1 = r.p1;
    o.p2 = r.p2;
    o.vx = r.vx;
    o.vy = r.vy;
    o.f = r.f;
    o.pad = 0;
    out[blockIdx.x] = o;
  }
}

// Descending bitonic sort of buf[0..n) in LDS (n <= p2 <= kListCap, padded with 0).
__device__ __forceinline__ void lds_sort_desc(uint64_t* buf, uint32_t n) {
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
}

// Append key k of every lane with q set to buf (wave-aggregated: one LDS
// atomic per wave); entries past cap are counted but dropped.
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

// FP32 block list: the block's points within tau_band of the block maximum,
// best first, at most kListC of them (exact top by key).
template <int LOGN>
__device__ __forceinline__ void select_list(const Cx<float> (&v)[pickE<LOGN>()], bool active, float sc,
                                            uint32_t fbase, int t, unsigned char* scratch, float tau_band,
                                            uint32_t fstart, uint32_t nactive, BlockList32* out) {
  constexpr int E = pickE<LOGN>();
  float P[E];
  float pm = -1.f, pn = 3.4e38f;
#pragma unroll
  for (int p = 0; p < E; ++p) {
    const float vx = v[p].x * sc, vy = v[p].y * sc;
    P[p] = active ? fmaf(vx, vx, vy * vy) : -1.f;
    pm = fmaxf(pm, P[p]);
    if (active) pn = fminf(pn, P[p]);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    pm = fmaxf(pm, __shfl_xor(pm, m));
    pn = fminf(pn, __shfl_xor(pn, m));
  }
  float* wmax = reinterpret_cast<float*>(scratch);                 // [16]
  float* wmin = reinterpret_cast<float*>(scratch + 64);            // [16]
  uint32_t* cnt = reinterpret_cast<uint32_t*>(scratch + 128);      // [1]
  uint64_t* wbest = reinterpret_cast<uint64_t*>(scratch + 256);    // [16]
  uint64_t* keys = reinterpret_cast<uint64_t*>(scratch + 512);     // [kListCap]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  if (lane == 0) {
    wmax[wave] = pm;
    wmin[wave] = pn;
  }
  if (tid == 0) *cnt = 0;
  __syncthreads();
  float pb = wmax[0], pbn = wmin[0];
  for (int w = 1; w < nw; ++w) {
    pb = fmaxf(pb, wmax[w]);
    pbn = fminf(pbn, wmin[w]);
  }
  BlockList32* o = out + blockIdx.x;

  if (pb == pbn) {
    // every value of the block is exactly equal (e.g. the r = 0 ring): the
    // best keys are the lowest flat indices
    const uint32_t c = nactive < uint32_t(kListC) ? nactive : uint32_t(kListC);
    for (uint32_t i = tid; i < c; i += blockDim.x) o->keys[i] = key32(pb, fstart + i);
    if (tid == 0) {
      o->pmax = pb;
      o->count = c;
      o->total = nactive;
      o->flags = uint32_t(kFlagFallback);
    }
    return;
  }

  const float theta = pb - pb * tau_band;
#pragma unroll
  for (int p = 0; p < E; ++p) {
    const bool q = P[p] >= theta && P[p] >= 0.f;
    wave_append(q, key32(P[p], fbase + uint32_t(out_bin<LOGN, E>(t, p))), cnt, keys, uint32_t(kListCap));
  }
  __syncthreads();
  const uint32_t n = *cnt;

  if (n <= uint32_t(kListCap)) {
    if (n <= 64) {
      for (uint32_t i = tid; i < n; i += blockDim.x) {
        const uint64_t ki = keys[i];
        uint32_t rank = 0;
        for (uint32_t j = 0; j < n; ++j) rank += keys[j] > ki ? 1u : 0u;
        o->keys[rank] = ki;  // rank < n <= 64 = kListC
      }
    } else {
      lds_sort_desc(keys, n);
      for (uint32_t i = tid; i < uint32_t(kListC); i += blockDim.x) o->keys[i] = keys[i];
    }
    if (tid == 0) {
      o->pmax = pb;
      o->count = n < uint32_t(kListC) ? n : uint32_t(kListC);
      o->total = n;
      o->flags = 0;
    }
    return;
  }

  // Exact fallback (more than kListCap points in the band, not all equal):
  // kListC rounds of block argmax.
  uint32_t taken = 0;
  uint32_t rounds = 0;
  for (; rounds < uint32_t(kListC); ++rounds) {
    uint64_t tb = 0;
#pragma unroll
    for (int p = 0; p < E; ++p) {
      if (!((taken >> p) & 1u) && P[p] >= theta) {
        const uint64_t k = key32(P[p], fbase + uint32_t(out_bin<LOGN, E>(t, p)));
        tb = k > tb ? k : tb;
      }
    }
    tb = wave_max_u64(tb);
    if (lane == 0) wbest[wave] = tb;
    __syncthreads();
    uint64_t b = wbest[0];
    for (int w = 1; w < nw; ++w) b = wbest[w] > b ? wbest[w] : b;
    __syncthreads();
    if (b == 0) break;
    if (tid == 0) o->keys[rounds] = b;
#pragma unroll
    for (int p = 0; p < E; ++p) {
      if (P[p] >= theta && key32(P[p], fbase + uint32_t(out_bin<LOGN, E>(t, p))) == b) taken |= 1u << p;
    }
  }
  if (tid == 0) {
    o->pmax = pb;
    o->count = rounds;
    o->total = n;
    o->flags = uint32_t(kFlagFallback);
  }
}

template <typename T, int LOGN, bool LIST>
__global__ __launch_bounds__(radius_threads<LOGN>()) void k_radius(RadiusParams prm) {
  constexpr int E = pickE<LOGN>();
  constexpr bool SPLIT = pickSplit<LOGN>();
  using S = Shape<LOGN, E>;
  constexpr int N = S::N, TPR = S::TPR;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int rl = tid / TPR, t = tid - rl * TPR;
  const int m = blockIdx.x * prm.rpb + rl;
  const bool active = m < prm.M;
  const int mm = active ? m : prm.M - 1;
  unsigned char* lds_r = smem + size_t(rl) * fft_region_bytes<T, LOGN>();
  unsigned char* scratch = smem + size_t(prm.rpb) * fft_region_bytes<T, LOGN>();

  const Cx<T>* __restrict__ c = reinterpret_cast<const Cx<T>*>(prm.c);
  const T* __restrict__ pw = reinterpret_cast<const T*>(prm.pw);
  const T* __restrict__ pv = reinterpret_cast<const T*>(prm.pv);
  const T* __restrict__ scale = reinterpret_cast<const T*>(prm.scale);
  const Cx<T>* __restrict__ tw = reinterpret_cast<const Cx<T>*>(prm.tw);

  // weighted spectrum f(l) = r_m^l c_l, l = t + TPR i, r^l = r^t r^(TPR i)
  const T rt = pw[size_t(mm) * TPR + t];
  Cx<T> v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const Cx<T> x = c[t + TPR * i];
    const T w = rt * pv[size_t(mm) * E + i];
    v[i] = {x.x * w, x.y * w};
  }
  fft_regs<T, LOGN, E, +1, SPLIT>(v, t, lds_r, tw);

  const T sc = scale[mm];
  const uint32_t fbase = uint32_t(mm) * uint32_t(N);
  if constexpr (LIST) {
    const uint32_t r0 = uint32_t(blockIdx.x) * uint32_t(prm.rpb);
    const uint32_t ract = uint32_t(prm.M) - r0 < uint32_t(prm.rpb) ? uint32_t(prm.M) - r0 : uint32_t(prm.rpb);
    select_list<LOGN>(v, active, sc, fbase, t, scratch, prm.tau_band, r0 * uint32_t(N), ract * uint32_t(N),
                      reinterpret_cast<BlockList32*>(prm.out));
  } else {
    select_best<LOGN, T>(v, active, sc, fbase, t, scratch, reinterpret_cast<BlockBest64*>(prm.out));
  }
}

// ---------------------------------------------------------------- small block helpers
__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, uint64_t* wb) {
  v = wave_max_u64(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wb[wave] = v;
  __syncthreads();
  uint64_t b = wb[0];
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = 1; w < nw; ++w) b = wb[w] > b ? wb[w] : b;
  __syncthreads();
  return b;
}

// deterministic tree sum of one double per thread (blockDim.x = 256)
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (int(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- FP64 merge
__global__ __launch_bounds__(1024) void k_merge64(const BlockBest64* __restrict__ blocks, int nb, int N, int logn,
                                                  Winner* __restrict__ w) {
  __shared__ Best wb[16];
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const BlockBest64 o = blocks[i];
    Best x{o.p1, o.p2, o.vx, o.vy, o.f};
    best_merge(b, x);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) best_merge(b, best_shfl(b, m));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wb[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    Best r = wb[0];
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) best_merge(r, wb[i]);
    Winner o;
    const bool valid = r.f != 0xffffffffu;  // false only if every value was NaN
    o.m = valid ? int32_t(r.f >> logn) : 0;
    o.j = valid ? int32_t(r.f & uint32_t(N - 1)) : 0;
    o.kcount = 0;
    o.flags = 0;
    o.ax = o.ay = 0.0;  // filled by k_update's reader from the radius and angle
    o.cx = valid ? r.vx : 0.0;
    o.cy = valid ? r.vy : 0.0;
    o.margin = !valid ? __builtin_nan("") : r.p1 > 0.0 ? (r.p1 - r.p2) / r.p1 : 0.0;
    o.pad = 0.0;
    *w = o;
  }
}

// ---------------------------------------------------------------- FP32 short-list
// Global short-list from the per-block lists (each: its points within the
// re-check band of the block maximum, best first): every listed point within
// tau_band of the FP32 maximum, sorted by key and cut at kKMax; if that is
// fewer than recheck_k points, the best points of the next-best blocks are
// appended until it is not.  A gather that overflows kSelCap (a flat grid:
// all-zero or exactly tied values) falls back to an exact pop-merge.
__device__ __forceinline__ float block_max_f32(float v, float* wf) {
  v = wave_max_f32(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wf[wave] = v;
  __syncthreads();
  float b = wf[0];
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = 1; w < nw; ++w) b = fmaxf(b, wf[w]);
  __syncthreads();
  return b;
}

__global__ __launch_bounds__(1024) void k_select32(const BlockList32* __restrict__ lists, int nb, int recheck_k,
                                                   float tau_band, uint32_t* __restrict__ heads,
                                                   CandList* __restrict__ cand) {
  __shared__ uint64_t buf[kSelCap];
  __shared__ uint32_t cblk[kSelCap];
  __shared__ uint64_t wb[16];
  __shared__ float wf[16];
  __shared__ uint32_t scount, sblocks, sflags;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  float pm = -1.f;
  uint32_t fl = 0;
  for (int b = tid; b < nb; b += blockDim.x) {
    fl |= lists[b].flags;
    if (lists[b].count > 0) pm = fmaxf(pm, lists[b].pmax);
  }
  if (tid == 0) {
    sflags = 0;
    scount = 0;
    sblocks = 0;
  }
  const float pg = block_max_f32(pm, wf);  // its barriers order the initialisation above
  if (fl) atomicOr(&sflags, fl & uint32_t(kFlagFallback));
  const float theta = pg - pg * tau_band;
  // blocks whose maximum reaches the band
  for (int b0 = 0; b0 < nb; b0 += blockDim.x) {
    const int b = b0 + tid;
    const bool q = b < nb && lists[b].count > 0 && lists[b].pmax >= theta;
    const uint64_t mask = __ballot(q);
    if (mask) {
      const int leader = __ffsll(static_cast<long long>(mask)) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&sblocks, uint32_t(__popcll(mask)));
      base = __shfl(base, leader);
      if (q) {
        const uint32_t pos = base + uint32_t(__popcll(mask & ((uint64_t(1) << lane) - 1)));
        if (pos < uint32_t(kSelCap)) cblk[pos] = uint32_t(b);
      }
    }
  }
  __syncthreads();
  const uint32_t ncb = sblocks < uint32_t(kSelCap) ? sblocks : uint32_t(kSelCap);
  // one wave per candidate block: its band prefix, one coalesced load of 64 keys
  for (uint32_t i = wave; i < ncb; i += nw) {
    const BlockList32* L = lists + cblk[i];
    const uint32_t cnt = L->count;
    const uint64_t k = lane < int(cnt) ? L->keys[lane] : 0;
    const bool q = lane < int(cnt) && key_p(k) >= theta;
    wave_append(q, k, &scount, buf, uint32_t(kSelCap));
    if (lane == 0 && cnt > 0 && L->total > cnt && key_p(L->keys[cnt - 1]) >= theta)
      atomicOr(&sflags, uint32_t(kFlagListTruncated));
  }
  __syncthreads();
  const uint32_t band = scount;

  if (band <= uint32_t(kSelCap) && sblocks <= uint32_t(kSelCap)) {
    lds_sort_desc(buf, band);
    uint32_t keff = band < uint32_t(kKMax) ? band : uint32_t(kKMax);
    if (band > uint32_t(kKMax) && tid == 0) atomicOr(&sflags, uint32_t(kFlagBandTruncated));
    for (uint32_t i = tid; i < keff; i += blockDim.x) cand->keys[i] = buf[i];
    if (keff < uint32_t(recheck_k)) {
      // top up with the best points of the next-best blocks (maxima below the band)
      uint64_t tb = 0;
      int tbb = -1;
      for (int b = tid; b < nb; b += blockDim.x) {
        heads[b] = 0;
        if (lists[b].count > 0 && lists[b].pmax < theta && lists[b].keys[0] > tb) {
          tb = lists[b].keys[0];
          tbb = b;
        }
      }
      while (keff < uint32_t(recheck_k)) {
        const uint64_t g = block_max_u64(tb, wb);
        if (g == 0) break;
        if (tid == 0) cand->keys[keff] = g;
        ++keff;
        if (tbb >= 0 && tb == g) {
          heads[tbb] = 1;
          tb = 0;
          tbb = -1;
          for (int b = tid; b < nb; b += blockDim.x) {
            if (heads[b] == 0 && lists[b].count > 0 && lists[b].pmax < theta && lists[b].keys[0] > tb) {
              tb = lists[b].keys[0];
              tbb = b;
            }
          }
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      cand->count = int32_t(keff);
      cand->flags = int32_t(sflags);
      cand->pmax32 = pg;
    }
    return;
  }

  // Exact fallback (a flat grid: more band points or band blocks than the
  // gather holds): pop-merge of the sorted per-block lists.
  uint64_t tb = 0;
  int tbb = -1;
  for (int b = tid; b < nb; b += blockDim.x) {
    heads[b] = 0;
    if (lists[b].count > 0 && lists[b].keys[0] > tb) {
      tb = lists[b].keys[0];
      tbb = b;
    }
  }
  const int want = recheck_k > kListC ? recheck_k : kListC;
  int r = 0;
  for (; r < want; ++r) {
    const uint64_t g = block_max_u64(tb, wb);
    if (g == 0) break;
    if (tid == 0) cand->keys[r] = g;
    if (tbb >= 0 && tb == g) {
      const uint32_t h = ++heads[tbb];
      if (h >= lists[tbb].count && lists[tbb].total > lists[tbb].count) atomicOr(&sflags, uint32_t(kFlagListTruncated));
      tb = 0;
      tbb = -1;
      for (int b = tid; b < nb; b += blockDim.x) {
        const uint32_t hb = heads[b];
        if (hb < lists[b].count && lists[b].keys[hb] > tb) {
          tb = lists[b].keys[hb];
          tbb = b;
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    atomicOr(&sflags, uint32_t(kFlagFallback) | uint32_t(kFlagBandTruncated));
    cand->count = r;
    cand->flags = int32_t(sflags);
    cand->pmax32 = pg;
  }
}

__global__ void k_force(const int32_t* __restrict__ forced, int step, int N, CandList* __restrict__ cand) {
  if (threadIdx.x == 0) {
    const uint32_t m = uint32_t(forced[2 * step]), j = uint32_t(forced[2 * step + 1]);
    cand->count = 1;
    cand->flags = 8;  // forced step
    cand->pmax32 = 0.f;
    cand->keys[0] = (uint64_t(0) << 32) | uint64_t(~(m * uint32_t(N) + j));
  }
}

// ---------------------------------------------------------------- FP64 direct re-check
// partial sums over a chunk of samples of G[n] / (1 - r_m e^{2 pi i (j - n)/N})
__global__ __launch_bounds__(256) void k_recheck(const CandList* __restrict__ cand, const double* __restrict__ g,
                                                 const double* __restrict__ omega, const double* __restrict__ radii,
                                                 int N, int logn, int nch, double* __restrict__ partials) {
  __shared__ double sh[256];
  const int chunk = blockIdx.y;
  const int cl = N / nch;
  const int count = cand->count;
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const uint32_t f = key_f(cand->keys[i]);
    const int m = int(f >> logn), j = int(f & uint32_t(N - 1));
    const double r = radii[m];
    double ax = 0.0, ay = 0.0;
    for (int n = chunk * cl + threadIdx.x; n < (chunk + 1) * cl; n += blockDim.x) {
      const int d = (j - n) & (N - 1);
      const double ox = omega[2 * d], oy = omega[2 * d + 1];
      const double dx = fma(-r, ox, 1.0), dy = -r * oy;
      const double inv = 1.0 / fma(dx, dx, dy * dy);
      const double gx = g[2 * n], gy = g[2 * n + 1];
      ax += fma(gx, dx, gy * dy) * inv;
      ay += fma(gy, dx, -gx * dy) * inv;
    }
    const double sx = block_sum256(ax, sh);
    const double sy = block_sum256(ay, sh);
    if (threadIdx.x == 0) {
      partials[2 * (size_t(i) * nch + chunk)] = sx;
      partials[2 * (size_t(i) * nch + chunk) + 1] = sy;
    }
  }
}

__global__ __launch_bounds__(256) void k_finalize(const CandList* __restrict__ cand,
                                                  const double* __restrict__ partials,
                                                  const double* __restrict__ radii, const double* __restrict__ omega,
                                                  int N, int logn, int nch, Winner* __restrict__ w) {
  __shared__ Best wb[4];
  const int count = cand->count;
  const int forced = cand->flags & 8;
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const uint32_t f = key_f(cand->keys[i]);
    const double r = radii[f >> logn];
    double ax = 0.0, ay = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      ax += partials[2 * (size_t(i) * nch + ch)];
      ay += partials[2 * (size_t(i) * nch + ch) + 1];
    }
    const double s = sqrt((1.0 - r) * (1.0 + r)) / double(N);
    const Best x{(ax * s) * (ax * s) + (ay * s) * (ay * s), -1.0, ax * s, ay * s, f};
    best_merge(b, x);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) best_merge(b, best_shfl(b, m));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wb[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    Best r = wb[0];
    for (int i = 1; i < 4; ++i) best_merge(r, wb[i]);
    Winner o;
    const bool valid = count > 0 && r.f != 0xffffffffu;
    o.m = valid ? int32_t(r.f >> logn) : 0;
    o.j = valid ? int32_t(r.f & uint32_t(N - 1)) : 0;
    o.cx = valid ? r.vx : 0.0;
    o.cy = valid ? r.vy : 0.0;
    if (forced || count < 2 || !valid) o.margin = __builtin_nan("");
    else o.margin = r.p1 > 0.0 ? (r.p1 - r.p2) / r.p1 : 0.0;
    o.kcount = forced ? 1 : count;
    o.flags = cand->flags & 7;
    o.ax = o.ay = 0.0;
    o.pad = 0.0;
    *w = o;
  }
}

// ---------------------------------------------------------------- update / energy
constexpr int kUpdThreads = 256;
constexpr int kUpdPerThread = 4;

__global__ __launch_bounds__(256) void k_prepare(double* __restrict__ g64, float* __restrict__ g32, int N,
                                                 double* __restrict__ epart, int* __restrict__ nonfinite) {
  __shared__ double sh[256];
  double acc = 0.0;
  int bad = 0;
#pragma unroll
  for (int s = 0; s < kUpdPerThread; ++s) {
    const int n = blockIdx.x * (kUpdThreads * kUpdPerThread) + s * kUpdThreads + threadIdx.x;
    if (n < N) {
      const double x = g64[2 * n], y = g64[2 * n + 1];
      if (!isfinite(x) || !isfinite(y)) bad = 1;
      if (g32) {
        g32[2 * n] = float(x);
        g32[2 * n + 1] = float(y);
      }
      acc += fma(x, x, y * y);
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  const double tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) epart[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_update(const Winner* __restrict__ w, const double* __restrict__ radii,
                                                const double* __restrict__ omega, double* __restrict__ g64,
                                                float* __restrict__ g32, int N, int M, double* __restrict__ epart) {
  __shared__ double sh[256];
  Winner W = *w;
  W.m = min(max(W.m, 0), M - 1);
  W.j = W.j & (N - 1);
  const double r = radii[W.m];
  const double s = sqrt((1.0 - r) * (1.0 + r));
  const double cx = W.cx, cy = W.cy;
  const double wjx = omega[2 * W.j], wjy = -omega[2 * W.j + 1];  // e^{-2 pi i j/N}
  const double csx = cx * s, csy = cy * s;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kUpdPerThread; ++q) {
    const int n = blockIdx.x * (kUpdThreads * kUpdPerThread) + q * kUpdThreads + threadIdx.x;
    if (n < N) {
      const int d = (n - W.j) & (N - 1);
      const double ox = omega[2 * d], oy = omega[2 * d + 1];
      const double gx = g64[2 * n], gy = g64[2 * n + 1];
      // num = G (1 - r w^d) - c s
      const double ux = fma(-r, ox, 1.0), uy = -r * oy;
      const double nx = fma(gx, ux, -gy * uy) - csx;
      const double ny = fma(gx, uy, gy * ux) - csy;
      // / (w^d - r)
      const double dx = ox - r, dy = oy;
      const double inv = 1.0 / fma(dx, dx, dy * dy);
      const double qx = fma(nx, dx, ny * dy) * inv;
      const double qy = fma(ny, dx, -nx * dy) * inv;
      // * e^{-2 pi i j/N}
      const double hx = fma(qx, wjx, -qy * wjy);
      const double hy = fma(qx, wjy, qy * wjx);
      g64[2 * n] = hx;
      g64[2 * n + 1] = hy;
      if (g32) {
        g32[2 * n] = float(hx);
        g32[2 * n + 1] = float(hy);
      }
      acc += fma(hx, hx, hy * hy);
    }
  }
  const double tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) epart[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_record(const Winner* __restrict__ w, const double* __restrict__ radii,
                                                const double* __restrict__ omega, const double* __restrict__ epart,
                                                int nparts, int N, int M, int step, int32_t* __restrict__ idx,
                                                double* __restrict__ a, double* __restrict__ coef,
                                                double* __restrict__ energy, double* __restrict__ margin,
                                                int32_t* __restrict__ kcount, int32_t* __restrict__ flags) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += epart[i];
  const double tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) {
    const double E = tot / double(N);
    if (step < 0) {
      energy[0] = E;
    } else {
      Winner W = *w;
      W.m = min(max(W.m, 0), M - 1);
      W.j = W.j & (N - 1);
      const double r = radii[W.m];
      idx[2 * step] = W.m;
      idx[2 * step + 1] = W.j;
      a[2 * step] = r * omega[2 * W.j];
      a[2 * step + 1] = r * omega[2 * W.j + 1];
      coef[2 * step] = W.cx;
      coef[2 * step + 1] = W.cy;
      energy[step + 1] = E;
      margin[step] = W.margin;
      kcount[step] = W.kcount;
      flags[step] = W.flags;
    }
  }
}

// ---------------------------------------------------------------- host-side geometry
template <int LOGN>
static FftGeom geom_of(bool fp64) {
  constexpr int E = pickE<LOGN>();
  using S = Shape<LOGN, E>;
  FftGeom g;
  g.E = E;
  g.tpr = S::TPR;
  g.twsize = S::twsize();
  g.split = pickSplit<LOGN>();
  g.lds_elems = S::LDS_ELEMS;
  (void)fp64;
  return g;
}

template <int LOGN>
static void twiddles_of(double* out) {
  constexpr int E = pickE<LOGN>();
  using S = Shape<LOGN, E>;
  for (int p = 1; p < S::NP; ++p) {
    const int ns = S::ns(p), R = S::radix(p), off = S::twoff(p);
    const long double L = (long double)ns * R;
    for (int k = 0; k < ns; ++k) {
      const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)k / L;
      out[2 * (off + k)] = (double)cosl(ang);
      out[2 * (off + k) + 1] = (double)sinl(ang);
    }
  }
}

#define AFD_LOGN_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

FftGeom fft_geom(int logn, bool fp64) {
  switch (logn) {
#define X(L) \
  case L:    \
    return geom_of<L>(fp64);
    AFD_LOGN_CASES(X)
#undef X
    default:
      return FftGeom{0, 0, 0, false, 0};
  }
}

void fft_twiddles(int logn, bool fp64, double* out) {
  (void)fp64;
  switch (logn) {
#define X(L)             \
  case L:                \
    twiddles_of<L>(out); \
    break;
    AFD_LOGN_CASES(X)
#undef X
    default:
      break;
  }
}

template <int LOGN>
static int radius_lds_of(bool fp64, int rpb) {
  const size_t fr = fp64 ? fft_region_bytes<double, LOGN>() : fft_region_bytes<float, LOGN>();
  return int(size_t(rpb) * fr + kScratchBytes);
}

int radius_lds_bytes(int logn, bool fp64, int rpb, bool list) {
  (void)list;
  switch (logn) {
#define X(L) \
  case L:    \
    return radius_lds_of<L>(fp64, rpb);
    AFD_LOGN_CASES(X)
#undef X
    default:
      return 0;
  }
}

template <int LOGN>
static int fwd_lds_of(bool fp64) {
  return int(fp64 ? fft_region_bytes<double, LOGN>() : fft_region_bytes<float, LOGN>());
}

hipError_t setup_kernel_attributes() {
  const int big = 160 * 1024;
  hipError_t e = hipSuccess;
#define X(L)                                                                                                   \
  if (e == hipSuccess)                                                                                         \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_radius<double, L, false>),                         \
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);                                  \
  if (e == hipSuccess)                                                                                         \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_radius<float, L, true>),                           \
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);                                  \
  if (e == hipSuccess)                                                                                         \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_fft_fwd<double, L>),                               \
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);                                  \
  if (e == hipSuccess)                                                                                         \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_fft_fwd<float, L>),                                \
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  AFD_LOGN_CASES(X)
#undef X
  return e;
}

hipError_t launch_fft_fwd(int logn, bool fp64, const void* g, const void* tw, void* c, hipStream_t s) {
  switch (logn) {
#define X(L)                                                                                                     \
  case L: {                                                                                                      \
    const int thr = Shape<L, pickE<L>()>::TPR;                                                                   \
    if (fp64)                                                                                                    \
      hipLaunchKernelGGL((k_fft_fwd<double, L>), dim3(1), dim3(thr), fwd_lds_of<L>(true), s,                    \
                         reinterpret_cast<const Cx<double>*>(g), reinterpret_cast<const Cx<double>*>(tw),        \
                         reinterpret_cast<Cx<double>*>(c));                                                      \
    else                                                                                                         \
      hipLaunchKernelGGL((k_fft_fwd<float, L>), dim3(1), dim3(thr), fwd_lds_of<L>(false), s,                    \
                         reinterpret_cast<const Cx<float>*>(g), reinterpret_cast<const Cx<float>*>(tw),          \
                         reinterpret_cast<Cx<float>*>(c));                                                       \
    return hipGetLastError();                                                                                    \
  }
    AFD_LOGN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_radius(int logn, bool fp64, const RadiusParams& p, int blocks, hipStream_t s) {
  switch (logn) {
#define X(L)                                                                                                  \
  case L: {                                                                                                   \
    const int thr = Shape<L, pickE<L>()>::TPR * p.rpb;                                                        \
    const int lds = radius_lds_of<L>(fp64, p.rpb);                                                            \
    if (fp64)                                                                                                 \
      hipLaunchKernelGGL((k_radius<double, L, false>), dim3(blocks), dim3(thr), lds, s, p);                  \
    else                                                                                                      \
      hipLaunchKernelGGL((k_radius<float, L, true>), dim3(blocks), dim3(thr), lds, s, p);                    \
    return hipGetLastError();                                                                                 \
  }
    AFD_LOGN_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

static int ilog2i(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

hipError_t launch_merge64(const BlockBest64* blocks, int nblocks, int N, Winner* w, hipStream_t s) {
  hipLaunchKernelGGL(k_merge64, dim3(1), dim3(1024), 0, s, blocks, nblocks, N, ilog2i(N), w);
  return hipGetLastError();
}

hipError_t launch_select32(const BlockList32* lists, int nblocks, int recheck_k, float tau_band, CandList* cand,
                           hipStream_t s) {
  // the per-block heads live right after the candidate list record
  uint32_t* heads = reinterpret_cast<uint32_t*>(cand + 1);
  hipLaunchKernelGGL(k_select32, dim3(1), dim3(1024), 0, s, lists, nblocks, recheck_k, tau_band, heads, cand);
  return hipGetLastError();
}

hipError_t launch_force(const int32_t* forced, int step, int N, CandList* cand, hipStream_t s) {
  hipLaunchKernelGGL(k_force, dim3(1), dim3(64), 0, s, forced, step, N, cand);
  return hipGetLastError();
}

hipError_t launch_recheck(const CandList* cand, const double* g, const double* omega, const double* radii, int N,
                          int nch, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_recheck, dim3(kKMax, nch), dim3(256), 0, s, cand, g, omega, radii, N, ilog2i(N), nch,
                     partials);
  return hipGetLastError();
}

hipError_t launch_finalize(const CandList* cand, const double* partials, const double* radii, const double* omega,
                           int N, int nch, Winner* w, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, cand, partials, radii, omega, N, ilog2i(N), nch, w);
  return hipGetLastError();
}

int update_blocks(int N) { return (N + kUpdThreads * kUpdPerThread - 1) / (kUpdThreads * kUpdPerThread); }

hipError_t launch_prepare(const double* g, double* g64, float* g32, int N, double* epart, int* nonfinite,
                          hipStream_t s) {
  (void)g;
  hipLaunchKernelGGL(k_prepare, dim3(update_blocks(N)), dim3(kUpdThreads), 0, s, g64, g32, N, epart, nonfinite);
  return hipGetLastError();
}

hipError_t launch_update(const Winner* w, const double* radii, const double* omega, double* g64, float* g32, int N,
                         int M, double* epart, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(update_blocks(N)), dim3(kUpdThreads), 0, s, w, radii, omega, g64, g32, N, M,
                     epart);
  return hipGetLastError();
}

hipError_t launch_record(const Winner* w, const double* radii, const double* omega, const double* epart, int nparts,
                         int N, int M, int step, int32_t* idx, double* a, double* coef, double* energy,
                         double* margin, int32_t* kcount, int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_record, dim3(1), dim3(256), 0, s, w, radii, omega, epart, nparts, N, M, step, idx, a, coef,
                     energy, margin, kcount, flags);
  return hipGetLastError();
}

}  // namespace afd
