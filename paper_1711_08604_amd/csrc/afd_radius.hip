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
// the winner, FP32 into the short-list for the double re-check.
#include "afd_select.h"

namespace afd {

constexpr size_t kScratchBytes = 512 + sizeof(uint64_t) * (kListCap + kListC);

template <typename T, int LOGN>
__host__ __device__ constexpr int radius_threads() {
  return Shape<LOGN, pickE<T, LOGN>()>::TPR < 64 ? 64 : Shape<LOGN, pickE<T, LOGN>()>::TPR;
}

// Waves per SIMD the register budget must allow: two workgroups per CU for
// the 512-thread single-precision transforms (at most 128 VGPRs), no
// constraint otherwise.
template <typename T, int LOGN>
__host__ __device__ constexpr int radius_min_waves() {
  return (sizeof(T) == 4 && radius_threads<T, LOGN>() == 512) ? 4 : 1;
}

template <typename T, int LOGN>
static size_t radius_lds(int rpb) {
  const size_t need = size_t(rpb) * fft_region_bytes<T, LOGN, pickSplit<T, LOGN>()>() + kScratchBytes;
  return need > sizeof(MergeScratch) ? need : sizeof(MergeScratch);
}

// FP64 workgroup selection: best point (value, flat index, grid value) and the
// runner-up value.  Within a thread the bins are visited in increasing index
// order, so a strict comparison keeps the lowest index among equal values.
template <int LOGN, typename T>
__device__ __forceinline__ void select_best(const Cx<T> (&v)[pickE<T, LOGN>()], bool active, T sc, uint32_t fbase,
                                            int t, Best* wb, BlockBest64* out) {
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
    b.f = fbase + uint32_t(t + Shape<LOGN, E>::TPR * bitrev(i1, LE));
    // exact |.|^2 of the scaled grid value, as compared across radii
    b.p1 = b.vx * b.vx + b.vy * b.vy;
    b.p2 = fmin(y2 * s2, b.p1);
  }
  const Best r = block_best(b, wb);
  if (threadIdx.x == 0) {
    BlockBest64* o = out + blockIdx.x;
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
template <int LOGN>
__device__ __forceinline__ void select_list(const Cx<float> (&v)[pickE<float, LOGN>()], bool active, float sc,
                                            uint32_t fbase, int t, unsigned char* scratch, float tau_band,
                                            uint32_t fstart, uint32_t nactive, BlockList32* out) {
  constexpr int E = pickE<float, LOGN>();
  constexpr int TPR = Shape<LOGN, E>::TPR;
  constexpr int LE = ilog2c(E);
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
  BlockList32* o = out + blockIdx.x;

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
      base = __shfl(base, leader);
      if (q) {
        const uint32_t pos = base + uint32_t(__popcll(mask & ((uint64_t(1) << lane) - 1)));
        if (pos < uint32_t(kListCap)) keys[pos] = key32(Y[p] * s2, fbase + uint32_t(t + TPR * bitrev(p, LE)));
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
    if (tid == 0) {
      st_agent(&o->pmax, pb);
      st_agent(&o->count, n < uint32_t(kListC) ? n : uint32_t(kListC));
      st_agent(&o->total, n);
      st_agent(&o->flags, 0u);
    }
    return;
  }

  // More than kListCap points in the band.  If every value is exactly equal
  // (e.g. the r = 0 ring) the best keys are the lowest flat indices;
  // otherwise kListC rounds of exact workgroup argmax.
  float pn = 3.4e38f;
  if (active) {
#pragma unroll
    for (int p = 0; p < E; ++p) pn = fminf(pn, Y[p] * s2);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) pn = fminf(pn, __shfl_xor(pn, m));
  if (lane == 0) wmin[wave] = pn;
  __syncthreads();
  float pbn = wmin[0];
  for (int w = 1; w < nw; ++w) pbn = fminf(pbn, wmin[w]);
  if (pb == pbn) {
    const uint32_t c = nactive < uint32_t(kListC) ? nactive : uint32_t(kListC);
    if (uint32_t(tid) < c) st_agent(&o->keys[tid], key32(pb, fstart + uint32_t(tid)));  // wave 0 (c <= 64)
    if (tid == 0) {
      st_agent(&o->pmax, pb);
      st_agent(&o->count, c);
      st_agent(&o->total, nactive);
      st_agent(&o->flags, uint32_t(kFlagFallback));
    }
    return;
  }
  uint32_t taken = 0;
  uint32_t rounds = 0;
  for (; rounds < uint32_t(kListC); ++rounds) {
    uint64_t tb = 0;
#pragma unroll
    for (int p = 0; p < E; ++p) {
      if (!((taken >> p) & 1u) && Y[p] >= ty) {
        const uint64_t k = key32(Y[p] * s2, fbase + uint32_t(t + TPR * bitrev(p, LE)));
        tb = k > tb ? k : tb;
      }
    }
    const uint64_t b = block_max_u64(tb, wbest);
    if (b == 0) break;
    if (tid == 0) st_agent(&o->keys[rounds], b);
#pragma unroll
    for (int p = 0; p < E; ++p) {
      if (Y[p] >= ty && key32(Y[p] * s2, fbase + uint32_t(t + TPR * bitrev(p, LE))) == b) taken |= 1u << p;
    }
  }
  if (tid == 0) {
    st_agent(&o->pmax, pb);
    st_agent(&o->count, rounds);
    st_agent(&o->total, n);
    st_agent(&o->flags, uint32_t(kFlagFallback));
  }
}

template <typename T, int LOGN, bool LIST>
__global__ __launch_bounds__((radius_threads<T, LOGN>())) __attribute__((amdgpu_waves_per_eu(
    radius_min_waves<T, LOGN>()))) void k_radius(RadiusParams prm) {
  constexpr int E = pickE<T, LOGN>();
  constexpr bool SPLIT = pickSplit<T, LOGN>();
  using S = Shape<LOGN, E>;
  constexpr int N = S::N, TPR = S::TPR;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int rl = tid / TPR, t = tid - rl * TPR;
  const int m = blockIdx.x * prm.rpb + rl;
  const bool active = m < prm.M;
  const int mm = active ? m : prm.M - 1;
  constexpr size_t region = fft_region_bytes<T, LOGN, SPLIT>();
  unsigned char* lds_r = smem + size_t(rl) * region;
  unsigned char* scratch = smem + size_t(prm.rpb) * region;

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
    // double precision: bound the loads in flight (128-register budget)
    if (sizeof(T) == 8 && (i % 4) == 3) __builtin_amdgcn_sched_barrier(0);
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
    select_best<LOGN, T>(v, active, sc, fbase, t, reinterpret_cast<Best*>(scratch),
                         reinterpret_cast<BlockBest64*>(prm.out));
  }

  if (!last_workgroup(prm.counter, &s_last)) return;
  MergeScratch* Sm = reinterpret_cast<MergeScratch*>(smem);
  if constexpr (LIST) {
    select32_tail(reinterpret_cast<const BlockList32*>(prm.out), int(gridDim.x), prm.recheck_k, prm.tau_band,
                  prm.cand, Sm);
  } else {
    merge64_tail(reinterpret_cast<const BlockBest64*>(prm.out), int(gridDim.x), N, LOGN, prm.winner, Sm);
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

hipError_t setup_radius_attributes() {
  hipError_t e = hipSuccess;
#define X(L)                                                                                  \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<double, L, false>));                 \
  if (e == hipSuccess)                                                                        \
    e = set_max_dynamic_lds(reinterpret_cast<const void*>(k_radius<float, L, true>));
  AFD_LDS_LOGN_CASES(X)
#undef X
  return e;
}

hipError_t launch_radius(int logn, bool fp64, const RadiusParams& p, int blocks, hipStream_t s) {
  switch (logn) {
#define X(L)                                                                                 \
  case L: {                                                                                  \
    if (fp64) {                                                                              \
      constexpr int thr = radius_threads<double, L>();                                       \
      const size_t lds = radius_lds<double, L>(p.rpb);                                       \
      hipLaunchKernelGGL((k_radius<double, L, false>), dim3(blocks), dim3(thr), lds, s, p);  \
    } else {                                                                                 \
      constexpr int thr = radius_threads<float, L>();                                        \
      const size_t lds = radius_lds<float, L>(p.rpb);                                        \
      hipLaunchKernelGGL((k_radius<float, L, true>), dim3(blocks), dim3(thr), lds, s, p);    \
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
