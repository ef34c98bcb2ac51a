// Per-step kernels around the radius kernel:
//   k_prepare   copy-in checks, complex64 copy of the samples, E_0
//   k_force     forced grid point (first_a_zero, replay) as a one-entry short-list
//   k_recheck   the direct rule of Sec. 3.1, eq. term81, in double for each
//               short-listed point, in partial sums over chunks of samples; the
//               last workgroup picks the winner (largest |.|^2, lowest flat
//               index) and its coefficient c_k = <G_k, e_{a_k}>~ (eq. (3))
//   k_update    G_{k+1} = (G_k - c_k e_{a_k}) (1 - conj(a_k) z)/(z - a_k) (eq. (7))
//               in double; the last workgroup sums E_k = (1/N) sum |G_{k+1}|^2
//               and records the step's outputs
//   k_merge     the radius kernel's per-workgroup records merged into the
//               winner (FP64) or the short-list (FP32) in a launch of its own
//   k_pick      a replayed step: the selection's own choice is recorded and
//               the forced point takes its place
//   k_zero      counters cleared by a kernel in a captured decomposition
#include "afd_update.h"

namespace afd {

constexpr int kUpdThreads = 256;
constexpr int kUpdPerThread = 4;

int update_blocks(int N) { return (N + kUpdThreads * kUpdPerThread - 1) / (kUpdThreads * kUpdPerThread); }
int recheck_chunks(int N) { return (N + 2047) / 2048; }

// Batched launches: signal b = blockIdx.y works on
// its own slices of every per-signal buffer.
__global__ __launch_bounds__(256) void k_prepare(double* __restrict__ g64, float* __restrict__ g32, int N,
                                                 double* __restrict__ epart, int* __restrict__ nonfinite,
                                                 unsigned int* __restrict__ counter, RecordArgs R) {
  __shared__ double wd[16];
  __shared__ int s_last;
  const int b = blockIdx.y;
  g64 += 2 * size_t(N) * b;
  if (g32) g32 += 2 * size_t(N) * b;
  epart += size_t(gridDim.x) * b;
  counter += b;
  R = record_of(R, b);
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
  const double tot = block_sum_f64(acc, wd);
  if (threadIdx.x == 0) st_agent(epart + blockIdx.x, tot);
  if (!last_arrival(counter, gridDim.x, &s_last)) return;
  const double E = energy_from_parts(epart, int(gridDim.x), N, wd);
  if (threadIdx.x == 0) write_record(R, -1, E);
}

__global__ void k_force(const int32_t* __restrict__ forced, int fstride, int step, int N,
                        CandList* __restrict__ cand) {
  const int b = blockIdx.x;
  forced += size_t(fstride) * b;
  cand += b;
  if (threadIdx.x == 0) {
    const uint32_t m = uint32_t(forced[2 * step]), j = uint32_t(forced[2 * step + 1]);
    cand->count = 1;
    cand->flags = kFlagForced;
    cand->pmax32 = 0.f;
    cand->keys[0] = uint64_t(~(m * uint32_t(N) + j));  // P = 0: the re-check supplies the value
  }
}

// Partial sums over a chunk of samples of G[n] / (1 - r_m e^{2 pi i (j - n)/N})
// for every short-listed point (m, j): each workgroup holds its chunk's
// samples and unit roots in registers and runs through the candidates, with
// e^{2 pi i (j - n)/N} = e^{2 pi i j/N} conj(e^{2 pi i n/N}), so the samples
// are read once per step rather than once per candidate.  The wave sums of
// every candidate meet in LDS and are added in wave order after the loop.
// Non-uniform samples (S.z non-null): the NS samples sit at S.z[n] in place of
// e^{2 pi i n/N}, each term carries the quadrature weight S.w[n], and the sum
// is scaled by sqrt(1 - r^2) instead of sqrt(1 - r^2)/N.  Workgroup z of
// the grid's third dimension takes candidates z, z + gridDim.z, ...; their
// radii and angles are fetched together before the sums.
constexpr int kRecheckPerThread = 8;  // chunk of 2048 samples over 256 threads
__global__ __launch_bounds__(256) void k_recheck(const CandList* __restrict__ cand, const double* __restrict__ g,
                                                 const double* __restrict__ omega, const double* __restrict__ radii,
                                                 int N, int nch, double* __restrict__ partials,
                                                 unsigned int* __restrict__ counter, Winner* __restrict__ w,
                                                 RecheckSamples S) {
  __shared__ double wsum[kKMax][4][2];  // [candidate][wave] (re, im)
  __shared__ double cpar[kKMax][3];     // [candidate] r, e^{2 pi i j/N}
  __shared__ double wd[16];
  __shared__ Best bb[16];
  __shared__ int s_last;
  const int chunk = blockIdx.x;
  const int ns = S.z ? S.ns : N;  // samples
  const double* __restrict__ zs = S.z ? S.z : omega;
  const int cl = (ns + nch - 1) / nch;  // samples per chunk (the last may hold fewer)
  const int b = blockIdx.y;
  const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
  cand += b;
  g += 2 * size_t(ns) * b;
  partials += 2 * size_t(kKMax) * size_t(nch) * b;
  counter += b;
  w += b;
  const int count = min(max(cand->count, 0), kKMax);
  const int c0 = int(blockIdx.z), cs = int(gridDim.z);
  // this workgroup's candidates: radius and angle, all in one round trip
  for (int c = c0 + cs * tid; c < count; c += cs * int(blockDim.x)) {
    const uint32_t f = key_f(cand->keys[c]);
    const int m = int(f / uint32_t(N)), j = int(f % uint32_t(N));
    cpar[c][0] = radii[m];
    cpar[c][1] = omega[2 * j];
    cpar[c][2] = omega[2 * j + 1];
  }
  double gx[kRecheckPerThread], gy[kRecheckPerThread], ox[kRecheckPerThread], oy[kRecheckPerThread];
#pragma unroll
  for (int q = 0; q < kRecheckPerThread; ++q) {
    const int i = tid + 256 * q;
    const int n = chunk * cl + i;
    const bool in = i < cl && n < ns;
    gx[q] = in ? g[2 * n] : 0.0;
    gy[q] = in ? g[2 * n + 1] : 0.0;
    ox[q] = in ? zs[2 * n] : 1.0;
    oy[q] = in ? zs[2 * n + 1] : 0.0;
    if (S.w && in) {
      const double wn = S.w[n];
      gx[q] *= wn;
      gy[q] *= wn;
    }
  }
  __syncthreads();
  for (int c = c0; c < count; c += cs) {
    const double r = cpar[c][0];
    const double wjx = cpar[c][1], wjy = cpar[c][2];
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int q = 0; q < kRecheckPerThread; ++q) {
      // e^{2 pi i (j - n)/N}
      const double ux = fma(wjx, ox[q], wjy * oy[q]);
      const double uy = fma(wjy, ox[q], -wjx * oy[q]);
      const double dx = fma(-r, ux, 1.0), dy = -r * uy;
      const double inv = 1.0 / fma(dx, dx, dy * dy);
      ax += fma(gx[q], dx, gy[q] * dy) * inv;
      ay += fma(gy[q], dx, -gx[q] * dy) * inv;
    }
    ax = wave_sum_f64(ax);
    ay = wave_sum_f64(ay);
    if (lane == 0) {
      wsum[c][wave][0] = ax;
      wsum[c][wave][1] = ay;
    }
  }
  __syncthreads();
  for (int c = c0 + cs * tid; c < count; c += cs * int(blockDim.x)) {
    double sx = 0.0, sy = 0.0;
    for (int v = 0; v < nwaves(); ++v) {
      sx += wsum[c][v][0];
      sy += wsum[c][v][1];
    }
    st_agent(partials + 2 * (size_t(c) * nch + chunk), sx);
    st_agent(partials + 2 * (size_t(c) * nch + chunk) + 1, sy);
  }
  if (!last_arrival(counter, gridDim.x * gridDim.z, &s_last)) return;
  static_assert(kKMax <= 256, "one candidate per thread");
  uint64_t key = 0;
  double rk = 0.0;
  if (tid < count) {
    key = cand->keys[tid];
    rk = radii[key_f(key) / uint32_t(N)];
  }
  winner_from_partials(count, cand->flags, key, rk, partials, N, S.z ? 1.0 : double(N), nch, w, bb, wd);
}

// Same merge functions, workgroup size and record order as the fused step
// tail, so the result is the one the tail reaches.
__global__ __launch_bounds__(256) void k_merge(int fp64, const void* __restrict__ recs,
                                               const uint64_t* __restrict__ heads,
                                               const uint64_t* __restrict__ seconds, int nrec, int N,
                                               int recheck_k, float tau_band, unsigned int* __restrict__ flagword,
                                               CandList* __restrict__ cand, Winner* __restrict__ w) {
  extern __shared__ __align__(16) unsigned char smem[];
  MergeScratch* Sm = reinterpret_cast<MergeScratch*>(smem);
  const int b = blockIdx.x;
  if (fp64) {
    merge64_tail<4>(reinterpret_cast<const BlockBest64*>(recs) + size_t(nrec) * b, nrec, N, w + b, Sm);
  } else {
    select32_tail<4>(reinterpret_cast<const BlockList32*>(recs) + size_t(nrec) * b, heads + size_t(nrec) * b,
                     seconds + size_t(nrec) * b, nrec, recheck_k, tau_band, flagword + b, cand + b, Sm, true);
  }
}

__global__ __launch_bounds__(64) void k_pick(PickArgs a) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const int32_t* fp = a.forced + size_t(a.fstride) * b + 2 * a.step;
  const uint32_t fm = uint32_t(fp[0]), fj = uint32_t(fp[1]);
  const uint32_t ff = fm * uint32_t(a.N) + fj;
  Winner* w = a.winner + b;
  CandList* cand = a.cand + b;
  const Winner own = *w;
  // FP32: was the forced point among the re-checked candidates?
  bool listed = false;
  if (!a.fp64) {
    const int count = min(max(cand->count, 0), kKMax);
    for (int i = lane; i < count; i += 64) listed |= key_f(cand->keys[i]) == ff;
  }
  listed = __ballot(listed) != 0;
  __syncthreads();  // every lane has read the short-list
  if (lane != 0) return;
  const size_t s = size_t(a.steps) * size_t(b) + size_t(a.step);
  a.idx[2 * s] = own.m;
  a.idx[2 * s + 1] = own.j;
  a.p[s] = own.cx * own.cx + own.cy * own.cy;  // as the selection compared it
  a.margin[s] = own.margin;
  a.flags[s] = (own.flags & 7) | (listed ? kFlagForcedListed : 0);
  if (a.fp64) {
    Winner o = own;
    o.m = int32_t(fm);
    o.j = int32_t(fj);
    o.cx = a.probe[2 * b];
    o.cy = a.probe[2 * b + 1];
    o.margin = __builtin_nan("");
    o.kcount = 0;
    o.fp32err = 0.0;
    *w = o;
  } else {
    cand->count = 1;
    cand->flags = kFlagForced | (own.flags & 7);
    cand->pmax32 = 0.f;
    cand->keys[0] = uint64_t(~ff);  // P = 0: the re-check supplies the value
  }
}

__global__ __launch_bounds__(256) void k_zero(ZeroArgs z) {
  for (int r = 0; r < z.n; ++r)
    for (int i = int(threadIdx.x); i < z.words[r]; i += int(blockDim.x)) z.p[r][i] = 0u;
}

__global__ __launch_bounds__(256) void k_update(double* __restrict__ g64, float* __restrict__ g32, UpdateArgs U) {
  __shared__ double wd[16];
  __shared__ int s_last;
  const int b = blockIdx.y;
  g64 += 2 * size_t(U.N) * b;
  if (g32) g32 += 2 * size_t(U.N) * b;
  U.epart += size_t(gridDim.x) * b;
  U.counter += b;
  U.R = record_of(U.R, b);
  const Blaschke B = blaschke_of(U);
  const int N = U.N;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kUpdPerThread; ++q) {
    const int n = blockIdx.x * (kUpdThreads * kUpdPerThread) + q * kUpdThreads + threadIdx.x;
    if (n < N) {
      double hx, hy;
      blaschke_apply(B, U.omega, N, n, g64[2 * n], g64[2 * n + 1], hx, hy);
      g64[2 * n] = hx;
      g64[2 * n + 1] = hy;
      if (g32) {
        g32[2 * n] = float(hx);
        g32[2 * n + 1] = float(hy);
      }
      acc += fma(hx, hx, hy * hy);
    }
  }
  update_finish(U, acc, wd, &s_last);
}

// ---------------------------------------------------------------- launchers
hipError_t launch_prepare(double* g64, float* g32, int N, double* epart, int* nonfinite, unsigned int* counter,
                          const RecordArgs& R, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3(update_blocks(N), batch), dim3(kUpdThreads), 0, s, g64, g32, N, epart,
                     nonfinite, counter, R);
  return hipGetLastError();
}

hipError_t launch_force(const int32_t* forced, int fstride, int step, int N, CandList* cand, int batch,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_force, dim3(batch), dim3(64), 0, s, forced, fstride, step, N, cand);
  return hipGetLastError();
}

hipError_t launch_merge(bool fp64, const void* recs, const uint64_t* heads, const uint64_t* seconds, int nrec, int N,
                        int recheck_k, float tau_band, unsigned int* flagword, CandList* cand, Winner* w,
                        int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_merge, dim3(batch), dim3(256), uint32_t(sizeof(MergeScratch)), s, fp64 ? 1 : 0, recs, heads,
                     seconds, nrec, N, recheck_k, tau_band, flagword, cand, w);
  return hipGetLastError();
}

hipError_t launch_zero(const ZeroArgs& z, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, z);
  return hipGetLastError();
}

hipError_t launch_pick(const PickArgs& a, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_pick, dim3(batch), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_recheck(const CandList* cand, const double* g, const double* omega, const double* radii, int N,
                          double* partials, unsigned int* counter, Winner* w, int batch, hipStream_t s,
                          const RecheckSamples& S) {
  const int ns = S.z ? S.ns : N;
  const int nch = recheck_chunks(ns);
  if ((ns + nch - 1) / nch > 256 * kRecheckPerThread) return hipErrorInvalidValue;  // a chunk fits the registers
  // candidate groups: at least a few hundred workgroups for a short signal
  const int groups = nch >= 128 ? 1 : nch >= 32 ? 2 : nch >= 8 ? 4 : 8;
  hipLaunchKernelGGL(k_recheck, dim3(nch, batch, groups), dim3(256), 0, s, cand, g, omega, radii, N, nch, partials,
                     counter, w, S);
  return hipGetLastError();
}

hipError_t launch_update(double* g64, float* g32, const UpdateArgs& U, int batch, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  launch_ev(k_update, dim3(update_blocks(U.N), batch), dim3(kUpdThreads), 0u, s, e0, e1, g64, g32, U);
  return hipGetLastError();
}

}  // namespace afd
