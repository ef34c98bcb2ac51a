// The re-check winner, the remainder update of Sec. 2, eq. (7), per sample,
// and the record of a finished step: shared by the stand-alone re-check and
// update kernels and by the fused step tail (afd_advance.hip).
#pragma once

#include "afd_select.h"

namespace afd {

// Per-step constants of G' = (G (1 - r w^d) - c s) e^{-2 pi i j/N} / (w^d - r),
// a = r e^{2 pi i j/N}, z_n = e^{2 pi i n/N}, w^d = e^{2 pi i (n - j)/N},
// s = sqrt(1 - r^2): the same rational map as eq. (7), written with the
// sample angles relative to the selected angle.
struct Blaschke {
  double r, csx, csy, wjx, wjy;
  int j;
};

__device__ __forceinline__ Blaschke blaschke_of(Winner W, const double* __restrict__ radii,
                                                const double* __restrict__ omega, int N, int M) {
  W.m = min(max(W.m, 0), M - 1);
  Blaschke B;
  B.j = min(max(W.j, 0), N - 1);
  B.r = radii[W.m];
  const double s = sqrt((1.0 - B.r) * (1.0 + B.r));
  B.wjx = omega[2 * B.j];
  B.wjy = -omega[2 * B.j + 1];  // e^{-2 pi i j/N}
  B.csx = W.cx * s;
  B.csy = W.cy * s;
  return B;
}

__device__ __forceinline__ Blaschke blaschke_of(const UpdateArgs& U) {
  return blaschke_of(*U.R.w, U.radii, U.omega, U.N, U.M);
}

__device__ __forceinline__ void blaschke_apply(const Blaschke& B, const double* __restrict__ omega, int N, int n,
                                               double gx, double gy, double& hx, double& hy) {
  const int d = n >= B.j ? n - B.j : n - B.j + N;  // (n - j) mod N
  const double ox = omega[2 * d], oy = omega[2 * d + 1];
  const double ux = fma(-B.r, ox, 1.0), uy = -B.r * oy;
  const double nx = fma(gx, ux, -gy * uy) - B.csx;
  const double ny = fma(gx, uy, gy * ux) - B.csy;
  const double dx = ox - B.r, dy = oy;
  const double inv = 1.0 / fma(dx, dx, dy * dy);
  const double qx = fma(nx, dx, ny * dy) * inv;
  const double qy = fma(ny, dx, -nx * dy) * inv;
  hx = fma(qx, B.wjx, -qy * B.wjy);
  hy = fma(qx, B.wjy, qy * B.wjx);
}

// Winner of the short-list from the chunk partial sums of the direct rule
// (Sec. 3.1, eq. term81): partials[i][ch] holds the (re, im) sum of
// G[n] / (1 - r_i e^{2 pi i (j_i - n)/N}) over chunk ch of the samples for
// candidate i; the inner product is that sum times sqrt(1 - r_i^2)/div (div = N,
// or 1 for weighted non-uniform samples).  One
// candidate per thread (count <= kKMax <= blockDim.x): thread i passes its
// key and radius (ignored for i >= count).  Largest |.|^2 wins, ties to the
// lowest flat index.  Thread 0 writes the result to *w (any address space);
// `bb`, `wd`: LDS Best[16], double[16].
__device__ __forceinline__ void winner_from_partials(int count, int cflags, uint64_t key, double r,
                                                     const double* __restrict__ partials, int N, double div,
                                                     int nch, Winner* w, Best* bb, double* wd) {
  const bool forced = (cflags & kFlagForced) != 0;
  Best b{-1.0, -1.0, 0.0, 0.0, 0xffffffffu};
  double err = 0.0;
  if (int(threadIdx.x) < count) {
    const double* pp = partials + 2 * size_t(threadIdx.x) * nch;
    double ax = 0.0, ay = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      ax += ld_agent(pp + 2 * ch);
      ay += ld_agent(pp + 2 * ch + 1);
    }
    const double s = sqrt((1.0 - r) * (1.0 + r)) / div;
    const Best x{(ax * s) * (ax * s) + (ay * s) * (ay * s), -1.0, ax * s, ay * s, key_f(key)};
    err = fabs(double(key_p(key)) - x.p1);
    b = x;
  }
  const Best rb = block_best(b, bb);
  err = wave_max_f64(err);
  if ((threadIdx.x & 63) == 0) wd[threadIdx.x >> 6] = err;
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = wd[0];
    for (int i = 1; i < nwaves(); ++i) e = fmax(e, wd[i]);
    Winner o;
    const bool valid = count > 0 && rb.f != 0xffffffffu;
    o.m = valid ? int32_t(rb.f / uint32_t(N)) : 0;
    o.j = valid ? int32_t(rb.f % uint32_t(N)) : 0;
    o.cx = valid ? rb.vx : 0.0;
    o.cy = valid ? rb.vy : 0.0;
    if (forced || count < 2 || !valid) o.margin = __builtin_nan("");
    else o.margin = rb.p1 > 0.0 ? (rb.p1 - rb.p2) / rb.p1 : 0.0;
    o.kcount = forced ? 1 : count;
    o.flags = cflags & 7;
    o.ax = o.ay = 0.0;
    o.fp32err = (forced || !valid || !(rb.p1 > 0.0)) ? 0.0 : e / rb.p1;
    *w = o;
  }
}

// The record of signal b of a batch.
__device__ __forceinline__ RecordArgs record_of(RecordArgs R, int b) {
  const size_t s = size_t(R.steps) * size_t(b);
  R.w += b;
  R.idx += 2 * s;
  R.a += 2 * s;
  R.coef += 2 * s;
  R.energy += s + size_t(b);
  R.margin += s;
  R.kcount += s;
  R.flags += s;
  R.fp32err += s;
  return R;
}

__device__ __forceinline__ void write_record(const RecordArgs& R, int step, double E) {
  if (step < 0) {
    R.energy[0] = E;
    return;
  }
  Winner W = *R.w;
  W.m = min(max(W.m, 0), R.M - 1);
  W.j = min(max(W.j, 0), R.N - 1);
  const double r = R.radii[W.m];
  R.idx[2 * step] = W.m;
  R.idx[2 * step + 1] = W.j;
  R.a[2 * step] = r * R.omega[2 * W.j];
  R.a[2 * step + 1] = r * R.omega[2 * W.j + 1];
  R.coef[2 * step] = W.cx;
  R.coef[2 * step + 1] = W.cy;
  R.energy[step + 1] = E;
  R.margin[step] = W.margin;
  R.kcount[step] = W.kcount;
  R.flags[step] = W.flags;
  R.fp32err[step] = W.fp32err;
}

// energy of the samples from the per-workgroup partial sums, in index order
__device__ __forceinline__ double energy_from_parts(const double* __restrict__ epart, int nparts, int N,
                                                    double* wd) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += ld_agent(epart + i);
  return block_sum_f64(acc, wd) / double(N);
}

// End of an update launch: publish this workgroup's energy partial; the last
// workgroup sums them and records the step.  `wd`: LDS double[16], `flag`: LDS int.
// (U: this signal's view, see k_update)
__device__ __forceinline__ void update_finish(const UpdateArgs& U, double acc, double* wd, int* flag) {
  const double tot = block_sum_f64(acc, wd);
  if (threadIdx.x == 0) st_agent(U.epart + blockIdx.x, tot);
  if (!last_arrival(U.counter, gridDim.x, flag)) return;
  const double E = energy_from_parts(U.epart, int(gridDim.x), U.N, wd);
  if (threadIdx.x == 0) write_record(U.R, U.step, E);
}

}  // namespace afd
