// Non-uniform samples (Sec. 3.2, the remark after Step 2): the samples sit
// at z_n = e^{2 pi i t_n} (positions t_n in turns), the inner product is the
// quadrature sum_n w_n G(z_n) conj(F(z_n)), and the DFT of the samples
// becomes a non-uniform DFT.  With c_l = sum_n w_n G_n e^{-2 pi i l t_n} the
// grid value on the uniform polar grid a = r e^{2 pi i j/N} is
//   sqrt(1 - r^2) sum_{l >= 0} r^l c_l e^{2 pi i l j/N}        (eq. ku12),
// the geometric expansion of the Szego kernel; unlike the uniform case c_l
// is not N-periodic, so the series is not folded into 1/(1 - r^N).  A plan
// accepts only radii whose terms beyond l = N - 1 are negligible (the same
// 2^-60 / 2^-40 cut as the uniform path's), so the radius kernel runs
// unchanged on c_0..c_{N-1} with the scale sqrt(1 - r^2).
//
//   k_nudft, k_nudft_sum  c_l, l < N: partial sums over chunks of samples,
//                         then summed over the chunks in order
//   k_nu_prepare          E_0 = sum_n w_n |G_n|^2 and the non-finite check
//   k_nu_update           eq. (7) at the sample points and the quadrature
//                         energy; the last workgroup records the step
// All in double precision; the FP32 mode's spectrum is the double one
// rounded once.  One signal per plan.
#include "afd_update.h"

namespace afd {

constexpr int kNuThreads = 128;  // k_nudft workgroup
constexpr int kNuL = 4;          // consecutive frequencies per thread
constexpr int kNuChunk = 256;    // samples per workgroup (grid dimension y)
constexpr int kNuUpdThreads = 256;
constexpr int kNuUpdPer = 4;

int nudft_chunks(int ns) { return (ns + kNuChunk - 1) / kNuChunk; }
int nu_update_blocks(int ns) { return (ns + kNuUpdThreads * kNuUpdPer - 1) / (kNuUpdThreads * kNuUpdPer); }
static_assert(kNuUpdThreads * kNuUpdPer == 1024, "the plan sizes the energy partials with update_blocks()");

// frac(l t) for an integer l < 2^24 and a double t, to a rounding of the
// result: l t = p + e exactly (e from the fused multiply-add), p - rint(p) is
// exact, and adding e rounds once.
__device__ __forceinline__ double frac_of_product(double l, double t) {
#pragma clang fp contract(off)
  // (no contraction: p must be the rounded product for e to be its error)
  const double p = l * t;
  const double e = fma(l, t, -p);
  return (p - rint(p)) + e;
}

// part[chunk][l] = sum over the chunk's samples of u_n e^{-2 pi i l t_n},
// u_n = w_n G_n.  Thread: kNuL consecutive l; e^{-2 pi i l0 t_n} from the
// exact fractional turn and sincospi, the next ones by multiplying with
// conj(z_n).
__global__ __launch_bounds__(kNuThreads) void k_nudft(const double* __restrict__ g, const double* __restrict__ wt,
                                                      const double* __restrict__ turns, const double* __restrict__ z,
                                                      int ns, int N, double* __restrict__ part) {
  __shared__ double su[kNuChunk][2];
  __shared__ double sz[kNuChunk][2];
  __shared__ double st[kNuChunk];
  const int n0 = blockIdx.y * kNuChunk;
  const int cnt = min(kNuChunk, ns - n0);
  for (int i = threadIdx.x; i < cnt; i += kNuThreads) {
    const int n = n0 + i;
    const double w = wt[n];
    su[i][0] = w * g[2 * n];
    su[i][1] = w * g[2 * n + 1];
    sz[i][0] = z[2 * n];
    sz[i][1] = z[2 * n + 1];
    st[i] = turns[n];
  }
  __syncthreads();
  const int l0 = (blockIdx.x * kNuThreads + threadIdx.x) * kNuL;
  if (l0 >= N) return;
  double ax[kNuL], ay[kNuL];
#pragma unroll
  for (int i = 0; i < kNuL; ++i) ax[i] = ay[i] = 0.0;
  const double dl0 = double(l0);
  for (int i = 0; i < cnt; ++i) {
    const double f = frac_of_product(dl0, st[i]);
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);
    double ex = cs, ey = -sn;  // e^{-2 pi i l0 t}
    const double ux = su[i][0], uy = su[i][1];
    const double zx = sz[i][0], zy = -sz[i][1];  // conj(z_n)
#pragma unroll
    for (int q = 0; q < kNuL; ++q) {
      ax[q] = fma(ux, ex, fma(-uy, ey, ax[q]));
      ay[q] = fma(ux, ey, fma(uy, ex, ay[q]));
      if (q + 1 < kNuL) {
        const double nx = fma(ex, zx, -ey * zy);
        const double ny = fma(ex, zy, ey * zx);
        ex = nx;
        ey = ny;
      }
    }
  }
  double* o = part + 2 * (size_t(blockIdx.y) * N + l0);
#pragma unroll
  for (int q = 0; q < kNuL; ++q) {
    if (l0 + q < N) {
      o[2 * q] = ax[q];
      o[2 * q + 1] = ay[q];
    }
  }
}

// c_l = sum over the chunks, in chunk order, of part[chunk][l]; written in
// the precision of the radius transforms.
template <typename T>
__global__ __launch_bounds__(256) void k_nudft_sum(const double* __restrict__ part, int nchunk, int N,
                                                   Cx<T>* __restrict__ c) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= N) return;
  double x = 0.0, y = 0.0;
  for (int k = 0; k < nchunk; ++k) {
    x += part[2 * (size_t(k) * N + l)];
    y += part[2 * (size_t(k) * N + l) + 1];
  }
  c[l] = {T(x), T(y)};
}

// End of a pass over the samples: this workgroup's weighted energy partial
// is published; the last workgroup sums them in index order and records.
__device__ __forceinline__ void nu_finish(double acc, double* __restrict__ epart, unsigned int* counter,
                                          const RecordArgs& R, int step, double* wd, int* flag) {
  const double tot = block_sum_f64(acc, wd);
  if (threadIdx.x == 0) st_agent(epart + blockIdx.x, tot);
  if (!last_arrival(counter, gridDim.x, flag)) return;
  const double E = energy_from_parts(epart, int(gridDim.x), 1, wd);
  if (threadIdx.x == 0) write_record(R, step, E);
}

__global__ __launch_bounds__(kNuUpdThreads) void k_nu_prepare(const double* __restrict__ g,
                                                              const double* __restrict__ wt, int ns,
                                                              double* __restrict__ epart, int* __restrict__ nonfinite,
                                                              unsigned int* __restrict__ counter, RecordArgs R) {
  __shared__ double wd[16];
  __shared__ int s_last;
  double acc = 0.0;
  int bad = 0;
#pragma unroll
  for (int q = 0; q < kNuUpdPer; ++q) {
    const int n = blockIdx.x * (kNuUpdThreads * kNuUpdPer) + q * kNuUpdThreads + threadIdx.x;
    if (n < ns) {
      const double x = g[2 * n], y = g[2 * n + 1];
      if (!isfinite(x) || !isfinite(y)) bad = 1;
      acc += wt[n] * fma(x, x, y * y);
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  nu_finish(acc, epart, counter, R, -1, wd, &s_last);
}

// G' = (G (1 - r w) - c s) / (w - r) * conj(e^{2 pi i j/N}) with w = z_n
// conj(e^{2 pi i j/N}), s = sqrt(1 - r^2): eq. (7) with a = r e^{2 pi i j/N},
// the same rational map as the uniform update with the sample at z_n.
__global__ __launch_bounds__(kNuUpdThreads) void k_nu_update(double* __restrict__ g, const double* __restrict__ wt,
                                                             const double* __restrict__ z, int ns, UpdateArgs U) {
  __shared__ double wd[16];
  __shared__ int s_last;
  const Blaschke B = blaschke_of(U);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kNuUpdPer; ++q) {
    const int n = blockIdx.x * (kNuUpdThreads * kNuUpdPer) + q * kNuUpdThreads + threadIdx.x;
    if (n < ns) {
      const double zx = z[2 * n], zy = z[2 * n + 1];
      const double ox = fma(zx, B.wjx, -zy * B.wjy), oy = fma(zx, B.wjy, zy * B.wjx);
      const double gx = g[2 * n], gy = g[2 * n + 1];
      const double ux = fma(-B.r, ox, 1.0), uy = -B.r * oy;
      const double nx = fma(gx, ux, -gy * uy) - B.csx;
      const double ny = fma(gx, uy, gy * ux) - B.csy;
      const double dx = ox - B.r, dy = oy;
      const double inv = 1.0 / fma(dx, dx, dy * dy);
      const double qx = fma(nx, dx, ny * dy) * inv;
      const double qy = fma(ny, dx, -nx * dy) * inv;
      const double hx = fma(qx, B.wjx, -qy * B.wjy);
      const double hy = fma(qx, B.wjy, qy * B.wjx);
      g[2 * n] = hx;
      g[2 * n + 1] = hy;
      acc += wt[n] * fma(hx, hx, hy * hy);
    }
  }
  nu_finish(acc, U.epart, U.counter, U.R, U.step, wd, &s_last);
}

// ---------------------------------------------------------------- launchers
hipError_t launch_nudft(const double* g, const double* wt, const double* turns, const double* z, int ns, int N,
                        double* part, bool fp64, void* c, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int lpb = kNuThreads * kNuL;
  const dim3 grid((N + lpb - 1) / lpb, nudft_chunks(ns));
  launch_ev(k_nudft, grid, dim3(kNuThreads), 0u, s, e0, nullptr, g, wt, turns, z, ns, N, part);
  if (fp64)
    launch_ev(k_nudft_sum<double>, dim3((N + 255) / 256), dim3(256), 0u, s, nullptr, e1,
              static_cast<const double*>(part), nudft_chunks(ns), N, static_cast<Cx<double>*>(c));
  else
    launch_ev(k_nudft_sum<float>, dim3((N + 255) / 256), dim3(256), 0u, s, nullptr, e1,
              static_cast<const double*>(part), nudft_chunks(ns), N, static_cast<Cx<float>*>(c));
  return hipGetLastError();
}

hipError_t launch_nu_prepare(const double* g, const double* wt, int ns, double* epart, int* nonfinite,
                             unsigned int* counter, const RecordArgs& R, hipStream_t s) {
  hipLaunchKernelGGL(k_nu_prepare, dim3(nu_update_blocks(ns)), dim3(kNuUpdThreads), 0, s, g, wt, ns, epart,
                     nonfinite, counter, R);
  return hipGetLastError();
}

hipError_t launch_nu_update(double* g, const double* wt, const double* z, int ns, const UpdateArgs& U, hipStream_t s,
                            hipEvent_t e0, hipEvent_t e1) {
  launch_ev(k_nu_update, dim3(nu_update_blocks(ns)), dim3(kNuUpdThreads), 0u, s, e0, e1, g, wt, z, ns, U);
  return hipGetLastError();
}

}  // namespace afd
