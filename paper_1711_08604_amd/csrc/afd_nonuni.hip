// Non-uniform samples (Sec. 3.2, the remark after Step 2): the samples sit
// at z_n = e^{2 pi i t_n} (positions t_n in turns), the inner product is the
// quadrature sum_n w_n G(z_n) conj(F(z_n)), and the DFT of the samples
// becomes a non-uniform DFT.  With c_l = sum_n w_n G_n e^{-2 pi i l t_n} the
// grid value on the uniform polar grid a = r e^{2 pi i j/N} is
//   sqrt(1 - r^2) sum_{l >= 0} r^l c_l e^{2 pi i l j/N}        (eq. ku12),
// the geometric expansion of the Szego kernel; unlike the uniform case c_l
// is not N-periodic, so the series is not folded into 1/(1 - r^N).  A plan
// computes the modes l < K N (K a power of two) that the largest radius
// needs (the same 2^-60 / 2^-40 cut as the uniform path's radius tables);
// the radius kernel runs on c_0..c_{N-1} with the scale sqrt(1 - r^2), and a
// radius whose terms outlast N reads its own folded spectrum
// cf[l] = sum_k (r^N)^k c_(l + kN) (k_nu_fold).
//
// c_l, l < K N, comes from a gridding non-uniform FFT (type 1) with the
// "exponential of semicircle" kernel phi(x) = exp(beta (sqrt(1 - (2x/W)^2) - 1)),
// |x| < W/2 grid cells (Barnett, Magland, af Klinteberg, SIAM J. Sci. Comput.
// 2019): with the modes shifted to l' = l - KN/2 (strengths times
// e^{-2 pi i (KN/2) t_n}), each point k of a grid of G = 4KN cells gathers
// b_k = sum_n u'_n phi(G t_n - k) (wrapped), a length-G forward FFT gives
// B_{l'}, and c_l = B_{l'} / Phi(l'/G), Phi the kernel's Fourier transform
// (tabled per plan).  W = 12 and beta = 2.69 W keep the error near 1e-14 of
// max |c| (measured against the exact sum).
//
//   k_nu_spread           b_k from the samples within W/2 of cell k (index
//                         ranges per cell, samples in position order)
//   (FFT)                 the forward transforms of afd_fwd.hip, length G
//   k_nu_deconv           c_l = B_{l'} / Phi(l'/G), in the precision of the
//                         radius transforms
//   k_nu_fold             the folded spectra of the radii that need more
//                         than N terms
//   k_nu_prepare          E_0 = sum_n w_n |G_n|^2 and the non-finite check
//   k_nu_update           eq. (7) at the sample points and the quadrature
//                         energy; the last workgroup records the step
// All in double precision; the FP32 mode's spectrum is the double one
// rounded once.  A batch (grid dimension y) shares the positions, weights and
// tables; each signal has its own samples, grid, spectrum and records.
#include <algorithm>
#include <vector>

#include "afd_update.h"

namespace afd {

constexpr int kNuUpdThreads = 256;
constexpr int kNuUpdPer = 4;

int nu_update_blocks(int ns) { return (ns + kNuUpdThreads * kNuUpdPer - 1) / (kNuUpdThreads * kNuUpdPer); }
static_assert(kNuUpdThreads * kNuUpdPer == 1024, "the plan sizes the energy partials with update_blocks()");

int nu_grid_log2(int logn) { return logn + 2 < 6 ? 6 : logn + 2; }  // G = 4N, at least 64 > 2W

// b_k = sum of u_n phi(x), u_n = G_n ws_n (ws_n = w_n e^{-2 pi i (N/2) t_n}),
// x = G t_n - k wrapped to [-G/2, G/2), over the samples of cell k's ranges
// (rng[k] = {lo1, hi1, lo2, hi2}: a window that wraps around t = 0 has two).
__global__ __launch_bounds__(256) void k_nu_spread(const double* __restrict__ g, const double* __restrict__ ws,
                                                   const double* __restrict__ turns, const int4* __restrict__ rng,
                                                   int G, int ns, double* __restrict__ b) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= G) return;
  g += 2 * size_t(ns) * blockIdx.y;
  b += 2 * size_t(G) * blockIdx.y;
  const int4 r = rng[k];
  const double dG = double(G), half = 0.5 * dG;
  double ax = 0.0, ay = 0.0;
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    const int lo = part ? r.z : r.x, hi = part ? r.w : r.y;
    for (int n = lo; n < hi; ++n) {
      double x = turns[n] * dG - double(k);  // exact: G is a power of two
      if (x >= half) x -= dG;
      if (x < -half) x += dG;
      const double z = x * (2.0 / kEsWidth);
      const double phi = exp(kEsBeta * (sqrt(fmax(1.0 - z * z, 0.0)) - 1.0));
      const double gx = g[2 * n], gy = g[2 * n + 1], sx = ws[2 * n], sy = ws[2 * n + 1];
      const double ux = fma(gx, sx, -gy * sy), uy = fma(gx, sy, gy * sx);
      ax = fma(ux, phi, ax);
      ay = fma(uy, phi, ay);
    }
  }
  b[2 * k] = ax;
  b[2 * k + 1] = ay;
}

// c_l = B_q / Phi((l - NM/2)/G), q = (l - NM/2) mod G, for the NM modes
// l < NM (NM = N, or K N when radii need K N terms): l < N into c, the
// rest into ctail[l - N].  From 2^15 points the forward transform leaves B
// in column order (bin q at (q mod N2) N1 + q / N2).
template <typename T>
__global__ __launch_bounds__(256) void k_nu_deconv(const double* __restrict__ B, const double* __restrict__ dinv,
                                                   int N, int NM, int G, int cols_l1, int cols_l2,
                                                   Cx<T>* __restrict__ c, Cx<T>* __restrict__ ctail) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= NM) return;
  B += 2 * size_t(G) * blockIdx.y;
  const int q = l >= NM / 2 ? l - NM / 2 : l - NM / 2 + G;
  const int pos = cols_l2 ? ((q & ((1 << cols_l2) - 1)) << cols_l1) + (q >> cols_l2) : q;
  const double d = dinv[l];
  const Cx<T> v{T(B[2 * pos] * d), T(B[2 * pos + 1] * d)};
  if (l < N)
    c[size_t(N) * blockIdx.y + l] = v;
  else
    ctail[size_t(NM - N) * blockIdx.y + (l - N)] = v;
}

// Folded spectra of the radii whose series outlasts N terms (Sec. 3.1,
// eq. ku12 with e^{2 pi i l j/N} depending on l mod N only): with
// rho = r^N, cf[l] = sum_k rho^k c_(l + kN), k < K, so that r^l cf[l] holds
// every term r^(l + kN) c_(l + kN) of the series (the radius kernel applies
// r^l).  Summed in double precision in the order of k.
template <typename T>
__global__ __launch_bounds__(256) void k_nu_fold(const Cx<T>* __restrict__ c, const Cx<T>* __restrict__ ctail,
                                                 const double* __restrict__ rho, int N, int K, int nfold,
                                                 Cx<T>* __restrict__ cfold) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= N) return;
  const int b = blockIdx.z;
  c += size_t(N) * b;
  ctail += size_t(N) * (K - 1) * b;
  // folded spectra f = blockIdx.y, blockIdx.y + gridDim.y, ... (grid y
  // holds at most kMaxGridY)
  for (int f = blockIdx.y; f < nfold; f += gridDim.y) {
    const double p = rho[f];
    double ax = double(c[l].x), ay = double(c[l].y), pk = 1.0;
    for (int k = 1; k < K; ++k) {
      pk *= p;
      const Cx<T> x = ctail[size_t(k - 1) * N + l];
      ax = fma(pk, double(x.x), ax);
      ay = fma(pk, double(x.y), ay);
    }
    cfold[(size_t(b) * nfold + f) * N + l] = {T(ax), T(ay)};
  }
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
  const int b = blockIdx.y;
  g += 2 * size_t(ns) * b;
  epart += size_t(gridDim.x) * b;
  counter += b;
  R = record_of(R, b);
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
  const int b = blockIdx.y;
  g += 2 * size_t(ns) * b;
  U.epart += size_t(gridDim.x) * b;
  U.counter += b;
  U.R = record_of(U.R, b);
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
hipError_t launch_nu_fourier(const double* g, const NuTables& t, int logn, bool fp64, void* c, int ns, int batch,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int N = 1 << logn;
  const int NM = 1 << t.lognm;  // modes: N, or K N for the folded radii
  const int K = NM / N;
  const int lg = nu_grid_log2(t.lognm);
  const int G = 1 << lg;
  launch_ev(k_nu_spread, dim3((G + 255) / 256, batch), dim3(256), 0u, s, e0, nullptr, g, t.ws, t.turns, t.rng, G, ns,
            t.b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_fwd(lg, true, t.b, t.tw1, t.tw2, t.omega, t.xt, t.B, batch, s);
  if (e != hipSuccess) return e;
  const FwdPlan fp = fwd_plan(lg, true);
  const int cl1 = lg > kMaxLdsLogN ? fp.l1 : 0, cl2 = lg > kMaxLdsLogN ? fp.l2 : 0;
  hipEvent_t ed = t.nfold > 0 ? nullptr : e1;
  if (fp64)
    launch_ev(k_nu_deconv<double>, dim3((NM + 255) / 256, batch), dim3(256), 0u, s, nullptr, ed,
              static_cast<const double*>(t.B), t.dinv, N, NM, G, cl1, cl2, static_cast<Cx<double>*>(c),
              static_cast<Cx<double>*>(t.ctail));
  else
    launch_ev(k_nu_deconv<float>, dim3((NM + 255) / 256, batch), dim3(256), 0u, s, nullptr, ed,
              static_cast<const double*>(t.B), t.dinv, N, NM, G, cl1, cl2, static_cast<Cx<float>*>(c),
              static_cast<Cx<float>*>(t.ctail));
  if (t.nfold > 0) {
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((N + 255) / 256, t.nfold < kMaxGridY ? t.nfold : kMaxGridY, batch);
    if (fp64)
      launch_ev(k_nu_fold<double>, grid, dim3(256), 0u, s, nullptr, e1, static_cast<const Cx<double>*>(c),
                static_cast<const Cx<double>*>(t.ctail), t.rho, N, K, t.nfold, static_cast<Cx<double>*>(t.cfold));
    else
      launch_ev(k_nu_fold<float>, grid, dim3(256), 0u, s, nullptr, e1, static_cast<const Cx<float>*>(c),
                static_cast<const Cx<float>*>(t.ctail), t.rho, N, K, t.nfold, static_cast<Cx<float>*>(t.cfold));
  }
  return hipGetLastError();
}

hipError_t launch_nu_prepare(const double* g, const double* wt, int ns, double* epart, int* nonfinite,
                             unsigned int* counter, const RecordArgs& R, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_nu_prepare, dim3(nu_update_blocks(ns), batch), dim3(kNuUpdThreads), 0, s, g, wt, ns, epart,
                     nonfinite, counter, R);
  return hipGetLastError();
}

hipError_t launch_nu_update(double* g, const double* wt, const double* z, int ns, const UpdateArgs& U, int batch,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_ev(k_nu_update, dim3(nu_update_blocks(ns), batch), dim3(kNuUpdThreads), 0u, s, e0, e1, g, wt, z, ns, U);
  return hipGetLastError();
}

// ---------------------------------------------------------------- plan tables (host)
// 1/Phi(l'/G), l' = l - N/2, l < N: Phi(xi) = 2 int_0^{W/2} phi(x) cos(2 pi xi x) dx
// by Gauss-Legendre quadrature (nodes by Newton's method on P_q) in long double.
void nu_deconv_table(int N, int G, double* dinv) {
  constexpr int q = 100;
  long double xs[q], ws[q];
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < q; ++i) {
    long double z = cosl(pi * ((long double)i + 0.75L) / ((long double)q + 0.5L));
    long double pp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int j = 2; j <= q; ++j) {
        const long double p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / (long double)j;
        p0 = p1;
        p1 = p2;
      }
      pp = (long double)q * (z * p1 - p0) / (z * z - 1.0L);
      const long double dz = p1 / pp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    // node on [0, W/2]
    xs[i] = (z + 1.0L) * (long double)kEsWidth / 4.0L;
    ws[i] = 2.0L / ((1.0L - z * z) * pp * pp) * (long double)kEsWidth / 4.0L;
  }
  long double phi[q];
  for (int i = 0; i < q; ++i) {
    const long double zz = 2.0L * xs[i] / (long double)kEsWidth;
    phi[i] = expl((long double)kEsBeta * (sqrtl(1.0L - zz * zz) - 1.0L)) * ws[i];
  }
  for (int l = 0; l < N; ++l) {
    const long double xi = (long double)(l - N / 2) / (long double)G;
    long double acc = 0.0L;
    for (int i = 0; i < q; ++i) acc += phi[i] * cosl(2.0L * pi * xi * xs[i]);
    dinv[l] = (double)(1.0L / (2.0L * acc));
  }
}

// Per cell k of the G-cell grid: the samples with |G t_n - k| < W/2 (mod G),
// as up to two index ranges {lo1, hi1, lo2, hi2} (positions increasing).
void nu_cell_ranges(const double* turns, int ns, int G, int32_t* rng) {
  std::vector<double> p(ns);
  for (int n = 0; n < ns; ++n) p[n] = turns[n] * double(G);  // exact
  const double h = kEsWidth / 2.0;
  auto above = [&](double a) { return int32_t(std::upper_bound(p.begin(), p.end(), a) - p.begin()); };
  auto below = [&](double b) { return int32_t(std::lower_bound(p.begin(), p.end(), b) - p.begin()); };
  for (int k = 0; k < G; ++k) {
    const double a = double(k) - h, b = double(k) + h;
    int32_t* r = rng + 4 * size_t(k);
    r[2] = r[3] = 0;
    if (a < 0.0) {
      r[0] = 0;
      r[1] = below(b);
      r[2] = above(a + double(G));
      r[3] = ns;
    } else if (b > double(G)) {
      r[0] = above(a);
      r[1] = ns;
      r[2] = 0;
      r[3] = below(b - double(G));
    } else {
      r[0] = above(a);
      r[1] = below(b);
    }
  }
}

}  // namespace afd
