// Outputs on either side of the maximal-selection loop:
//   k_recon, k_recon_sum  the partial sum S_n of expansion (Sn) on the N
//                         circle points, with the Takenaka-Malmquist system
//                         of Sec. 2, eq. (2), and the relative errors
//                         delta_k = ||G - S_k||_N^2 / ||G||_N^2 of Sec. 4,
//                         eq. er, for every k;
//   k_analytic_mask/out   the analytic (H^2) part of boundary samples,
//                         g = IDFT(h . DFT(x)), as two forward DFTs:
//                         IDFT(y) = conj(DFT(conj(y)))/N.
// All in double precision; signal b of a batch in grid dimension y.
#include "afd_select.h"

namespace afd {

constexpr int kRecThreads = 256;

// One thread per sample z = e^{2 pi i n/N} (or, for non-uniform samples, the
// point omega[n] of N = samples points).  With P_0 = 1 and
// d_k = 1 - conj(a_k) z: B_k = sqrt(1 - |a_k|^2) P_k / d_k, S += c_k B_k,
// P_{k+1} = P_k (z - a_k)/d_k.  With wpart, the wave sums of |G - S_k|^2
// (k = 0: |G|^2), times the quadrature weight wt[n] when wt is given, go to
// wpart[b][k][wave] for a fixed-order total.
__global__ __launch_bounds__(kRecThreads) void k_recon(const double* __restrict__ ak, const double* __restrict__ ck,
                                                       int steps, int N, const double* __restrict__ omega,
                                                       const double* __restrict__ G, double* __restrict__ S,
                                                       double* __restrict__ wpart, const double* __restrict__ wt) {
  const int b = blockIdx.y;
  const int n = int(blockIdx.x) * kRecThreads + int(threadIdx.x);
  const bool valid = n < N;
  const int nwt = int(gridDim.x) * (kRecThreads / 64);
  const int wv = int(blockIdx.x) * (kRecThreads / 64) + int(threadIdx.x >> 6);
  const bool lead = (threadIdx.x & 63) == 0;
  ak += 2 * size_t(steps) * b;
  ck += 2 * size_t(steps) * b;
  if (wpart) wpart += size_t(steps + 1) * size_t(nwt) * b;
  const double zx = valid ? omega[2 * n] : 1.0, zy = valid ? omega[2 * n + 1] : 0.0;
  double gx = 0.0, gy = 0.0;
  if (G && valid) {
    gx = G[2 * (size_t(N) * b + n)];
    gy = G[2 * (size_t(N) * b + n) + 1];
  }
  const double wn = (wt && valid) ? wt[n] : 1.0;
  if (wpart) {
    const double e = wave_sum_f64(wn * fma(gx, gx, gy * gy));
    if (lead) wpart[wv] = e;
  }
  double px = 1.0, py = 0.0, sx = 0.0, sy = 0.0;
  for (int k = 0; k < steps; ++k) {
    const double ax = ak[2 * k], ay = ak[2 * k + 1];
    const double cx = ck[2 * k], cy = ck[2 * k + 1];
    const double s = sqrt(fma(-ax, ax, fma(-ay, ay, 1.0)));
    const double dx = 1.0 - fma(ax, zx, ay * zy), dy = fma(ay, zx, -ax * zy);
    const double inv = 1.0 / fma(dx, dx, dy * dy);
    const double bx = s * fma(px, dx, py * dy) * inv, by = s * fma(py, dx, -px * dy) * inv;
    sx += fma(cx, bx, -cy * by);
    sy += fma(cx, by, cy * bx);
    const double nx = zx - ax, ny = zy - ay;
    const double qx = fma(nx, dx, ny * dy) * inv, qy = fma(ny, dx, -nx * dy) * inv;
    const double tx = fma(px, qx, -py * qy);
    py = fma(px, qy, py * qx);
    px = tx;
    if (wpart) {
      const double ex = gx - sx, ey = gy - sy;
      const double e = wave_sum_f64(valid ? wn * fma(ex, ex, ey * ey) : 0.0);
      if (lead) wpart[size_t(k + 1) * nwt + wv] = e;
    }
  }
  if (S && valid) {
    S[2 * (size_t(N) * b + n)] = sx;
    S[2 * (size_t(N) * b + n) + 1] = sy;
  }
}

// delta[b][k-1] = (sum of wpart[b][k]) / (sum of wpart[b][0]), k = 1..steps;
// one workgroup per k, the same fixed summation order for every row.
__global__ __launch_bounds__(kRecThreads) void k_recon_sum(const double* __restrict__ wpart, int steps, int nwt,
                                                           double* __restrict__ delta) {
  __shared__ double wd[16];
  const int b = blockIdx.y, k = int(blockIdx.x) + 1;
  wpart += size_t(steps + 1) * size_t(nwt) * b;
  double e0 = 0.0, ek = 0.0;
  for (int i = threadIdx.x; i < nwt; i += kRecThreads) {
    e0 += wpart[i];
    ek += wpart[size_t(k) * nwt + i];
  }
  e0 = block_sum_f64(e0, wd);
  ek = block_sum_f64(ek, wd);
  if (threadIdx.x == 0) delta[size_t(steps) * b + (k - 1)] = ek / e0;
}

// Position of DFT bin l in the forward transform's output: natural order, or
// with cols (N > 2^14) bin l = k2 + N2 k1 at k2 N1 + k1.
__device__ __forceinline__ int bin_pos(int l, int cols_l1, int cols_l2) {
  return cols_l2 ? ((l & ((1 << cols_l2) - 1)) << cols_l1) + (l >> cols_l2) : l;
}

// Y[l] = conj(h_l X_l), natural order; flags non-finite spectra.
__global__ __launch_bounds__(kRecThreads) void k_analytic_mask(const double* __restrict__ X, double* __restrict__ Y,
                                                               int N, int cols_l1, int cols_l2, int* flag) {
  const int b = blockIdx.y;
  const int l = int(blockIdx.x) * kRecThreads + int(threadIdx.x);
  if (l >= N) return;
  const size_t base = 2 * size_t(N) * b;
  const int p = bin_pos(l, cols_l1, cols_l2);
  const double xr = X[base + 2 * p], xi = X[base + 2 * p + 1];
  if (!isfinite(xr) || !isfinite(xi)) atomicOr(flag, 1);
  const double h = (l == 0 || 2 * l == N) ? 1.0 : (2 * l < N ? 2.0 : 0.0);
  Y[base + 2 * l] = h * xr;
  Y[base + 2 * l + 1] = -(h * xi);
}

// g[n] = conj(Z[n]) / N (Z the DFT of Y); nothing is written if the input was flagged.
__global__ __launch_bounds__(kRecThreads) void k_analytic_out(const double* __restrict__ Z, double* __restrict__ g,
                                                              int N, int cols_l1, int cols_l2,
                                                              const int* __restrict__ flag) {
  if (*flag & 1) return;
  const int b = blockIdx.y;
  const int n = int(blockIdx.x) * kRecThreads + int(threadIdx.x);
  if (n >= N) return;
  const size_t base = 2 * size_t(N) * b;
  const int p = bin_pos(n, cols_l1, cols_l2);
  const double inv = 1.0 / double(N);
  g[base + 2 * n] = Z[base + 2 * p] * inv;
  g[base + 2 * n + 1] = -(Z[base + 2 * p + 1] * inv);
}

// ---------------------------------------------------------------- launchers
int recon_waves(int N) { return (N + kRecThreads - 1) / kRecThreads * (kRecThreads / 64); }

hipError_t launch_recon(const double* a, const double* c, int steps, int N, const double* omega, const double* G,
                        double* S, double* wpart, double* delta, int batch, hipStream_t s, const double* wt) {
  const int blocks = (N + kRecThreads - 1) / kRecThreads;
  hipLaunchKernelGGL(k_recon, dim3(blocks, batch), dim3(kRecThreads), 0, s, a, c, steps, N, omega, G, S, wpart, wt);
  if (wpart && delta && steps > 0)
    hipLaunchKernelGGL(k_recon_sum, dim3(steps, batch), dim3(kRecThreads), 0, s, wpart, steps, recon_waves(N),
                       delta);
  return hipGetLastError();
}

hipError_t launch_analytic_mask(const double* X, double* Y, int N, int cols_l1, int cols_l2, int* flag, int batch,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_analytic_mask, dim3((N + kRecThreads - 1) / kRecThreads, batch), dim3(kRecThreads), 0, s, X,
                     Y, N, cols_l1, cols_l2, flag);
  return hipGetLastError();
}

hipError_t launch_analytic_out(const double* Z, double* g, int N, int cols_l1, int cols_l2, const int* flag,
                               int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_analytic_out, dim3((N + kRecThreads - 1) / kRecThreads, batch), dim3(kRecThreads), 0, s, Z,
                     g, N, cols_l1, cols_l2, flag);
  return hipGetLastError();
}

}  // namespace afd
