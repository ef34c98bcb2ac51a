// Internal interface between the host plan (afd_api.hip) and the kernels
// (afd_fwd.hip, afd_radius.hip, afd_step.hip): device record layouts and
// launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <cmath>

namespace afd {

constexpr int kMaxLogN = 20;       // N <= 2^20
constexpr int kMaxLdsLogN = 14;    // single-workgroup (LDS-resident) transforms up to 2^14
constexpr int kListC = 64;         // per-workgroup candidate list length (FP32 mode)
constexpr int kListCap = 1024;     // per-workgroup LDS gather capacity before the exact fallback
constexpr int kKMax = 256;         // longest short-list re-checked in double
constexpr int kSelCap = 1024;      // global gather capacity of the short-list selection
// Default re-check band (relative to the FP32 maximum): 4e-6 up to 2^14
// points, then x 2^(1/3) per doubling (1.6e-5 at 2^20), about eight times the
// largest FP32 error of |.|^2 measured at those sizes.
inline float default_tau_band(int logn) {
  return logn <= 14 ? 4e-6f : float(4e-6 * std::exp2((logn - 14) / 3.0));
}

// flags (per step; bits 0-2 are reported)
constexpr int kFlagBandTruncated = 1;
constexpr int kFlagListTruncated = 2;
constexpr int kFlagFallback = 4;
constexpr int kFlagForced = 8;

// FP64 mode: best and runner-up of one radius workgroup
struct BlockBest64 {
  double p1, p2, vx, vy;
  uint32_t f;
  uint32_t pad;
};

// FP32 mode: exact top entries (key order) among the workgroup's points within
// the re-check band of the workgroup maximum
struct BlockList32 {
  float pmax;
  uint32_t count;   // entries written (<= kListC)
  uint32_t total;   // points that passed the band (may exceed count)
  uint32_t flags;
  uint64_t keys[kListC];
};

struct CandList {
  int32_t count;
  int32_t flags;
  float pmax32;
  int32_t pad;
  uint64_t keys[kKMax];
};

struct Winner {
  int32_t m, j;
  int32_t kcount, flags;
  double ax, ay;
  double cx, cy;
  double margin;
  double fp32err;  // FP32 mode: max |P32 - P64| / P64max over the re-checked points
};

struct RadiusParams {
  const void* c;      // spectrum, N complex (T)
  const void* pw;     // [M][TPR]  r_m^t
  const void* pv;     // [M][E]    r_m^(TPR v)
  const void* pq;     // [M][E]    r_m^((TPR/R0) v), R0 the radix of the first pass
  const int* lsig;    // [M]       significant spectrum length: the terms l >= lsig[m] are dropped
  const int* order;   // [M][2]    (radius, lsig) of workgroup b when one radius per workgroup (lsig descending)
  const void* scale;  // [M]       sqrt(1-r^2) / (N (1 - r^N))
  const void* tw;     // Stockham twiddles of the inverse transform
  int M;
  int rpb;            // radii per workgroup
  float tau_band;     // FP32 lists: relative band below the workgroup maximum
  int recheck_k;      // FP32: minimum short-list length
  void* out;          // BlockBest64[blocks] or BlockList32[blocks]
  uint64_t* heads;    // FP32: [blocks] head key (best point) of each workgroup list
  uint64_t* seconds;  // FP32: [blocks] second key of each workgroup list (0: none)
  unsigned int* flagword;  // FP32: fallback flag of the step (zero between steps)
  unsigned int* counter;  // last-workgroup counter (zero between launches)
  CandList* cand;     // FP32 short-list (written by the last workgroup)
  Winner* winner;     // FP64 winner (written by the last workgroup)
  int tail;           // 1: the last workgroup merges the records; 0: the step tail merges them
  int nrec;           // record slots per signal (the records' stride)
  unsigned int* queue;  // non-null (single signal, tail = 0): slots come from this work queue
  unsigned int qbase;   // the queue's value at this launch (it only grows during a call)
  // double precision, non-null: the grid point (m, j) at probe[probe_stride b] of signal b
  // (a replayed step's forced point) has its scaled grid value stored to probe_out[2b], [2b+1]
  const int32_t* probe;
  int probe_stride;
  double* probe_out;
  // non-uniform samples with radii whose series outlasts N terms: radius m
  // with fslot[m] >= 0 reads its own folded spectrum cfold[b][fslot[m]][N]
  // (the FOLD instantiations of the radius kernel only)
  const void* cfold;
  const int* fslot;
  int nfold;
};

// Radius transforms beyond the LDS (N > 2^kMaxLdsLogN): per radius a
// four-step transform over N = N1 N2 through an intermediate in HBM, run
// over chunks of radii (see afd_large.hip).
struct BigParams {
  const void* c;      // spectrum in column order: c_{N2 l1 + l2} at [l2][l1] (T complex)
  const void* c0;     // [N2 2^kBigMedShift2] c_l for l < N2 2^kBigMedShift2 in natural order (T complex)
  const void* pa;     // [M][N1]  r_m^(N2 l1)
  const void* pb;     // [M][N2]  r_m^l2
  const void* scale;  // [M]      sqrt(1-r^2) / (N (1 - r^N))
  const int* lsig;    // [M]      significant spectrum length (later terms dropped)
  const void* wl;     // e^{2 pi i e/N}, e < 2^sw (T complex)
  const void* wh;     // e^{2 pi i h 2^sw/N}, h < N/2^sw (T complex)
  const void* tw1;    // Stockham twiddles of the length-N1 transforms
  const void* tw2;    // Stockham twiddles of the length-N2 transforms
  const void* tw2m[2];  // Stockham twiddles of the length-(N2 2^kBigMedShift), (N2 2^kBigMedShift2) transforms
  void* z;            // [chunk][N1][N2] intermediate (T complex)
  const int* border;  // [M] launch order of the radii: short spectra first, then long ones
  int M;
  int m0;             // position in border of the launch's first radius
  float tau_band;
  int recheck_k;
  void* blocks;       // [M][gstride] per-workgroup records (BlockList32 or BlockBest64)
  int gstride;        // record slots per radius (the larger record count of the two row passes)
  int med;            // 1: radii with N2 < L <= N2 2^kBigMedShift2 ran in the shifted splits' row passes
  void* rrec;         // [M] per-radius records (same type)
  uint64_t* heads;    // FP32: [M] head key of each per-radius record
  unsigned int* flagword;  // FP32: fallback flag of the step (zero between steps)
  unsigned int* counter_g;  // radius arrivals of the step's merge (zero between steps)
  CandList* cand;
  Winner* winner;
  // double precision, non-null: the grid value at the point (m, j) = (probe[0], probe[1])
  // is stored to probe_out[0], [1] (as in RadiusParams; one signal)
  const int32_t* probe;
  double* probe_out;
};

// Radii of medium spectrum length run in a row-only pass over a shifted
// split: N2 < L <= 4 N2 over N1/4 x 4 N2 (kBigMedShift), 4 N2 < L <= 16 N2
// over N1/16 x 16 N2 (kBigMedShift2).
constexpr int kBigMedShift = 2;
constexpr int kBigMedShift2 = 4;
struct BigGeom {
  int l1, l2;     // N1 = 2^l1 (column transforms), N2 = 2^l2 (row transforms)
  int g_med[2], thr_b_med[2];  // the medium radii's row passes: records per radius, threads
  size_t lds_b_med[2];
  int gstride;    // record slots per radius: the largest record count of the three row passes
  int sw;         // twiddle split: e = h 2^sw + low
  int ca, thr_a;  // columns and threads per column workgroup
  int rb, thr_b;  // rows and threads per row workgroup
  int g;          // row workgroups (records) per radius
  size_t lds_a, lds_b;
  size_t rec_bytes;  // one per-workgroup record
};
BigGeom big_geom(int logn, bool fp64);
hipError_t setup_big_attributes();
// The `nr` radii at launch positions p.m0.. (p.border): the column pass
// (with `cols`; the radii with short spectra need none), then the row pass
// with the selection.  e0 stamps the first launch's start, e1 the row pass's
// end; r0 / r1 stamp the row pass alone.
// med (1, 2): the row pass of the split shifted by kBigMedShift, kBigMedShift2 (radii of
// medium spectrum length; no column pass).
hipError_t launch_big(int logn, bool fp64, const BigParams& p, int nr, bool cols, int med, hipStream_t s,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, hipEvent_t r0 = nullptr,
                      hipEvent_t r1 = nullptr);
// After the last chunk of a step: the radius records into the winner (FP64)
// or the short-list (FP32); e1 stamps its end.
hipError_t launch_big_merge(int logn, bool fp64, const BigParams& p, hipStream_t s, hipEvent_t e1 = nullptr);

// Step outputs written by the last workgroup of k_update / k_prepare.
struct RecordArgs {
  const Winner* w;
  const double* radii;
  const double* omega;
  int N, M;
  int steps;  // per-signal length of the step arrays (batched plans hold signals back to back)
  int32_t* idx;
  double* a;
  double* coef;
  double* energy;
  double* margin;
  int32_t* kcount;
  int32_t* flags;
  double* fp32err;
};

// A replayed step (afd_replay): the point the step's own selection chose is
// recorded, then the forced point takes its place as the winner.  Arrays
// are per signal, `steps` entries apart (index: 2 per step).
struct PickArgs {
  const int32_t* forced;  // [B][fstride] (m, j) per step
  int fstride;
  int step;
  int N, logn, M, steps;
  int fp64;
  CandList* cand;         // FP32: the short-list (read), then the forced point as a one-entry list
  Winner* winner;         // the selection's winner (read); FP64: replaced by the forced point
  const double* probe;    // FP64: [B][2] the FFT-form grid value at the forced point
  int32_t* idx;           // (m, j) the selection chose
  double* p;              // its |<G_k, e_a>~|^2
  double* margin;         // its margin
  int32_t* flags;         // its flags; bit 4: FP32, the forced point was on the short-list
};
constexpr int kFlagForcedListed = 16;

// Everything a kernel needs to apply step `step`'s remainder update (eq. (7))
// and record the step (see afd_update.h).
struct UpdateArgs {
  const double* radii;
  const double* omega;
  int N, M;
  double* epart;          // per-workgroup energy partial sums
  unsigned int* counter;  // last-workgroup counter (zero between launches)
  RecordArgs R;
  int step;
};

// Grid barriers of the fused step tail count arrivals on kBarGroups
// counters: workgroup w arrives on counter w mod kBarGroups.
constexpr int kBarGroups = 8;
__host__ __device__ constexpr unsigned long long bar_group_count(int nw, int g) {
  return nw > g ? (unsigned long long)((nw - 1 - g) / kBarGroups + 1) : 0ull;
}

// Step tail for 2^10 <= N <= 2^14 (afd_advance.hip): re-check, winner,
// remainder update and the forward DFT of the new remainder.
struct AdvanceArgs {
  const CandList* cand;     // short-list (FP32 mode) or forced point
  Winner* winner;           // written here after a re-check, else read (FP64 grid maximum)
  double* g64;              // remainder samples, updated in place
  const double* radii;
  const double* omega;      // e^{2 pi i n/N}
  const void* omega_t;      // e^{2 pi i n/N} in the transform precision (T complex)
  const void* tw1;          // Stockham twiddles of the length-N1 row DFTs
  const void* tw2;          // Stockham twiddles of the length-N2 column DFTs
  void* xt;                 // [N2][N1] intermediate (T complex)
  void* c;                  // spectrum of the new remainder (T complex)
  double* partials;         // [kKMax][nch] (re, im) re-check partial sums
  double* epart;            // [nb] energy partial sums
  unsigned long long* bar;  // grid barrier counters, kBarGroups of them (zero at the start of a call)
  unsigned long long bar_base[kBarGroups];  // per counter: arrivals of the call's earlier launches
  int* status;              // bit 1: a grid barrier wait ran out
  // the radius kernel's per-workgroup records, merged here when nrec > 0
  // (otherwise the short-list is in cand, or the winner in winner)
  const void* recs;         // [B][nrec] BlockList32 (FP32) or BlockBest64 (FP64)
  const uint64_t* heads;    // FP32: [B][nrec] head keys
  const uint64_t* seconds;  // FP32: [B][nrec] second keys
  int nrec;
  int recheck_k;
  float tau_band;
  unsigned int* flagword;   // FP32: [B] fallback flag of the step, cleared here after the merges
  RecordArgs R;
  int step;
  int M;
  int update;   // 1: apply the step's update and record it; 0: transform the samples as they are
  int recheck;  // 1: re-check the short-list; 0: the winner is already in `winner`
  int fft;      // 1: transform the new remainder
  int phase;    // set by the launcher
};
struct AdvGeom {
  int l1, l2;     // N1 = 2^l1 (row DFT length), N2 = 2^l2 (column DFT length)
  int nb;         // transform workgroups (also the energy partial sums)
  int ga;         // re-check workgroups
  int nch;        // re-check chunks
  int tw1_size, tw2_size;
};
bool advance_supported(int logn);
AdvGeom advance_geom(int logn);
// Stockham twiddle table of the length-2^l DFTs of the step tail (l = 6, 7).
void advance_twiddles(int l, double* out_interleaved);
// Add the grid barrier arrivals of one launch_advance with batch 1 to a.bar_base.
void advance_bar_advance(int logn, AdvanceArgs& a);
// One launch with grid barriers for batch 1 when `fused`; one launch per
// phase otherwise (the barriers need every workgroup resident at once).
hipError_t launch_advance(int logn, bool fp64, const AdvanceArgs& a, int batch, bool fused, hipStream_t s,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Geometry of the LDS-resident transform for 2^logn points.
struct FftGeom {
  int E;        // values per thread
  int tpr;      // threads per transform
  int twsize;   // twiddle table entries
  bool split;   // exchange re/im separately through half the LDS
  int lds_elems;
};
FftGeom fft_geom(int logn, bool fp64);
// Fill the Stockham twiddle table (e^{+2 pi i k/(Ns R)} per pass) in double.
void fft_twiddles(int logn, bool fp64, double* out_interleaved);

// Forward DFT: one workgroup below 2^12 points (table tw1 of size 2^logn),
// else two passes of sizes 2^l2 (columns, table tw2) and 2^l1 (rows, tw1).
struct FwdPlan {
  bool two_pass;
  int l1, l2;
  int tw1_size, tw2_size;
};
FwdPlan fwd_plan(int logn, bool fp64);

int radius_lds_bytes(int logn, bool fp64, int rpb);
int radius_slots(int logn, bool fp64, int rpb);
// Radix of the first Stockham pass of the LDS-resident radius transform.
int radius_first_radix(int logn, bool fp64);
// Significant spectrum length of radius r: the smallest L with
// r^L / (1 - r) <= 2^-bits (so the dropped weights sum to at most 2^-bits),
// at least 1 and at most n.
int significant_length(double r, int bits, int64_t n);
int radius_threads_of(int logn, bool fp64);
int update_blocks(int N);
int recheck_chunks(int N);

// Allow a kernel the whole 160 KB of LDS less its static LDS.
inline hipError_t set_max_dynamic_lds(const void* fn) {
  hipFuncAttributes a;
  hipError_t e = hipFuncGetAttributes(&a, fn);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(160 * 1024 - a.sharedSizeBytes));
}

// Launch with optional timing events: a non-null e0 / e1 takes the start /
// end timestamp of this dispatch itself (no extra packets on the stream).
template <typename F, typename... Args>
inline void launch_ev(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                      Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

hipError_t setup_radius_attributes();
hipError_t setup_fwd_attributes();
hipError_t setup_pp_attributes();

// N = P^K for P = 3 (K <= 8), 5 (K <= 6), 7 (K <= 4) (afd_primepow.hip):
// transform geometry, twiddle table (2 * (twsize + 1) doubles, interleaved),
// the forward DFT and the fused radius kernel (one radius per workgroup,
// records merged by the last workgroup).
struct PpGeom {
  int prime;    // P; 0: not supported
  int k;        // N = P^k
  int E;        // values per thread
  int tpr;      // threads holding values (N / E)
  int threads;  // workgroup size (tpr rounded up to whole waves)
  int twsize;   // twiddle entries
};
bool pp_supported(int prime, int k);
PpGeom pp_geom(int prime, int k);
void pp_twiddles(int prime, int k, double* tw);
int pp_lds_bytes(int prime, int k, bool fp64);
int pp_first_radix(int prime, int k);
// From 2048 points the forward DFT runs in two passes through xt (N complex,
// the transform's precision) with the split's tables tw1 (rows) and tw2
// (columns) and the unit roots omega; below, one workgroup with tw.
int pp_fwd_twsize(int prime, int k, bool rows);
hipError_t launch_fwd_pp(int prime, int k, bool fp64, const void* g, const void* tw, const void* tw1,
                         const void* tw2, const double* omega, void* xt, void* c, int batch, hipStream_t s,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_radius_pp(int prime, int k, bool fp64, const RadiusParams& p, int batch, hipStream_t s,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Mixed-radix N (afd_mixed.hip): N = 2^a 3^b 5^c 7^d <= kMaxMixedN with at
// least two distinct primes, E values per thread (a multiple of each prime
// of N, E <= 30), TPR = N/E threads, run-time pass radices (the last is E).
constexpr int kMaxMixedPasses = 12;
constexpr int kMaxMixedN = 16384;
struct MixedGeom {
  int E;        // values per thread; 0: N is not taken by the mixed-radix path
  int tpr;      // threads holding values (N / E)
  int threads;  // workgroup size (tpr rounded up to whole waves)
  int np;       // passes
  int twsize;   // twiddle entries
  int radix[kMaxMixedPasses];  // pass radices, each dividing E
  int ns[kMaxMixedPasses];     // product of the earlier radices
  int twoff[kMaxMixedPasses];  // twiddle-table offset of each pass (from pass 1)
};
// kernel arguments: the pass table lives in device memory (3 ints per pass:
// radix, ns, twiddle offset), so no kernel indexes its arguments at run time
struct MixedArgs {
  const int* passes;
  int np, tpr, threads, E;
};
MixedGeom mixed_geom(int64_t n);
void mixed_twiddles(const MixedGeom& g, double* tw);
void mixed_pass_table(const MixedGeom& g, int* out);
hipError_t setup_mixed_attributes();
int mixed_lds_bytes(const MixedGeom& g, bool fp64);
// one workgroup per signal: c = DFT(sig) with the inverse's table, conjugated
hipError_t launch_fwd_mixed(const MixedGeom& g, const int* passes, bool fp64, const void* sig, const void* tw,
                            void* c, int batch, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_radius_mixed(const MixedGeom& g, const int* passes, bool fp64, const RadiusParams& p, int batch,
                               hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Batched launches cover `batch` signals (grid dimension y, or z for the
// re-check); each signal's buffers follow the previous signal's.  For
// N > 2^14, c0 (nullable) also receives the bins l < N2 2^kBigMedShift2 in natural order.
hipError_t launch_fwd(int logn, bool fp64, const void* g, const void* tw1, const void* tw2, const double* omega,
                      void* xt, void* c, int batch, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                      void* c0 = nullptr);
hipError_t launch_radius(int logn, bool fp64, const RadiusParams& p, int blocks, int batch, hipStream_t s,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_prepare(double* g64, float* g32, int N, double* epart, int* nonfinite, unsigned int* counter,
                          const RecordArgs& R, int batch, hipStream_t s);
// forced: per signal `fstride` int32 apart (0: the same point for every signal)
hipError_t launch_force(const int32_t* forced, int fstride, int step, int N, CandList* cand, int batch,
                        hipStream_t s);
// One workgroup per signal merges the radius kernel's per-workgroup records
// (as the fused step tail does): FP64 into the winner, FP32 into the short-list.
hipError_t launch_merge(bool fp64, const void* recs, const uint64_t* heads, const uint64_t* seconds, int nrec, int N,
                        int recheck_k, float tau_band, unsigned int* flagword, CandList* cand, Winner* w,
                        int batch, hipStream_t s);
hipError_t launch_pick(const PickArgs& a, int batch, hipStream_t s);
// Up to 6 word ranges set to zero by one kernel (in place of memsets where a
// call is captured into a graph).
struct ZeroArgs {
  unsigned int* p[6];
  int words[6];
  int n;
};
hipError_t launch_zero(const ZeroArgs& z, hipStream_t s);
// Samples of the re-check: uniform (z null: e^{2 pi i n/N}, n < N) or the
// non-uniform positions z[ns] (interleaved complex) with quadrature weights w.
struct RecheckSamples {
  const double* z;
  const double* w;
  int ns;
};
hipError_t launch_recheck(const CandList* cand, const double* g, const double* omega, const double* radii, int N,
                          double* partials, unsigned int* counter, Winner* w, int batch, hipStream_t s,
                          const RecheckSamples& S = RecheckSamples{nullptr, nullptr, 0});
hipError_t launch_update(double* g64, float* g32, const UpdateArgs& U, int batch, hipStream_t s,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Non-uniform samples (afd_nonuni.hip): per signal of a batch, ns samples g
// (interleaved complex, signals back to back), at positions `turns`, points
// z = e^{2 pi i turns} (interleaved), quadrature weights wt, shared by the
// batch.  launch_nu_fourier writes c_l, l < N = 2^logn, per signal in the
// radius transforms' precision (and the folded spectra of the radii that
// need more than N terms) by a gridding non-uniform FFT of NM = 2^t.lognm
// modes on a grid of G = 2^nu_grid_log2(t.lognm) cells (kernel width
// kEsWidth cells).
constexpr int kMaxNuSamples = 1 << 16;
constexpr int kMaxNuLogModes = 18;  // NM <= 2^18 modes (grids of up to 2^20 cells)
// Largest grid dimension y or z of one launch: launches whose radii or
// folded spectra run along y take at most this many per launch.
constexpr int kMaxGridY = 65535;
constexpr double kEsWidth = 12.0;
constexpr double kEsBeta = 2.69 * 12.0;
int nu_grid_log2(int logn);
struct NuTables {
  const double* turns;  // [ns]
  const double* ws;     // [ns] complex: w_n e^{-2 pi i (N/2) t_n}
  const int4* rng;      // [G] sample index ranges of each cell
  double* b;            // [batch][G] complex: the gridded strengths
  double* B;            // [batch][G] complex: their forward DFT
  void* xt;             // [batch][G] complex: four-step intermediate
  const void* tw1;      // forward-DFT twiddles of length G (fwd_plan(log2 G, true))
  const void* tw2;
  const double* omega;  // [G] complex e^{2 pi i k/G}
  const double* dinv;   // [NM] 1/Phi((l - NM/2)/G)
  int lognm;            // NM = 2^lognm modes: N, or K N when radii need K N terms (G = 4 NM)
  void* ctail;          // [batch][NM - N] modes l >= N (the radius transforms' precision)
  int nfold;            // radii whose series outlasts N terms
  const double* rho;    // [nfold] r^N of each
  void* cfold;          // [batch][nfold][N] their folded spectra
};
void nu_deconv_table(int N, int G, double* dinv);
void nu_cell_ranges(const double* turns, int ns, int G, int32_t* rng);
hipError_t launch_nu_fourier(const double* g, const NuTables& t, int logn, bool fp64, void* c, int ns, int batch,
                             hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_nu_prepare(const double* g, const double* wt, int ns, double* epart, int* nonfinite,
                             unsigned int* counter, const RecordArgs& R, int batch, hipStream_t s);
hipError_t launch_nu_update(double* g, const double* wt, const double* z, int ns, const UpdateArgs& U, int batch,
                            hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Reconstruction and analytic front end (afd_recon.hip), double precision.
int recon_waves(int N);  // wave partial sums per signal and step in `wpart`
// N points omega (e^{2 pi i n/N}, or a non-uniform plan's sample points) with
// quadrature weights wt (nullable: equal weights).  S (nullable): partial sums
// [batch][N]; wpart/delta (nullable, together): [batch][steps+1][recon_waves(N)]
// scratch and [batch][steps] relative errors.
hipError_t launch_recon(const double* a, const double* c, int steps, int N, const double* omega, const double* G,
                        double* S, double* wpart, double* delta, int batch, hipStream_t s,
                        const double* wt = nullptr);
// cols_l2 > 0: the forward DFT's column-order output (bin k2 + 2^cols_l2 k1 at k2 2^cols_l1 + k1)
hipError_t launch_analytic_mask(const double* X, double* Y, int N, int cols_l1, int cols_l2, int* flag, int batch,
                                hipStream_t s);
hipError_t launch_analytic_out(const double* Z, double* g, int N, int cols_l1, int cols_l2, const int* flag,
                               int batch, hipStream_t s);

}  // namespace afd
