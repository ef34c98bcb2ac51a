// Internal interface between the host plan (afd_api.hip) and the kernels
// (afd_kernels.hip): device record layouts and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

namespace afd {

constexpr int kMaxLogN = 20;       // N <= 2^20
constexpr int kMaxLdsLogN = 14;    // single-workgroup (LDS-resident) transforms up to 2^14
constexpr int kListC = 64;         // per-block candidate list length (FP32 mode)
constexpr int kListCap = 1024;     // per-block LDS gather capacity before the exact fallback
constexpr int kKMax = 256;         // longest short-list re-checked in double
constexpr int kSelCap = 1024;      // global gather capacity of the short-list selection
constexpr float kTauBandDefault = 4e-6f;  // default re-check band (relative to the FP32 maximum)

// flags (per step)
constexpr int kFlagBandTruncated = 1;
constexpr int kFlagListTruncated = 2;
constexpr int kFlagFallback = 4;

// FP64 mode: best and runner-up of one radius block
struct BlockBest64 {
  double p1, p2, vx, vy;
  uint32_t f;
  uint32_t pad;
};

// FP32 mode: exact top entries (key order) among the block's points within
// the list band of the block maximum
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
  double pad;
};

struct RadiusParams {
  const void* c;      // spectrum, N complex (T)
  const void* pw;     // [M][TPR]  r_m^t
  const void* pv;     // [M][E]    r_m^(TPR v)
  const void* scale;  // [M]       sqrt(1-r^2) / (N (1 - r^N))
  const void* tw;     // Stockham twiddles of the inverse transform
  int M;
  int rpb;            // radii per block
  float tau_band;     // FP32 lists: relative band below the block maximum
  void* out;          // BlockBest64[blocks] or BlockList32[blocks]
};

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

int radius_lds_bytes(int logn, bool fp64, int rpb, bool list);

hipError_t setup_kernel_attributes();

hipError_t launch_fft_fwd(int logn, bool fp64, const void* g, const void* tw, void* c, hipStream_t s);
hipError_t launch_radius(int logn, bool fp64, const RadiusParams& p, int blocks, hipStream_t s);
hipError_t launch_merge64(const BlockBest64* blocks, int nblocks, int N, Winner* w, hipStream_t s);
hipError_t launch_select32(const BlockList32* lists, int nblocks, int recheck_k, float tau_band, CandList* cand,
                           hipStream_t s);
hipError_t launch_force(const int32_t* forced, int step, int N, CandList* cand, hipStream_t s);
hipError_t launch_recheck(const CandList* cand, const double* g, const double* omega, const double* radii,
                          int N, int nch, double* partials, hipStream_t s);
hipError_t launch_finalize(const CandList* cand, const double* partials, const double* radii,
                           const double* omega, int N, int nch, Winner* w, hipStream_t s);
hipError_t launch_prepare(const double* g, double* g64, float* g32, int N, double* epart, int* nonfinite,
                          hipStream_t s);
hipError_t launch_update(const Winner* w, const double* radii, const double* omega, double* g64, float* g32,
                         int N, int M, double* epart, hipStream_t s);
hipError_t launch_record(const Winner* w, const double* radii, const double* omega, const double* epart, int nparts,
                         int N, int M, int step, int32_t* idx, double* a, double* coef, double* energy,
                         double* margin, int32_t* kcount, int32_t* flags, hipStream_t s);
int update_blocks(int N);

}  // namespace afd
