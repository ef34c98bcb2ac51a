// Host side of libafd: plan validation, double-precision tables, device
// workspace, and the stream-ordered step driver behind the C ABI of afd.h.
#include "../../include/afd.h"
#include "afd_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

using namespace afd;

// Static scratch of afd_decompose_noalloc: the per-call staging of the
// results, which afd_decompose keeps in memory the plan allocates on first
// use.  HIP places one copy on every device the library runs on; each is
// held until the process ends.  Host code reaches a copy only through the
// address hipGetSymbolAddress returns for it (scratch_of).
constexpr size_t kScratchBytes = size_t(512) << 10;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_last_error;

afd_status fail(afd_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

afd_status hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return AFD_E_HIP;
}

// Device address of `scratch` on `device`, which must be current: looked up
// once per device and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

afd_status scratch_of(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(AFD_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch[device];
  return AFD_OK;
}

int ilog2_exact(int64_t n) {
  if (n < 2 || (n & (n - 1)) != 0) return -1;
  int r = 0;
  while ((int64_t(1) << r) < n) ++r;
  return r;
}

// k if n = prime^k with k >= 1, else -1
int ilogp_exact(int64_t n, int prime) {
  if (n < prime) return -1;
  int k = 0;
  while (n % prime == 0) {
    n /= prime;
    ++k;
  }
  return n == 1 ? k : -1;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

enum TimedKind { kTimeNone = 0, kTimeRadius = 1, kTimeFft = 2, kTimeUpdate = 3, kTimeRows = 4 };

// Device arena layout for one plan.
struct Layout {
  size_t radii, omega, tw, twf1, twf2, pw, pv, scale, g64, g32, c, xt, blocks, cand, partials, winner, epart,
      nonfinite, forced0, counters, bar, omega_t, rqueue, probe, border;
  // truncated / pruned spectrum of the LDS-resident radius transforms
  size_t pq, lsig, order;
  // FP32 head and second keys of the workgroup (or per-radius) records
  size_t heads, seconds;
  // mixed-radix pass table (radix, ns, twiddle offset per pass)
  size_t mixp;
  // radius transforms beyond the LDS
  size_t wl, wh, z, c0, rrec, bcounters, twm, twm2;
  // non-uniform samples: positions (turns), quadrature weights, points, DFT partial sums
  size_t nu_t, nu_w, nu_z;
  // and the gridding non-uniform FFT: shifted weights, cell ranges, deconvolution,
  // grid, its transform, intermediate, twiddles and unit roots of the G-cell grid
  size_t nu_ws, nu_rng, nu_dinv, nu_b, nu_B, nu_xt, nu_tw1, nu_tw2, nu_omega;
  // and radii whose series outlasts N terms: modes l >= N, folded spectra, r^N, slots
  size_t nu_ctail, nu_cfold, nu_rho, nu_fslot;
  size_t total;
};

// Budget of the intermediate of the two-pass radius transforms: it bounds the
// radii per chunk (128 single / 64 double precision at N = 2^20).  Each chunk
// costs two launch boundaries per step, where the device drains and refills.
constexpr size_t kBigChunkBytes = size_t(1) << 30;

struct Config {
  int logn;
  int64_t N;
  int M;
  bool fp64;
  FftGeom geom;
  FwdPlan fwd;
  int rpb;
  int nblocks;
  int nch;
  int nparts;
  int batch;    // signals per call
  bool big;     // N > 2^kMaxLdsLogN: two-pass radius transforms
  BigGeom bg;
  bool adv;     // 2^10 <= N <= 2^14: fused step tail (afd_advance.hip)
  AdvGeom ag;
  int chunk;    // radii per two-pass chunk (of the radii with long spectra)
  int nshort;   // N > 2^14: radii whose significant spectrum fits in N2 terms (no intermediate)
  int nmed[2];  // N > 2^14: radii with N2 < L <= 4 N2, 4 N2 < L <= 16 N2 (the shifted splits' row passes)
  int twm_size[2];  // N > 2^14: twiddle entries of the length-4 N2 and -16 N2 transforms
  int prime;    // N = prime^pk (prime = 3, 5, 7; radix-prime transforms, afd_primepow.hip)
  int pk;       // 0: N = 2^logn
  bool mixed;   // N = 2^a 3^b 5^c 7^d with several primes (mixed-radix transforms, afd_mixed.hip)
  MixedGeom mg;
  bool nu;      // non-uniform samples (afd_nonuni.hip)
  int ns;       // samples per signal (N unless nu)
  int nu_lognm; // non-uniform samples: 2^nu_lognm modes of the non-uniform DFT (N, or K N)
  int nfold;    // non-uniform samples: radii whose series outlasts N terms (folded spectra)
};

constexpr int kNumCounters = 5;  // radius, recheck, update, prepare; FP32 fallback flag word

afd_status validate(const afd_plan_desc* d, Config* cfg) {
  if (!d) return fail(AFD_E_INVALID, "desc is NULL");
  if (d->n > (int64_t(1) << kMaxLogN) && ilog2_exact(d->n) > 0)
    return fail(AFD_E_UNSUPPORTED, "N > 2^20 is not supported");
  int prime = 0, pk = -1;
  for (const int q : {3, 5, 7}) {
    const int k = ilogp_exact(d->n, q);
    if (k > 0) prime = q, pk = k;
  }
  if (pk > 0 && !pp_supported(prime, pk))
    return fail(AFD_E_UNSUPPORTED, "N = 3^K needs K <= 8, N = 5^K K <= 6, N = 7^K K <= 4");
  const int logn = pk > 0 ? 0 : ilog2_exact(d->n);
  const MixedGeom mg = logn < 1 && pk < 1 ? mixed_geom(d->n) : MixedGeom{};
  if (logn < 1 && pk < 1 && mg.E == 0) {
    int64_t v = d->n;
    for (const int q : {2, 3, 5, 7})
      while (v > 1 && v % q == 0) v /= q;
    if (d->n >= 2 && v == 1)
      return fail(AFD_E_UNSUPPORTED,
                  "mixed-radix N needs N <= 16384, the product of its distinct primes <= 30 and N/E threads "
                  "within the workgroup");
    return fail(AFD_E_INVALID, "N must be a power of two >= 2 or a product of powers of 2, 3, 5 and 7");
  }
  if (d->m < 1) return fail(AFD_E_INVALID, "M must be >= 1");
  if (!d->radii) return fail(AFD_E_INVALID, "radii is NULL");
  // flat grid indices f = m N + j are unsigned 32-bit, 2^32 - 1 marking "no point"
  if (int64_t(d->m) * d->n >= (int64_t(1) << 32) - 1) return fail(AFD_E_INVALID, "M*N must be < 2^32 - 1");
  if (d->precision != AFD_FP64 && d->precision != AFD_FP32_RECHECK) return fail(AFD_E_INVALID, "bad precision");
  if (d->recheck_k < 0 || d->recheck_k > kListC) return fail(AFD_E_INVALID, "recheck_k must be in 0..64");
  if (!(d->recheck_band >= 0.0) || d->recheck_band > 1e-4)
    return fail(AFD_E_INVALID, "recheck_band must be in [0, 1e-4]");
  bool has_zero = false;
  for (int i = 0; i < d->m; ++i) {
    const double r = d->radii[i];
    if (!std::isfinite(r) || r < 0.0 || r >= 1.0) return fail(AFD_E_INVALID, "radius outside [0, 1)");
    if (r == 0.0) has_zero = true;
  }
  if (d->first_a_zero && !has_zero) return fail(AFD_E_INVALID, "first_a_zero needs a radius equal to 0");
  if (d->batch < 0 || d->batch > 65535) return fail(AFD_E_INVALID, "batch must be in 0..65535");
  const int batch = d->batch == 0 ? 1 : d->batch;
  const bool nu = d->sample_turns != nullptr;
  if (nu) {
    if (d->samples < 1) return fail(AFD_E_INVALID, "samples must be >= 1 with sample_turns");
    if (d->samples > kMaxNuSamples) return fail(AFD_E_UNSUPPORTED, "non-uniform samples: at most 2^16");
    double prev = -1.0;
    for (int64_t i = 0; i < d->samples; ++i) {
      const double t = d->sample_turns[i];
      if (!std::isfinite(t) || t < 0.0 || t >= 1.0 || !(t > prev))
        return fail(AFD_E_INVALID, "sample_turns must be finite, strictly increasing and in [0, 1)");
      prev = t;
      if (d->sample_weights && !std::isfinite(d->sample_weights[i]))
        return fail(AFD_E_INVALID, "sample_weights must be finite");
    }
    if (logn < 1 || logn > kMaxLdsLogN)
      return fail(AFD_E_UNSUPPORTED, "non-uniform samples need a grid of N = 2^K <= 2^14 angles");
    // the modes of the non-uniform DFT: N, or the power of two K N >= the
    // longest significant series (radii beyond N terms get folded spectra)
    const int bits = d->precision == AFD_FP64 ? 60 : 40;
    int64_t lmax = d->n;
    int nfold = 0;
    for (int i = 0; i < d->m; ++i) {
      const int64_t L = significant_length(d->radii[i], bits, int64_t(1) << 30);
      lmax = L > lmax ? L : lmax;
      if (L > d->n) ++nfold;
    }
    int lognm = logn;
    while ((int64_t(1) << lognm) < lmax && lognm <= kMaxNuLogModes) ++lognm;
    if (lognm > kMaxNuLogModes)
      return fail(AFD_E_UNSUPPORTED,
                  "non-uniform samples: a radius is too close to 1 (its kernel series needs more than 2^18 terms)");
    if (cfg) {
      cfg->nu_lognm = lognm;
      cfg->nfold = nfold;
    }
  } else if (d->samples != 0) {
    return fail(AFD_E_INVALID, "samples needs sample_turns");
  }
  if (batch > 1 && logn > kMaxLdsLogN) return fail(AFD_E_UNSUPPORTED, "batch > 1 needs N <= 2^14");
  if (int64_t(batch) * d->n * d->m >= (int64_t(1) << 40) || int64_t(batch) * d->n >= (int64_t(1) << 31))
    return fail(AFD_E_INVALID, "batch * N (* M) too large");
  if (cfg) {
    cfg->logn = logn;
    cfg->N = d->n;
    cfg->M = d->m;
    cfg->batch = batch;
    cfg->fp64 = d->precision == AFD_FP64;
    cfg->pk = pk > 0 ? pk : 0;
    cfg->prime = pk > 0 ? prime : 0;
    cfg->mixed = mg.E > 0;
    cfg->mg = mg;
    cfg->fwd = cfg->pk || cfg->mixed ? FwdPlan{} : fwd_plan(logn, cfg->fp64);
    cfg->nch = recheck_chunks(int(d->n));
    cfg->nparts = update_blocks(int(d->n));
    cfg->big = logn > kMaxLdsLogN;
    cfg->nu = nu;
    cfg->ns = nu ? int(d->samples) : int(d->n);
    if (!nu) cfg->nu_lognm = cfg->nfold = 0;  // (set with the checks of the samples otherwise)
    if (nu) {
      cfg->fwd = FwdPlan{};
      cfg->nch = recheck_chunks(cfg->ns);
      cfg->nparts = update_blocks(cfg->ns);
    }
    cfg->adv = !cfg->pk && !cfg->mixed && !nu && advance_supported(logn);
    cfg->ag = cfg->adv ? advance_geom(logn) : AdvGeom{};
    if (cfg->adv) {
      cfg->fwd.tw1_size = cfg->ag.tw1_size;
      cfg->fwd.tw2_size = cfg->ag.tw2_size;
      cfg->nch = cfg->ag.nch;
      cfg->nparts = cfg->ag.nb;
    }
    if (cfg->big) {
      cfg->geom = FftGeom{0, 0, 0, false, 0};
      cfg->bg = big_geom(logn, cfg->fp64);
      // only the radii with long spectra go through the intermediate, in
      // chunks; those of medium length run in the shifted split's row pass
      cfg->nshort = 0;
      cfg->nmed[0] = cfg->nmed[1] = 0;
      for (int i = 0; i < d->m; ++i) {
        const int64_t L = significant_length(d->radii[i], cfg->fp64 ? 60 : 40, d->n);
        if (L <= (int64_t(1) << cfg->bg.l2)) ++cfg->nshort;
        else if (L <= (int64_t(1) << (cfg->bg.l2 + kBigMedShift))) ++cfg->nmed[0];
        else if (L <= (int64_t(1) << (cfg->bg.l2 + kBigMedShift2))) ++cfg->nmed[1];
      }
      cfg->twm_size[0] = fft_geom(cfg->bg.l2 + kBigMedShift, cfg->fp64).twsize;
      cfg->twm_size[1] = fft_geom(cfg->bg.l2 + kBigMedShift2, cfg->fp64).twsize;
      const size_t nlong = size_t(d->m - cfg->nshort - cfg->nmed[0] - cfg->nmed[1]);
      const size_t per_radius = size_t(d->n) * (cfg->fp64 ? 16 : 8);
      const size_t fit = kBigChunkBytes / per_radius;
      cfg->chunk = nlong == 0 ? 0 : int(fit < 1 ? 1 : fit > nlong ? nlong : fit);
      cfg->rpb = 1;
      cfg->nblocks = d->m * cfg->bg.gstride;  // record slots of every radius of a step
    } else if (cfg->pk) {
      // one radius per workgroup; the inverse and forward transforms share
      // the twiddle table
      const PpGeom tg = pp_geom(cfg->prime, cfg->pk);
      cfg->geom = FftGeom{tg.E, tg.tpr, tg.twsize, false, 0};
      // the forward DFT's split (from 2048 points): row and column tables, intermediate
      cfg->fwd.two_pass = pp_fwd_twsize(cfg->prime, cfg->pk, true) > 0;
      cfg->fwd.tw1_size = pp_fwd_twsize(cfg->prime, cfg->pk, true);
      cfg->fwd.tw2_size = pp_fwd_twsize(cfg->prime, cfg->pk, false);
      cfg->bg = BigGeom{};
      cfg->chunk = 0;
      cfg->nshort = 0;
      cfg->rpb = 1;
      cfg->nblocks = d->m;
    } else if (cfg->mixed) {
      // one radius per workgroup; the one-workgroup forward transform takes
      // the inverse's table, conjugated
      cfg->geom = FftGeom{mg.E, mg.tpr, mg.twsize, false, 0};
      cfg->bg = BigGeom{};
      cfg->chunk = 0;
      cfg->nshort = 0;
      cfg->rpb = 1;
      cfg->nblocks = d->m;
    } else {
      cfg->geom = fft_geom(logn, cfg->fp64);
      cfg->bg = BigGeom{};
      cfg->chunk = 0;
      cfg->nshort = 0;
      const int tpr = cfg->geom.tpr;
      cfg->rpb = tpr >= 64 ? 1 : 64 / tpr;
      cfg->nblocks = (d->m + cfg->rpb - 1) / cfg->rpb;
    }
  }
  return AFD_OK;
}

Layout layout_of(const Config& c) {
  Layout L{};
  size_t o = 0;
  const size_t real = c.fp64 ? 8 : 4;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.radii = take(8 * size_t(c.M));
  L.mixp = take(c.mixed ? sizeof(int) * 3 * kMaxMixedPasses : 0);
  L.omega = take(16 * size_t(c.N));
  L.tw = take(2 * real * size_t(c.geom.twsize + 1));
  L.twf1 = take(2 * real * size_t(c.fwd.tw1_size + 1));
  L.twf2 = take(2 * real * size_t(c.fwd.tw2_size + 1));
  // LDS path: r^t [M][TPR] and r^(TPR v) [M][E]; two-pass path: r^(N2 l1) [M][N1] and r^l2 [M][N2]
  L.pw = take(real * size_t(c.M) * (c.big ? (size_t(1) << c.bg.l1) : size_t(c.geom.tpr)));
  L.pv = take(real * size_t(c.M) * (c.big ? (size_t(1) << c.bg.l2) : size_t(c.geom.E)));
  L.scale = take(real * size_t(c.M));
  L.pq = take(c.big ? 0 : real * size_t(c.M) * c.geom.E);
  L.lsig = take(4 * size_t(c.M));
  L.order = take(c.big ? 0 : 8 * size_t(c.M));
  // per-signal buffers: `batch` copies back to back
  const size_t B = size_t(c.batch);
  L.heads = take(c.fp64 ? 0 : 8 * size_t(c.big ? c.M : c.nblocks) * B);
  L.seconds = take(c.fp64 || c.big ? 0 : 8 * size_t(c.nblocks) * B);
  L.g64 = take(16 * size_t(c.ns) * B);
  L.g32 = take(c.fp64 || c.adv || c.nu ? 0 : 8 * size_t(c.N) * B);
  L.c = take(2 * real * size_t(c.N) * B);
  // the four-step intermediate of the forward DFT, or of the fused step tail's
  L.xt = take(c.fwd.two_pass || c.adv ? 2 * real * size_t(c.N) * B : 0);
  L.blocks = take((c.fp64 ? sizeof(BlockBest64) : sizeof(BlockList32)) * size_t(c.nblocks) * B);
  L.wl = take(c.big ? 2 * real * (size_t(1) << c.bg.sw) : 0);
  L.wh = take(c.big ? 2 * real * (size_t(1) << (c.logn - c.bg.sw)) : 0);
  L.z = take(c.big ? 2 * real * size_t(c.chunk) * size_t(c.N) : 0);
  L.c0 = take(c.big ? 2 * real * (size_t(1) << (c.bg.l2 + kBigMedShift2)) * B : 0);
  L.twm = take(c.big ? 2 * real * size_t(c.twm_size[0] + 1) : 0);
  L.twm2 = take(c.big ? 2 * real * size_t(c.twm_size[1] + 1) : 0);
  L.rrec = take(c.big ? (c.fp64 ? sizeof(BlockBest64) : sizeof(BlockList32)) * size_t(c.M) : 0);
  L.bcounters = take(c.big ? 4 : 0);
  L.border = take(c.big ? 4 * size_t(c.M) : 0);  // radii with short spectra first
  L.cand = take(sizeof(CandList) * B);
  L.partials = take(16 * size_t(kKMax) * c.nch * B);
  L.winner = take(sizeof(Winner) * B);
  L.epart = take(8 * size_t(c.nparts) * B);
  L.nonfinite = take(4);
  L.forced0 = take(8);
  L.counters = take(4 * kNumCounters * B);  // [kind][signal]
  L.bar = take(8 * 16 * kBarGroups);  // counters 128 bytes apart
  L.rqueue = take(4);                  // work queue of the radius slots
  L.probe = take(16 * B);              // replay: the grid value at each signal's forced point
  // fused step tail in single precision: the unit roots rounded to float
  L.omega_t = take(c.adv && !c.fp64 ? 8 * size_t(c.N) : 0);
  L.nu_t = take(c.nu ? 8 * size_t(c.ns) : 0);
  L.nu_w = take(c.nu ? 8 * size_t(c.ns) : 0);
  L.nu_z = take(c.nu ? 16 * size_t(c.ns) : 0);
  const size_t G = c.nu ? size_t(1) << nu_grid_log2(c.nu_lognm) : 0;
  const size_t NM = c.nu ? size_t(1) << c.nu_lognm : 0;
  const FwdPlan gp = c.nu ? fwd_plan(nu_grid_log2(c.nu_lognm), true) : FwdPlan{};
  L.nu_ws = take(16 * size_t(c.nu ? c.ns : 0));
  L.nu_rng = take(16 * G);
  L.nu_dinv = take(8 * NM);
  L.nu_ctail = take(c.nu ? 2 * real * (NM - size_t(c.N)) * B : 0);
  L.nu_cfold = take(c.nu ? 2 * real * size_t(c.nfold) * size_t(c.N) * B : 0);
  L.nu_rho = take(c.nu ? 8 * size_t(c.nfold) : 0);
  L.nu_fslot = take(c.nu && c.nfold > 0 ? 4 * size_t(c.M) : 0);
  L.nu_b = take(16 * G * B);
  L.nu_B = take(16 * G * B);
  L.nu_xt = take(16 * G * B);
  L.nu_tw1 = take(c.nu ? 16 * size_t(gp.tw1_size + 1) : 0);
  L.nu_tw2 = take(c.nu ? 16 * size_t(gp.tw2_size + 1) : 0);
  L.nu_omega = take(16 * G);
  L.total = o;
  return L;
}

bool is_device_pointer(const void* p) {
  hipPointerAttribute_t attr;
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace

struct afd_plan_s {
  Config cfg{};
  Layout L{};
  int device = 0;
  hipStream_t stream = nullptr;
  int recheck_k = 8;
  float tau_band = 1e-5f;
  bool first_a_zero = false;
  bool concurrent = false;  // the stream runs beside other streams' kernels: no grid barriers
  int rslots = 0;  // radius workgroups resident at once (queued launches), 0: none
  // launch choices that leave the results unchanged (afd_plan_tune): the
  // three-launch step tail, no double-precision work queue, radii per
  // two-pass chunk (at most cfg.chunk, whose intermediate is allocated)
  bool split_tail = false;
  bool no_queue = false;
  int chunk = 0;
  int zero_m = -1;
  unsigned char* arena = nullptr;
  // per-call result staging on the device
  unsigned char* res = nullptr;
  int res_steps = -1;
  int32_t* forced = nullptr;
  int forced_steps = -1;
  // scratch of afd_reconstruct / afd_analytic, grown on demand
  unsigned char* aux = nullptr;
  size_t aux_bytes = 0;
  // timing
  int time_kind = kTimeNone;
  int time_every = 1;      // time every time_every-th unit of the class
  int64_t time_seen = 0;   // units of the class seen since timing was enabled
  double time_ms = 0.0;
  int64_t time_launches = 0;
  std::vector<hipEvent_t> events;

  template <typename P>
  P* at(size_t off) const {
    return reinterpret_cast<P*>(arena + off);
  }
};

// Decompositions of several plans captured into one graph (afd_group_create).
struct afd_group_s {
  std::vector<afd_plan_s*> plans;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// A decomposition captured into a HIP graph (afd_graph_create).
struct afd_graph_s {
  afd_plan_s* plan = nullptr;
  afd_result out{};
  int steps = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

afd_status build_tables(afd_plan_s* p, const afd_plan_desc* d) {
  const double* radii = d->radii;
  const Config& c = p->cfg;
  const int64_t N = c.N;
  const int M = c.M, tpr = c.geom.tpr, E = c.geom.E;
  std::vector<double> omega(2 * size_t(N));
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int64_t n = 0; n < N; ++n) {
    const long double ang = two_pi * (long double)n / (long double)N;
    omega[2 * n] = (double)cosl(ang);
    omega[2 * n + 1] = (double)sinl(ang);
  }
  std::vector<double> tw(2 * size_t(c.geom.twsize + 1), 0.0);
  if (c.pk)
    pp_twiddles(c.prime, c.pk, tw.data());
  else if (c.mixed)
    mixed_twiddles(c.mg, tw.data());
  else
    fft_twiddles(c.logn, c.fp64, tw.data());
  std::vector<double> twf1(2 * size_t(c.fwd.tw1_size + 1), 0.0), twf2(2 * size_t(c.fwd.tw2_size + 1), 0.0);
  if (c.pk) {
    // N = P^K: the one-workgroup forward transform takes the inverse's table,
    // conjugated; the split one the tables of its rows and columns
    if (c.fwd.two_pass) {
      pp_twiddles(c.prime, c.pk / 2, twf1.data());
      pp_twiddles(c.prime, c.pk - c.pk / 2, twf2.data());
    }
  } else if (c.nu || c.mixed) {
    // (non-uniform samples: no forward FFT; mixed radix: the inverse's table)
  } else if (c.adv) {
    advance_twiddles(c.ag.l1, twf1.data());
    advance_twiddles(c.ag.l2, twf2.data());
  } else {
    fft_twiddles(c.fwd.two_pass ? c.fwd.l1 : c.logn, c.fp64, twf1.data());
    if (c.fwd.two_pass) fft_twiddles(c.fwd.l2, c.fp64, twf2.data());
  }
  // r^l = pw[m][a] * pv[m][b]: l = a + TPR b (LDS path) or l = N2 a + b (two-pass path, pw = r^(N2 a))
  const int na = c.big ? (1 << c.bg.l1) : tpr, nb = c.big ? (1 << c.bg.l2) : E;
  const long double sa = c.big ? (long double)nb : 1.0L, sb = c.big ? 1.0L : (long double)tpr;
  std::vector<double> pw(size_t(M) * na), pv(size_t(M) * nb), sc(M);
  for (int m = 0; m < M; ++m) {
    const long double r = radii[m];
    for (int a = 0; a < na; ++a) pw[size_t(m) * na + a] = a == 0 ? 1.0 : (double)powl(r, sa * (long double)a);
    for (int b = 0; b < nb; ++b) pv[size_t(m) * nb + b] = b == 0 ? 1.0 : (double)powl(r, sb * (long double)b);
    const long double rN = powl(r, (long double)N);
    // non-uniform samples: the series is not folded (its terms from l = N on are negligible)
    sc[m] = c.nu ? (double)sqrtl((1.0L - r) * (1.0L + r))
                 : (double)(sqrtl((1.0L - r) * (1.0L + r)) / ((long double)N * (1.0L - rN)));
  }
  // LDS path: r^((TPR/R0) v) for the pruned start, and the significant
  // spectrum length of each radius (weights below 2^-40 single / 2^-60 double
  // precision of the largest term, summed, are dropped)
  std::vector<double> pq;
  std::vector<int32_t> lsig(M);
  for (int m = 0; m < M; ++m) lsig[m] = significant_length(radii[m], c.fp64 ? 60 : 40, N);
  if (!c.big) {
    const int r0 = c.pk      ? pp_first_radix(c.prime, c.pk)
                   : c.mixed ? (c.mg.np >= 2 ? c.mg.ns[1] : 1)
                             : radius_first_radix(c.logn, c.fp64);
    const long double step = (long double)(tpr / (r0 > 0 ? r0 : 1));
    pq.resize(size_t(M) * E);
    for (int m = 0; m < M; ++m) {
      const long double r = radii[m];
      for (int v = 0; v < E; ++v) pq[size_t(m) * E + v] = v == 0 ? 1.0 : (double)powl(r, step * (long double)v);
    }
  }
  // two-pass path: e^{2 pi i e/N} = wh[e >> sw] * wl[e mod 2^sw]
  std::vector<double> wl, wh;
  if (c.big) {
    const int64_t nl = int64_t(1) << c.bg.sw, nh = N >> c.bg.sw;
    wl.resize(2 * size_t(nl));
    wh.resize(2 * size_t(nh));
    for (int64_t e = 0; e < nl; ++e) {
      wl[2 * e] = omega[2 * e];
      wl[2 * e + 1] = omega[2 * e + 1];
    }
    for (int64_t h = 0; h < nh; ++h) {
      wh[2 * h] = omega[2 * (h * nl)];
      wh[2 * h + 1] = omega[2 * (h * nl) + 1];
    }
  }
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpy(p->arena + off, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e = up(p->L.radii, radii, 8 * size_t(M));
  if (e == hipSuccess) e = up(p->L.omega, omega.data(), omega.size() * 8);
  if (e == hipSuccess && c.mixed) {
    int table[3 * kMaxMixedPasses] = {};
    mixed_pass_table(c.mg, table);
    e = up(p->L.mixp, table, sizeof(table));
  }
  if (c.fp64) {
    if (e == hipSuccess) e = up(p->L.tw, tw.data(), tw.size() * 8);
    if (e == hipSuccess) e = up(p->L.twf1, twf1.data(), twf1.size() * 8);
    if (e == hipSuccess) e = up(p->L.twf2, twf2.data(), twf2.size() * 8);
    if (e == hipSuccess) e = up(p->L.pw, pw.data(), pw.size() * 8);
    if (e == hipSuccess) e = up(p->L.pv, pv.data(), pv.size() * 8);
    if (e == hipSuccess) e = up(p->L.scale, sc.data(), sc.size() * 8);
    if (e == hipSuccess && c.big) e = up(p->L.wl, wl.data(), wl.size() * 8);
    if (e == hipSuccess && c.big) e = up(p->L.wh, wh.data(), wh.size() * 8);
    if (e == hipSuccess && !c.big) e = up(p->L.pq, pq.data(), pq.size() * 8);
  } else {
    auto f32 = [](const std::vector<double>& v) {
      std::vector<float> o(v.size());
      for (size_t i = 0; i < v.size(); ++i) o[i] = float(v[i]);
      return o;
    };
    const std::vector<float> tw32 = f32(tw), pw32 = f32(pw), pv32 = f32(pv), sc32 = f32(sc);
    const std::vector<float> twf1_32 = f32(twf1), twf2_32 = f32(twf2), wl32 = f32(wl), wh32 = f32(wh),
                             pq32 = f32(pq);
    if (e == hipSuccess) e = up(p->L.tw, tw32.data(), tw32.size() * 4);
    if (e == hipSuccess) e = up(p->L.twf1, twf1_32.data(), twf1_32.size() * 4);
    if (e == hipSuccess) e = up(p->L.twf2, twf2_32.data(), twf2_32.size() * 4);
    if (e == hipSuccess) e = up(p->L.pw, pw32.data(), pw32.size() * 4);
    if (e == hipSuccess) e = up(p->L.pv, pv32.data(), pv32.size() * 4);
    if (e == hipSuccess) e = up(p->L.scale, sc32.data(), sc32.size() * 4);
    if (e == hipSuccess && c.big) e = up(p->L.wl, wl32.data(), wl32.size() * 4);
    if (e == hipSuccess && c.big) e = up(p->L.wh, wh32.data(), wh32.size() * 4);
    if (e == hipSuccess && !c.big) e = up(p->L.pq, pq32.data(), pq32.size() * 4);
  }
  if (e == hipSuccess) e = up(p->L.lsig, lsig.data(), lsig.size() * 4);
  if (e == hipSuccess && c.adv && !c.fp64) {
    std::vector<float> om(2 * size_t(N));
    for (size_t i = 0; i < om.size(); ++i) om[i] = float(omega[i]);
    e = up(p->L.omega_t, om.data(), om.size() * 4);
  }
  if (!c.big) {
    // workgroup order: longest significant spectrum first (ties by index)
    std::vector<int32_t> order(M);
    for (int m = 0; m < M; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return lsig[a] > lsig[b]; });
    std::vector<int32_t> wi(2 * size_t(M));
    for (int b = 0; b < M; ++b) {
      wi[2 * size_t(b)] = order[b];
      wi[2 * size_t(b) + 1] = lsig[order[b]];
    }
    if (e == hipSuccess) e = up(p->L.order, wi.data(), wi.size() * 4);
  }
  if (c.nu && e == hipSuccess) {
    // positions, quadrature weights (periodic trapezoid unless given) and
    // points z_n = e^{2 pi i t_n} in long double, rounded once
    const int ns = c.ns;
    std::vector<double> w(ns), z(2 * size_t(ns));
    for (int n = 0; n < ns; ++n) {
      const double t = d->sample_turns[n];
      if (d->sample_weights) {
        w[n] = d->sample_weights[n];
      } else if (ns == 1) {
        w[n] = 1.0;
      } else {
        const double nx = n + 1 < ns ? d->sample_turns[n + 1] : d->sample_turns[0] + 1.0;
        const double pv = n > 0 ? d->sample_turns[n - 1] : d->sample_turns[ns - 1] - 1.0;
        w[n] = (nx - pv) / 2.0;
      }
      const long double ang = two_pi * (long double)t;
      z[2 * size_t(n)] = (double)cosl(ang);
      z[2 * size_t(n) + 1] = (double)sinl(ang);
    }
    e = up(p->L.nu_t, d->sample_turns, 8 * size_t(ns));
    if (e == hipSuccess) e = up(p->L.nu_w, w.data(), 8 * size_t(ns));
    if (e == hipSuccess) e = up(p->L.nu_z, z.data(), 16 * size_t(ns));
    // the non-uniform FFT of NM modes: strengths' factor w_n e^{-2 pi i (NM/2) t_n}
    // (the fractional turn of (NM/2) t_n is exact), cell ranges,
    // deconvolution, and the forward-transform tables of the G-cell grid
    const int64_t NM = int64_t(1) << c.nu_lognm;
    std::vector<double> ws(2 * size_t(ns));
    for (int n = 0; n < ns; ++n) {
      const double h = double(NM / 2) * d->sample_turns[n];  // exact: NM/2 is a power of two
      const long double ang = two_pi * (long double)(h - std::nearbyint(h));
      ws[2 * size_t(n)] = (double)((long double)w[n] * cosl(ang));
      ws[2 * size_t(n) + 1] = (double)(-(long double)w[n] * sinl(ang));
    }
    const int lg = nu_grid_log2(c.nu_lognm);
    const int64_t G = int64_t(1) << lg;
    std::vector<int32_t> rng(4 * size_t(G));
    nu_cell_ranges(d->sample_turns, ns, int(G), rng.data());
    std::vector<double> dinv(static_cast<size_t>(NM));
    nu_deconv_table(int(NM), int(G), dinv.data());
    // radii whose series outlasts N terms: their slots and r^N
    if (c.nfold > 0) {
      std::vector<int32_t> fslot(M, -1);
      std::vector<double> rho;
      for (int m = 0; m < M; ++m)
        if (significant_length(radii[m], c.fp64 ? 60 : 40, int64_t(1) << 30) > N) {
          fslot[m] = int32_t(rho.size());
          rho.push_back((double)powl((long double)radii[m], (long double)N));
        }
      if (e == hipSuccess) e = up(p->L.nu_fslot, fslot.data(), 4 * fslot.size());
      if (e == hipSuccess) e = up(p->L.nu_rho, rho.data(), 8 * rho.size());
    }
    const FwdPlan gp = fwd_plan(lg, true);
    std::vector<double> gtw1(2 * size_t(gp.tw1_size + 1), 0.0), gtw2(2 * size_t(gp.tw2_size + 1), 0.0);
    fft_twiddles(gp.two_pass ? gp.l1 : lg, true, gtw1.data());
    if (gp.two_pass) fft_twiddles(gp.l2, true, gtw2.data());
    std::vector<double> gom(2 * size_t(G));
    for (int64_t k = 0; k < G; ++k) {
      const long double ang = two_pi * (long double)k / (long double)G;
      gom[2 * k] = (double)cosl(ang);
      gom[2 * k + 1] = (double)sinl(ang);
    }
    if (e == hipSuccess) e = up(p->L.nu_ws, ws.data(), 8 * ws.size());
    if (e == hipSuccess) e = up(p->L.nu_rng, rng.data(), 4 * rng.size());
    if (e == hipSuccess) e = up(p->L.nu_dinv, dinv.data(), 8 * dinv.size());
    if (e == hipSuccess) e = up(p->L.nu_tw1, gtw1.data(), 8 * gtw1.size());
    if (e == hipSuccess) e = up(p->L.nu_tw2, gtw2.data(), 8 * gtw2.size());
    if (e == hipSuccess) e = up(p->L.nu_omega, gom.data(), 8 * gom.size());
  }
  const int32_t f0[2] = {p->zero_m < 0 ? 0 : p->zero_m, 0};
  if (e == hipSuccess) e = up(p->L.forced0, f0, sizeof(f0));
  if (e == hipSuccess) e = hipMemset(p->arena + p->L.nonfinite, 0, 4);
  if (e == hipSuccess) e = hipMemset(p->arena + p->L.counters, 0, 4 * kNumCounters * size_t(c.batch));
  if (e == hipSuccess && c.big) e = hipMemset(p->arena + p->L.bcounters, 0, 4);
  if (c.big) {
    // launch order of the radii beyond the LDS: the short spectra (one row
    // launch, no intermediate), the medium ones (one row launch of the
    // shifted split), then the long ones (chunks through the intermediate)
    std::vector<int32_t> order;
    const int n2 = 1 << c.bg.l2, n2m = n2 << kBigMedShift, n2m2 = n2 << kBigMedShift2;
    for (int m = 0; m < M; ++m)
      if (lsig[m] <= n2) order.push_back(m);
    for (int m = 0; m < M; ++m)
      if (lsig[m] > n2 && lsig[m] <= n2m) order.push_back(m);
    for (int m = 0; m < M; ++m)
      if (lsig[m] > n2m && lsig[m] <= n2m2) order.push_back(m);
    for (int m = 0; m < M; ++m)
      if (lsig[m] > n2m2) order.push_back(m);
    if (e == hipSuccess) e = up(p->L.border, order.data(), 4 * size_t(M));
    for (int k = 0; k < 2; ++k) {
      std::vector<double> twm(2 * size_t(c.twm_size[k] + 1), 0.0);
      fft_twiddles(c.bg.l2 + (k == 0 ? kBigMedShift : kBigMedShift2), c.fp64, twm.data());
      const size_t at = k == 0 ? p->L.twm : p->L.twm2;
      if (c.fp64) {
        if (e == hipSuccess) e = up(at, twm.data(), twm.size() * 8);
      } else {
        std::vector<float> twm32(twm.begin(), twm.end());
        if (e == hipSuccess) e = up(at, twm32.data(), twm32.size() * 4);
      }
    }
  }
  if (e != hipSuccess) return hip_fail(e, "uploading plan tables");
  return AFD_OK;
}

// Result staging: idx(2s i32) a(2s) coef(2s) energy(s+1) margin(s) kcount(s i32) flags(s i32)
struct ResPtrs {
  int32_t* idx;
  double* a;
  double* coef;
  double* energy;
  double* margin;
  int32_t* kcount;
  int32_t* flags;
  double* fp32err;
  // replay: the selection's own choice per step
  int32_t* pidx;
  double* pp;
  double* pmargin;
  int32_t* pflags;
  size_t total;
};

ResPtrs res_layout(unsigned char* base, int steps, int batch) {
  ResPtrs r{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return base + at;
  };
  // signal-major: signal b's arrays follow signal b-1's
  const size_t s = size_t(steps < 1 ? 1 : steps), B = size_t(batch);
  r.idx = reinterpret_cast<int32_t*>(take(8 * s * B));
  r.a = reinterpret_cast<double*>(take(16 * s * B));
  r.coef = reinterpret_cast<double*>(take(16 * s * B));
  r.energy = reinterpret_cast<double*>(take(8 * (s + 1) * B));
  r.margin = reinterpret_cast<double*>(take(8 * s * B));
  r.kcount = reinterpret_cast<int32_t*>(take(4 * s * B));
  r.flags = reinterpret_cast<int32_t*>(take(4 * s * B));
  r.fp32err = reinterpret_cast<double*>(take(8 * s * B));
  r.pidx = reinterpret_cast<int32_t*>(take(8 * s * B));
  r.pp = reinterpret_cast<double*>(take(8 * s * B));
  r.pmargin = reinterpret_cast<double*>(take(8 * s * B));
  r.pflags = reinterpret_cast<int32_t*>(take(4 * s * B));
  r.total = o;
  return r;
}

afd_status ensure_res(afd_plan_s* p, int steps) {
  if (p->res && p->res_steps >= steps) return AFD_OK;
  if (p->res) {
    (void)hipFree(p->res);
    p->res = nullptr;
  }
  const size_t bytes = res_layout(nullptr, steps, p->cfg.batch).total;
  hipError_t e = hipMalloc(&p->res, bytes);
  if (e != hipSuccess) {
    p->res = nullptr;
    return fail(AFD_E_NOMEM, std::string("result staging: ") + hipGetErrorString(e));
  }
  p->res_steps = steps;
  return AFD_OK;
}

afd_status ensure_forced(afd_plan_s* p, int steps) {
  if (p->forced && p->forced_steps >= steps) return AFD_OK;
  if (p->forced) {
    (void)hipFree(p->forced);
    p->forced = nullptr;
  }
  hipError_t e = hipMalloc(&p->forced, 8 * size_t(steps < 1 ? 1 : steps) * size_t(p->cfg.batch));
  if (e != hipSuccess) {
    p->forced = nullptr;
    return fail(AFD_E_NOMEM, std::string("forced indices: ") + hipGetErrorString(e));
  }
  p->forced_steps = steps;
  return AFD_OK;
}

// Per-kernel timing: the events are handed to the launch itself, which
// stamps the dispatch's start and end (no extra packets on the stream).
struct Timer {
  afd_plan_s* p;
  bool off = false;  // no timing in this call (it creates no events)
  size_t next = 0;
  // events for one timed unit of kind k, or nulls when k is not timed
  hipError_t pair(int k, hipEvent_t* a, hipEvent_t* b) {
    *a = *b = nullptr;
    if (off || p->time_kind != k) return hipSuccess;
    if (p->time_seen++ % p->time_every != 0) return hipSuccess;  // not sampled
    if (next >= p->events.size() / 2) {
      hipEvent_t x, y;
      hipError_t e = hipEventCreate(&x);
      if (e != hipSuccess) return e;
      e = hipEventCreate(&y);
      if (e != hipSuccess) {
        (void)hipEventDestroy(x);
        return e;
      }
      p->events.push_back(x);
      p->events.push_back(y);
    }
    *a = p->events[2 * next];
    *b = p->events[2 * next + 1];
    ++next;
    return hipSuccess;
  }
  hipError_t collect() {
    for (size_t i = 0; i < next; ++i) {
      float ms = 0.f;
      const hipError_t e = hipEventElapsedTime(&ms, p->events[2 * i], p->events[2 * i + 1]);
      if (e != hipSuccess) return e;
      p->time_ms += ms;
      p->time_launches += 1;
    }
    return hipSuccess;
  }
};

#define HIPCHK(expr, where)                     \
  do {                                          \
    const hipError_t _e = (expr);               \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

// A replayed step after its selection: the records are merged (when the
// radius kernel left them to the step tail) and, in single precision, the
// short-list re-checked, as afd_decompose does; then k_pick records that
// choice and puts the forced point in its place, whose coefficient is the
// FFT-form grid value (double precision) or the direct rule in double (a
// one-entry re-check).  The winner is then in p->L.winner.
// The non-uniform FFT's device tables of a plan.
NuTables nu_tables(afd_plan_s* p) {
  NuTables t{};
  t.turns = p->at<double>(p->L.nu_t);
  t.ws = p->at<double>(p->L.nu_ws);
  t.rng = p->at<int4>(p->L.nu_rng);
  t.b = p->at<double>(p->L.nu_b);
  t.B = p->at<double>(p->L.nu_B);
  t.xt = p->at<void>(p->L.nu_xt);
  t.tw1 = p->at<void>(p->L.nu_tw1);
  t.tw2 = p->at<void>(p->L.nu_tw2);
  t.omega = p->at<double>(p->L.nu_omega);
  t.lognm = p->cfg.nu_lognm;
  t.ctail = p->at<void>(p->L.nu_ctail);
  t.nfold = p->cfg.nfold;
  t.rho = p->at<double>(p->L.nu_rho);
  t.cfold = p->at<void>(p->L.nu_cfold);
  t.dinv = p->at<double>(p->L.nu_dinv);
  return t;
}

// The re-check's samples: the plan's non-uniform positions and weights, or
// the uniform points (null).
RecheckSamples samples_of(afd_plan_s* p) {
  if (!p->cfg.nu) return RecheckSamples{nullptr, nullptr, 0};
  return RecheckSamples{p->at<double>(p->L.nu_z), p->at<double>(p->L.nu_w), p->cfg.ns};
}

afd_status replay_pick(afd_plan_s* p, int k, bool merged, PickArgs pk) {
  const Config& c = p->cfg;
  const int B = c.batch;
  hipStream_t s = p->stream;
  CandList* cand = p->at<CandList>(p->L.cand);
  Winner* win = p->at<Winner>(p->L.winner);
  unsigned int* counters = p->at<unsigned int>(p->L.counters);
  const double* omega = p->at<double>(p->L.omega);
  const double* radii = p->at<double>(p->L.radii);
  double* g64 = p->at<double>(p->L.g64);
  double* partials = p->at<double>(p->L.partials);
  if (!merged)
    HIPCHK(launch_merge(c.fp64, p->at<void>(p->L.blocks), c.fp64 ? nullptr : p->at<uint64_t>(p->L.heads),
                        c.fp64 ? nullptr : p->at<uint64_t>(p->L.seconds), c.nblocks, int(c.N), p->recheck_k,
                        p->tau_band, counters + 4 * B, cand, win, B, s),
           "k_merge");
  if (!c.fp64)
    HIPCHK(launch_recheck(cand, g64, omega, radii, int(c.N), partials, counters + 1 * B, win, B, s, samples_of(p)),
           "k_recheck");
  pk.step = k;
  HIPCHK(launch_pick(pk, B, s), "k_pick");
  if (!c.fp64)
    HIPCHK(launch_recheck(cand, g64, omega, radii, int(c.N), partials, counters + 1 * B, win, B, s, samples_of(p)),
           "k_recheck");
  return AFD_OK;
}

// Steps of a plan with the fused step tail: per step the radius kernel (or a
// forced point), then one launch_advance that re-checks, updates and
// transforms the new remainder for the next step.  A replayed step runs the
// radius kernel and the selection too (replay_pick), and the step tail then
// updates with the forced point.
afd_status run_adv(afd_plan_s* p, int steps, const int32_t* forced_user, const RecordArgs& rec,
                   RadiusParams rp, const PickArgs& pk, Timer& tm) {
  const Config& c = p->cfg;
  const int B = c.batch;
  hipStream_t s = p->stream;
  const bool replay = forced_user != nullptr;
  auto forced_at = [&](int k) { return !replay && p->first_a_zero && k == 0; };
  AdvanceArgs a{};
  a.cand = p->at<CandList>(p->L.cand);
  a.winner = p->at<Winner>(p->L.winner);
  a.g64 = p->at<double>(p->L.g64);
  a.radii = p->at<double>(p->L.radii);
  a.omega = p->at<double>(p->L.omega);
  a.omega_t = c.fp64 ? p->at<void>(p->L.omega) : p->at<void>(p->L.omega_t);
  a.tw1 = p->at<void>(p->L.twf1);
  a.tw2 = p->at<void>(p->L.twf2);
  a.xt = p->at<void>(p->L.xt);
  a.c = p->at<void>(p->L.c);
  a.partials = p->at<double>(p->L.partials);
  a.epart = p->at<double>(p->L.epart);
  a.bar = p->at<unsigned long long>(p->L.bar);
  a.status = p->at<int>(p->L.nonfinite);
  a.recs = p->at<void>(p->L.blocks);
  a.heads = c.fp64 ? nullptr : p->at<uint64_t>(p->L.heads);
  a.seconds = c.fp64 ? nullptr : p->at<uint64_t>(p->L.seconds);
  a.recheck_k = p->recheck_k;
  a.tau_band = p->tau_band;
  a.flagword = p->at<unsigned int>(p->L.counters) + 4 * B;
  a.R = rec;
  a.M = c.M;
  // one signal on a stream that has the device to itself: one launch with grid barriers
  const bool fused = B == 1 && !p->concurrent && !p->split_tail;
  auto advance = [&](hipEvent_t e0, hipEvent_t e1) -> hipError_t {
    const hipError_t e = launch_advance(c.logn, c.fp64, a, B, fused, s, e0, e1);
    if (fused) advance_bar_advance(c.logn, a);
    return e;
  };
  if (steps > 0 && !forced_at(0)) {
    hipEvent_t e0, e1;
    HIPCHK(tm.pair(kTimeFft, &e0, &e1), "event");
    a.update = 0;
    a.recheck = 0;
    a.nrec = 0;
    a.fft = 1;
    a.step = -1;
    HIPCHK(advance(e0, e1), "k_advance");
  }
  for (int k = 0; k < steps; ++k) {
    const bool forced = forced_at(k);
    if (forced) {
      HIPCHK(launch_force(p->at<int32_t>(p->L.forced0), 0, 0, int(c.N), p->at<CandList>(p->L.cand), B, s),
             "k_force");
    } else {
      hipEvent_t e0, e1;
      HIPCHK(tm.pair(kTimeRadius, &e0, &e1), "event");
      const int grid = rp.queue ? p->rslots : c.nblocks;
      if (replay && c.fp64) rp.probe = p->forced + 2 * k;
      HIPCHK(launch_radius(c.logn, c.fp64, rp, grid, B, s, e0, e1), "k_radius");
      // the queue hands out the slots past the grid: every processed slot
      // takes one ticket (each workgroup's last one comes back past the end),
      // nblocks tickets per launch
      if (rp.queue) rp.qbase += unsigned(c.nblocks);
      if (replay) {
        const afd_status st = replay_pick(p, k, false, pk);
        if (st != AFD_OK) return st;
      }
    }
    hipEvent_t u0, u1;
    HIPCHK(tm.pair(kTimeUpdate, &u0, &u1), "event");
    a.update = 1;
    // a forced point comes as a one-entry short-list; a replayed step's winner is ready
    a.recheck = (!replay && (!c.fp64 || forced)) ? 1 : 0;
    a.nrec = (forced || replay) ? 0 : c.nblocks;
    a.fft = (k + 1 < steps && !forced_at(k + 1)) ? 1 : 0;
    a.step = k;
    HIPCHK(advance(u0, u1), "k_advance");
  }
  return AFD_OK;
}

// `staging`: where the results are staged on the device (the static scratch
// of afd_decompose_noalloc), or null for the plan's own staging.  `graph`:
// the call is being captured into a HIP graph (afd_graph_create): the
// records go straight into the caller's device arrays (staging only for the
// null ones), counters are cleared by a kernel, nothing is timed, and the
// host neither waits nor checks the flag (afd_graph_status reads it).
afd_status run(afd_plan_s* p, const double* signal, int steps, const int32_t* forced_user, afd_result* out,
               unsigned char* staging = nullptr, bool graph = false) {
  if (!p) return fail(AFD_E_INVALID, "plan is NULL");
  if (!signal) return fail(AFD_E_INVALID, "signal is NULL");
  if (!out) return fail(AFD_E_INVALID, "out is NULL");
  if (steps < 0) return fail(AFD_E_INVALID, "steps must be >= 0");
  if (!out->energy || (steps > 0 && (!out->index || !out->a || !out->coef)))
    return fail(AFD_E_INVALID, "out.energy (and out.index, out.a, out.coef when steps > 0) are required");
  const Config& c = p->cfg;
  const int N = int(c.N);
  const int NS = c.ns;  // samples per signal
  const int B = c.batch;
  HIPCHK(hipSetDevice(p->device), "hipSetDevice");

  const bool sig_dev = is_device_pointer(signal);
  if (graph) {
    const void* dev[] = {signal, out->index, out->a, out->coef, out->energy, out->margin, out->remainder,
                         out->recheck_count, out->flags, out->fp32_error};
    for (const void* q : dev)
      if (q && !is_device_pointer(q))
        return fail(AFD_E_INVALID, "a captured decomposition needs device pointers for the signal and outputs");
  }
  if (!sig_dev) {
    for (int64_t i = 0; i < 2 * int64_t(NS) * B; ++i)
      if (!std::isfinite(signal[i])) return fail(AFD_E_NONFINITE, "signal holds NaN or Inf");
  }
  std::vector<int32_t> forced_host;
  if (forced_user) {
    const size_t nf = 2 * size_t(steps) * size_t(B);
    forced_host.resize(nf);
    if (steps > 0)
      HIPCHK(hipMemcpy(forced_host.data(), forced_user, 4 * nf, hipMemcpyDefault), "reading forced indices");
    for (size_t k = 0; k < nf; k += 2) {
      if (forced_host[k] < 0 || forced_host[k] >= c.M || forced_host[k + 1] < 0 || forced_host[k + 1] >= N)
        return fail(AFD_E_INVALID, "forced index outside [0,M) x [0,N)");
    }
    afd_status st = ensure_forced(p, steps);
    if (st != AFD_OK) return st;
    if (steps > 0)
      HIPCHK(hipMemcpyAsync(p->forced, forced_host.data(), 4 * nf, hipMemcpyHostToDevice, p->stream),
             "uploading forced indices");
  }
  afd_status st = AFD_OK;
  if (!staging) {
    st = ensure_res(p, steps);
    if (st != AFD_OK) return st;
  }
  const ResPtrs R = res_layout(staging ? staging : p->res, steps, B);

  hipStream_t s = p->stream;
  double* g64 = p->at<double>(p->L.g64);
  float* g32 = c.fp64 || c.adv ? nullptr : p->at<float>(p->L.g32);
  void* cspec = p->at<void>(p->L.c);
  const double* radii = p->at<double>(p->L.radii);
  const double* omega = p->at<double>(p->L.omega);
  Winner* win = p->at<Winner>(p->L.winner);
  CandList* cand = p->at<CandList>(p->L.cand);
  double* partials = p->at<double>(p->L.partials);
  double* epart = p->at<double>(p->L.epart);
  int* nonfinite = p->at<int>(p->L.nonfinite);
  const int32_t* forced0 = p->at<int32_t>(p->L.forced0);
  unsigned int* counters = p->at<unsigned int>(p->L.counters);

  RecordArgs rec{};
  rec.w = win;
  rec.radii = radii;
  rec.omega = omega;
  rec.N = N;
  rec.M = c.M;
  rec.steps = steps;
  rec.idx = graph ? out->index : R.idx;
  rec.a = graph ? out->a : R.a;
  rec.coef = graph ? out->coef : R.coef;
  rec.energy = graph ? out->energy : R.energy;
  rec.margin = graph && out->margin ? out->margin : R.margin;
  rec.kcount = graph && out->recheck_count ? out->recheck_count : R.kcount;
  rec.flags = graph && out->flags ? out->flags : R.flags;
  rec.fp32err = graph && out->fp32_error ? out->fp32_error : R.fp32err;

  // flags and last-workgroup counters start at zero (also after an aborted
  // call); in a captured graph by a kernel (no memset nodes)
  if (graph) {
    ZeroArgs z{};
    auto add = [&](void* q, size_t bytes) {
      z.p[z.n] = static_cast<unsigned int*>(q);
      z.words[z.n] = int(bytes / 4);
      ++z.n;
    };
    add(nonfinite, 4);
    add(counters, 4 * kNumCounters * size_t(B));
    if (c.adv) add(p->arena + p->L.bar, 8 * 16 * kBarGroups);
    if (c.adv) add(p->arena + p->L.rqueue, 4);
    if (c.big) add(p->arena + p->L.bcounters, 4);
    HIPCHK(launch_zero(z, s), "k_zero");
  } else {
    HIPCHK(hipMemsetAsync(nonfinite, 0, 4, s), "clearing flag");
    HIPCHK(hipMemsetAsync(counters, 0, 4 * kNumCounters * size_t(B), s), "clearing counters");
    if (c.adv) HIPCHK(hipMemsetAsync(p->arena + p->L.bar, 0, 8 * 16 * kBarGroups, s), "clearing counters");
    if (c.adv) HIPCHK(hipMemsetAsync(p->arena + p->L.rqueue, 0, 4, s), "clearing counters");
    if (c.big) HIPCHK(hipMemsetAsync(p->arena + p->L.bcounters, 0, 4, s), "clearing counters");
  }
  HIPCHK(hipMemcpyAsync(g64, signal, 16 * size_t(NS) * B, sig_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        s),
         "copying signal");
  // counters are [kind][signal]: radius, recheck, update, prepare, FP32 fallback flags
  const RecheckSamples smp = samples_of(p);
  const double* nu_w = c.nu ? p->at<double>(p->L.nu_w) : nullptr;
  if (c.nu)
    HIPCHK(launch_nu_prepare(g64, nu_w, NS, epart, nonfinite, counters + 3 * B, rec, B, s), "k_nu_prepare");
  else
    HIPCHK(launch_prepare(g64, g32, N, epart, nonfinite, counters + 3 * B, rec, B, s), "k_prepare");

  RadiusParams rp{};
  rp.c = cspec;
  rp.pw = p->at<void>(p->L.pw);
  rp.pv = p->at<void>(p->L.pv);
  rp.pq = p->at<void>(p->L.pq);
  rp.lsig = p->at<int>(p->L.lsig);
  rp.order = p->at<int>(p->L.order);
  rp.scale = p->at<void>(p->L.scale);
  rp.tw = p->at<void>(p->L.tw);
  rp.M = c.M;
  rp.rpb = c.rpb;
  rp.tau_band = p->tau_band;
  rp.recheck_k = p->recheck_k;
  rp.out = p->at<void>(p->L.blocks);
  rp.counter = counters + 0 * B;
  rp.heads = p->at<uint64_t>(p->L.heads);
  rp.seconds = p->at<uint64_t>(p->L.seconds);
  rp.flagword = counters + 4 * B;
  rp.cand = cand;
  rp.winner = win;
  rp.tail = c.adv ? 0 : 1;  // with the fused step tail, the tail merges the records
  rp.nrec = c.nblocks;
  // one signal with more radius workgroups than fit at once: a work queue
  // (double precision; see radius_queued)
  const bool queued =
      c.fp64 && c.adv && B == 1 && c.rpb == 1 && p->rslots > 0 && p->rslots < c.nblocks && !p->no_queue;
  rp.queue = queued ? p->at<unsigned int>(p->L.rqueue) : nullptr;
  rp.qbase = 0;
  rp.probe = nullptr;  // set per replayed step (double precision)
  rp.probe_stride = 2 * steps;
  rp.probe_out = p->at<double>(p->L.probe);
  // non-uniform samples: radii whose series outlasts N terms read folded spectra
  rp.cfold = c.nu && c.nfold > 0 ? p->at<void>(p->L.nu_cfold) : nullptr;
  rp.fslot = c.nu && c.nfold > 0 ? p->at<int>(p->L.nu_fslot) : nullptr;
  rp.nfold = c.nu ? c.nfold : 0;

  BigParams bp{};
  if (c.big) {
    bp.c = cspec;
    bp.c0 = p->at<void>(p->L.c0);
    bp.pa = p->at<void>(p->L.pw);
    bp.pb = p->at<void>(p->L.pv);
    bp.scale = p->at<void>(p->L.scale);
    bp.lsig = p->at<int>(p->L.lsig);
    bp.wl = p->at<void>(p->L.wl);
    bp.wh = p->at<void>(p->L.wh);
    bp.tw1 = p->at<void>(p->L.twf1);
    bp.tw2 = p->at<void>(p->L.twf2);
    bp.tw2m[0] = p->at<void>(p->L.twm);
    bp.tw2m[1] = p->at<void>(p->L.twm2);
    bp.gstride = c.bg.gstride;
    bp.med = 1;
    bp.z = p->at<void>(p->L.z);
    bp.M = c.M;
    bp.m0 = 0;
    bp.tau_band = p->tau_band;
    bp.recheck_k = p->recheck_k;
    bp.blocks = p->at<void>(p->L.blocks);
    bp.rrec = p->at<void>(p->L.rrec);
    bp.counter_g = p->at<unsigned int>(p->L.bcounters);
    bp.heads = p->at<uint64_t>(p->L.heads);
    bp.flagword = counters + 4 * B;
    bp.cand = cand;
    bp.winner = win;
    bp.probe = nullptr;
    bp.probe_out = p->at<double>(p->L.probe);
    bp.border = p->at<int>(p->L.border);
  }
  const bool replay = forced_user != nullptr;
  PickArgs pk{};
  pk.forced = p->forced;
  pk.fstride = 2 * steps;
  pk.N = N;
  pk.logn = c.logn;
  pk.M = c.M;
  pk.steps = steps;
  pk.fp64 = c.fp64 ? 1 : 0;
  pk.cand = cand;
  pk.winner = win;
  pk.probe = p->at<double>(p->L.probe);
  pk.idx = R.pidx;
  pk.p = R.pp;
  pk.margin = R.pmargin;
  pk.flags = R.pflags;

  Timer tm{p};
  tm.off = staging != nullptr || graph;
  UpdateArgs upd{};
  upd.radii = radii;
  upd.omega = omega;
  upd.N = N;
  upd.M = c.M;
  upd.epart = epart;
  upd.counter = counters + 2 * B;
  upd.R = rec;
  if (c.adv) {
    st = run_adv(p, steps, forced_user, rec, rp, pk, tm);
    if (st != AFD_OK) return st;
  }
  for (int k = 0; k < (c.adv ? 0 : steps); ++k) {
    if (!replay && p->first_a_zero && k == 0) {
      HIPCHK(launch_force(forced0, 0, 0, N, cand, B, s), "k_force");
      HIPCHK(launch_recheck(cand, g64, omega, radii, N, partials, counters + 1 * B, win, B, s, smp), "k_recheck");
    } else {
      hipEvent_t e0, e1;
      HIPCHK(tm.pair(kTimeFft, &e0, &e1), "event");
      const void* gin = c.fp64 ? static_cast<const void*>(g64) : static_cast<const void*>(g32);
      if (c.nu)
        HIPCHK(launch_nu_fourier(g64, nu_tables(p), c.logn, c.fp64, cspec, NS, B, s, e0, e1), "non-uniform DFT");
      else if (c.mixed)
        HIPCHK(launch_fwd_mixed(c.mg, p->at<int>(p->L.mixp), c.fp64, gin, p->at<void>(p->L.tw), cspec, B, s, e0, e1),
               "forward DFT");
      else if (c.pk)
        HIPCHK(launch_fwd_pp(c.prime, c.pk, c.fp64, gin, p->at<void>(p->L.tw), p->at<void>(p->L.twf1),
                             p->at<void>(p->L.twf2), omega, p->at<void>(p->L.xt), cspec, B, s, e0, e1),
               "forward DFT");
      else
        HIPCHK(launch_fwd(c.logn, c.fp64, gin, p->at<void>(p->L.twf1), p->at<void>(p->L.twf2), omega,
                          p->at<void>(p->L.xt), cspec, B, s, e0, e1, c.big ? p->at<void>(p->L.c0) : nullptr),
               "forward DFT");
      HIPCHK(tm.pair(kTimeRadius, &e0, &e1), "event");
      if (replay && c.fp64) {
        rp.probe = p->forced + 2 * k;
        bp.probe = p->forced + 2 * k;
      }
      if (c.big) {
        // the radii with short spectra in one row launch, then the others in
        // chunks through the intermediate (launch order in p->L.border)
        bool first = true;
        for (int m0 = 0; m0 < c.M;) {
          // launch positions: short radii, the two medium classes, then chunks of long ones
          const int b1 = c.nshort, b2 = b1 + c.nmed[0], b3 = b2 + c.nmed[1];
          const int med = m0 < b1 ? 0 : m0 < b2 ? 1 : m0 < b3 ? 2 : 0;
          const bool longs = m0 >= b3;
          int nr = m0 < b1 ? b1 - m0 : m0 < b2 ? b2 - m0 : m0 < b3 ? b3 - m0
                                                                 : (c.M - m0 < p->chunk ? c.M - m0 : p->chunk);
          if (nr > kMaxGridY) nr = kMaxGridY;  // radii run along grid y
          bp.m0 = m0;
          hipEvent_t r0, r1;
          HIPCHK(tm.pair(kTimeRows, &r0, &r1), "event");
          HIPCHK(launch_big(c.logn, c.fp64, bp, nr, longs, med, s, first ? e0 : nullptr, nullptr, r0, r1), "k_big");
          first = false;
          m0 += nr;
        }
        HIPCHK(launch_big_merge(c.logn, c.fp64, bp, s, e1), "k_big_merge");
      } else if (c.pk) {
        HIPCHK(launch_radius_pp(c.prime, c.pk, c.fp64, rp, B, s, e0, e1), "k_radius_pp");
      } else if (c.mixed) {
        HIPCHK(launch_radius_mixed(c.mg, p->at<int>(p->L.mixp), c.fp64, rp, B, s, e0, e1), "k_radius_mixed");
      } else {
        HIPCHK(launch_radius(c.logn, c.fp64, rp, c.nblocks, B, s, e0, e1), "k_radius");
      }
      if (replay) {
        // the radius kernel's last workgroup merged the records
        st = replay_pick(p, k, true, pk);
        if (st != AFD_OK) return st;
      } else if (!c.fp64) {
        HIPCHK(launch_recheck(cand, g64, omega, radii, N, partials, counters + 1 * B, win, B, s, smp), "k_recheck");
      }
    }
    hipEvent_t u0, u1;
    HIPCHK(tm.pair(kTimeUpdate, &u0, &u1), "event");
    upd.step = k;
    if (c.nu)
      HIPCHK(launch_nu_update(g64, nu_w, smp.z, NS, upd, B, s, u0, u1), "k_nu_update");
    else
      HIPCHK(launch_update(g64, g32, upd, B, s, u0, u1), "k_update");
  }
  if (graph) {
    if (out->remainder)
      HIPCHK(hipMemcpyAsync(out->remainder, g64, 16 * size_t(NS) * B, hipMemcpyDeviceToDevice, s), "copy remainder");
    return AFD_OK;
  }
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, nonfinite, 4, hipMemcpyDeviceToHost, s), "reading flag");
  HIPCHK(hipStreamSynchronize(s), "hipStreamSynchronize");
  HIPCHK(tm.collect(), "hipEventElapsedTime");
  if (bad & 2) return fail(AFD_E_HIP, "a grid barrier of the step tail timed out");
  if (bad) return fail(AFD_E_NONFINITE, "signal holds NaN or Inf");

  // staged signal-major with per-signal stride `steps`: the caller's layout
  const size_t S = size_t(steps), BB = size_t(B);
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s) : hipSuccess;
  };
  HIPCHK(cp(out->index, R.idx, 8 * S * BB), "copy index");
  HIPCHK(cp(out->a, R.a, 16 * S * BB), "copy a");
  HIPCHK(cp(out->coef, R.coef, 16 * S * BB), "copy coef");
  HIPCHK(cp(out->energy, R.energy, 8 * (S + 1) * BB), "copy energy");
  if (out->margin) HIPCHK(cp(out->margin, R.margin, 8 * S * BB), "copy margin");
  if (out->recheck_count) HIPCHK(cp(out->recheck_count, R.kcount, 4 * S * BB), "copy recheck_count");
  if (out->flags) HIPCHK(cp(out->flags, R.flags, 4 * S * BB), "copy flags");
  if (out->fp32_error) HIPCHK(cp(out->fp32_error, R.fp32err, 8 * S * BB), "copy fp32_error");
  if (replay) {
    if (out->pick_index) HIPCHK(cp(out->pick_index, R.pidx, 8 * S * BB), "copy pick_index");
    if (out->pick_p) HIPCHK(cp(out->pick_p, R.pp, 8 * S * BB), "copy pick_p");
    if (out->pick_margin) HIPCHK(cp(out->pick_margin, R.pmargin, 8 * S * BB), "copy pick_margin");
    if (out->pick_flags) HIPCHK(cp(out->pick_flags, R.pflags, 4 * S * BB), "copy pick_flags");
  }
  if (out->remainder) HIPCHK(cp(out->remainder, g64, 16 * size_t(NS) * BB), "copy remainder");
  HIPCHK(hipStreamSynchronize(s), "hipStreamSynchronize");
  g_last_error.clear();
  return AFD_OK;
}

afd_status ensure_aux(afd_plan_s* p, size_t bytes) {
  if (p->aux && p->aux_bytes >= bytes) return AFD_OK;
  if (p->aux) {
    (void)hipFree(p->aux);
    p->aux = nullptr;
    p->aux_bytes = 0;
  }
  const hipError_t e = hipMalloc(&p->aux, bytes);
  if (e != hipSuccess) {
    p->aux = nullptr;
    return fail(AFD_E_NOMEM, std::string("scratch: ") + hipGetErrorString(e));
  }
  p->aux_bytes = bytes;
  return AFD_OK;
}

// Copy n doubles from host or device memory into `dst` (host).
hipError_t fetch(std::vector<double>& dst, const double* src, size_t n) {
  dst.resize(n);
  return n ? hipMemcpy(dst.data(), src, 8 * n, hipMemcpyDefault) : hipSuccess;
}

afd_status reconstruct(afd_plan_s* p, const double* a, const double* coef, int steps, const double* signal,
                       double* partial_sum, double* delta) {
  if (!p) return fail(AFD_E_INVALID, "plan is NULL");
  if (steps < 0) return fail(AFD_E_INVALID, "steps must be >= 0");
  if (steps > 0 && (!a || !coef)) return fail(AFD_E_INVALID, "a and coef are required when steps > 0");
  if (delta && !signal) return fail(AFD_E_INVALID, "delta needs the signal");
  const Config& c = p->cfg;
  // (non-uniform samples: the partial sums at the sample points, the errors in the quadrature norm)
  const int N = c.ns, B = c.batch;
  HIPCHK(hipSetDevice(p->device), "hipSetDevice");
  const size_t nk = 2 * size_t(steps) * B;
  std::vector<double> ah, ch, gh;
  HIPCHK(fetch(ah, a, nk), "reading a");
  HIPCHK(fetch(ch, coef, nk), "reading coef");
  for (size_t i = 0; i < nk; i += 2) {
    if (!std::isfinite(ah[i]) || !std::isfinite(ah[i + 1]) || !std::isfinite(ch[i]) || !std::isfinite(ch[i + 1]))
      return fail(AFD_E_NONFINITE, "a or coef holds NaN or Inf");
    if (!(ah[i] * ah[i] + ah[i + 1] * ah[i + 1] < 1.0)) return fail(AFD_E_INVALID, "|a_k| >= 1");
  }
  const size_t nsig = 2 * size_t(N) * B;
  if (signal) {
    HIPCHK(fetch(gh, signal, nsig), "reading signal");
    for (double v : gh)
      if (!std::isfinite(v)) return fail(AFD_E_NONFINITE, "signal holds NaN or Inf");
  }
  // scratch: a, coef, signal, partial sums, wave sums, delta
  const size_t wps = (delta && steps > 0) ? size_t(steps + 1) * recon_waves(N) * B : 0;
  const size_t o_a = 0, o_c = align_up(o_a + 8 * nk, 256), o_g = align_up(o_c + 8 * nk, 256);
  const size_t o_s = align_up(o_g + (signal ? 8 * nsig : 0), 256);
  const size_t o_w = align_up(o_s + (partial_sum ? 8 * nsig : 0), 256);
  const size_t o_d = align_up(o_w + 8 * wps, 256);
  const size_t total = align_up(o_d + 8 * size_t(steps) * B, 256) + 256;
  afd_status st = ensure_aux(p, total);
  if (st != AFD_OK) return st;
  hipStream_t s = p->stream;
  double* da = reinterpret_cast<double*>(p->aux + o_a);
  double* dc = reinterpret_cast<double*>(p->aux + o_c);
  double* dg = signal ? reinterpret_cast<double*>(p->aux + o_g) : nullptr;
  double* ds = partial_sum ? reinterpret_cast<double*>(p->aux + o_s) : nullptr;
  double* dw = wps ? reinterpret_cast<double*>(p->aux + o_w) : nullptr;
  double* dd = reinterpret_cast<double*>(p->aux + o_d);
  if (nk) {
    HIPCHK(hipMemcpyAsync(da, ah.data(), 8 * nk, hipMemcpyHostToDevice, s), "uploading a");
    HIPCHK(hipMemcpyAsync(dc, ch.data(), 8 * nk, hipMemcpyHostToDevice, s), "uploading coef");
  }
  if (dg) HIPCHK(hipMemcpyAsync(dg, gh.data(), 8 * nsig, hipMemcpyHostToDevice, s), "uploading signal");
  if (ds || dw)
    HIPCHK(launch_recon(da, dc, steps, N, p->at<double>(c.nu ? p->L.nu_z : p->L.omega), dg, ds, dw,
                        delta ? dd : nullptr, B, s, c.nu ? p->at<double>(p->L.nu_w) : nullptr),
           "k_recon");
  if (partial_sum) HIPCHK(hipMemcpyAsync(partial_sum, ds, 8 * nsig, hipMemcpyDefault, s), "copy partial sum");
  if (delta && steps > 0)
    HIPCHK(hipMemcpyAsync(delta, dd, 8 * size_t(steps) * B, hipMemcpyDefault, s), "copy delta");
  HIPCHK(hipStreamSynchronize(s), "hipStreamSynchronize");
  g_last_error.clear();
  return AFD_OK;
}

afd_status analytic(afd_plan_s* p, const double* x, double* g) {
  if (!p) return fail(AFD_E_INVALID, "plan is NULL");
  if (!x || !g) return fail(AFD_E_INVALID, "x and g are required");
  const Config& c = p->cfg;
  if (c.pk || c.mixed || c.nu) return fail(AFD_E_UNSUPPORTED, "afd_analytic needs N = 2^K uniform samples");
  const int N = int(c.N), B = c.batch, logn = c.logn;
  HIPCHK(hipSetDevice(p->device), "hipSetDevice");
  const size_t nsig = 2 * size_t(N) * B;
  const bool x_dev = is_device_pointer(x);
  std::vector<double> xh;
  if (!x_dev) {
    for (size_t i = 0; i < nsig; ++i)
      if (!std::isfinite(x[i])) return fail(AFD_E_NONFINITE, "x holds NaN or Inf");
  }
  // double-precision forward DFT tables of the standard (non-fused) plan
  const FwdPlan fp = fwd_plan(logn, true);
  std::vector<double> tw1(2 * size_t(fp.tw1_size + 1), 0.0), tw2(2 * size_t(fp.tw2_size + 1), 0.0);
  fft_twiddles(fp.two_pass ? fp.l1 : logn, true, tw1.data());
  if (fp.two_pass) fft_twiddles(fp.l2, true, tw2.data());
  const size_t o_x = 0, o_y = align_up(8 * nsig, 256), o_t = align_up(o_y + 8 * nsig, 256);
  const size_t o_w1 = align_up(o_t + (fp.two_pass ? 8 * nsig : 0), 256);
  const size_t o_w2 = align_up(o_w1 + 8 * tw1.size(), 256);
  const size_t o_f = align_up(o_w2 + 8 * tw2.size(), 256);
  afd_status st = ensure_aux(p, o_f + 256);
  if (st != AFD_OK) return st;
  hipStream_t s = p->stream;
  double* X = reinterpret_cast<double*>(p->aux + o_x);
  double* Y = reinterpret_cast<double*>(p->aux + o_y);
  void* xt = p->aux + o_t;
  void* w1 = p->aux + o_w1;
  void* w2 = p->aux + o_w2;
  int* flag = reinterpret_cast<int*>(p->aux + o_f);
  HIPCHK(hipMemcpyAsync(w1, tw1.data(), 8 * tw1.size(), hipMemcpyHostToDevice, s), "uploading twiddles");
  HIPCHK(hipMemcpyAsync(w2, tw2.data(), 8 * tw2.size(), hipMemcpyHostToDevice, s), "uploading twiddles");
  HIPCHK(hipMemsetAsync(flag, 0, 4, s), "clearing flag");
  HIPCHK(hipMemcpyAsync(Y, x, 8 * nsig, x_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s), "copying x");
  const int cl1 = logn > kMaxLdsLogN ? fp.l1 : 0, cl2 = logn > kMaxLdsLogN ? fp.l2 : 0;
  HIPCHK(launch_fwd(logn, true, Y, w1, w2, p->at<double>(p->L.omega), xt, X, B, s), "forward DFT");
  HIPCHK(launch_analytic_mask(X, Y, N, cl1, cl2, flag, B, s), "k_analytic_mask");
  HIPCHK(launch_fwd(logn, true, Y, w1, w2, p->at<double>(p->L.omega), xt, X, B, s), "forward DFT");
  // the result goes to the caller's memory, or through Y to the host
  const bool g_dev = is_device_pointer(g);
  HIPCHK(launch_analytic_out(X, g_dev ? g : Y, N, cl1, cl2, flag, B, s), "k_analytic_out");
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, s), "reading flag");
  HIPCHK(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (bad) return fail(AFD_E_NONFINITE, "x holds NaN or Inf");
  if (!g_dev) HIPCHK(hipMemcpy(g, Y, 8 * nsig, hipMemcpyDeviceToHost), "copy g");
  g_last_error.clear();
  return AFD_OK;
}

// Launch choices found by afd_plan_tune, per device and plan shape; a plan
// created later with the same shape starts from them.
struct TuneKey {
  int device;
  int64_t n;
  int ns, m, fp64, batch, pk, nu;
  bool operator<(const TuneKey& o) const {
    return std::tie(device, n, ns, m, fp64, batch, pk, nu) <
           std::tie(o.device, o.n, o.ns, o.m, o.fp64, o.batch, o.pk, o.nu);
  }
};
struct TuneChoice {
  bool split_tail, no_queue;
  int chunk;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;

TuneKey tune_key(const afd_plan_s* p) {
  const Config& c = p->cfg;
  return TuneKey{p->device, c.N, c.ns, c.M, c.fp64 ? 1 : 0, c.batch, c.pk, c.nu ? 1 : 0};
}

}  // namespace

extern "C" {

afd_status afd_plan_create(const afd_plan_desc* desc, void* hip_stream, afd_plan* out) {
  if (!out) return fail(AFD_E_INVALID, "out is NULL");
  *out = nullptr;
  Config cfg;
  afd_status st = validate(desc, &cfg);
  if (st != AFD_OK) return st;
  afd_plan_s* p = new (std::nothrow) afd_plan_s();
  if (!p) return fail(AFD_E_NOMEM, "host allocation failed");
  p->cfg = cfg;
  p->L = layout_of(cfg);
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  p->recheck_k = desc->recheck_k == 0 ? 8 : desc->recheck_k;
  p->tau_band = desc->recheck_band == 0.0 ? default_tau_band(cfg.logn) : float(desc->recheck_band);
  p->first_a_zero = desc->first_a_zero != 0;
  p->concurrent = desc->concurrent != 0;
  for (int i = 0; i < desc->m; ++i)
    if (desc->radii[i] == 0.0) {
      p->zero_m = i;
      break;
    }
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) {
    static bool attrs_done = false;
    if (!attrs_done) {
      e = setup_radius_attributes();
      if (e == hipSuccess) e = setup_fwd_attributes();
      if (e == hipSuccess) e = setup_big_attributes();
      if (e == hipSuccess) e = setup_pp_attributes();
      if (e == hipSuccess) e = setup_mixed_attributes();
      if (e == hipSuccess) attrs_done = true;
    }
  }
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "device setup");
  }
  p->rslots = cfg.big || cfg.pk || cfg.mixed ? 0 : radius_slots(cfg.logn, cfg.fp64, cfg.rpb);
  p->chunk = cfg.chunk;
  {
    // a shape tuned earlier in this process starts from its choices
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(tune_key(p));
    if (it != g_tune.end()) {
      p->split_tail = it->second.split_tail;
      p->no_queue = it->second.no_queue;
      if (it->second.chunk > 0 && it->second.chunk <= cfg.chunk) p->chunk = it->second.chunk;
    }
  }
  e = hipMalloc(&p->arena, p->L.total);
  if (e != hipSuccess) {
    p->arena = nullptr;
    delete p;
    return fail(AFD_E_NOMEM, std::string("workspace: ") + hipGetErrorString(e));
  }
  st = build_tables(p, desc);
  if (st != AFD_OK) {
    afd_plan_destroy(p);
    return st;
  }
  *out = p;
  g_last_error.clear();
  return AFD_OK;
}

afd_status afd_decompose(afd_plan plan, const double* signal, int32_t steps, afd_result* out) {
  return run(plan, signal, steps, nullptr, out);
}

afd_status afd_graph_create(afd_plan plan, const double* signal, int32_t steps, const afd_result* out,
                            afd_graph* graph) {
  if (!graph) return fail(AFD_E_INVALID, "graph is NULL");
  *graph = nullptr;
  if (!plan) return fail(AFD_E_INVALID, "plan is NULL");
  if (!out) return fail(AFD_E_INVALID, "out is NULL");
  if (steps < 0) return fail(AFD_E_INVALID, "steps must be >= 0");
  HIPCHK(hipSetDevice(plan->device), "hipSetDevice");
  // the staging of the outputs the caller leaves null, allocated before the capture
  afd_status st = ensure_res(plan, steps);
  if (st != AFD_OK) return st;
  afd_graph_s* g = new (std::nothrow) afd_graph_s();
  if (!g) return fail(AFD_E_NOMEM, "host allocation failed");
  g->plan = plan;
  g->out = *out;
  g->steps = steps;
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "hipStreamCreateWithFlags");
  }
  // the plan's calls run on plan->stream: the capture swaps in its own stream
  hipStream_t own = plan->stream;
  plan->stream = cap;
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    afd_result o = *out;
    st = run(plan, signal, steps, nullptr, &o, nullptr, true);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cap, &gr);
    g->graph = gr;
    if (st == AFD_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
    if (st == AFD_OK) {
      e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
    }
  } else {
    st = hip_fail(e, "hipStreamBeginCapture");
  }
  plan->stream = own;
  (void)hipStreamDestroy(cap);
  if (st != AFD_OK) {
    afd_graph_destroy(g);
    return st;
  }
  *graph = g;
  g_last_error.clear();
  return AFD_OK;
}

void afd_group_destroy(afd_group group) {
  if (!group) return;
  if (group->exec) (void)hipGraphExecDestroy(group->exec);
  if (group->graph) (void)hipGraphDestroy(group->graph);
  delete group;
}

// The capture: a fork event on the group's stream, which every member's own
// capture stream waits on (joining the capture), the member's decomposition
// on its stream, and a join event per member that the group's stream waits
// on before the capture ends.
afd_status afd_group_create(const afd_plan* plans, int32_t count, const double* const* signals,
                            const int32_t* steps, const afd_result* outs, afd_group* group) {
  if (!group) return fail(AFD_E_INVALID, "group is NULL");
  *group = nullptr;
  if (!plans || !signals || !steps || !outs) return fail(AFD_E_INVALID, "NULL argument");
  if (count < 1) return fail(AFD_E_INVALID, "count must be >= 1");
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return fail(AFD_E_INVALID, "a plan is NULL");
    if (steps[i] < 0) return fail(AFD_E_INVALID, "steps must be >= 0");
    if (plans[i]->device != plans[0]->device) return fail(AFD_E_INVALID, "plans of different devices");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(AFD_E_INVALID, "a plan appears twice");
  }
  HIPCHK(hipSetDevice(plans[0]->device), "hipSetDevice");
  for (int i = 0; i < count; ++i) {
    const afd_status st = ensure_res(plans[i], steps[i]);
    if (st != AFD_OK) return st;
  }
  afd_group_s* g = new (std::nothrow) afd_group_s();
  if (!g) return fail(AFD_E_NOMEM, "host allocation failed");
  g->plans.assign(plans, plans + count);
  std::vector<hipStream_t> cap(size_t(count) + 1, nullptr);
  std::vector<hipEvent_t> ev(size_t(count) + 1, nullptr);
  afd_status st = AFD_OK;
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < cap.size() && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&cap[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) st = hip_fail(e, "creating capture streams");
  std::vector<hipStream_t> own(static_cast<size_t>(count));
  std::vector<bool> conc(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    own[i] = plans[i]->stream;
    conc[i] = plans[i]->concurrent;
  }
  if (st == AFD_OK) {
    e = hipStreamBeginCapture(cap[0], hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamBeginCapture");
  }
  if (st == AFD_OK) {
    e = hipEventRecord(ev[0], cap[0]);
    for (int i = 0; i < count && e == hipSuccess && st == AFD_OK; ++i) {
      e = hipStreamWaitEvent(cap[i + 1], ev[0], 0);
      if (e != hipSuccess) break;
      plans[i]->stream = cap[i + 1];
      plans[i]->concurrent = true;
      afd_result o = outs[i];
      st = run(plans[i], signals[i], steps[i], nullptr, &o, nullptr, true);
      if (st == AFD_OK) e = hipEventRecord(ev[i + 1], cap[i + 1]);
      if (st == AFD_OK && e == hipSuccess) e = hipStreamWaitEvent(cap[0], ev[i + 1], 0);
    }
    if (st == AFD_OK && e != hipSuccess) st = hip_fail(e, "forking the capture");
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cap[0], &gr);
    g->graph = gr;
    if (st == AFD_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
    if (st == AFD_OK) {
      e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
    }
  }
  for (int i = 0; i < count; ++i) {
    plans[i]->stream = own[i];
    plans[i]->concurrent = conc[i];
  }
  for (size_t i = 0; i < cap.size(); ++i) {
    if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (cap[i]) (void)hipStreamDestroy(cap[i]);
  }
  if (st != AFD_OK) {
    afd_group_destroy(g);
    return st;
  }
  *group = g;
  g_last_error.clear();
  return AFD_OK;
}

afd_status afd_group_launch(afd_group group) {
  if (!group) return fail(AFD_E_INVALID, "group is NULL");
  afd_plan_s* p0 = group->plans[0];
  HIPCHK(hipSetDevice(p0->device), "hipSetDevice");
  HIPCHK(hipGraphLaunch(group->exec, p0->stream), "hipGraphLaunch");
  return AFD_OK;
}

afd_status afd_group_status(afd_group group) {
  if (!group) return fail(AFD_E_INVALID, "group is NULL");
  afd_plan_s* p0 = group->plans[0];
  HIPCHK(hipSetDevice(p0->device), "hipSetDevice");
  HIPCHK(hipStreamSynchronize(p0->stream), "hipStreamSynchronize");
  for (afd_plan_s* p : group->plans) {
    int bad = 0;
    HIPCHK(hipMemcpy(&bad, p->arena + p->L.nonfinite, 4, hipMemcpyDeviceToHost), "reading flag");
    if (bad & 2) return fail(AFD_E_HIP, "a grid barrier of the step tail timed out");
    if (bad) return fail(AFD_E_NONFINITE, "a member's signal holds NaN or Inf");
  }
  return AFD_OK;
}

afd_status afd_graph_launch(afd_graph graph) {
  if (!graph) return fail(AFD_E_INVALID, "graph is NULL");
  HIPCHK(hipSetDevice(graph->plan->device), "hipSetDevice");
  HIPCHK(hipGraphLaunch(graph->exec, graph->plan->stream), "hipGraphLaunch");
  return AFD_OK;
}

afd_status afd_graph_status(afd_graph graph) {
  if (!graph) return fail(AFD_E_INVALID, "graph is NULL");
  afd_plan_s* p = graph->plan;
  HIPCHK(hipSetDevice(p->device), "hipSetDevice");
  HIPCHK(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  int bad = 0;
  HIPCHK(hipMemcpy(&bad, p->arena + p->L.nonfinite, 4, hipMemcpyDeviceToHost), "reading flag");
  if (bad & 2) return fail(AFD_E_HIP, "a grid barrier of the step tail timed out");
  if (bad) return fail(AFD_E_NONFINITE, "signal holds NaN or Inf");
  return AFD_OK;
}

void afd_graph_destroy(afd_graph graph) {
  if (!graph) return;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
}

afd_status afd_decompose_noalloc(afd_plan plan, const double* signal, int32_t steps, afd_result* out) {
  if (!plan) return fail(AFD_E_INVALID, "plan is NULL");
  if (steps < 0) return fail(AFD_E_INVALID, "steps must be >= 0");
  const size_t need = res_layout(nullptr, steps, plan->cfg.batch).total;
  if (need > kScratchBytes)
    return fail(AFD_E_INVALID, "steps * batch too large for the static scratch of afd_decompose_noalloc (" +
                                   std::to_string(need) + " > " + std::to_string(kScratchBytes) + " bytes)");
  hipError_t e = hipSetDevice(plan->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  unsigned char* staging = nullptr;
  const afd_status st = scratch_of(plan->device, &staging);
  if (st != AFD_OK) return st;
  return run(plan, signal, steps, nullptr, out, staging);
}

afd_status afd_replay(afd_plan plan, const double* signal, int32_t steps, const int32_t* forced_index,
                      afd_result* out) {
  if (!forced_index && steps > 0) return fail(AFD_E_INVALID, "forced_index is NULL");
  static const int32_t none[2] = {0, 0};
  return run(plan, signal, steps, forced_index ? forced_index : none, out);
}

size_t afd_workspace_bytes(const afd_plan_desc* desc) {
  Config cfg;
  if (validate(desc, &cfg) != AFD_OK) return 0;
  return layout_of(cfg).total;
}

void afd_plan_destroy(afd_plan plan) {
  if (!plan) return;
  for (hipEvent_t ev : plan->events) (void)hipEventDestroy(ev);
  if (plan->arena) (void)hipFree(plan->arena);
  if (plan->res) (void)hipFree(plan->res);
  if (plan->forced) (void)hipFree(plan->forced);
  if (plan->aux) (void)hipFree(plan->aux);
  delete plan;
}

const char* afd_status_string(afd_status status) {
  switch (status) {
    case AFD_OK: return "AFD_OK";
    case AFD_E_INVALID: return "AFD_E_INVALID: invalid argument";
    case AFD_E_NONFINITE: return "AFD_E_NONFINITE: non-finite input";
    case AFD_E_NOMEM: return "AFD_E_NOMEM: allocation failed";
    case AFD_E_HIP: return "AFD_E_HIP: HIP runtime error";
    case AFD_E_UNSUPPORTED: return "AFD_E_UNSUPPORTED: unsupported size";
  }
  return "unknown afd_status";
}

const char* afd_last_error(void) { return g_last_error.c_str(); }

afd_status afd_reconstruct(afd_plan plan, const double* a, const double* coef, int32_t steps, const double* signal,
                           double* partial_sum, double* delta) {
  return reconstruct(plan, a, coef, steps, signal, partial_sum, delta);
}

afd_status afd_analytic(afd_plan plan, const double* x, double* g) { return analytic(plan, x, g); }

afd_status afd_plan_set_timing(afd_plan plan, const char* kernel, int32_t enable) {
  if (!plan || !kernel) return fail(AFD_E_INVALID, "plan or kernel is NULL");
  int kind = kTimeNone;
  if (std::strcmp(kernel, "radius") == 0) kind = kTimeRadius;
  else if (std::strcmp(kernel, "fft") == 0) kind = kTimeFft;
  else if (std::strcmp(kernel, "update") == 0) kind = kTimeUpdate;
  else if (std::strcmp(kernel, "rows") == 0) kind = kTimeRows;
  else return fail(AFD_E_INVALID, "unknown kernel class");
  if (enable < 0) return fail(AFD_E_INVALID, "enable must be >= 0");
  plan->time_kind = enable ? kind : kTimeNone;
  plan->time_every = enable > 0 ? enable : 1;
  plan->time_seen = 0;
  plan->time_ms = 0.0;
  plan->time_launches = 0;
  return AFD_OK;
}

afd_status afd_plan_kernel_time(afd_plan plan, double* ms, int64_t* launches) {
  if (!plan || !ms || !launches) return fail(AFD_E_INVALID, "NULL argument");
  *ms = plan->time_ms;
  *launches = plan->time_launches;
  return AFD_OK;
}

afd_status afd_plan_tune(afd_plan plan, const double* signal, int32_t steps, afd_tuning* out) {
  if (!plan) return fail(AFD_E_INVALID, "plan is NULL");
  if (steps < 0) return fail(AFD_E_INVALID, "steps must be >= 0");
  if (steps > 0 && !signal) return fail(AFD_E_INVALID, "signal is NULL");
  const Config& c = plan->cfg;
  // the candidates: every combination of the choices that apply to this plan
  const bool tail_opt = c.adv && c.batch == 1;
  const bool queue_opt =
      c.fp64 && c.adv && c.batch == 1 && c.rpb == 1 && plan->rslots > 0 && plan->rslots < c.nblocks;
  std::vector<int> chunks{c.chunk};
  if (c.big && c.chunk > 1) {
    for (int d : {2, 4})
      if (std::max(1, c.chunk / d) != chunks.back()) chunks.push_back(std::max(1, c.chunk / d));
  }
  std::vector<TuneChoice> cands;
  for (int split = 0; split <= (tail_opt ? 1 : 0); ++split)
    for (int nq = 0; nq <= (queue_opt ? 1 : 0); ++nq)
      for (int ch : chunks) cands.push_back(TuneChoice{split != 0, nq != 0, ch});
  afd_tuning rep{};
  TuneChoice best{plan->split_tail, plan->no_queue, plan->chunk};
  if (steps > 0 && cands.size() > 1) {
    const size_t S = size_t(steps) * size_t(c.batch);
    std::vector<int32_t> idx(2 * S);
    std::vector<double> a(2 * S), coef(2 * S), energy(S + size_t(c.batch));
    afd_result r{};
    r.index = idx.data();
    r.a = a.data();
    r.coef = coef.data();
    r.energy = energy.data();
    double best_ms = 0.0;
    // every candidate must give the first one's results bit for bit
    std::vector<int32_t> idx0;
    std::vector<double> coef0, energy0;
    for (size_t i = 0; i < cands.size(); ++i) {
      plan->split_tail = cands[i].split_tail;
      plan->no_queue = cands[i].no_queue;
      plan->chunk = cands[i].chunk;
      double ms = 0.0;
      for (int rep_i = 0; rep_i < 3; ++rep_i) {  // one warm-up, then the faster of two
        const auto t0 = std::chrono::steady_clock::now();
        const afd_status st = run(plan, signal, steps, nullptr, &r);
        const auto t1 = std::chrono::steady_clock::now();
        if (st != AFD_OK) {
          plan->split_tail = best.split_tail;
          plan->no_queue = best.no_queue;
          plan->chunk = best.chunk;
          return st;
        }
        const double t = std::chrono::duration<double, std::milli>(t1 - t0).count();
        if (rep_i == 1 || (rep_i == 2 && t < ms)) ms = t;
      }
      if (i == 0) {
        rep.ms_default = ms;
        idx0 = idx;
        coef0 = coef;
        energy0 = energy;
      } else if (idx != idx0 || std::memcmp(coef.data(), coef0.data(), 8 * coef.size()) != 0 ||
                 std::memcmp(energy.data(), energy0.data(), 8 * energy.size()) != 0) {
        plan->split_tail = best.split_tail;
        plan->no_queue = best.no_queue;
        plan->chunk = best.chunk;
        return fail(AFD_E_HIP, "a launch choice changed the results");
      }
      if (i == 0 || ms < best_ms) {
        best_ms = ms;
        best = cands[i];
      }
    }
    rep.ms = best_ms;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tune[tune_key(plan)] = best;
    }
  }
  plan->split_tail = best.split_tail;
  plan->no_queue = best.no_queue;
  plan->chunk = best.chunk;
  rep.split_tail = best.split_tail ? 1 : 0;
  rep.no_queue = best.no_queue ? 1 : 0;
  rep.chunk = c.big ? best.chunk : 0;
  rep.candidates = int32_t(cands.size());
  if (out) *out = rep;
  g_last_error.clear();
  return AFD_OK;
}

afd_status afd_plan_radius_launch(afd_plan plan, int64_t* blocks, int32_t* threads, int32_t* lds_bytes) {
  if (!plan || !blocks || !threads || !lds_bytes) return fail(AFD_E_INVALID, "NULL argument");
  const Config& c = plan->cfg;
  if (c.big) {  // the row pass, which carries the selection
    *blocks = int64_t(c.bg.g) * c.M;
    *threads = c.bg.thr_b;
    *lds_bytes = int32_t(c.bg.lds_b);
  } else if (c.pk) {
    const PpGeom tg = pp_geom(c.prime, c.pk);
    *blocks = c.nblocks;
    *threads = tg.threads;
    *lds_bytes = pp_lds_bytes(c.prime, c.pk, c.fp64);
  } else if (c.mixed) {
    *blocks = c.nblocks;
    *threads = c.mg.threads;
    *lds_bytes = mixed_lds_bytes(c.mg, c.fp64);
  } else {
    const bool queued = c.fp64 && c.adv && c.batch == 1 && c.rpb == 1 && plan->rslots > 0 &&
                        plan->rslots < c.nblocks && !plan->no_queue;
    *blocks = queued ? plan->rslots : c.nblocks;
    *threads = radius_threads_of(c.logn, c.fp64);
    *lds_bytes = radius_lds_bytes(c.logn, c.fp64, c.rpb);
  }
  return AFD_OK;
}

}  // extern "C"
