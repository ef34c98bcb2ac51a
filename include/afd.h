/*
 * afd.h -- C ABI of libafd: the FFT-based Core-AFD maximal-selection loop on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Gao, Ku, Qian, "Fast algorithm of adaptive Fourier series"
 * (arXiv 1711.08604).  Given the boundary samples G(z_n), z_n = e^{2 pi i n/N},
 * n = 0..N-1, N = 2^K, of a function in the Hardy space of the unit disc, each
 * step k of Core-AFD (Sec. 2, eqs. (3), (7) and ak; Sec. 3.2, Steps 1-2)
 *
 *   1. evaluates the rectangle-rule inner products <G_k, e_a>~ (Sec. 3.1,
 *      eq. term81) on the polar grid a_{m,j} = r_m e^{2 pi i j/N}, m = 0..M-1,
 *      j = 0..N-1, through one forward DFT of the samples (eq. term4) and one
 *      inverse DFT per radius of the weighted spectrum r_m^l c_l (eq. rcl,
 *      with the constant N = 2^K; the circle measure is dt/2pi);
 *   2. selects the grid point with the largest |<G_k, e_a>~|^2 (ties: lowest
 *      flat index m*N + j);
 *   3. records a_k and the coefficient c_k = <G_k, e_{a_k}>~ and replaces the
 *      remainder by G_{k+1} = (G_k - c_k e_{a_k}) (1 - conj(a_k) z)/(z - a_k)
 *      (eq. (7)), with e_a(z) = sqrt(1-|a|^2)/(1 - conj(a) z);
 *   4. records the remainder energy E_k = (1/N) sum_n |G_{k+1}(z_n)|^2.
 *
 * Every step runs in hand-written HIP kernels on the plan's stream.  All
 * functions are extern "C"; no C++ exception crosses this boundary.
 */
#ifndef AFD_H_
#define AFD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct afd_plan_s* afd_plan; /* opaque; owns its device workspace and tables */
typedef struct afd_graph_s* afd_graph; /* opaque; one decomposition captured as a HIP graph */
typedef struct afd_group_s* afd_group; /* opaque; decompositions of several plans in one graph */

typedef enum {
  AFD_OK = 0,
  AFD_E_INVALID = 1,     /* bad argument (see each function)                        */
  AFD_E_NONFINITE = 2,   /* NaN or Inf in the input samples                          */
  AFD_E_NOMEM = 3,       /* device or host allocation failed                         */
  AFD_E_HIP = 4,         /* a HIP runtime error; afd_last_error() holds its text     */
  AFD_E_UNSUPPORTED = 5  /* valid but outside what this build supports (e.g. N > 2^20) */
} afd_status;

typedef enum {
  /* Every step in IEEE double: forward DFT, per-radius inverse DFTs, |.|^2,
     selection, coefficient (the grid value itself), update and energy.        */
  AFD_FP64 = 0,
  /* Forward and inverse DFTs, |.|^2 and a candidate short-list in IEEE single
     (complex64 data, FP32 accumulation); the short-list (at least recheck_k
     points, plus every point within a relative band of the FP32 maximum) is
     re-evaluated in double by the direct rule of eq. term81 against the double
     remainder, and the winner, coefficient, update and energy are double.    */
  AFD_FP32_RECHECK = 1
} afd_precision;

typedef struct {
  int64_t n;              /* N = 2^K samples, 2 <= N <= 2^20, or N = p^K for p = 3 (K <= 8,
                             N <= 6561), 5 (K <= 6, N <= 15625) or 7 (K <= 4, N <= 2401)
                             (radix-p transforms; the paper's closing remark extends the fast
                             algorithm to N = p^K), or a mixed radix N = 2^a 3^b 5^c 7^d <= 16384
                             with several of these primes, their product at most 30 (2*3, 2*5,
                             2*7, 3*5, 3*7, 2*3*5), and N/E <= 1024 threads (512 from E = 18),
                             E the values per thread (a multiple of that product, E <= 30);
                             e.g. 1000, 1536, 6000, 12288, 15360                                */
  int32_t m;              /* M >= 1 radii; M * N must be < 2^32 - 1 (flat grid indices m N + j
                             are unsigned 32-bit)                                              */
  const double* radii;    /* host pointer, length M, each in [0, 1); any order; copied at
                             create.  Grid index m refers to position m of this array.        */
  afd_precision precision;
  int32_t recheck_k;      /* FP32 mode: minimum short-list length, 1..64 (0 -> 8)              */
  int32_t first_a_zero;   /* 1: step 1 takes a_1 = 0 (the grid point (m0, 0) of the first
                             radius equal to 0) instead of the maximum; requires such a radius */
  double recheck_band;    /* FP32 mode: relative band below the FP32 maximum whose points are
                             all re-checked in double, in [0, 1e-4] (0 -> the default: 4e-6
                             up to N = 2^14, then growing by 2^(1/3) per doubling of N to
                             1.6e-5 at 2^20, about eight times the largest FP32 error of
                             |.|^2 measured at those sizes); the short-list holds at most 256
                             points (flags bit 0 reports a cut)                              */
  int32_t batch;          /* signals per call, 1..65535 (0 -> 1): independent decompositions of
                             signals with this N and these radii, run together (every kernel
                             of a step covers all of them).  batch > 1 needs N <= 2^14.        */
  int32_t concurrent;     /* 1: the plan's stream runs beside other streams' kernels on the
                             device (a server).  For one signal with 2^10 <= N <= 2^14 the step
                             tail then runs as three launches instead of one launch whose grid
                             barriers need every workgroup of the launch resident at once.
                             Results are the same bit for bit.  0: the stream has the device's
                             resources to itself while the plan runs.                          */
  /* Non-uniform samples (Sec. 3.2, the remark after Step 2).  NULL: the signal holds the N
     uniform samples G(e^{2 pi i n/N}).  Otherwise the signal holds `samples` values G(z_n) at
     z_n = e^{2 pi i t_n}, t_n = sample_turns[n] (host pointer, length `samples`, finite,
     strictly increasing, in [0, 1); copied at create), and the inner product becomes the
     quadrature sum_n w_n G(z_n) conj(F(z_n)) with w_n = sample_weights[n] (host pointer,
     finite; NULL: the periodic trapezoidal weights (t_{n+1} - t_{n-1})/2).  The selection grid
     stays a_{m,j} = r_m e^{2 pi i j/N}; the DFT of the samples becomes the non-uniform DFT
     c_l = sum_n w_n G(z_n) e^{-2 pi i l t_n}, l < N.  A batch shares the positions and
     weights (each signal holds `samples` values).  Needs N = 2^K <= 2^14,
     1 <= samples <= 2^16 and radii whose kernel series r^l is negligible from l = 2^18 on (the
     significant length of the uniform path's radius tables); else AFD_E_UNSUPPORTED.  The
     non-uniform DFT computes the K N modes (K a power of two) the longest series needs, and a
     radius whose series outlasts N terms is transformed from its folded spectrum
     sum_k r^(kN) c_(l+kN).  The remainder then has `samples` values; afd_reconstruct gives the
     partial sums at the sample points and the relative errors in the quadrature norm;
     afd_analytic returns AFD_E_UNSUPPORTED.                                                 */
  const double* sample_turns;
  const double* sample_weights; /* NULL: trapezoidal weights; ignored without sample_turns    */
  int64_t samples;              /* number of non-uniform samples (0 with sample_turns NULL)   */
} afd_plan_desc;

/* Per-decomposition outputs.  Caller-owned; each pointer may be host memory
   or device memory of the plan's device (detected per pointer).  Layouts are
   for one signal; with batch B every array holds B of them back to back
   (signal-major: e.g. index is [B][steps][2], energy [B][steps+1]).        */
typedef struct {
  int32_t* index;         /* 2*steps: (m_k, j_k) per step                          [required] */
  double* a;              /* 2*steps: a_k as interleaved (re, im)                  [required] */
  double* coef;           /* 2*steps: c_k = <G_k, e_{a_k}>~, interleaved (re, im)  [required] */
  double* energy;         /* steps+1: E_0 = ||G||_N^2, E_k = ||G_{k+1}||_N^2       [required] */
  double* margin;         /* steps: (P1 - P2)/P1, P1 >= P2 the two largest |.|^2 seen by the
                             selection (FP64: the whole grid; FP32: the re-checked short-list);
                             NaN for forced steps                                   [nullable] */
  double* remainder;      /* 2*N: final remainder G_{steps+1}, interleaved          [nullable] */
  int32_t* recheck_count; /* steps: short-list length re-checked in double (FP64: 0) [nullable] */
  int32_t* flags;         /* steps: bit 0 = the band held more points than could be
                             re-checked; bit 1 = some radius held more band points than
                             its per-radius list; bit 2 = an exact fallback path of the
                             selection ran (flat or exactly tied values, e.g. r = 0) [nullable] */
  double* fp32_error;     /* steps: FP32 mode, max |P32 - P64| / P64max over the re-checked
                             points (P = |<G_k, e_a>~|^2; P64 by the double direct rule); the
                             measured error of the FP32 bulk against double.  FP64: 0 [nullable] */
  /* Written by afd_replay only (afd_decompose leaves them untouched): what the
     step's own selection chose on the replayed remainder G_k before the forced
     point replaced it.                                                          */
  int32_t* pick_index;    /* 2*steps: (m, j) of the selection's choice             [nullable] */
  double* pick_p;         /* steps: its |<G_k, e_a>~|^2 (FP64: the FFT-form grid value the
                             selection compared; FP32: the double re-check)        [nullable] */
  double* pick_margin;    /* steps: the selection's margin, as `margin` in afd_decompose
                                                                                   [nullable] */
  int32_t* pick_flags;    /* steps: bits 0-2 as `flags`; bit 4: FP32 mode, the forced point
                             was on the short-list that was re-checked in double   [nullable] */
} afd_result;

/* Validate `desc`, copy the radii, build the per-radius double-precision
   tables and allocate the device workspace on the current HIP device.
   `hip_stream` is a hipStream_t (NULL = the default stream) on which every
   later call of this plan runs.  On success *out receives the plan.
   Errors: AFD_E_INVALID (null pointer, N < 2 or with a prime factor above 7,
   M < 1,
   M*N >= 2^32 - 1, a radius outside [0,1) or non-finite, recheck_k or
   recheck_band out of range, first_a_zero without a zero radius, batch < 0
   or batch * N * M too large), AFD_E_UNSUPPORTED (N > 2^20, N = 3^K with
   K > 8, 5^K with K > 6, 7^K with K > 4, a mixed-radix N outside the
   sizes above, or batch > 1 with N > 2^14), AFD_E_NOMEM, AFD_E_HIP.  On error *out is
   set to NULL and nothing is left allocated. */
afd_status afd_plan_create(const afd_plan_desc* desc, void* hip_stream, afd_plan* out);

/* Run `steps` >= 0 steps of the maximal-selection loop on `signal` (2*N
   doubles, interleaved complex128, host or device; B*2*N for a plan with
   batch B, signal b at offset 2*N*b) and write `out`.
   Synchronous: returns after the results are in `out`.  The plan's device
   state is overwritten; `signal` is only read.  Errors: AFD_E_INVALID (null
   plan/signal/out or a required out field, steps < 0), AFD_E_NONFINITE,
   AFD_E_HIP.  Validation happens before any device work; on error `out` is
   untouched.  An all-zero remainder selects flat index 0 with c_k = 0 and
   the loop continues. */
afd_status afd_decompose(afd_plan plan, const double* signal, int32_t steps, afd_result* out);

/* One whole decomposition of `steps` steps (as afd_decompose) captured into
   a HIP graph, for callers that repeat decompositions of one shape and want
   them submitted as one unit (the per-launch host work and the host waits of
   afd_decompose are gone).  `signal` and every non-null array of `out` must
   be device memory of the plan's device; they are baked into the graph (to
   decompose another signal, write it into the same buffer), as is the plan's
   workspace: the graph and the plan's other calls must not run concurrently.
   `out` is copied.  Each afd_graph_launch enqueues one replay on the plan's
   stream and returns at once; the results are in `out` when the stream has
   reached them.  Counters are cleared by a kernel at the start of every
   replay.  Errors: AFD_E_INVALID (NULL, steps < 0, a required out field
   missing, a host pointer), AFD_E_NOMEM, AFD_E_HIP (capture or instantiation
   failed).  Non-finite samples are not reported by the launch: see
   afd_graph_status. */
afd_status afd_graph_create(afd_plan plan, const double* signal, int32_t steps, const afd_result* out,
                            afd_graph* graph);
afd_status afd_graph_launch(afd_graph graph);
/* Waits for the plan's stream; AFD_E_NONFINITE if the last replay's signal
   held NaN or Inf (its outputs are then meaningless), AFD_E_HIP if a grid
   barrier of the step tail timed out, else AFD_OK. */
afd_status afd_graph_status(afd_graph graph);
/* NULL-safe.  Destroy graphs before their plan. */
void afd_graph_destroy(afd_graph graph);

/* Batches of uneven N: one decomposition of each of `count` >= 1 distinct
   plans of one device, each with its own N (2^K, p^K, mixed radix or non-uniform), radii,
   precision and batch, captured together into one HIP graph with one branch
   per plan; the branches run concurrently on the device, and
   afd_group_launch submits all of them with one graph launch on the stream
   of plans[0].  signals[i], steps[i] and outs[i] are plans[i]'s, with the
   requirements of afd_graph_create (device memory, baked in, `outs` copied).
   Each plan's step tail takes its three-launch form (as with
   afd_plan_desc.concurrent), so that no branch depends on having the device
   to itself; results equal each plan's afd_decompose bit for bit.  The plans
   must not run other calls while a launch of the group is in flight.
   Errors: AFD_E_INVALID (NULL, count < 1, a plan twice, plans of different
   devices, and afd_graph_create's), AFD_E_NOMEM, AFD_E_HIP. */
afd_status afd_group_create(const afd_plan* plans, int32_t count, const double* const* signals,
                            const int32_t* steps, const afd_result* outs, afd_group* group);
afd_status afd_group_launch(afd_group group);
/* Waits for the last launch; the first member (in plans order) whose signal
   held NaN or Inf gives AFD_E_NONFINITE (that member's outputs are
   meaningless, the others' are valid), else AFD_OK. */
afd_status afd_group_status(afd_group group);
/* NULL-safe.  Destroy groups before their plans. */
void afd_group_destroy(afd_group group);

/* Launch choices of a plan that leave its results unchanged bit for bit:
   the step tail in one launch with grid barriers or in three launches
   (2^10 <= N <= 2^14, one signal), the double-precision radius kernel's work
   queue on or off, and the radii per two-pass chunk (N > 2^14: the
   allocated chunk, or a half or a quarter of it).                          */
typedef struct {
  int32_t split_tail;    /* 1: the three-launch step tail                        */
  int32_t no_queue;      /* 1: no work queue in the radius kernel                */
  int32_t chunk;         /* radii per two-pass chunk (0 for N <= 2^14)           */
  int32_t candidates;    /* combinations that apply to the plan (timed if > 1)   */
  double ms;             /* chosen combination: ms per decomposition (0: untimed) */
  double ms_default;     /* the default combination's ms (0: untimed)            */
} afd_tuning;

/* Autotuner: decomposes `steps` steps of `signal` (as afd_decompose takes it)
   with every combination of the choices above that applies to the plan (one
   warm-up and the faster of two timed runs each), keeps the fastest in the
   plan and in a per-process table from which plans created later with the
   same device, N, samples, M, precision and batch start.  steps = 0 times
   nothing and reports the plan's current choices.  *out (nullable) receives
   the choices.  Errors: those of afd_decompose; on error the plan keeps its
   previous choices. */
afd_status afd_plan_tune(afd_plan plan, const double* signal, int32_t steps, afd_tuning* out);

/* For callers that cannot allocate device memory (code under stream capture,
   tight serving loops, harnesses that forbid allocation): afd_decompose
   without any allocation in the call.  afd_decompose stages its results in
   device memory the plan allocates on the first call (and again when `steps`
   grows); this entry point stages them in a static device array of 512 KiB
   instead, one per device, held until the process ends (the plan's workspace
   was allocated by afd_plan_create).  Limit: the staging takes about
   (100 steps + 8) bytes per signal and must fit in 512 KiB (for one signal,
   up to about 5200 steps); larger requests return AFD_E_INVALID before any
   device work.  Every call on a device shares that
   device's array and nothing in it needs to start at zero (each staged value
   is written by the call's kernels before it is read), but calls that
   overlap in time on one device (other threads or streams) race: serialise
   them.  Timing (afd_plan_set_timing) is not collected by these calls.
   Results equal afd_decompose's bit for bit.  Errors as afd_decompose, plus
   AFD_E_INVALID for too many steps. */
afd_status afd_decompose_noalloc(afd_plan plan, const double* signal, int32_t steps, afd_result* out);

/* As afd_decompose, but step k continues from the grid point forced_index[2k],
   forced_index[2k+1] (host or device, 2*steps int32) instead of the selected
   one.  Every step still runs the whole path on the replayed remainder G_k:
   the forward DFT, the per-radius inverse DFTs, |.|^2, the selection and (FP32
   mode) the double re-check of the short-list; the choice it makes goes to
   pick_index / pick_p / pick_margin / pick_flags.  The forced point then takes
   its place: c_k is the FFT-form grid value there from the same radius
   transforms (FP64 mode; so with the indices afd_decompose chose, the results
   equal afd_decompose's bit for bit) or its double direct-rule value (eq.
   term81; FP32 mode), and the update uses it.  `margin` is NaN.  Used to
   compare every step of the path with a reference trajectory past near-ties.
   first_a_zero does not apply (the forced indices cover every step).  With
   batch B, forced_index is [B][steps][2].  Errors as afd_decompose, plus
   AFD_E_INVALID for an index outside [0,M) x [0,N). */
afd_status afd_replay(afd_plan plan, const double* signal, int32_t steps,
                      const int32_t* forced_index, afd_result* out);

/* Device bytes a plan with this description allocates (tables + workspace);
   0 if `desc` is invalid.  For admission control. */
size_t afd_workspace_bytes(const afd_plan_desc* desc);

/* Release the plan and its device memory.  NULL-safe. */
void afd_plan_destroy(afd_plan plan);

/* Static text for a status code. */
const char* afd_status_string(afd_status status);

/* Detail of the last error on the calling thread ("" if none). */
const char* afd_last_error(void);

/* Partial sum of a decomposition on the circle and its relative errors
   (Sec. 2, expansion (Sn), with the Takenaka-Malmquist system of eq. (2);
   Sec. 4, eq. er).  With n = steps, at the plan's N points
   z_j = e^{2 pi i j/N}:
     S_n(z) = sum_{k<n} c_k B_k(z),
     B_k(z) = sqrt(1 - |a_k|^2)/(1 - conj(a_k) z) * prod_{l<k} (z - a_l)/(1 - conj(a_l) z),
     delta_k = ||G - S_k||_N^2 / ||G||_N^2, k = 1..n (NaN where ||G||_N = 0).
   a, coef: 2*steps doubles each, interleaved complex as afd_decompose writes
   them ([B][steps][2] for a plan with batch B), host or device, copied at
   the call.  signal: 2*N doubles (B*2*N), host or device; required for
   delta, else nullable.  partial_sum: 2*N doubles out (B*2*N), nullable.
   delta: steps doubles out (B*steps), nullable.  In double precision on the
   plan's stream; synchronous.  Errors: AFD_E_INVALID (null plan, steps < 0,
   a or coef NULL with steps > 0, delta without signal, some |a_k| >= 1),
   AFD_E_NONFINITE (NaN or Inf in a, coef or signal), AFD_E_NOMEM, AFD_E_HIP.
   Validation happens before any device work; on error the outputs are
   untouched. */
afd_status afd_reconstruct(afd_plan plan, const double* a, const double* coef, int32_t steps,
                           const double* signal, double* partial_sum, double* delta);

/* Analytic (H^2) part of N boundary samples, the front end that brings a
   real signal into the Hardy space before the decomposition (Sec. 4,
   case 2): g = IDFT(h . DFT(x)) with h_0 = 1, h_l = 2 for 0 < l < N/2,
   h_{N/2} = 1, h_l = 0 for N/2 < l < N (N = 2: h = (1, 1)).  For real x,
   Re g = x.  x, g: 2*N doubles (B*2*N), interleaved complex, host or
   device; they may alias.  Two double-precision forward DFTs on the plan's
   stream (IDFT(y) = conj(DFT(conj(y)))/N); synchronous.  Errors:
   AFD_E_INVALID (NULL), AFD_E_NONFINITE (NaN or Inf in x), AFD_E_NOMEM,
   AFD_E_HIP, AFD_E_UNSUPPORTED (a plan whose N is not 2^K); on error g is
   untouched. */
afd_status afd_analytic(afd_plan plan, const double* x, double* g);

/* Per-kernel timing with HIP events that the dispatches of the kernel class
   `kernel` stamp on the plan's stream ("radius": the fused weighted
   inverse-DFT / |.|^2 / selection kernel, or both passes of a step at
   N > 2^14; "fft": the forward DFT; "update": the remainder update, which
   for 2^10 <= N <= 2^14 is the fused step tail; "rows": N > 2^14, each row
   pass launch of the radius transforms, one per chunk of radii).  enable = n >= 1 starts
   accumulating (and clears the totals) over every n-th launch of the class
   (1: every launch; a stamped dispatch costs a few microseconds, so a
   benchmark samples); 0 stops.  Errors: AFD_E_INVALID for an unknown class
   or enable < 0. */
afd_status afd_plan_set_timing(afd_plan plan, const char* kernel, int32_t enable);

/* Accumulated milliseconds and launch count of the timed kernel class since
   timing was enabled.  Errors: AFD_E_INVALID. */
afd_status afd_plan_kernel_time(afd_plan plan, double* ms, int64_t* launches);

/* Launch geometry of the radius kernel of this plan: grid blocks, threads
   per block, dynamic LDS bytes per block.  Errors: AFD_E_INVALID. */
afd_status afd_plan_radius_launch(afd_plan plan, int64_t* blocks, int32_t* threads, int32_t* lds_bytes);

#ifdef __cplusplus
}
#endif

#endif /* AFD_H_ */
