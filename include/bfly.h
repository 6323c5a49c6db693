/*
 * bfly.h -- C ABI of the MI355X butterfly library (libbfly.so).
 *
 * The library applies the butterfly algorithm of Poulson, Demanet, Maxwell &
 * Ying, "A Parallel Butterfly Algorithm", to kernels K(x, y) = exp(i Phi(x, y))
 * with a smooth real phase Phi (Sec. 1.4, Eq. (6)), using analytic
 * tensor-product Chebyshev interpolation (Sec. 1.4 "Avoiding quadratic
 * precomputation"):
 *
 *   f(x) ~= sum_y exp(i Phi(x, y)) g(y)            (Sec. 1, Eq. 1 over all boxes)
 *
 * evaluated in O(r^2 N^d log N) work (Sec. 1) on one GPU.  The steps are the
 * sequential algorithm's (Alg. "alg:serial"): leaf initialisation, log2 N
 * merge-and-split stages (Sec. 1.1) with the column-to-row "middle switch"
 * at stage floor(log2 N / 2), and final evaluation at the targets.
 *
 * Conventions (all entry points)
 * ------------------------------
 *  - Phi = 2 pi tau; the phase ids below define tau, the phase in turns.
 *  - Points are row-major FP64 [n][d] arrays in DEVICE memory, any order.
 *  - Values are complex128 (interleaved re, im doubles) in DEVICE memory;
 *    right-hand side k of g starts at g + 2*k*ldg doubles (ldg >= n_src).
 *    Input and output are complex128 in every precision mode.
 *  - The caller owns every device buffer, including the workspace.  No entry
 *    point allocates device memory, and apply calls never synchronise: all
 *    work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *    Buffers must stay valid until that work completes.
 *  - Errors are return codes; nothing is thrown.  Argument validation happens
 *    on the host, before any HIP call, so invalid arguments never reach the
 *    GPU.  A device error from earlier asynchronous work is reported as
 *    BFLY_EDEVICE by the next call.  bfly_last_error() returns a
 *    thread-local message describing the last failure.
 *  - Points outside the plan's boxes are clamped into the nearest leaf box;
 *    NaN coordinates go to leaf 0.  Accuracy degrades gracefully there.
 *  - The plan does not check the butterfly condition (Sec. 1: diam(A)
 *    diam(B) <= D for every interacting pair); choosing N for the boxes and
 *    phase is the caller's job.
 *  - Plans are immutable and hold no device memory; one plan may be used
 *    concurrently on several streams with distinct workspaces.
 */
#ifndef BFLY_H
#define BFLY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfly_plan_s* bfly_plan_t;

/* status codes */
enum {
  BFLY_OK = 0,
  BFLY_EINVAL = 1,       /* an argument is out of range or NULL                */
  BFLY_EUNSUPPORTED = 2, /* valid, but not supported (e.g. phase id for this d) */
  BFLY_ENOMEM = 3,       /* host allocation failed                              */
  BFLY_EDEVICE = 4,      /* a HIP call or earlier device work failed            */
  BFLY_EWORKSPACE = 5    /* workspace missing or smaller than required          */
};

/* phase ids (tau = Phi / 2 pi; N is the plan's N)
 *  FOURIER      tau = x . y                                  any d  (Sec. 3)
 *  HYPRADON2    tau = N x0 sqrt(y0^2 + x1^2 y1^2)            d = 2  (Sec. 3.1 family)
 *  GENRADON3    tau = N (x.y + sqrt(g0^2 y0^2 + g1^2 y1^2 + y2^2)),
 *               g0 = (2 + sin 2pi x0 sin 2pi x1)/3,
 *               g1 = (2 + cos 2pi x0 cos 2pi x1)/3           d = 3  (Sec. 3.2 family)
 *  SEPARABLE_TEST tau = N (sum_j x_j^2 + sum_j y_j^3)        any d  (rank-one kernel:
 *               the butterfly is exact, used to check results at any size)
 *  GENRADON3_PI tau = (x.p + sqrt(gamma^2 + kappa^2)) / 2, gamma = p0 g0(x),
 *               kappa = p1 g1(x) with g0, g1 as above: the Sec. 3.2 phase as
 *               printed, Phi = pi (...), no N inside (the scale comes from the
 *               source box, e.g. p in [-N/2, N/2)^3)          d = 3 */
enum {
  BFLY_PHASE_FOURIER = 0,
  BFLY_PHASE_HYPRADON2 = 1,
  BFLY_PHASE_GENRADON3 = 2,
  BFLY_PHASE_SEPARABLE_TEST = 3,
  BFLY_PHASE_GENRADON3_PI = 4
};

/* precision modes (internal arithmetic; I/O is always complex128)
 *  FP64     everything in FP64 (the paper computes in double precision, Sec. 3).
 *  FP32     phase tau and its reduction modulo 1 in FP64, then FP32
 *           sine/cosine, FP32 weights and FP32 contractions.
 *  SPLIT32  hi/lo pairs of FP32 values with error-free accumulation: NOT
 *           implemented.  Every entry point that takes a precision returns
 *           BFLY_EUNSUPPORTED for it.  On gfx950 an FP64 multiply-add costs
 *           about twice an FP32 one (measured 58.7 against 112 TFLOP/s),
 *           while a double-float multiply-add takes 18 FP32 instructions
 *           (measured 7.3x slower than an FP64 multiply-add), so the FP64
 *           mode gives near-FP64 results faster. */
enum { BFLY_FP64 = 0, BFLY_FP32 = 1, BFLY_SPLIT32 = 2 };

/* Create a plan.
 *  d        1, 2 or 3
 *  N        leaf boxes per dimension, a power of two, 1 <= N, N^d < 2^31
 *  src_lo/src_hi  host double[d]: source box Y = prod [lo, hi), hi > lo, finite
 *  tgt_lo/tgt_hi  host double[d]: target box X
 *  phase_id one of BFLY_PHASE_*, valid for d
 *  q        Chebyshev nodes per dimension (rank r = q^d):
 *           d = 1: 2..16, d = 2: 2..12, d = 3: 2..5
 *  out      receives the plan (host object; no device memory, no HIP call)
 * Returns BFLY_OK, BFLY_EINVAL, BFLY_EUNSUPPORTED or BFLY_ENOMEM. */
int bfly_plan(int d, int64_t N, const double* src_lo, const double* src_hi,
              const double* tgt_lo, const double* tgt_hi, int phase_id, int q,
              bfly_plan_t* out);

/* Destroy a plan (NULL is accepted).  Returns BFLY_OK. */
int bfly_plan_destroy(bfly_plan_t plan);

/* Query a plan: out[0..4] = d, N, q, r = q^d, switch level floor(log2 N / 2)
 * of the forward apply (the adjoint switches at log2 N minus that).
 * Returns BFLY_OK or BFLY_EINVAL. */
int bfly_plan_info(bfly_plan_t plan, int64_t* out5);

/* Device workspace, in bytes, needed by one apply (forward or adjoint) with
 * n_in input points, nrhs right-hand sides and precision prec.  n_in is
 * n_src for bfly_apply and n_tgt for bfly_apply_adjoint.  A host
 * computation only: no HIP call, no allocation.
 * Returns BFLY_OK or BFLY_EINVAL. */
int bfly_workspace_size(bfly_plan_t plan, int64_t n_in, int nrhs, int prec, size_t* bytes);

/* Forward apply f = B g  (B ~= K restricted to the points).
 *  n_src, y   sources, device double[n_src][d]            (n_src >= 0)
 *  g, ldg     device complex128 [nrhs][ldg], ldg >= n_src
 *  n_tgt, x   targets, device double[n_tgt][d]            (n_tgt >= 0)
 *  f, ldf     device complex128 [nrhs][ldf], ldf >= n_tgt; entries
 *             [k][0..n_tgt) are overwritten, in the caller's target order
 *  nrhs       1 .. 4096
 *  prec       BFLY_FP64 or BFLY_FP32
 *  ws         device workspace of ws_bytes >= bfly_workspace_size(plan, n_src, nrhs, prec)
 *  stream     hipStream_t (NULL = default stream)
 * f must not alias g, x, y or ws.
 * Returns BFLY_OK, BFLY_EINVAL, BFLY_EWORKSPACE or BFLY_EDEVICE. */
int bfly_apply(bfly_plan_t plan,
               int64_t n_src, const double* y, const void* g, int64_t ldg,
               int64_t n_tgt, const double* x, void* f, int64_t ldf,
               int nrhs, int prec, void* ws, size_t ws_bytes, void* stream);

/* Forward apply without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * bfly_apply; the workspace is a device array inside the library, one copy
 * per GPU, of BFLY_NOALLOC_MAX_BYTES bytes, held from the library's load on
 * that GPU to the end of the process.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); its first call on a
 * device looks up that device's copy (hipGetSymbolAddress).
 * Limits and sharing:
 *  - an apply whose bfly_workspace_size(plan, n_src, nrhs, prec) exceeds
 *    BFLY_NOALLOC_MAX_BYTES returns BFLY_EWORKSPACE before any HIP call
 *    (e.g. 2-D, q = 5, one right-hand side: N = 256 fits in FP64 and FP32,
 *    N = 1024 does not);
 *  - every call on one GPU uses that GPU's one array: calls that overlap in
 *    time on one GPU (several streams or host threads) race and give wrong
 *    results; calls in one stream's order are safe.  Nothing in the array
 *    needs to start at zero, so the previous call's contents do no harm.
 * Returns BFLY_OK, BFLY_EINVAL, BFLY_EWORKSPACE or BFLY_EDEVICE. */
#define BFLY_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int bfly_apply_noalloc(bfly_plan_t plan,
                       int64_t n_src, const double* y, const void* g, int64_t ldg,
                       int64_t n_tgt, const double* x, void* f, int64_t ldf,
                       int nrhs, int prec, void* stream);

/* Adjoint apply g_out = B' f_in, where B' is the butterfly for the adjoint
 * kernel K^H(y, x) = exp(-i Phi(x, y)): the same steps with the roles of
 * the two point sets swapped and the phase negated (Sec. 1: the low-rank
 * condition is symmetric in diam(A) diam(B)).  B' approximates K^H to the
 * same accuracy.  Its middle switch sits at level L - floor(L/2), the mirror
 * of the forward apply's floor(L/2) (Sec. 1.4), so each of its steps is the
 * transpose of a step of B and B' = B^H exactly (up to rounding): gradients
 * through B computed with B' are exact for the computed forward.
 *  n_tgt, x       the plan's targets (now the inputs), device double[n_tgt][d]
 *  f_in, ldf      device complex128 [nrhs][ldf], ldf >= n_tgt
 *  n_src, y       the plan's sources (now the outputs), device double[n_src][d]
 *  g_out, ldg     device complex128 [nrhs][ldg], ldg >= n_src, overwritten
 *  ws             ws_bytes >= bfly_workspace_size(plan, n_tgt, nrhs, prec)
 * Other arguments and returns as bfly_apply. */
int bfly_apply_adjoint(bfly_plan_t plan,
                       int64_t n_tgt, const double* x, const void* f_in, int64_t ldf,
                       int64_t n_src, const double* y, void* g_out, int64_t ldg,
                       int nrhs, int prec, void* ws, size_t ws_bytes, void* stream);

/* One instance of a batched apply (bfly_apply_batched): a forward apply
 * (adjoint = 0: inputs g at the plan's sources, outputs f at its targets) or
 * an adjoint apply (adjoint = 1: inputs f at the targets, outputs g at the
 * sources), with the sizes, layouts and ownership of bfly_apply /
 * bfly_apply_adjoint:
 *  plan               any plan; instances may use different plans
 *  nrhs               1 .. 4096
 *  n_in, pts_in       input points, device double[n_in][d]
 *  in, ld_in          device complex128 [nrhs][ld_in], ld_in >= n_in
 *  n_out, pts_out     output points, device double[n_out][d]
 *  out, ld_out        device complex128 [nrhs][ld_out], ld_out >= n_out,
 *                     overwritten; must not alias any other buffer of the batch */
typedef struct {
  bfly_plan_t plan;
  int adjoint;
  int nrhs;
  int64_t n_in;
  const double* pts_in;
  const void* in;
  int64_t ld_in;
  int64_t n_out;
  const double* pts_out;
  void* out;
  int64_t ld_out;
} bfly_batch_item;

/* Device workspace, in bytes, for bfly_apply_batched on these n_items
 * (host array) in precision prec.  Returns BFLY_OK, BFLY_EINVAL or
 * BFLY_EDEVICE. */
int bfly_batch_workspace_size(int n_items, const bfly_batch_item* items, int prec, size_t* bytes);

/* Many applies at once, batched across instances: every instance gives the
 * result bfly_apply or
 * bfly_apply_adjoint would give it, bit for bit, but the instances are
 * binned in one sort and their level stages run level-synchronously, one
 * launch per step for all instances that share d, q, phase and direction,
 * so small instances share the GPU.  The call enqueues kernels only (no
 * allocation, no synchronisation, no host-to-device copy, no memset), so it
 * may be captured in a HIP graph; a captured call reads its descriptors of
 * pointers and sizes as they were at capture time.
 *  n_items    1 .. 4096 instances (host array `items`)
 *  prec       BFLY_FP64 or BFLY_FP32 for all of them
 *  ws         ws_bytes >= bfly_batch_workspace_size(n_items, items, prec),
 *             256-byte aligned
 * Limits: total input points below 2^31, total leaves (sum of N^d) at most
 * 2^31.  Returns BFLY_OK, BFLY_EINVAL, BFLY_EWORKSPACE or BFLY_EDEVICE. */
int bfly_apply_batched(int n_items, const bfly_batch_item* items, int prec, void* ws, size_t ws_bytes,
                       void* stream);

/* Autotune the launch shapes of one apply: the stages each launch fuses
 * (every cover of each half of the algorithm by launches the LDS can hold),
 * the fusion units per workgroup of the column-space and row-space launches,
 * and whether right-hand sides share phase factors in chunks.  The apply runs
 * repeatedly on the caller's buffers with candidate shapes, each timed with
 * HIP events on `stream` (the call synchronises the stream, so it cannot be
 * captured in a graph); a candidate replaces the best only when 0.5% faster.
 * The fastest is recorded for (device, d, q, N, nrhs, prec, phase id,
 * direction), and every later apply with that key uses it (also inside
 * graphs and batched applies).  Every candidate computes the same result bit
 * for bit; on return the outputs hold the apply with the chosen shapes.
 * With BFLY_TUNE_CACHE naming a file, records are read from it at the first
 * apply and the table is written to it after each tuning; the environment
 * overrides BFLY_UB, BFLY_KFUSE, BFLY_LDS, BFLY_KSPLIT take precedence over
 * recorded shapes.  For debugging, BFLY_STOP_STAGES=n makes every single
 * apply of the process stop after the level launches that end within its
 * first n merge-and-split stages, without the final evaluation (the outputs
 * are not written): the start of the workspace then holds that level's
 * weights.
 *  adjoint              0: the arguments of bfly_apply (inputs g at the
 *                       sources, outputs f at the targets); 1: those of
 *                       bfly_apply_adjoint (inputs at the targets)
 *  n_in .. ld_out, nrhs, prec, ws, ws_bytes, stream   as bfly_apply
 *  max_ms               stop trying candidates after this much GPU time
 *                       (>= 0; 0: try all)
 *  best_ms              (host, may be NULL) the chosen shapes' ms per apply
 * Returns BFLY_OK, BFLY_EINVAL, BFLY_EWORKSPACE or BFLY_EDEVICE. */
int bfly_tune(bfly_plan_t plan, int adjoint, int64_t n_in, const double* pts_in, const void* in, int64_t ld_in,
              int64_t n_out, const double* pts_out, void* out, int64_t ld_out, int nrhs, int prec, void* ws,
              size_t ws_bytes, double max_ms, double* best_ms, void* stream);

/* Forget every tuned record of this process; with BFLY_TUNE_CACHE set, the
 * next apply reads the file's records again.  Returns BFLY_OK. */
int bfly_tune_reset(void);

/* Per-step timing, for profiling.  While enabled, every apply records a HIP
 * event pair around each kernel launch on its stream (a few microseconds of
 * overhead per launch).  bfly_timing_read waits for the recorded events and
 * writes, per launch kind, the accumulated milliseconds, the number of
 * launches and the work those launches performed (merge-and-split stages,
 * leaf initialisations, middle switches) since the previous read, then
 * resets the counts.  Launch kinds (BFLY_STEP_*):
 *   0 binning (leaf keys, sort, CSR offsets)
 *   1 column-space launches: leaf initialisation, first-half stages, switch
 *   2 row-space launches: second-half stages
 *   3 final evaluation
 * All five arrays are host arrays of BFLY_NUM_STEPS entries.  The timing
 * state is process-wide; do not enable it while several threads apply.
 * Returns BFLY_OK, BFLY_EINVAL or BFLY_EDEVICE. */
enum { BFLY_NUM_STEPS = 4 };
int bfly_timing_enable(int on);
int bfly_timing_read(double* ms, int64_t* launches, int64_t* stages, int64_t* inits, int64_t* switches);

/* The launches that the last bfly_timing_read collected, one record each in
 * launch order: kind (BFLY_STEP_*), merge-and-split stages, leaf
 * initialisations and middle switches it performed, and its milliseconds.
 * Writes min(cap, total) records into the host arrays (each of cap entries)
 * and the total into *count.  Returns BFLY_OK or BFLY_EINVAL. */
int bfly_timing_launches(int cap, int* count, int* kind, int* stages, int* inits, int* switches, double* ms);

/* Phase-factor throughput, for the roofline accounting of an apply: each of
 * n_threads threads evaluates `iters` factors exp(2 pi i tau) with the
 * reduction and sine/cosine that the apply's kernels use in precision prec
 * (BFLY_FP64 or BFLY_FP32), at arguments spread over [0, span) turns, and
 * writes the sum of its factors to out[thread] (device complex128
 * [n_threads]).  The paper evaluates these factors in batches and they are
 * the bulk of the work (Sec. 3); timing this call (events around it on
 * `stream`) gives the cost of one factor.  Besides each factor the kernel
 * does three FP64 additions per factor (argument step and the sum).
 *  n_threads  1 .. 2^30;  iters  a positive multiple of 8;  0 <= span < 1e15
 * Enqueues one kernel; no allocation.  Returns BFLY_OK, BFLY_EINVAL or
 * BFLY_EDEVICE. */
int bfly_phase_rate(int prec, int64_t n_threads, int64_t iters, double span, void* out, void* stream);

/* FP32 multiply-add throughput of the two contraction units, for the choice
 * between them: unit 0 runs 32 independent v_fma_f32 chains per lane (VALU),
 * unit 1 eight independent v_mfma_f32_4x4x1_16b_f32 chains per wave (matrix
 * cores: 16 blocks of 4 x 4 x 1, 256 multiply-adds per instruction), unit 2
 * both in one instruction stream (per iteration 8 matrix instructions and
 * 32 vector multiply-adds per lane).  Each of n_threads threads (a multiple
 * of 64) runs `iters` iterations and writes one sum to out[thread] (device
 * float [n_threads]).  Per iteration a wave does 32 x 64 (unit 0), 8 x 256
 * (unit 1) or both (unit 2) multiply-adds.  Time the call with events on
 * `stream`.  Returns BFLY_OK, BFLY_EINVAL or BFLY_EDEVICE. */
int bfly_contraction_rate(int unit, int64_t n_threads, int64_t iters, void* out, void* stream);

/* Static description of a status code. */
const char* bfly_status_string(int status);

/* Thread-local detail message of the last failing call on this thread
 * ("" if none). */
const char* bfly_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BFLY_H */
