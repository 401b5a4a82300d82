/*
 * qdot.h -- C ABI of the MI355X (gfx950) qdot library.
 *
 * qdot is the error-bounded quantized dot product of Diffenderfer,
 * Osei-Kuffuor and Menon ("Qdot: Quantized Dot Product Kernel for
 * Approximate High Performance Computing", arXiv 2105.00115).  Given FP64
 * vectors x, y (or FP32 vectors, qdot_f32*) and a relative tolerance eps it
 *   1. bins the component products x_i y_i by their binary exponent
 *      (Def. 3.1 with exact binning, Sec. 3.2; Alg. 2),
 *   2. scores every non-empty bin (eq. bin-score-def) and gives it a
 *      precision -- double, single, half or perforate -- (eq.
 *      precision-def), so that the bound of Thm 3.3 / Thm 3.5 stays below
 *      eps,
 *   3. computes each kept product at its bin's precision after scaling the
 *      operands to exponent 0 and sums the results (Alg. 1, Sec. 3.3).
 *
 * Conventions for every entry point:
 *   - Vectors and matrices are device pointers (hipMalloc'd or any memory a
 *     gfx950 kernel may read), aligned to their element size, owned by the
 *     caller; the library never frees or retains them past the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Entry points named *_async only enqueue work and return; their
 *     results are written to device memory in stream order.  Others
 *     synchronise `stream` before returning.
 *   - Return value is a qdot_status.  Argument errors are detected on the
 *     host before anything is enqueued.  Data-dependent errors of async
 *     calls (non-finite input) land in the `status` field of the device
 *     result.  Nothing aborts, nothing throws across the ABI.
 *   - A handle is not thread-safe: use one handle per host thread/stream.
 *     Calls on one handle must be ordered on one stream (they share the
 *     handle's workspace).
 */
#ifndef QDOT_H
#define QDOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define QDOT_API __attribute__((visibility("default")))
#else
#define QDOT_API
#endif

/* ---- status codes ---------------------------------------------------- */
#define QDOT_OK 0
#define QDOT_E_INVAL 1      /* bad argument: n < 0, NULL with n > 0, tol <= 0
                               or not finite, unknown option value */
#define QDOT_E_NONFINITE 2  /* an input component is Inf or NaN (value NaN) */
#define QDOT_E_DEVICE 3     /* a HIP call failed; see qdot_last_error() */
#define QDOT_E_NOMEM 4      /* workspace allocation failed */
#define QDOT_E_BREAKDOWN 5  /* CG / power: a divisor was <= 0, not finite, or
                               qdot perforated every component */
#define QDOT_E_MAXIT 6      /* CG: iteration limit reached */

/* ---- precision classes (eq. precision-def) ------------------------- */
#define QDOT_DOUBLE 0
#define QDOT_SINGLE 1
#define QDOT_HALF 2
#define QDOT_PERF 3 /* perforated: left out of the sum */

/* ---- result flags ---------------------------------------------------- */
#define QDOT_F_UNATTAINABLE 1  /* some bin scored >= the input precision's
                                  mantissa width (52 for double inputs, 23
                                  for single): no precision row of eq.
                                  (precision-def) applies; it stays at the
                                  input precision and the bound may exceed
                                  eps */
#define QDOT_F_THM_ALL_DOUBLE 2 /* Thm 3.6 condition e_max - e_min <= -t - m
                                  holds (m = 23 for double inputs, 10 for
                                  single): every bin is at the input
                                  precision */
#define QDOT_F_ALL_PERF 4      /* no component kept; value is +0 */
#define QDOT_F_OVERFLOW 8      /* the final scaling by 2^e_max overflowed */
#define QDOT_F_GUARANTEED 16   /* guard_mode 1: the Thm 3.4 bound, taken with
                                  a certified lower bound of |x.y| in place
                                  of 2^E, is <= eps (see guard_mode) */
#define QDOT_F_RESELECTED 32   /* guard_mode 1: the classes were selected a
                                  second time and pass 2 was repeated */

/* ---- options --------------------------------------------------------- */
/* Zero-initialised = defaults. */
typedef struct qdot_options {
    /* 0: key = exponent of the product x_i*y_i (Def. 3.1, the theorems);
     * 1: key = E(x_i) + E(y_i) (Alg. 2, exponent preprocessing line), with
     *    the key taken as the bin's exponent u_k in the score and in
     *    bound_rel, as Alg. 2 is printed.  A bin of key k then holds
     *    products up to 2^(k+2), not 2^(k+1) as Thm 3.2 assumes, so under
     *    key_mode 1 bound_rel (and bound_abs) may understate the Thm 3.3
     *    bound of those bins by up to a factor 2 and is not an upper bound
     *    of the error. */
    int32_t key_mode;
    /* 0: score with eps / N_bins (experiments of Sec. 4.1), so that Thm 3.5
     *    bounds the relative error by eps;  1: score with eps itself. */
    int32_t score_mode;
    /* 0: eq. (precision-def) as printed (half-open intervals);
     * 1: the proof's wording (perforate when the score is <= 0, else the
     *    narrowest precision whose mantissa width is >= the score). */
    int32_t boundary_mode;
    /* 0: FP32 leaves summed in FP32 inside 64-element tiles of the index
     *    order (adjacent-pairwise tree), then at FP64 (two passes over x, y);
     * 1: one pass over x, y: the same classes and leaves (Alg. 1), summed
     *    exactly and rounded once.  While scanning the exponents, every
     *    block keeps per-bin candidate sums of all three precisions for the
     *    bins near its running maximum key and each kept bin takes its
     *    class's sum after the cutoff.  Accepted by qdot_async, qdot,
     *    qdot_power, qdot_cg and (for the qdot instances) the batched entry
     *    points when n <= 2^30 and the tolerance keeps every possibly kept
     *    bin within 255 exponents of e_max (ceil(log2 n) - t_min + 1 <=
     *    255, t_min the smallest t any histogram of n components can give:
     *    tol >= about 1e-60 at n = 2^27); QDOT_E_INVAL otherwise and in
     *    qdot_classes_async. */
    int32_t accum_mode;
    /* 0: the classes are selected once, against e_max (Alg. 2); the
     *    relative bound of Thm 3.3 then needs e_max <= flexp(x.y).
     * 1: guaranteed-eps mode (Thm 3.4, for data whose products cancel).
     *    After pass 2 the library bounds |x.y| from below by
     *      L = |S| (1 - 2^-52) - a            (units of 2^e_max)
     *    where S is the computed sum and a bounds every error of the call
     *    from the histogram and the classes alone:
     *      a = (Q + T + F) (1 + 2^-40),
     *      Q = sum_k M_k 2^(k-e_max+1) rho(class_k)  (quantisation; rho =
     *          2^-53, 3 2^-24 + 3 2^-48 + 2^-72, 2^-10 + 2^-22, 1 for
     *          double, single, half, perforated),
     *      T = g6 (1 + 2^-9) sum_{single, half bins} M_k 2^(k-e_max+1)
     *          (FP32 tile trees, g6 = 6u/(1-6u), u = 2^-24),
     *      F = 2^-52 |S| + 4 gn^2 (1 + 2^-8) sum_{kept bins} M_k 2^(k-e_max+1)
     *          + (2n + 4) 2^-1074  (FP64 stage and leaves scaled into
     *          the subnormal range, gn = n 2^-53 / (1 - n 2^-53)).
     *    When every non-zero product has the same sign, L is raised to
     *    1 (|x.y| >= max |x_i y_i| >= 2^e_max).  With E_lo = flexp(L) +
     *    e_max <= flexp(x.y), the call is certified (QDOT_F_GUARANTEED)
     *    when L > 0 and bound_rel 2^(e_max - E_lo) <= eps.  Otherwise the
     *    classes are selected again with the reference exponent e_ref =
     *    E_lo in place of e_max in the score (L > 0), or with e_ref =
     *    e_min - t - 22 - boundary_mode (single-precision inputs: - 9 -),
     *    which puts every bin at the input precision (L <= 0), pass 2 runs
     *    again (QDOT_F_RESELECTED) and the check is repeated with the
     *    larger of the two lower bounds.  Needs key_mode 0 and accum_mode
     *    0; accepted by qdot_async, qdot, qdot_classes_async, the qdot_f32
     *    entry points, qdot_power, qdot_cg and the batched entry points
     *    (every qdot instance and every CG system of the launch). */
    int32_t guard_mode;
    /* Binning strategy (Sec. 3.2), the partition of [e_min, e_max] into the
     * bins that are scored:
     * 0: exact bins, one exponent each (the default; bin_param unused);
     * 1: ranged bins of width w = bin_param (1..4196), (u_k - w, u_k] with
     *    u_k = e_min + k w - 1, k = 1, 2, ...;
     * 2: variable-width bins from at most s = bin_param (0..4196) splits:
     *    from the one bin (e_min - 1, e_max], each split halves, at
     *    l + ceil((u - l) / 2), the non-empty bin of more than one exponent
     *    whose Thm 3.2 term M_k 2^(u_k) is largest (ties to the higher u_k).
     * A bin is scored with its upper exponent u_k (eq. bin-score-def), its
     * class holds for all its keys, N_bins counts the non-empty bins and the
     * Thm 3.3 term of a bin is M_k 2^(u_k - e_max + 1) eps(class).  Modes 1
     * and 2 need accum_mode 0 and guard_mode 0 and are accepted by
     * qdot_async, qdot, qdot_classes_async, qdot_noalloc_async and the
     * qdot_f32 entry points; QDOT_E_INVAL elsewhere. */
    int32_t bin_mode;
    int32_t bin_param;
    /* 1: skip perforated tiles in pass 2 (Sec. 4.2 shows whole index ranges
     * of a solver's vectors falling into the perforated class).  Pass 1
     * also records, for every 64-component tile of the index order, the
     * largest key slot of its non-zero products; pass 2 reads neither x nor
     * y of a tile whose largest key lies below the lowest kept bin, since
     * every component of it is perforated.  Classes, counts and flags are
     * those of tile_skip 0, and so is the value, bit for bit, under the
     * dense accumulate form (qdot_tune acc_form 0; pass 2 with tile keys
     * always takes it, so a handle tuned to the compacting form gets a
     * value that may differ by the order of its FP64 additions).  Only the
     * bytes pass 2 reads change.  The handle keeps 2 bytes per tile (n / 32
     * bytes), grown at the first call with a larger n (an allocation, so
     * not while the stream is being captured: QDOT_E_INVAL then).  Needs
     * accum_mode 0 and guard_mode 0; accepted by qdot_async, qdot,
     * qdot_classes_async and the qdot_f32 entry points, QDOT_E_INVAL
     * elsewhere.  0: the default, no tile keys. */
    int32_t tile_skip;
} qdot_options;

/* ---- per-call result ------------------------------------------------- */
typedef struct qdot_result {
    double value;        /* the approximate dot product */
    int64_t count[4];    /* components per class DOUBLE, SINGLE, HALF, PERF;
                            PERF includes zero products */
    int64_t n_zero;      /* components with x_i == 0 or y_i == 0 */
    int32_t e_min, e_max;/* smallest / largest product exponent (keys) */
    int32_t n_bins;      /* non-empty exponent bins */
    int32_t t;           /* floor(log2(eps / N_bins)) (or of eps) */
    double part[3];      /* class sums DOUBLE, SINGLE, HALF (absolute) */
    double bound_rel;    /* sum_k M_k 2^(k - e_max + 1) eps(class_k)
                            (Thm 3.3 relative bound) */
    double bound_abs;    /* 2^e_max * bound_rel (Thm 3.2 absolute bound) */
    int32_t flags;       /* QDOT_F_* */
    int32_t status;      /* QDOT_OK or QDOT_E_NONFINITE (then value is
                            NaN and every other field 0) */
    double lower;        /* guard_mode 1: certified lower bound L 2^e_max
                            of |x.y| (0 when none is known; rounded to FP64,
                            exact unless subnormal); 0 otherwise */
    int32_t e_ref;       /* exponent the scores were taken against: e_max,
                            or the guard_mode 1 reselection's reference */
    int32_t passes;      /* sweeps over x, y that accumulated kept
                            components: 1 (pass 2, or the one-pass mode's
                            single sweep), 2 after a guard_mode 1
                            reselection, 0 when nothing was kept */
} qdot_result;

/* ---- CSR matrix (device arrays, host struct) -------------------------- */
typedef struct qdot_csr {
    int64_t n;             /* rows == columns */
    int64_t nnz;
    const int32_t *rowptr; /* n + 1 */
    const int32_t *col;    /* nnz, ascending within a row */
    const double *val;     /* nnz */
} qdot_csr;

typedef struct qdot_cg_result {
    int32_t iters;        /* iterations taken */
    int32_t status;       /* QDOT_OK, QDOT_E_BREAKDOWN or QDOT_E_MAXIT */
    double relres_est;    /* sqrt(c_k) / ||b|| at exit (c_k from the dot
                             product in use) */
    double relres_true;   /* ||b - A x|| / ||b|| recomputed at exit (FP64) */
} qdot_cg_result;

/* One CG system of a batched launch (all pointers device memory). */
typedef struct qdot_cg_system {
    qdot_csr A;          /* square, A.n rows */
    const double *b;     /* A.n right-hand side */
    double *x;           /* A.n: x0 on entry, solution on exit */
    double rtol;         /* stop when sqrt(c_k) <= rtol * ||b||_2 */
    double qtol;         /* qdot tolerance of both inner products */
    int32_t maxit;       /* iteration limit (QDOT_E_MAXIT beyond) */
    int32_t use_qdot;    /* 0: plain FP64 inner products */
} qdot_cg_system;

/* ---- launch configuration (autotuner) ---------------------------------- */
/* Launch shape of the two streaming passes.  Grids are persistent:
 * blocks_per_cu * CUs blocks of 256 threads, each thread keeping `unroll`
 * groups of 4 consecutive components in flight (1, 2 or 4).  Calls on
 * single-precision inputs (qdot_f32*) use twice the blocks per CU (at most
 * 8) and twice the unroll (at most 4) of their bucket: their groups are
 * half the bytes.  No setting changes a class, a count or an FP32 tile sum:
 * the 64-element tiles are fixed by the index order. */
typedef struct qdot_tune {
    int32_t scan_blocks_per_cu; /* exponent scan, 1..16 */
    int32_t scan_unroll;
    int32_t acc_blocks_per_cu;  /* accumulate pass and FP64 dot, 1..16 */
    int32_t acc_unroll;
    int32_t onepass_blocks_per_cu; /* one-pass scan (accum_mode 1), 1..16 */
    int32_t onepass_unroll;
    int32_t acc_form;    /* accumulate pass of double inputs: 0 every
                            candidate leaf formed in place, 1 kept
                            components compacted per wave and their leaves
                            formed 64 at a time (same tile sums bit for
                            bit); float inputs use 0 */
    int32_t hist_copies; /* global histogram copies the scan blocks of
                            double inputs spread their merges over: 1, 2, 4
                            or 8; float inputs use 8 */
    int32_t block_threads; /* threads per block of the scan and accumulate
                              passes of aligned double inputs: 128, 256 or
                              512 (the blocks-per-CU fields count blocks of
                              256 threads); other inputs use 256 */
} qdot_tune;

/* Tuning is kept per size bucket: n < 2^16, < 2^20, < 2^24, >= 2^24. */
#define QDOT_TUNE_BUCKETS 4

typedef struct qdot_handle qdot_handle;

/* Create a handle on `device` (HIP ordinal): allocates the workspace
 * (histogram, class table, per-block partials) once.
 * Returns QDOT_E_INVAL (h NULL or bad ordinal), QDOT_E_DEVICE, QDOT_E_NOMEM. */
QDOT_API int32_t qdot_create(qdot_handle **h, int32_t device);

/* Free the handle and its workspace.  NULL is a no-op. */
QDOT_API int32_t qdot_destroy(qdot_handle *h);

/* Text of the last error on this handle ("" if none).  Owned by the
 * handle, valid until the next call on it. */
QDOT_API const char *qdot_last_error(const qdot_handle *h);

/* Device the handle was created on and its compute-unit count. */
QDOT_API int32_t qdot_device_info(const qdot_handle *h, int32_t *device,
                         int32_t *num_cus);

/* Set / get the launch configuration of one size bucket (0..3, or -1 for
 * all buckets in qdot_set_tune).  NULL cfg in set restores the defaults. */
QDOT_API int32_t qdot_set_tune(qdot_handle *h, int32_t bucket, const qdot_tune *cfg);
QDOT_API int32_t qdot_get_tune(const qdot_handle *h, int32_t bucket, qdot_tune *cfg);

/* Load tuned configurations from a text file written by the autotuner: one
 * line per bucket, "bucket scan_bpc scan_unroll acc_bpc acc_unroll
 * [onepass_bpc onepass_unroll [acc_form hist_copies [block_threads]]]" (fields left out keep
 * the bucket's current values), and optionally one line "solver
 * batch_bpc batch_chunk cg_rows_per_block cg_gang_max spmv_bpc cg_bpc
 * power_scan_in_spmv"
 * (qdot_solver_tune);
 * '#' starts a comment.  Invalid lines are
 * rejected with QDOT_E_INVAL and leave the handle unchanged.  qdot_create
 * also loads the file named by the environment variable QDOT_TUNE_FILE when
 * it is set. */
QDOT_API int32_t qdot_load_tune(qdot_handle *h, const char *path);

/* Kernel timing (diagnostics).  While enabled, every qdot and FP64-dot call
 * on this handle records HIP events on its stream around each kernel it
 * launches (not allowed while the stream is being captured into a graph).
 * qdot_timing_read synchronises the recorded events and returns the summed
 * durations in milliseconds of the scan, cutoff, accumulate and finalize
 * kernels of qdot (ms[0..3]; with guard_mode 1, ms[3] also covers the guard
 * stages and the second sweep; in the one-pass mode ms[1] is the single
 * cutoff-and-pick kernel and ms[2], ms[3] are 0) and of the FP64 dot (ms[4], both of its kernels), the number
 * of qdot and FP64-dot calls timed (calls[0..1]), then clears the record. */
QDOT_API int32_t qdot_timing_enable(qdot_handle *h, int32_t enable);
QDOT_API int32_t qdot_timing_read(qdot_handle *h, double ms[5], int32_t calls[2]);

/* qdot(x, y, eps) -- Alg. 3: parameter selection (Alg. 2) then the
 * computation phase (Alg. 1).
 *   x, y : device FP64[n]; n >= 0; tol = eps > 0, finite (any size:
 *          eps > 1 is allowed, as in the CG study of Sec. 4.2).
 *   opt  : NULL for defaults.
 *   dev_out : device pointer to one qdot_result, written in stream order.
 * n == 0 or all-zero products give value +0 with QDOT_F_ALL_PERF.
 * Enqueues four kernels (eight with guard_mode 1, whose second pass-2
 * kernels return at once when no reselection is needed); performs no
 * allocation and no host sync, so it may be captured in a HIP graph
 * (tile_skip 1: except the first call with a larger n, which grows the
 * handle's tile keys). */
QDOT_API int32_t qdot_async(qdot_handle *h, const double *x, const double *y,
                   int64_t n, double tol, const qdot_options *opt,
                   void *stream, qdot_result *dev_out);

/* qdot_async without a handle and without any allocation, for callers that
 * cannot allocate device memory: code recorded under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments
 * (minus the handle), options, kernels, results and async errors as
 * qdot_async, on the current device, with the default launch shapes.
 *   Workspace: a fixed device array of about 2.2 MB inside the library
 *   (control block and histograms ~0.35 MB, partials for 4096 blocks,
 *   one-pass per-bin tables), one copy per GPU, held until the process
 *   ends.  Its size does not depend on n: every grid of the call is capped
 *   to the partials it holds, so no n is refused for lack of room (n is
 *   limited only as for qdot_async; accum_mode 1 needs n <= 2^30).
 *   The first call on a device also clears that device's array, in order
 *   on `stream`.  Every call on one GPU shares its array: calls must be
 *   ordered (one stream, or synchronised); calls that overlap on one GPU
 *   race and give wrong results.
 * Returns QDOT_E_INVAL for the argument errors of qdot_async, a NULL
 * dev_out or tile_skip 1 (the tile keys need memory), QDOT_E_DEVICE when a HIP call fails (no message is kept: there
 * is no handle).  Performs no hipMalloc, hipFree or host sync. */
QDOT_API int32_t qdot_noalloc_async(const double *x, const double *y, int64_t n,
                           double tol, const qdot_options *opt, void *stream,
                           qdot_result *dev_out);

/* Synchronous qdot: as qdot_async, then copies the result to host_out and
 * synchronises the stream.  Returns the result's status (QDOT_OK or
 * QDOT_E_NONFINITE) when the call itself succeeded. */
QDOT_API int32_t qdot(qdot_handle *h, const double *x, const double *y, int64_t n,
             double tol, const qdot_options *opt, void *stream,
             qdot_result *host_out);

/* Debug view of the parameter selection (Alg. 2): per-component class
 * dev_cls[n] (uint8, QDOT_DOUBLE..QDOT_PERF) and, if dev_hist is not NULL,
 * the exponent histogram dev_hist[4196] (int64, slot k + 2148 counts the
 * products with exponent k).  Also writes the full result to dev_out.
 * Async, same errors as qdot_async. */
QDOT_API int32_t qdot_classes_async(qdot_handle *h, const double *x, const double *y,
                           int64_t n, double tol, const qdot_options *opt,
                           void *stream, uint8_t *dev_cls, int64_t *dev_hist,
                           qdot_result *dev_out);

/* qdot of single-precision inputs (eq. (precision-def) with mu = m_single,
 * the input precision the table allows; Sec. 3.2).  As qdot_async for
 * device float vectors x, y (n components, 4-byte aligned; 16-byte aligned
 * vectors take the vector-load path).  Every float is exactly a double, so
 * keys, histogram, t and scores are those of the same values given as
 * doubles; the precision table has no double row, so a bin scoring at or
 * above m_single (23) stays single and sets QDOT_F_UNATTAINABLE, and
 * QDOT_F_THM_ALL_DOUBLE means every bin is at the input precision (Thm 3.6
 * with m_half: e_max - e_min <= -t - 10).  The result is FP64 and counts
 * no double class.  accum_mode 1 is the one-pass reading (same
 * admissibility as for double inputs); guard_mode 1 reselects with every
 * bin at most single.  No allocation, no host sync; graph-capturable. */
QDOT_API int32_t qdot_f32_async(qdot_handle *h, const float *x, const float *y,
                       int64_t n, double tol, const qdot_options *opt,
                       void *stream, qdot_result *dev_out);

/* Synchronous qdot_f32_async, as qdot is to qdot_async. */
QDOT_API int32_t qdot_f32(qdot_handle *h, const float *x, const float *y, int64_t n,
                 double tol, const qdot_options *opt, void *stream,
                 qdot_result *host_out);

/* qdot_classes_async for single-precision inputs (accum_mode 0). */
QDOT_API int32_t qdot_f32_classes_async(qdot_handle *h, const float *x, const float *y,
                               int64_t n, double tol, const qdot_options *opt,
                               void *stream, uint8_t *dev_cls, int64_t *dev_hist,
                               qdot_result *dev_out);

/* Minimal entry: qdot of device vectors x, y (n components, 8-byte
 * aligned) at tolerance tol with the default options, on a handle the
 * library keeps per device (created on the first call on the current
 * device, kept until the process ends), on the null stream, synchronous.
 * value (host) receives the approximate dot product; counts (host, may be
 * NULL) the DOUBLE, SINGLE, HALF, PERF counts.  Returns the status as qdot
 * does.  Calls are serialised across host threads. */
QDOT_API int32_t qdot_simple(const double *x, const double *y, int64_t n, double tol,
                             double *value, int64_t counts[4]);

/* Plain FP64 dot product sum_i x_i y_i (the full-precision kernel that
 * qdot approximates; the comparison baseline of Sec. 4.1).  dev_out: one
 * double in device memory.  Async. */
QDOT_API int32_t qdot_fp64_dot_async(qdot_handle *h, const double *x, const double *y,
                            int64_t n, void *stream, double *dev_out);

/* Batched ragged qdot: B independent instances stored back to back, all in
 * one persistent kernel launch.
 *   x_cat, y_cat : device FP64[offsets[B]]
 *   offsets      : device int64[B + 1], offsets[0] = 0, non-decreasing;
 *                  instance j is [offsets[j], offsets[j+1]).  Its 64-element
 *                  accumulation tiles start at offsets[j].
 *   host_offsets : host copy of offsets, used to plan the work queue.
 *   tols         : device FP64[B]; an instance whose tolerance is not finite
 *                  and > 0 gets status QDOT_E_INVAL (value NaN).
 *   dev_out      : device qdot_result[B].
 * Each instance's counts, classes, bins and value follow qdot on that
 * instance alone (same readings, same tiles).  The first call with a new
 * offsets layout plans it (allocates the per-layout state and uploads the
 * work list, synchronously); later calls with the same layout only launch
 * one kernel: no allocation, no memset, no host sync, graph-capturable.
 * Up to 8 layouts are kept per handle.  Calls on one handle must be ordered
 * on one stream.  Host-side argument errors return QDOT_E_INVAL.
 * guard_mode 1 runs the guaranteed mode on every instance (same decisions,
 * flags, lower bound and passes as qdot_async on it): a small instance is
 * certified by the block that runs it, a large one by the block that
 * finishes its last pass-2 chunk, which after a reselection sweeps that
 * instance again alone.  The pass-2 chunks of a large instance wait for its cutoff
 * with a spin limit; a chunk that waits past it gives that instance status
 * QDOT_E_DEVICE (the work order makes the wait end long before). */
QDOT_API int32_t qdot_batched_async(qdot_handle *h, const double *x_cat,
                                    const double *y_cat, const int64_t *offsets,
                                    const int64_t *host_offsets, const double *tols,
                                    int32_t B, const qdot_options *opt, void *stream,
                                    qdot_result *dev_out);

/* Launch shapes of the solvers and the batched launch.  Chosen by the
 * autotuner; the defaults are {4, 131072, 16384, 16, 8, 2, 0}. */
typedef struct qdot_solver_tune {
    int32_t batch_blocks_per_cu; /* batched launch (qdot_batched_async,
                                    qdot_batch_run_async, qdot_cg_batched):
                                    persistent grid, blocks per CU, 1..16
                                    (the resident ones are capped by
                                    occupancy) */
    int32_t batch_chunk;       /* components per pass-1 / pass-2 chunk of a
                                  large batched instance, and the largest
                                  instance one block takes whole: 2^13..2^22,
                                  a multiple of 2048 */
    int32_t cg_rows_per_block; /* a batched CG system of n rows gets
                                  ceil(n / this) gang blocks, >= 1024 ... */
    int32_t cg_gang_max;       /* ... and at most this many, 1..512 */
    int32_t spmv_blocks_per_cu; /* SpMV grid (qdot_spmv_async, the power
                                   method), blocks per CU, 1..16 */
    int32_t cg_blocks_per_cu;  /* qdot_cg: gang blocks per CU, 1..2 (capped by
                                  occupancy and by one block per 1024 rows) */
    int32_t power_scan_in_spmv; /* qdot_power, two-pass qdot: 1 takes pass 1
                                   of both inner products inside the SpMV
                                   after the first iteration, 0 in a kernel
                                   of its own (same results) */
} qdot_solver_tune;

/* Set (cfg NULL: defaults) or read the handle's solver and batched launch
 * shapes.  Setting them frees the handle's cached batch plans (after a
 * device sync); out-of-range values return QDOT_E_INVAL and change
 * nothing.  No value changes a class, a count or an FP32 tile sum
 * (instances and row slices are split along whole 2048-component groups);
 * values move only by the order of compensated FP64 sums, and a CG
 * iteration count only as far as that moves its stopping test. */
QDOT_API int32_t qdot_set_solver_tune(qdot_handle *h, const qdot_solver_tune *cfg);
QDOT_API int32_t qdot_get_solver_tune(const qdot_handle *h, qdot_solver_tune *cfg);

/* Plan a batched layout ahead of time (e.g. before capturing
 * qdot_batched_async into a graph).  Synchronous. */
QDOT_API int32_t qdot_batched_plan(qdot_handle *h, const int64_t *host_offsets,
                                   int32_t B);

/* Batched launch of qdot instances and CG systems together: the B ragged
 * instances (arguments as qdot_batched_async; B may be 0; with accum_mode 1
 * each instance is read once, and an instance whose tolerance does not
 * admit the one-pass mode gets status QDOT_E_INVAL) and S CG systems (their
 * inner products always use accum_mode 0)
 * (systems: host array of S descriptors; S may be 0) run in one persistent
 * kernel launch.  Each CG system follows qdot_cg on that system alone (Alg.
 * 4 with the same stopping rule and the same inner products); it is solved
 * by a gang of blocks (one per cg_rows_per_block rows, at most cg_gang_max:
 * qdot_solver_tune) that meet at barriers,
 * gangs are formed before the qdot work items are handed out, largest
 * system first.  dev_cg_out: device qdot_cg_result[S].  Planning happens on
 * the first call with a new layout (offsets and system descriptors,
 * compared by value) and is synchronous; later calls with the same layout
 * launch two kernels (a re-arm pass over the gangs and the batch), allocate
 * nothing and can be captured in a graph.  A gang barrier that does not
 * complete within its spin limit gives that system status QDOT_E_DEVICE.
 * guard_mode 1 runs the guaranteed mode on every qdot instance (as
 * qdot_batched_async) and on every inner product of every CG system (as
 * qdot_cg). */
QDOT_API int32_t qdot_batch_run_async(qdot_handle *h, const double *x_cat,
                                      const double *y_cat, const int64_t *offsets,
                                      const int64_t *host_offsets, const double *tols,
                                      int32_t B, const qdot_cg_system *systems, int32_t S,
                                      const qdot_options *opt, void *stream,
                                      qdot_result *dev_out, qdot_cg_result *dev_cg_out);

/* Plan a layout of qdot_batch_run_async ahead of time (e.g. before graph
 * capture); opt (NULL = defaults) must carry the accum_mode of the later
 * calls, whose plans differ.  Synchronous. */
QDOT_API int32_t qdot_batch_plan(qdot_handle *h, const int64_t *host_offsets, int32_t B,
                                 const qdot_cg_system *systems, int32_t S,
                                 const qdot_options *opt);

/* S CG systems in one persistent launch (qdot_batch_run_async with no qdot
 * instances); host_out: host qdot_cg_result[S].  Synchronous. */
QDOT_API int32_t qdot_cg_batched(qdot_handle *h, const qdot_cg_system *systems, int32_t S,
                                 const qdot_options *opt, void *stream,
                                 qdot_cg_result *host_out);

/* y = A x for a CSR matrix (rows summed in stored order, each product and
 * sum one FP64 rounding).  col entries must lie in [0, n); rows of any
 * length are accepted.  The grid holds up to 8 blocks per CU (environment
 * variable QDOT_SPMV_BPC, 1..16, overrides it).  Async. */
QDOT_API int32_t qdot_spmv_async(qdot_handle *h, const qdot_csr *A, const double *x,
                        double *y, void *stream);

/* Conjugate gradient, Alg. 4 (ACG): both inner products of every iteration
 * (r.r and p.Ap) by qdot at tolerance qtol when use_qdot != 0, else by the
 * plain FP64 dot.  x holds x0 on entry and the solution on exit.  Stops
 * when sqrt(c_k) <= rtol * ||b||_2 (||b|| by the FP64 dot) or after maxit
 * iterations.  trace: NULL or device qdot_result[2*maxit + 1] receiving
 * every qdot result in call order.  Synchronous; out (host) receives the
 * iteration count, status and residuals.  Returns out->status.
 * The whole solve is one persistent launch of up to two blocks per CU
 * (as many as can be resident together; at most 512, at least 1024 rows
 * per block; environment variable QDOT_CG_BLOCKS caps the count).  A gang
 * barrier that does not complete within its spin limit ends the solve with
 * QDOT_E_DEVICE.  guard_mode 1 runs the guaranteed mode on every qdot of
 * the solve (same decisions, flags, lower bound and passes as qdot_async; a
 * reselected product costs one more sweep of the gang's rows and one more
 * gang barrier).  accum_mode 1 runs every qdot in the one-pass reading
 * (admissibility as for qdot_async, else QDOT_E_INVAL); each block reads its
 * rows once, and the last block to arrive at the one barrier of an inner
 * product selects and picks for the gang.  The first such call allocates
 * the gang's one-pass tables (2 x 4196 x 6 doubles) on the handle. */
QDOT_API int32_t qdot_cg(qdot_handle *h, const qdot_csr *A, const double *b, double *x,
                double rtol, double qtol, int32_t maxit, int32_t use_qdot,
                const qdot_options *opt, void *stream, qdot_cg_result *out,
                qdot_result *trace);

/* Power method (Alg. 5 with the Rayleigh quotient of the current unit
 * iterate): per iteration w = A x, lambda = dot(x, w), c = dot(w, w),
 * x = w / sqrt(c), with both dots by qdot at qtol when use_qdot != 0.
 * x: device FP64[n], unit vector on entry, last iterate on exit.
 * lambda (host): last lambda.  lambda_trace: NULL or device FP64[iters].
 * trace: NULL or device qdot_result[2 * iters]: with use_qdot != 0, the
 * results of iteration k's two qdot calls, lambda = qdot(x, w) at 2k and
 * c = qdot(w, w) at 2k + 1 (their counts are the per-precision component
 * shares the APM study of Sec. 4.3 plots); not written when use_qdot is 0.
 * After a breakdown, entries past the iteration that broke down are
 * unspecified.
 * opt: as qdot_async (the one-pass and guaranteed modes included).  With
 * the two-pass qdot the two inner products of an iteration are computed
 * side by side: one pass-1 kernel reads x and w once for both, and the
 * cutoff, pass-2 and combine kernels each run once for the pair, with the
 * results of two separate qdot calls.  Each iteration's SpMV also applies
 * the previous iteration's x = w / sqrt(c).  The handle keeps 2n doubles
 * of scratch (grown on demand) and, from the first call with the two-pass
 * qdot, a second workspace.
 * Synchronous.  QDOT_E_BREAKDOWN if c <= 0 or not finite. */
QDOT_API int32_t qdot_power(qdot_handle *h, const qdot_csr *A, double *x,
                   int32_t iters, double qtol, int32_t use_qdot,
                   const qdot_options *opt, void *stream, double *lambda,
                   double *lambda_trace, qdot_result *trace);

#ifdef __cplusplus
}
#endif
#endif /* QDOT_H */
