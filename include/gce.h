/*
 * gce.h -- C ABI of the MI355X conditional-entropy period search.
 *
 * The library evaluates, for every light curve c, every period P_p and every
 * period derivative Pdot_q of a search grid, the conditional entropy H_c of
 * Katz et al. 2020 ("GPU-Accelerated Periodic Source Identification in
 * Large-Scale Surveys: Measuring P and Pdot"), Sec. 2.3:
 *
 *   fold (Eq. (3)):    x = (t - t0) / P,   phi = frac(x - Pdot x^2 / 2)
 *   histogram:         (magnitude bin, phase bin) counts, n_mag x n_phase
 *   entropy (Eq. (4)): H_c = sum_ij p(m_i, phi_j) ln(p(phi_j) / p(m_i, phi_j))
 *
 * and the per-curve minimum of H_c over the grid (Sec. 2.3, Sec. 4: the
 * minimum CE locates the period; batches keep their minimum and parameters).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: epochs and periods in days, Pdot dimensionless.
 *  - t0 is the earliest epoch of each curve.  Magnitudes are normalised per
 *    curve onto [0, 1] by their minimum and maximum (u = (m - min) / (max -
 *    min), each operation correctly rounded) and cut into n_mag equal bins:
 *    bin floor(u * n_mag) of the exact product (not of its rounding), at
 *    most n_mag - 1 (the maximum falls in the last bin; a constant curve has
 *    one bin).
 *  - Fold arithmetic is IEEE binary64 in this order: invP = 1.0 / P
 *    (correctly rounded), x = dt * invP, x2 = x * x,
 *    y = fma(-(0.5 * Pdot), x2, x), phi = y - floor(y); the phase bin is the
 *    floor of the exact product phi * n_phase (not of its rounding), at most
 *    n_phase - 1.  The FP64 path reproduces these bins bit for bit.
 *  - Curves are ragged: epochs of curve c occupy [offsets[c], offsets[c+1])
 *    of the concatenated `times` / `mags` arrays.
 *  - The CE cube is row-major [curve][pdot][period] (period fastest); the
 *    flat index of a trial is q * n_periods + p.  The per-curve minimum is
 *    the lowest flat index among the trials with the smallest H_c.
 *  - Pointers are device pointers (hipMalloc or equivalent) unless marked
 *    HOST.  The caller owns every buffer; the library keeps no pointer to
 *    caller memory after the work it enqueued has completed.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work and return; results are valid once the stream has been synchronised.
 *  - Errors: every entry point returns GCE_OK (0) or a negative GCE_E* code;
 *    gce_status_string() describes the last error of the calling thread.
 *    Argument errors are detected on the host before anything is enqueued.
 *    Bad data values (non-finite epochs or magnitudes, a period outside
 *    [1e-12, 1e12] days or NaN, |Pdot| > 1 or NaN, epochs of one curve
 *    spanning more than 1e12 days) cannot be reported synchronously: the affected
 *    curves (all curves for a bad grid) get flat_index = -1, ce_min = NaN and
 *    NaN CE values.  Split-precision plans (GCE_PRECISION_SPLIT_FP32) form
 *    x^2 = (t - t0)^2 / P^2 in FP32 and accept only periods of at least
 *    1e-6 days and curves spanning at most 1e10 days (x below 1e16 cycles);
 *    other values are bad data values in the same sense.
 *  - Test hook: with the environment variable GCE_FAIL_ALLOC=1, the entry
 *    points that allocate device memory (gce_plan_create, gce_search,
 *    gce_autotune) return GCE_ENOMEM after checking their arguments, before
 *    any device call.
 *  - Limits: 1 <= n_phase_bins <= 128, 1 <= n_mag_bins <= 255,
 *    1 <= points per curve <= 65535 (counts are 16-bit; overlapping bins
 *    that count an epoch twice halve this, see gce_opts).
 */
#ifndef GCE_H
#define GCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCE_OK 0
#define GCE_EINVAL (-1)        /* bad argument (pointer, count, size, offsets) */
#define GCE_ENOMEM (-2)        /* device or host allocation failed */
#define GCE_EHIP (-3)          /* a HIP runtime call failed */
#define GCE_EWORKSPACE (-4)    /* caller workspace too small */
#define GCE_ENODEV (-5)        /* no usable gfx950 device */
#define GCE_EUNSUPPORTED (-6)  /* option combination not supported */

/* Precision of the fold / entropy arithmetic. */
#define GCE_PRECISION_FP64 0        /* bit-exact bins, FP64 entropy */
#define GCE_PRECISION_SPLIT_FP32 1  /* FP32 Pdot term and binning, FP64 entropy;
                                       approximate bins, FP32 CE cube.  Its
                                       phase is within E = 2^-22 + 2^-20 A
                                       + 2^-52 x cycles of the FP64 phase
                                       (x = (t - t0) / P, A = |Pdot| x^2 / 2;
                                       E = 0 at x = 0), so an epoch's bin
                                       differs from the FP64 bin only if its
                                       FP64 phase lies within E of a bin edge */

/* Per-curve result (48 bytes). */
typedef struct {
    int64_t flat_index;   /* q * n_periods + p of the minimum; -1 if invalid */
    int32_t period_index; /* p; -1 if invalid */
    int32_t pdot_index;   /* q; -1 if invalid */
    double ce_min;        /* H_c at flat_index; NaN if invalid */
    double ce_mean;       /* mean of H_c over the curve's trials; NaN if invalid */
    double ce_std;        /* population standard deviation of those H_c */
    double significance;  /* Eq. (5): (ce_mean - ce_min) / ce_std; 0 when
                             ce_std = 0; NaN if invalid */
} gce_best_t;

/*
 * gce_search -- one-call FP64 search (Sec. 2.3, Eqs. (3)-(4)).
 *
 *  times, mags     : device, [offsets[n_curves]] doubles, curve-major.
 *  curve_offsets   : HOST, [n_curves + 1], offsets[0] = 0, strictly
 *                    increasing, each curve 1..65535 epochs.
 *  periods         : device, [n_periods] doubles (days), any order.
 *  pdots           : device, [n_pdots] doubles, any order.
 *  n_phase_bins, n_mag_bins : histogram shape.
 *  out_ce          : device, [n_curves][n_pdots][n_periods] doubles, or NULL
 *                    to skip the cube (minimum only).
 *  out_best        : device, [n_curves] gce_best_t.
 *  stream          : hipStream_t.
 *
 * Allocates a workspace once per device, stream and shape (a small cache of
 * plans; the least recently used of more than four is destroyed, which
 * synchronises the device).  Calls on one stream share that stream's plan and
 * are ordered by the stream; calls on different streams never share a
 * workspace.  Not safe to call during stream capture unless an identical
 * call on the same stream has already run.  Returns GCE_OK or a negative
 * GCE_E* code.
 */
int gce_search(const double *times, const double *mags,
               const int64_t *curve_offsets, int64_t n_curves,
               const double *periods, int64_t n_periods, const double *pdots,
               int64_t n_pdots, int32_t n_phase_bins, int32_t n_mag_bins,
               double *out_ce, gce_best_t *out_best, void *stream);

/*
 * gce_search_noalloc -- gce_search for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It calls no hipMalloc, hipFree or other allocating
 * routine: the workspace lives in one device array of
 * GCE_NOALLOC_SCRATCH_BYTES owned by the library, one per device, held
 * from the library's first use of that device until the process ends.
 *
 * Arguments and results as for gce_search (FP64 bins, bit-exact with the
 * documented arithmetic).  Curves are searched in their given order with the
 * c ln c table in global memory.  The offsets are copied from HOST memory
 * with hipMemcpyAsync on `stream`.  Every part of the array is written by a
 * call before that call reads it, so nothing depends on an earlier call's
 * contents.  All calls on one device share its array: calls that overlap on
 * one device (on different streams, or from several threads) race on it.
 *
 * Returns GCE_EWORKSPACE, before touching the device, for shapes whose
 * workspace exceeds the array (roughly: 40 bytes per work unit of 64
 * periods x the heuristic Pdot trials per lane, plus 8 bytes per epoch,
 * period and Pdot value); GCE_ENODEV without a gfx950 device; GCE_EHIP if a
 * launch or the copy fails.
 */
#define GCE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gce_search_noalloc(const double *times, const double *mags,
                       const int64_t *curve_offsets, int64_t n_curves,
                       const double *periods, int64_t n_periods, const double *pdots,
                       int64_t n_pdots, int32_t n_phase_bins, int32_t n_mag_bins,
                       double *out_ce, gce_best_t *out_best, void *stream);

/* --------------------------------------------------------------------------
 * Plans: validation, scheduling and allocation once; execution many times.
 * gce_plan_execute allocates nothing and copies nothing between host and
 * device, so it may be captured into a HIP graph.
 * ------------------------------------------------------------------------ */
typedef struct gce_plan_s *gce_plan_t;

typedef struct {
    int32_t precision;       /* GCE_PRECISION_* */
    int32_t trials_per_lane; /* Pdot trials per lane: 0 = automatic, else
                                1, 2, 4 or 8 */
    int32_t phase_overlap;   /* nonzero: 50%-overlapping phase bins (Sec. 2.3):
                                bin k spans phases [k, k + 2) / n_phase, wrapping,
                                so every epoch counts in two bins and the
                                probabilities of Eq. (4) are counts over the
                                histogram total (2N without magnitude
                                overlap) */
    int32_t table_placement; /* c ln c table read by the entropy sums:
                                0 = automatic, 1 = global memory, 2 = a copy in
                                LDS shared by the two waves of a block (pays
                                off when there are many histogram cells per
                                epoch; counts at most 8191, and the table and
                                histograms must fit 64 KiB).  Automatic may
                                also search a ragged batch's shortest curves
                                in a second launch with the table in LDS. */
    int32_t mag_overlap;     /* nonzero: 50%-overlapping magnitude bins (Sec.
                                2.3): bin j spans [j, j + 2) / (n_mag + 1) of
                                the normalised magnitude u, i.e. with
                                s = min(floor(u * (n_mag + 1)), n_mag) (the
                                floor of the exact product) the
                                epoch is in bins s - 1 and s where they exist
                                (one bin in the first and last half-bin).  The
                                probabilities of Eq. (4) are counts over the
                                histogram's total count.  Curves may then hold
                                at most 32767 epochs (at most 4095 with the
                                table in LDS); with phase_overlap and
                                n_phase_bins = 1 the limits halve again
                                (GCE_EUNSUPPORTED beyond them). */
    int32_t waves_per_unit;  /* waves that search one work unit (64 periods x
                                trials_per_lane Pdot values of one curve):
                                0 = automatic, 1, or 2 = two waves that split
                                each magnitude bin's epochs and the phase bins
                                of the entropy sums between them and add into
                                one LDS copy of the unit's histograms (half
                                the LDS per wave, so more waves per CU where
                                histograms are large).  2 is compiled for 10
                                and 20 phase bins at 4 and 8 (10) or 2, 4
                                and 8 (20) trials per lane, and for 50 phase
                                bins at 1, 2 and 4 (GCE_EUNSUPPORTED
                                elsewhere); automatic takes 2 there when one
                                wave's histograms would hold 8 KiB or more. */
    int32_t refine_units;    /* split path only (no effect on FP64 plans):
                                0 = none; k in [1, 64] = after the split
                                search, the k work units of each curve with
                                the smallest split minima are searched again
                                with the FP64 kernel, and the curve's reported
                                minimum (flat, period and Pdot index, ce_min)
                                is the FP64 minimum over those units' trials,
                                its CE value the FP64 one; ce_mean and ce_std
                                stay those of the split CE values over the
                                whole grid, and the significance is formed
                                from them and the FP64 ce_min.  The CE cube
                                keeps the split values.  About k work units
                                per curve of extra FP64 work. */
} gce_opts;

#define GCE_TABLE_AUTO 0
#define GCE_TABLE_GLOBAL 1
#define GCE_TABLE_LDS 2

/*
 * gce_plan_create -- validate the shape and the HOST offsets, build the
 * schedule (curves ordered by decreasing length), allocate the device
 * workspace and upload the per-curve metadata.  Synchronous.
 *  plan          : out, the new plan.
 *  curve_offsets : HOST, [n_curves + 1] as for gce_search (copied).
 *  opts          : may be NULL (FP64, automatic tiling, disjoint bins).
 *                  Zero-initialise it and set the fields wanted.
 *  device        : HIP device ordinal the plan runs on.
 */
int gce_plan_create(gce_plan_t *plan, const int64_t *curve_offsets,
                    int64_t n_curves, int64_t n_periods, int64_t n_pdots,
                    int32_t n_phase_bins, int32_t n_mag_bins,
                    const gce_opts *opts, int32_t device);

/*
 * gce_plan_execute -- enqueue the whole search on `stream`: grid check,
 * per-curve preparation (t0, magnitude bins, points grouped by magnitude
 * bin), the search kernel, and the per-curve minimum (for split plans with
 * refine_units, then the FP64 search of each curve's best work units and
 * the FP64 minimum over them).  Allocates nothing and copies nothing
 * between host and device, so it can be captured in a HIP graph.
 *  times, mags : device, laid out as the plan's offsets describe.
 *  periods     : device, [n_periods].  pdots : device, [n_pdots].
 *  out_ce      : device cube [n_curves][n_pdots][n_periods] or NULL.
 *                FP64 plans write doubles; SPLIT_FP32 plans write floats
 *                through the same pointer (cast by the caller).
 *  out_best    : device, [n_curves].
 * Calls that overlap on one plan race on its workspace.
 */
int gce_plan_execute(gce_plan_t plan, const double *times, const double *mags,
                     const double *periods, const double *pdots,
                     void *out_ce, gce_best_t *out_best, void *stream);

/*
 * gce_plan_debug_counts -- test hook: the [n_mag][n_phase] histogram of
 * selected trials, binned by the same device code as the search.
 *  trial_curve, trial_flat : device, [n_trials] int64 (curve, flat index).
 *  out_counts  : device, [n_trials][n_mag][n_phase] uint32.
 * Out-of-range trial ids give all-zero histograms.
 */
int gce_plan_debug_counts(gce_plan_t plan, const double *times,
                          const double *mags, const double *periods,
                          const double *pdots, const int64_t *trial_curve,
                          const int64_t *trial_flat, int64_t n_trials,
                          uint32_t *out_counts, void *stream);

/*
 * gce_plan_set_timing -- measurement hook.  With capacity > 0 the plan keeps
 * a ring of `capacity` HIP event pairs and records one pair around the
 * search kernel of every later gce_plan_execute, on that call's stream
 * (leave it off under graph capture).  capacity = 0 disables it and frees
 * the events.  Returns GCE_EINVAL for capacity < 0 or > 65536.
 */
int gce_plan_set_timing(gce_plan_t plan, int32_t capacity);

/*
 * gce_plan_search_times -- search-kernel durations in milliseconds of the
 * most recent min(executes since enabling, capacity) executes, oldest first.
 * Waits for the recorded events.  out_ms: HOST, room for max values;
 * *n_out receives the number written.
 */
int gce_plan_search_times(gce_plan_t plan, float *out_ms, int32_t max,
                          int32_t *n_out);

/* What a plan chose: tiling and resources of its search kernel. */
typedef struct {
    int32_t precision;          /* GCE_PRECISION_* */
    int32_t trials_per_lane;    /* Pdot trials per lane actually used */
    int32_t lds_bytes_per_wave; /* LDS of one search wave */
    int32_t table_in_lds;       /* where the c ln c table is read: 0 global
                                   memory, 1 LDS, 2 global for the longer
                                   curves and LDS in a second search launch
                                   over the curves of at most
                                   4 * n_phase * n_mag epochs (automatic
                                   placement of a ragged batch) */
    int64_t work_units;         /* work units of one search launch */
    int64_t workspace_bytes;    /* device workspace held by the plan */
    int32_t waves_per_unit;     /* waves that search one work unit: 1 or 2 */
    int32_t refine_units;       /* work units per curve searched again in
                                   FP64 (split plans with refine_units) */
} gce_plan_info_t;

/* Fill *info for the plan.  Returns GCE_EINVAL for NULL arguments. */
int gce_plan_get_info(gce_plan_t plan, gce_plan_info_t *info);

/*
 * gce_merge_results -- combine per-curve results of searches over parts of
 * one grid (Sec. 4: batches over Pdot values or periods keep their minimum and
 * statistics, and the batches are combined).  HOST arrays, no GPU work.
 *  acc        : [n_curves] running result, flat indices in the full grid.
 *  acc_trials : trials already merged into acc (the same for every curve);
 *               0 means acc is empty and is overwritten.
 *  part       : [n_curves] result of one execute over the sub-grid of
 *               part_n_periods periods starting at period part_p_offset and
 *               part_n_pdots Pdot values starting at part_q_offset.
 *  n_periods  : period count of the full grid.
 * The minimum is the lexicographic (H_c, full-grid flat index) minimum, the
 * mean and population standard deviation are merged exactly (Chan et al.),
 * and the significance is recomputed.  Invalid curves stay invalid.
 */
int gce_merge_results(gce_best_t *acc, int64_t acc_trials,
                      const gce_best_t *part, int64_t n_curves,
                      int64_t n_periods, int64_t part_p_offset,
                      int64_t part_n_periods, int64_t part_q_offset,
                      int64_t part_n_pdots);

/*
 * gce_autotune -- measure the search kernel's tilings -- Pdot trials per
 * lane (1, 2, 4, 8) and c ln c table placement (global, LDS), those that fit
 * in LDS -- on a slice of the given workload and remember the fastest for
 * its shape class: precision, phase and magnitude overlap, phase and
 * magnitude bin counts, Pdot count (1, 2, 3-4, 5-8, more) and median curve
 * length (<128, <512, <2048, more).  Later plans created with automatic tiling
 * (trials_per_lane = 0) in this process use the remembered choice.  If the
 * environment variable GCE_TUNE_CACHE names a file, choices are read from it
 * at the first plan creation and appended to it here.
 * The slice: up to 128 curves spread over the length range, the first
 * min(n_periods, 8192) periods, all Pdot values, minimum only (no cube).
 * Inputs as for gce_search (times, mags, periods, pdots device; curve_offsets
 * HOST).  Allocates and synchronises `stream`; not for graph capture.
 *  best_tq  : out, the chosen trials per lane.
 *  best_placement : out (may be NULL), GCE_TABLE_GLOBAL or GCE_TABLE_LDS.
 *  ms       : out (may be NULL), [8] search-kernel milliseconds for 1, 2, 4,
 *             8 trials per lane with the table in global memory, then the
 *             same with the table in LDS; negative where not run.
 */
int gce_autotune(const double *times, const double *mags,
                 const int64_t *curve_offsets, int64_t n_curves,
                 const double *periods, int64_t n_periods, const double *pdots,
                 int64_t n_pdots, int32_t n_phase_bins, int32_t n_mag_bins,
                 int32_t precision, int32_t phase_overlap, int32_t mag_overlap,
                 int32_t device, void *stream, int32_t *best_tq,
                 int32_t *best_placement, float *ms);

/* Bytes of device workspace the plan holds. */
size_t gce_plan_workspace_bytes(gce_plan_t plan);

/* Release the plan and its workspace (synchronises the device first). */
int gce_plan_destroy(gce_plan_t plan);

/* Human-readable text for a status code; for GCE_EHIP it includes the HIP
 * error of the calling thread's last failing call. */
const char *gce_status_string(int status);

/* Library version string ("gce-mi355x 0.4.0 (gfx950)"; 0.2.0 appended
 * mag_overlap to gce_opts and to gce_autotune's arguments, 0.3.0 appended
 * waves_per_unit to gce_opts and to gce_plan_info_t, 0.4.0 appended
 * refine_units to both). */
const char *gce_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GCE_H */
