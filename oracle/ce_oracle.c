/*
 * ce_oracle.c -- plain FP64 CPU reference of the conditional-entropy (CE)
 * search over period P and period derivative Pdot (Katz et al.,
 * arXiv:2006.06866, Sec. 2.3 "Conditional Entropy Implementation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * Every function is written for readability: one trial at a time, the fold of
 * Eq. (3) point by point, the entropy of Eq. (4) term by term.  Arithmetic is
 * IEEE double; build with -O2 -ffp-contract=off and without fast-math so the
 * operation sequence below is exactly what executes.
 *
 * Readings of the paper taken here (the paper is silent on these points):
 *   - time origin: t0 = the earliest epoch of the curve, dt = t - t0;
 *   - magnitude normalisation: the curve's magnitudes are mapped linearly onto
 *     [0, 1] by their min and max and cut into n_mag equal-width bins; the
 *     median/std scaling of Sec. 2.3 is affine and so leaves these bins alone;
 *   - right edges (m = m_max, phase rounding up to 1) fall in the last bin;
 *   - 50%-overlapping magnitude bins: the n_mag bins then have width
 *     2 / (n_mag + 1) and start every 1 / (n_mag + 1), so they tile [0, 1]
 *     with each bin sharing half of itself with each neighbour; an epoch in
 *     the first or last half-bin is in one bin, every other epoch in two.
 *     Probabilities of Eq. (4) are counts over the total count of the
 *     histogram (the same divisor as N, or 2N, without magnitude overlap);
 *   - the phase bin is floor(phi * n_phase) of the exact product (the
 *     computed phase phi itself is the rounded fold of Eq. (3)), and the
 *     magnitude bin likewise floor(u * n_mag) of the exact product with the
 *     normalised magnitude u (itself a rounded quotient): equal-width bins
 *     of the value at hand, not of a rounding of the product;
 *   - empty histogram cells contribute nothing to Eq. (4);
 *   - the minimum over the grid is the first strict minimum in flat order
 *     flat = q * n_periods + p (Pdot index q outer, period index p inner);
 *   - a curve whose epochs or magnitudes are not all finite is invalid: its
 *     best index is -1, its CE values and best CE are NaN.
 *
 * Parity pins: every function here is pinned by the CPU tests (hand-counted
 * histograms, exact dyadic folds, closed-form entropies, the library Shannon
 * entropy identity, brute force over tiny grids, injected-signal recovery).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* ---------------------------------------------------------------------------
 * Equal-width bins of [0, 1] (Sec. 2.3): value v in [0, 1] lies in bin
 * floor(v * n), the floor taken of the exact product: v * n is split into its
 * rounded value p and the exact remainder v*n - p (one fused multiply-add,
 * the error-free product of Ogita, Rump and Oishi 2005), and a product that
 * rounds up onto an integer is moved back below it.  v = 1 (and a v that
 * rounds up to 1) falls in the last bin.
 * ------------------------------------------------------------------------- */
static int32_t equal_width_bin(double v, int32_t n_bins)
{
    double n = (double)n_bins;
    double p = v * n;
    double f = floor(p);
    /* floor(p) is the exact floor unless p rounded up onto an integer */
    if (f == p && fma(v, n, -p) < 0.0)   /* v * n == p + remainder */
        f -= 1.0;
    int32_t b = (int32_t)f;
    if (b >= n_bins) b = n_bins - 1;
    return b;
}

/* ---------------------------------------------------------------------------
 * Sec. 2.3: magnitudes normalised per light curve, then binned into n_mag
 * magnitude bins.  u = (m - m_min) / (m_max - m_min) lies in [0, 1].
 *   disjoint bins (overlap = 0): bin j is [j, j + 1) / n_mag, so the epoch
 *     is in bin floor(u * n_mag); bin2 (if not NULL) is -1;
 *   50%-overlapping bins (overlap = 1): bin j is [j, j + 2) / (n_mag + 1);
 *     with s = floor(u * (n_mag + 1)) the epoch lies in the sub-interval
 *     [s, s + 1) / (n_mag + 1), which belongs to bins s - 1 and s where
 *     those exist: bin[k] is the lower of them, bin2[k] the other or -1.
 * u = 1 (m = m_max) counts as inside the last sub-interval.  A constant curve
 * has every epoch in bin 0 alone.  Returns 0, or ORACLE_EINVAL for n <= 0 /
 * n_mag < 1 / overlap with bin2 NULL, or 1 if a magnitude is not finite.
 * ------------------------------------------------------------------------- */
int ce_oracle_mag_bins2(const double *mags, int64_t n, int32_t n_mag,
                        int32_t overlap, int32_t *bin, int32_t *bin2)
{
    if (n <= 0 || n_mag < 1 || !mags || !bin || (overlap && !bin2))
        return ORACLE_EINVAL;
    double lo = mags[0], hi = mags[0];
    for (int64_t k = 0; k < n; ++k) {
        if (!isfinite(mags[k]))
            return 1;
        if (mags[k] < lo) lo = mags[k];
        if (mags[k] > hi) hi = mags[k];
    }
    for (int64_t k = 0; k < n; ++k) {
        if (bin2)
            bin2[k] = -1;
        if (hi == lo) {
            bin[k] = 0;          /* constant curve: one magnitude bin */
            continue;
        }
        double u = (mags[k] - lo) / (hi - lo); /* normalised to [0, 1] */
        if (!overlap) {
            bin[k] = equal_width_bin(u, n_mag);  /* m == m_max: last bin */
            continue;
        }
        /* sub-interval of width 1 / (n_mag + 1); m == m_max: the last one */
        int32_t s = equal_width_bin(u, n_mag + 1);
        if (s == 0) {                 /* first half-bin: bin 0 only */
            bin[k] = 0;
        } else if (s == n_mag) {      /* last half-bin: bin n_mag - 1 only */
            bin[k] = n_mag - 1;
        } else {                      /* bins s - 1 and s */
            bin[k] = s - 1;
            bin2[k] = s;
        }
    }
    return ORACLE_OK;
}

/* Disjoint magnitude bins only (the original interface). */
int ce_oracle_mag_bins(const double *mags, int64_t n, int32_t n_mag,
                       int32_t *bin)
{
    return ce_oracle_mag_bins2(mags, n, n_mag, 0, bin, NULL);
}

/* ---------------------------------------------------------------------------
 * Sec. 2.3: n_phase equal-width phase bins; phase phi lies in bin
 * floor(phi * n_phase) of the exact product.  A phase that rounds up to 1
 * falls in the last bin.
 * ------------------------------------------------------------------------- */
static int32_t phase_bin(double phi, int32_t n_phase)
{
    return equal_width_bin(phi, n_phase);
}

/* ---------------------------------------------------------------------------
 * Eq. (3): the quadratic phase fold.  With x = dt / P the folded phase is
 *     phi = frac( x - (1/2) * Pdot * x^2 ),
 * which is Eq. (3) divided through by P.  1/P is taken once per trial by a
 * correctly rounded division; (1/2)*Pdot is exact.  The square of x is formed
 * first and the Pdot term is applied with one fused multiply-add.
 * Returns the phase bin in [0, n_phase).
 * ------------------------------------------------------------------------- */
static double fold_phase(double dt, double inv_p, double half_pdot)
{
    double x = dt * inv_p;
    double x2 = x * x;
    double y = fma(-half_pdot, x2, x);
    return y - floor(y);
}

static int32_t fold_bin(double dt, double inv_p, double half_pdot,
                        int32_t n_phase)
{
    return phase_bin(fold_phase(dt, inv_p, half_pdot), n_phase);
}

/* The classic P-only fold (Pdot absent): phi = frac(dt / P). */
static int32_t fold_bin_ponly(double dt, double inv_p, int32_t n_phase)
{
    double y = dt * inv_p;
    double phi = y - floor(y);
    return phase_bin(phi, n_phase);
}

/* ---------------------------------------------------------------------------
 * Eq. (3) phases of one curve's n epochs under one (P, Pdot) trial, with the
 * curve's earliest epoch as time origin: out_phi[k] in [0, 1) (a phase that
 * rounds up to 1 is returned as 1.0 and binned into the last bin).
 * Returns 0, ORACLE_EINVAL, or 1 if an epoch is not finite.
 * ------------------------------------------------------------------------- */
int ce_oracle_phases(const double *times, int64_t n, double period, double pdot,
                     double *out_phi)
{
    if (n <= 0 || !times || !out_phi)
        return ORACLE_EINVAL;
    double t0 = times[0];
    for (int64_t k = 0; k < n; ++k) {
        if (!isfinite(times[k]))
            return 1;
        if (times[k] < t0) t0 = times[k];
    }
    double inv_p = 1.0 / period, half_pdot = 0.5 * pdot;
    for (int64_t k = 0; k < n; ++k)
        out_phi[k] = fold_phase(times[k] - t0, inv_p, half_pdot);
    return ORACLE_OK;
}

/* Exposed for the exact-arithmetic fold tests. */
int32_t ce_oracle_fold_bin(double dt, double period, double pdot,
                           int32_t n_phase)
{
    return fold_bin(dt, 1.0 / period, 0.5 * pdot, n_phase);
}

/* ---------------------------------------------------------------------------
 * Eq. (4): H_c = sum_{i,j} p(m_i, phi_j) ln( p(phi_j) / p(m_i, phi_j) ),
 * with p(m_i, phi_j) = c[i][j] / N and p(phi_j) = sum_i c[i][j] / N.
 * counts is [n_mag][n_phase] (magnitude bin i outer, phase bin j inner).
 * Phase bin outer, magnitude bin inner; cells with c = 0 are skipped.
 * ------------------------------------------------------------------------- */
double ce_oracle_entropy(const uint32_t *counts, int32_t n_mag,
                         int32_t n_phase)
{
    double total = 0.0;
    for (int32_t i = 0; i < n_mag; ++i)
        for (int32_t j = 0; j < n_phase; ++j)
            total += (double)counts[(int64_t)i * n_phase + j];
    if (total <= 0.0)
        return NAN;
    double h = 0.0;
    for (int32_t j = 0; j < n_phase; ++j) {
        double col = 0.0;
        for (int32_t i = 0; i < n_mag; ++i)
            col += (double)counts[(int64_t)i * n_phase + j];
        double p_phi = col / total;
        for (int32_t i = 0; i < n_mag; ++i) {
            uint32_t c = counts[(int64_t)i * n_phase + j];
            if (c == 0)
                continue;
            double p_joint = (double)c / total;
            h += p_joint * log(p_phi / p_joint);
        }
    }
    return h;
}

/* Per-curve preparation shared by the search entry points below. */
typedef struct {
    int64_t n;
    double *dt;        /* t - t0 */
    int32_t *mbin;     /* magnitude bin of each epoch */
    int32_t *mbin2;    /* second magnitude bin (overlapping bins) or -1 */
    int valid;
} curve_prep;

/* bits of the `overlap` arguments below */
#define OVERLAP_PHASE 1
#define OVERLAP_MAG 2

static int prep_curve(const double *t, const double *m, int64_t n,
                      int32_t n_mag, int overlap, curve_prep *cp)
{
    cp->n = n;
    cp->valid = 1;
    cp->dt = (double *)malloc((size_t)n * sizeof(double));
    cp->mbin = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    cp->mbin2 = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!cp->dt || !cp->mbin || !cp->mbin2)
        return ORACLE_ENOMEM;
    double t0 = t[0];
    for (int64_t k = 0; k < n; ++k) {
        if (!isfinite(t[k]))
            cp->valid = 0;
        if (t[k] < t0) t0 = t[k];
    }
    for (int64_t k = 0; k < n; ++k)
        cp->dt[k] = t[k] - t0;
    if (ce_oracle_mag_bins2(m, n, n_mag, (overlap & OVERLAP_MAG) != 0, cp->mbin,
                            cp->mbin2) != ORACLE_OK)
        cp->valid = 0;
    return ORACLE_OK;
}

static void free_prep(curve_prep *cp)
{
    free(cp->dt);
    free(cp->mbin);
    free(cp->mbin2);
    cp->dt = NULL;
    cp->mbin = NULL;
    cp->mbin2 = NULL;
}

/* Histogram of one trial: counts[n_mag][n_phase] is cleared and filled.
 * With overlapping phase bins (bit OVERLAP_PHASE), phase bin k spans
 * [k, k + 2) / n_phase (wrapping), i.e. each bin overlaps each neighbour by
 * half (Sec. 2.3): an epoch whose phase lies in [b, b + 1) / n_phase is inside
 * bins b and b - 1 (mod n_phase), so every epoch is counted in two phase bins.
 * With overlapping magnitude bins (bit OVERLAP_MAG) an epoch is counted in
 * each magnitude bin that contains it (one or two). */
static void trial_counts(const curve_prep *cp, double inv_p, double half_pdot,
                         int ponly, int overlap, int32_t n_phase, int32_t n_mag,
                         uint32_t *counts)
{
    memset(counts, 0, (size_t)n_mag * (size_t)n_phase * sizeof(uint32_t));
    for (int64_t k = 0; k < cp->n; ++k) {
        int32_t b = ponly ? fold_bin_ponly(cp->dt[k], inv_p, n_phase)
                          : fold_bin(cp->dt[k], inv_p, half_pdot, n_phase);
        int32_t prev = (b == 0) ? n_phase - 1 : b - 1;
        int32_t mb[2] = {cp->mbin[k], cp->mbin2[k]};
        for (int i = 0; i < 2; ++i) {
            if (mb[i] < 0)
                continue;
            counts[(int64_t)mb[i] * n_phase + b] += 1;
            if (overlap & OVERLAP_PHASE)
                counts[(int64_t)mb[i] * n_phase + prev] += 1;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Histogram of one (curve, P, Pdot) trial, as used by Eq. (4).
 * times/mags hold the curve's n epochs; counts is [n_mag][n_phase];
 * overlap holds the bits described at ce_oracle_search.
 * Returns 0, ORACLE_EINVAL, or 1 if the curve is invalid (non-finite data).
 * ------------------------------------------------------------------------- */
int ce_oracle_counts(const double *times, const double *mags, int64_t n,
                     double period, double pdot, int32_t n_phase,
                     int32_t n_mag, int32_t overlap, uint32_t *counts)
{
    if (n <= 0 || n_phase < 1 || n_mag < 1 || !times || !mags || !counts)
        return ORACLE_EINVAL;
    curve_prep cp;
    if (prep_curve(times, mags, n, n_mag, overlap, &cp) != ORACLE_OK) {
        free_prep(&cp);
        return ORACLE_ENOMEM;
    }
    int rc = cp.valid ? ORACLE_OK : 1;
    if (cp.valid)
        trial_counts(&cp, 1.0 / period, 0.5 * pdot, 0, overlap, n_phase, n_mag,
                     counts);
    free_prep(&cp);
    return rc;
}

static int check_offsets(const int64_t *off, int64_t n_curves)
{
    if (!off || n_curves < 1 || off[0] != 0)
        return ORACLE_EINVAL;
    for (int64_t c = 0; c < n_curves; ++c)
        if (off[c + 1] <= off[c])
            return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * The full grid search of Sec. 2.3: for every curve c, Pdot index q and
 * period index p, H_c of Eq. (4) after the fold of Eq. (3).
 *   times, mags      : [off[n_curves]] epochs and magnitudes, curve-major
 *   off              : [n_curves + 1] curve offsets, off[0] = 0, increasing
 *   periods, pdots   : [n_p], [n_pd] search grid (days, dimensionless)
 *   out_ce           : [n_curves][n_pd][n_p] or NULL
 *   best_flat        : [n_curves] first strict minimum, flat = q*n_p + p
 *   best_ce          : [n_curves] H_c at best_flat
 *   ponly            : nonzero => classic P-only fold, pdots ignored (n_pd
 *                      is still the size of the q axis of out_ce)
 *   overlap          : bit 0 (1): 50%-overlapping phase bins; bit 1 (2):
 *                      50%-overlapping magnitude bins
 *   n_threads        : OpenMP threads over (curve, q); <= 0 = runtime default
 * The result does not depend on n_threads.
 * ------------------------------------------------------------------------- */
static int search_impl(const double *times, const double *mags,
                       const int64_t *off, int64_t n_curves,
                       const double *periods, int64_t n_p,
                       const double *pdots, int64_t n_pd, int32_t n_phase,
                       int32_t n_mag, double *out_ce, int64_t *best_flat,
                       double *best_ce, int ponly, int overlap,
                       int32_t n_threads)
{
    if (!times || !mags || !periods || (!pdots && !ponly) || !best_flat ||
        !best_ce || n_p < 1 || n_pd < 1 || n_phase < 1 || n_mag < 1)
        return ORACLE_EINVAL;
    if (check_offsets(off, n_curves) != ORACLE_OK)
        return ORACLE_EINVAL;

    curve_prep *cps = (curve_prep *)calloc((size_t)n_curves, sizeof(curve_prep));
    if (!cps)
        return ORACLE_ENOMEM;
    int rc = ORACLE_OK;
    for (int64_t c = 0; c < n_curves && rc == ORACLE_OK; ++c)
        rc = prep_curve(times + off[c], mags + off[c], off[c + 1] - off[c],
                        n_mag, overlap, &cps[c]);
    /* A grid value that is not a finite positive period, or a non-finite
     * Pdot, invalidates every curve. */
    int grid_ok = 1;
    for (int64_t p = 0; p < n_p; ++p)
        if (!isfinite(periods[p]) || !(periods[p] > 0.0))
            grid_ok = 0;
    if (!ponly)
        for (int64_t q = 0; q < n_pd; ++q)
            if (!isfinite(pdots[q]))
                grid_ok = 0;

    /* per (curve, q) minimum, merged in flat order afterwards */
    double *row_min = (double *)malloc((size_t)(n_curves * n_pd) * sizeof(double));
    int64_t *row_arg = (int64_t *)malloc((size_t)(n_curves * n_pd) * sizeof(int64_t));
    if (rc != ORACLE_OK || !row_min || !row_arg) {
        rc = ORACLE_ENOMEM;
        goto done;
    }

    int64_t n_rows = n_curves * n_pd;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int alloc_fail = 0;
#pragma omp parallel
    {
        uint32_t *counts = (uint32_t *)malloc((size_t)n_mag * (size_t)n_phase *
                                              sizeof(uint32_t));
        if (!counts) {
#pragma omp atomic write
            alloc_fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n_rows; ++r) {
            if (!counts)
                continue;
            int64_t c = r / n_pd, q = r % n_pd;
            const curve_prep *cp = &cps[c];
            double *row = out_ce ? out_ce + r * n_p : NULL;
            double hmin = NAN;
            int64_t pmin = -1;
            if (!cp->valid || !grid_ok) {
                if (row)
                    for (int64_t p = 0; p < n_p; ++p)
                        row[p] = NAN;
            } else {
                double half_pdot = ponly ? 0.0 : 0.5 * pdots[q];
                for (int64_t p = 0; p < n_p; ++p) {
                    double inv_p = 1.0 / periods[p];
                    trial_counts(cp, inv_p, half_pdot, ponly, overlap, n_phase,
                                 n_mag, counts);
                    double h = ce_oracle_entropy(counts, n_mag, n_phase);
                    if (row)
                        row[p] = h;
                    if (pmin < 0 || h < hmin) {
                        hmin = h;
                        pmin = p;
                    }
                }
            }
            row_min[r] = hmin;
            row_arg[r] = pmin;
        }
        free(counts);
    }
    if (alloc_fail) {
        rc = ORACLE_ENOMEM;
        goto done;
    }
    for (int64_t c = 0; c < n_curves; ++c) {
        best_flat[c] = -1;
        best_ce[c] = NAN;
        for (int64_t q = 0; q < n_pd; ++q) {
            int64_t r = c * n_pd + q;
            if (row_arg[r] < 0)
                continue;
            if (best_flat[c] < 0 || row_min[r] < best_ce[c]) {
                best_ce[c] = row_min[r];
                best_flat[c] = q * n_p + row_arg[r];
            }
        }
    }
done:
    for (int64_t c = 0; c < n_curves; ++c)
        free_prep(&cps[c]);
    free(cps);
    free(row_min);
    free(row_arg);
    return rc;
}

int ce_oracle_search(const double *times, const double *mags,
                     const int64_t *off, int64_t n_curves,
                     const double *periods, int64_t n_p, const double *pdots,
                     int64_t n_pd, int32_t n_phase, int32_t n_mag,
                     int32_t overlap, double *out_ce, int64_t *best_flat,
                     double *best_ce, int32_t n_threads)
{
    return search_impl(times, mags, off, n_curves, periods, n_p, pdots, n_pd,
                       n_phase, n_mag, out_ce, best_flat, best_ce, 0, overlap,
                       n_threads);
}

/* Classic CE over periods only (Pdot absent from the fold); out_ce is
 * [n_curves][n_p]. */
int ce_oracle_search_ponly(const double *times, const double *mags,
                           const int64_t *off, int64_t n_curves,
                           const double *periods, int64_t n_p,
                           int32_t n_phase, int32_t n_mag, double *out_ce,
                           int64_t *best_flat, double *best_ce,
                           int32_t n_threads)
{
    return search_impl(times, mags, off, n_curves, periods, n_p, NULL, 1,
                       n_phase, n_mag, out_ce, best_flat, best_ce, 1, 0,
                       n_threads);
}

/* ---------------------------------------------------------------------------
 * Selected trials only, for checks at sizes where the full cube is too slow:
 * trial t is curve curve_ids[t] at flat index flat_ids[t] = q*n_p + p.
 * out_ce[t] receives H_c; out_counts (optional) receives [n_mag][n_phase]
 * counts per trial.  OpenMP over trials.
 * ------------------------------------------------------------------------- */
int ce_oracle_trials(const double *times, const double *mags,
                     const int64_t *off, int64_t n_curves,
                     const double *periods, int64_t n_p, const double *pdots,
                     int64_t n_pd, int32_t n_phase, int32_t n_mag,
                     int32_t overlap, const int64_t *curve_ids,
                     const int64_t *flat_ids, int64_t n_trials, double *out_ce,
                     uint32_t *out_counts, int32_t n_threads)
{
    if (!times || !mags || !periods || !pdots || !curve_ids || !flat_ids ||
        !out_ce || n_p < 1 || n_pd < 1 || n_phase < 1 || n_mag < 1 ||
        n_trials < 0)
        return ORACLE_EINVAL;
    if (check_offsets(off, n_curves) != ORACLE_OK)
        return ORACLE_EINVAL;
    for (int64_t t = 0; t < n_trials; ++t)
        if (curve_ids[t] < 0 || curve_ids[t] >= n_curves || flat_ids[t] < 0 ||
            flat_ids[t] >= n_p * n_pd)
            return ORACLE_EINVAL;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int fail = 0;
    size_t cells = (size_t)n_mag * (size_t)n_phase;
#pragma omp parallel
    {
        uint32_t *counts = (uint32_t *)malloc(cells * sizeof(uint32_t));
        curve_prep cp;
        int64_t cur = -1;
        cp.dt = NULL;
        cp.mbin = NULL;
        cp.mbin2 = NULL;
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < n_trials; ++t) {
            if (!counts) {
#pragma omp atomic write
                fail = 1;
                continue;
            }
            int64_t c = curve_ids[t];
            if (c != cur) {
                free_prep(&cp);
                if (prep_curve(times + off[c], mags + off[c],
                               off[c + 1] - off[c], n_mag, overlap,
                               &cp) != ORACLE_OK) {
#pragma omp atomic write
                    fail = 1;
                    cur = -1;
                    continue;
                }
                cur = c;
            }
            int64_t q = flat_ids[t] / n_p, p = flat_ids[t] % n_p;
            int ok = cp.valid && isfinite(periods[p]) && periods[p] > 0.0 &&
                     isfinite(pdots[q]);
            if (!ok) {
                out_ce[t] = NAN;
                if (out_counts)
                    memset(out_counts + (size_t)t * cells, 0,
                           cells * sizeof(uint32_t));
                continue;
            }
            trial_counts(&cp, 1.0 / periods[p], 0.5 * pdots[q], 0, overlap,
                         n_phase, n_mag, counts);
            out_ce[t] = ce_oracle_entropy(counts, n_mag, n_phase);
            if (out_counts)
                memcpy(out_counts + (size_t)t * cells, counts,
                       cells * sizeof(uint32_t));
        }
        free_prep(&cp);
        free(counts);
    }
    return fail ? ORACLE_ENOMEM : ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Eq. (5) and its inputs: over one curve's n CE values, the mean, the
 * population standard deviation (two passes) and the significance
 * rho = (mean - min) / std, taken as 0 when std = 0.
 * ------------------------------------------------------------------------- */
int ce_oracle_significance(const double *values, int64_t n, double *mean,
                           double *std_dev, double *rho)
{
    if (!values || n < 1 || !mean || !std_dev || !rho)
        return ORACLE_EINVAL;
    double sum = 0.0, lo = values[0];
    for (int64_t i = 0; i < n; ++i) {
        sum += values[i];
        if (values[i] < lo) lo = values[i];
    }
    const double mu = sum / (double)n;
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i)
        ss += (values[i] - mu) * (values[i] - mu);
    const double sd = sqrt(ss / (double)n);
    *mean = mu;
    *std_dev = sd;
    *rho = sd > 0.0 ? (mu - lo) / sd : 0.0;
    return ORACLE_OK;
}

int ce_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
