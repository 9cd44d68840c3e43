"""The error band of the split-precision bins.

The split path forms x = (t - t0) / P and frac(x) in binary64 exactly as
the FP64 path does, then converts frac(x) to binary32, forms x^2 as the
binary32 product of dt^2 and (1/P)^2 (each rounded to float from binary64),
applies the Pdot term with one fma, reduces mod 1 and floors n * phase, every
binary32 step rounding toward minus infinity (the bin floor is of the exact
product).  Against the binary64 phase phi of Eq. (3), its phase differs by at
most, in cycles (|a| = |Pdot| / 2, A = |a| x^2 the Pdot term):
    frac(x) to float                 < 2^-24
    fract of a negative y            < 2^-24
    the rounding of y                < ulp(1 + A) <= 2^-23 (1 + A)
    the Pdot term (a, dt^2 and (1/P)^2 to float, their product)  < 4 * 2^-23 * A
    the binary64 rounding of phi itself              < 2^-52 (x + A)
i.e. below E = 2^-22 + 2^-20 A + 2^-52 x (0 at x = 0, where every step is
exact).  A split bin can therefore differ
from the binary64 bin only for an epoch whose binary64 phase lies within E of
a bin edge k / n_phase.  These helpers find those epochs with the oracle's
phases and check a split histogram against a reference histogram: identical
when no epoch of the trial is in the band, else differing by at most the
band's epochs (each counted once per magnitude bin that holds it).

Nothing here calls the HIP path; the CPU tests check the check itself on
histograms binned from phases moved within, and beyond, the band.
"""
import numpy as np

import oracle


def phase_error_bound(x, half_pdot):
    """Strict bound, in cycles, on the split phase's distance from the
    binary64 phase for x = (t - t0) / P and the trial's Pdot / 2.  At x = 0
    (the curve's first epoch) every step is exact and the bound is 0."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    a = abs(float(half_pdot))
    e = 2.0 ** -22 + 2.0 ** -20 * a * x * x + 2.0 ** -52 * x
    return np.where(x == 0.0, 0.0, e)


def edge_distance(phi, n_phase):
    """Distance, in cycles, from each phase to the nearest bin edge k / n
    (0 and 1 are the same edge)."""
    v = np.asarray(phi, dtype=np.float64) * n_phase
    return np.abs(v - np.rint(v)) / n_phase


def trial_band(times, period, pdot, n_phase):
    """(in_band, bound) per epoch of one curve under one trial."""
    t = np.asarray(times, dtype=np.float64)
    phi = oracle.phases(t, period, pdot)
    e = phase_error_bound((t - t.min()) / period, 0.5 * pdot)
    return edge_distance(phi, n_phase) < e, e


def entries_per_epoch(mags, n_mag, mag_overlap):
    """Histogram rows each epoch is counted in (1, or 2 for an epoch inside
    two overlapping magnitude bins)."""
    if not mag_overlap:
        return np.ones(np.asarray(mags).size, dtype=np.int64)
    _, b2 = oracle.mag_bins_overlap(mags, n_mag)
    return 1 + (np.asarray(b2) >= 0).astype(np.int64)


def check_counts_in_band(w, curve_ids, flat_ids, cnt_split, cnt_ref,
                         phase_overlap=False, mag_overlap=False, label=""):
    """Assert the band property on sampled trials; returns a summary dict:
    trials with an epoch in the band, histogram entries moved, and the mean
    over trials of the union bound sum_k 2 n E_k (capped at 1) on the chance
    that a trial of uniformly spread phases has an epoch in the band."""
    cs = np.asarray(cnt_split, dtype=np.int64)
    cr = np.asarray(cnt_ref, dtype=np.int64)
    n_p = w.periods.size
    near_trials, moved_total, ub = 0, 0.0, 0.0
    for i, (c, f) in enumerate(zip(np.asarray(curve_ids), np.asarray(flat_ids))):
        a, b = int(w.offsets[c]), int(w.offsets[c + 1])
        t, m = w.times[a:b], w.mags[a:b]
        if not (np.all(np.isfinite(t)) and np.all(np.isfinite(m))):
            continue
        q, p = divmod(int(f), n_p)
        near, e = trial_band(t, w.periods[p], w.pdots[q], w.n_phase)
        allow = int(entries_per_epoch(m, w.n_mag, mag_overlap)[near].sum())
        moved = np.abs(cs[i] - cr[i]).sum() / 2.0
        if allow == 0:
            assert moved == 0, (label, "bins moved with no epoch in the band", int(c), int(f))
        else:
            assert moved <= allow, (label, "more bins moved than epochs in the band",
                                    int(c), int(f), moved, allow)
            near_trials += 1
        moved_total += moved
        ub += min(1.0, float(np.sum(2.0 * w.n_phase * e)))
    n = max(1, len(curve_ids))
    return {"trials": len(curve_ids), "trials_with_band_epochs": near_trials,
            "entries_moved": moved_total, "union_bound_mean": ub / n}


def argmin_gap_bound(w, c, flat_split, flat_ref, phase_overlap=False, mag_overlap=False):
    """Bound on H64(split minimum) - H64(FP64 minimum) for curve c.

    A split CE value differs from the FP64 one only through histogram
    entries of band epochs; moving one entry between phase bins changes two
    cells and two marginals, each c ln c term by at most ln(T) + 1 for a
    histogram total T, so N H moves by at most 4 (ln T + 1) per entry.  The
    split value is minimal at its own minimum, so the FP64 gap is at most the
    movable entries of both trials times that, plus the float rounding of the
    two split values compared (1e-6 for H <= ln 255)."""
    a, b = int(w.offsets[c]), int(w.offsets[c + 1])
    t, m = w.times[a:b], w.mags[a:b]
    per = entries_per_epoch(m, w.n_mag, mag_overlap)
    total = float(per.sum()) * (2.0 if phase_overlap else 1.0)
    moved = 0
    for f in (flat_split, flat_ref):
        q, p = divmod(int(f), w.periods.size)
        near, _ = trial_band(t, w.periods[p], w.pdots[q], w.n_phase)
        moved += int(per[near].sum())
    return moved * 4.0 * (np.log(max(total, 2.0)) + 1.0) / total + 1e-6
