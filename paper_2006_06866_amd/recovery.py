"""Injection-recovery bookkeeping for searches over synthetic binaries.

Sec. 3.1: a period is recovered when it lies within about 10% of the true
period or of one of its harmonics (2, 1, 1/2, 1/3, 1/4 and 1/6 of it);
Sec. 3.2: a source is detected when its significance (Eq. (5)) is at least
10.  These are host-side summaries of the per-curve results.
"""
from __future__ import annotations

import numpy as np

HARMONICS = (2.0, 1.0, 0.5, 1.0 / 3.0, 0.25, 1.0 / 6.0)
REL_TOL = 0.10
DETECTION_THRESHOLD = 10.0


def harmonic_error(best_period, true_period, harmonics=HARMONICS):
    """Smallest relative distance |P_best / (h P_true) - 1| over harmonics h."""
    b = np.asarray(best_period, dtype=np.float64)[..., None]
    t = np.asarray(true_period, dtype=np.float64)[..., None]
    h = np.asarray(harmonics, dtype=np.float64)
    return np.min(np.abs(b / (h * t) - 1.0), axis=-1)


def recovered(best_period, true_period, rel_tol=REL_TOL, harmonics=HARMONICS):
    return harmonic_error(best_period, true_period, harmonics) <= rel_tol


def detected(significance, threshold=DETECTION_THRESHOLD):
    s = np.asarray(significance, dtype=np.float64)
    return np.isfinite(s) & (s >= threshold)


def summary(fields, periods, true_period, mask=None):
    """Counts of recovered and detected sources among the masked curves.

    fields: per-curve result fields (period_index, significance, ...);
    periods: the search grid; true_period: injected P0 per curve (days)."""
    pi = np.asarray(fields["period_index"])
    ok = pi >= 0
    best_p = np.where(ok, np.asarray(periods)[np.clip(pi, 0, None)], np.nan)
    rec = ok & recovered(best_p, true_period)
    exact = ok & (harmonic_error(best_p, true_period, (1.0,)) <= REL_TOL)
    det = detected(fields["significance"])
    m = np.ones(pi.size, dtype=bool) if mask is None else np.asarray(mask, dtype=bool)
    sig = np.asarray(fields["significance"], dtype=np.float64)[m]
    return {
        "curves": int(m.sum()),
        "recovered_harmonic": int((rec & m).sum()),
        "recovered_fundamental": int((exact & m).sum()),
        "detected_rho_ge_10": int((det & m).sum()),
        "median_significance": float(np.nanmedian(sig)) if sig.size else float("nan"),
    }
