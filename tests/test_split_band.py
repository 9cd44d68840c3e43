"""CPU checks of the split-path band check (tests/split_band.py): histograms
binned from the oracle's phases moved by less than the error bound pass it,
and so do moves only of epochs inside the band; a single epoch moved from
outside the band fails it."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2006_06866_amd import synth
from split_band import (check_counts_in_band, edge_distance, phase_error_bound,
                        trial_band)


def _hist(phi, mags, n_phase, n_mag):
    mb = oracle.mag_bins(mags, n_mag)
    b = np.minimum(np.floor(np.asarray(phi) * n_phase).astype(np.int64), n_phase - 1)
    h = np.zeros((n_mag, n_phase), dtype=np.int64)
    np.add.at(h, (mb, b), 1)
    return h


def test_bound_terms():
    assert phase_error_bound(0.0, 1e-9) == 0.0
    assert phase_error_bound(1e-3, 0.0) == 2.0 ** -22 + 2.0 ** -52 * 1e-3
    # the Pdot term grows as x^2: 1e5 cycles at Pdot/2 = 5e-11 is 0.5 cycle
    e = phase_error_bound(1e5, 5e-11)
    assert math.isclose(e, 2.0 ** -22 + 2.0 ** -20 * 0.5 + 2.0 ** -52 * 1e5)
    assert edge_distance([0.0, 0.1, 0.99, 0.25], 10)[0] == 0.0
    assert np.allclose(edge_distance([0.1, 0.99, 0.25], 10), [0.0, 0.01, 0.05])


def test_check_accepts_moves_within_the_band_and_rejects_others():
    w = synth.random_curves(41, [200, 300, 500], n_freq=40, n_pdots=4, pdot_scale=1e-9)
    rng = np.random.default_rng(5)
    ci = rng.integers(0, w.n_curves, 60)
    fi = rng.integers(0, w.periods.size * w.pdots.size, 60)
    ref, moved_in_band, outside = [], [], []
    for c, f in zip(ci, fi):
        a, b = w.offsets[c], w.offsets[c + 1]
        t, m = w.times[a:b], w.mags[a:b]
        q, p = divmod(int(f), w.periods.size)
        phi = oracle.phases(t, w.periods[p], w.pdots[q])
        near, e = trial_band(t, w.periods[p], w.pdots[q], w.n_phase)
        ref.append(_hist(phi, m, w.n_phase, w.n_mag))
        # every phase moved by less than its bound (kept in [0, 1))
        shift = rng.uniform(-1.0, 1.0, phi.size) * e * 0.999
        moved_in_band.append(_hist(np.mod(phi + shift, 1.0), m, w.n_phase, w.n_mag))
        # one epoch outside the band moved by a whole bin
        k = int(np.flatnonzero(~near)[0])
        phi2 = phi.copy()
        phi2[k] = np.mod(phi2[k] + 1.0 / w.n_phase, 1.0)
        outside.append(_hist(phi2, m, w.n_phase, w.n_mag))
    s = check_counts_in_band(w, ci, fi, moved_in_band, ref, label="in band")
    assert s["trials"] == 60 and 0.0 <= s["union_bound_mean"] <= 1.0
    with pytest.raises(AssertionError):
        check_counts_in_band(w, ci[:1], fi[:1], outside[:1], ref[:1], label="outside")


def test_band_catches_a_phase_edge_epoch():
    """An epoch exactly on a bin edge is in the band, and so may move,
    except the first epoch, whose phase 0 both paths compute exactly."""
    t = np.array([0.0, 0.1, 0.35, 0.7])
    near, e = trial_band(t, 1.0, 0.0, 10)
    assert not near[0] and near[1] and not near[2] and near[3]


def test_one_moved_entry_changes_h_by_at_most_the_gap_bound():
    """Moving one histogram entry between phase bins (same magnitude row)
    changes H by at most 4 (ln T + 1) / T, T the histogram total: the
    per-entry term of argmin_gap_bound."""
    rng = np.random.default_rng(9)
    for _ in range(400):
        n_mag, n_phase = int(rng.integers(1, 6)), int(rng.integers(2, 12))
        h = rng.integers(0, 6, (n_mag, n_phase)).astype(np.uint32)
        h[rng.integers(0, n_mag), rng.integers(0, n_phase)] += 1
        j = int(rng.choice(np.flatnonzero(h.sum(axis=1) > 0)))
        b1 = int(rng.choice(np.flatnonzero(h[j] > 0)))
        b2 = int((b1 + rng.integers(1, n_phase)) % n_phase)
        g = h.copy()
        g[j, b1] -= 1
        g[j, b2] += 1
        t = float(h.sum())
        assert abs(oracle.entropy(g) - oracle.entropy(h)) <= 4.0 * (math.log(t) + 1.0) / t


def test_argmin_gap_bound_counts_band_epochs():
    from split_band import argmin_gap_bound
    w = synth.random_curves(43, [300], n_freq=8, n_pdots=1, pdot_scale=0.0)
    # a period grid point where no epoch is in the band gives the rounding
    # allowance alone; exact edges (t = k P / n) give more
    base = argmin_gap_bound(w, 0, 0, 0)
    assert base >= 1e-6
    t = w.times.copy()
    t[1:4] = t[0] + np.array([1, 2, 3]) * w.periods[0] / w.n_phase
    w2 = synth.Workload(w.name, t, w.mags, w.offsets, w.periods, w.pdots, w.n_phase, w.n_mag)
    assert argmin_gap_bound(w2, 0, 0, 0) > base


def _rd32(v):
    """binary32 rounding toward minus infinity of an exact rational v."""
    f = np.float32(float(v))            # round to nearest (via double)
    if Fraction(float(f)) > v:
        f = np.nextafter(f, np.float32(-np.inf))
    # the double rounding above can land one float32 step low only when v
    # lies exactly between; step back up while the next float32 is still <= v
    while Fraction(float(np.nextafter(f, np.float32(np.inf)))) <= v:
        f = np.nextafter(f, np.float32(np.inf))
    return f


def _split_phase(dt, period, pdot):
    """The split path's phase, step by step as the kernel computes it: x and
    frac(x) in binary64 (to nearest); dt^2 and (1/P)^2 formed in binary64
    and rounded to nearest float (the prepass, the work unit's set-up), and
    Pdot/2 rounded to nearest float; then every binary32 operation rounded
    toward minus infinity."""
    invp = 1.0 / period
    x = dt * invp
    f = x - math.floor(x)
    xf = _rd32(Fraction(f))
    d2f = np.float32(dt * dt)
    ip2f = np.float32(invp * invp)
    x2f = _rd32(Fraction(float(d2f)) * Fraction(float(ip2f)))
    ha = np.float32(0.5 * pdot)
    y = _rd32(Fraction(float(xf)) - Fraction(float(ha)) * Fraction(float(x2f)))
    return _rd32(Fraction(float(y)) - math.floor(float(y)))


def test_error_bound_holds_for_the_split_arithmetic():
    """The split phase (emulated exactly, rounding mode included) is within
    E = phase_error_bound of the oracle's binary64 phase, mod 1, on random
    trials whose Pdot term spans 0 to ~300 cycles, and on epochs at x = 0."""
    rng = np.random.default_rng(23)
    worst = 0.0
    for i in range(3000):
        period = 10 ** rng.uniform(-3.0, 0.0)
        dt = 0.0 if i % 50 == 0 else rng.uniform(0.0, 3650.0)
        pdot = rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(-14.0, -9.5)
        phi64 = oracle.phases(np.array([0.0, dt]), period, pdot)[1]
        ps = float(_split_phase(dt, period, pdot))
        d = abs(ps - phi64)
        d = min(d, 1.0 - d)
        e = float(phase_error_bound(dt / period, 0.5 * pdot))
        assert d < e or (e == 0.0 and d == 0.0), (dt, period, pdot, d, e)
        if e > 0:
            worst = max(worst, d / e)
    # the bound is not vacuous: the largest error uses a fair part of it
    assert 0.05 < worst < 1.0
