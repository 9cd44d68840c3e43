"""Full-size workloads in the launch configuration the benchmark uses, checked
on sampled outputs the oracle computes one by one, and by properties that hold
at any size (the minimum is not beaten by any sampled trial; its neighbours
in P and Pdot are checked exactly).  Katz et al. 2020, Sec. 2.3.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import synth
from gce_testlib import say, upload, ce_tolerance, check_counts_exact
from split_band import argmin_gap_bound, check_counts_in_band

pytestmark = pytest.mark.gpu

_CACHE = {}


def _workload(cfg):
    if cfg not in _CACHE:
        _CACHE.clear()
        _CACHE[cfg] = synth.make_config(cfg)
    return _CACHE[cfg]


def _sample(w, bf, rng, n_random, n_curves_nb):
    n_p, n_pd = w.periods.size, w.pdots.size
    ci = list(rng.integers(0, w.n_curves, n_random))
    fi = list(rng.integers(0, n_p * n_pd, n_random))
    nb_curves = rng.choice(w.n_curves, size=min(n_curves_nb, w.n_curves), replace=False)
    for c in nb_curves:
        if bf["flat_index"][c] < 0:
            continue
        q0, p0 = divmod(int(bf["flat_index"][c]), n_p)
        for dq in range(-2, 3):
            for dp in range(-2, 3):
                q, p = q0 + dq, p0 + dp
                if 0 <= q < n_pd and 0 <= p < n_p:
                    ci.append(int(c))
                    fi.append(q * n_p + p)
        # and a column of random trials of the same curve
        for f in rng.integers(0, n_p * n_pd, 64):
            ci.append(int(c))
            fi.append(int(f))
    return np.array(ci, dtype=np.int64), np.array(fi, dtype=np.int64), nb_curves


@pytest.mark.parametrize("cfg", [2, 4, 5, 6])
def test_fullsize_fp64_sampled(cfg):
    """Configs 2, 4, 5 with the full CE cube; config 6 (the paper-scale grid,
    whose cube would be 179 GB) minimum-only, as the benchmark runs it."""
    w = _workload(cfg)
    say(f"[fullsize] config {cfg}: {w.n_curves} curves, {w.point_trials:.3g} point-trials")
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    phase_overlap=w.phase_overlap)
    say(f"[fullsize] plan {plan.info()}")
    cube = plan.new_cube() if cfg != 6 else None
    _, best = plan.execute(t, m, P, Pd, out_ce=cube)
    torch.cuda.synchronize()
    bf = gce.best_fields(best)
    assert np.all(bf["flat_index"] >= 0)
    rng = np.random.default_rng(100 + cfg)
    ci, fi, nb = _sample(w, bf, rng, 3000, 12)
    h = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase, w.n_mag,
                      ci, fi, phase_overlap=w.phase_overlap)
    if cube is not None:
        q, p = np.divmod(fi, w.periods.size)
        idx = torch.from_numpy(ci).cuda(), torch.from_numpy(q).cuda(), torch.from_numpy(p).cuda()
        g = cube[idx].cpu().numpy()
        del cube
        tol = ce_tolerance(h, w.n_phase, w.n_mag, w.lengths[ci])
        bad = np.abs(g - h) > tol
        assert not bad.any(), (f"{bad.sum()} sampled CE values off; first "
                               f"curve {ci[bad][0]} flat {fi[bad][0]}: {g[bad][0]} vs {h[bad][0]}")
    # the reported minimum is the CE at its trial, and no sampled trial of
    # that curve is lower
    for c in nb:
        sel = ci == c
        tol_c = ce_tolerance(bf["ce_min"][c], w.n_phase, w.n_mag, w.lengths[c])
        at = sel & (fi == bf["flat_index"][c])
        assert at.any() and abs(h[at][0] - bf["ce_min"][c]) <= tol_c
        assert np.all(h[sel] >= bf["ce_min"][c] - tol_c)
    check_counts_exact(plan, (t, m, P, Pd), w, ci[:600], fi[:600], f"config {cfg}")
    has = w.truth["inj_p"] >= 0
    found = np.sum((bf["period_index"] == w.truth["inj_p"]) & has)
    say(f"[fullsize] config {cfg}: injected period recovered for {found}/{has.sum()}")
    plan.close()


@pytest.mark.parametrize("cfg", [2, 4, 5, 6])
def test_fullsize_split_vs_fp64(cfg):
    """Split path at full size in the benchmark's launch configuration:
    sampled bins against the oracle's within the error band
    (tests/split_band.py), and minima against the FP64 path's (whose cube
    is checked against the oracle above): identical for every curve whose
    injected signal the FP64 search recovers; elsewhere the FP64 CE at the
    split minimum is within 1e-5 of the FP64 minimum or within the gap the
    band epochs of the two trials allow.  Config 6 (the paper-scale grid,
    no cube, overlapping phase bins): the sampled bins only."""
    w = _workload(cfg)
    say(f"[fullsize] split config {cfg}")
    t, m, P, Pd = upload(w)
    po = w.phase_overlap
    p32 = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                   precision=gce.PRECISION_SPLIT_FP32, phase_overlap=po)
    rng = np.random.default_rng(7)
    n_s = {2: 2000, 4: 2000, 5: 600, 6: 800}[cfg]
    ci = rng.integers(0, w.n_curves, n_s)
    fi = rng.integers(0, w.periods.size * w.pdots.size, n_s)
    if cfg == 6:
        _, b32 = p32.execute(t, m, P, Pd)
        torch.cuda.synchronize()
        c32 = p32.debug_counts(t, m, P, Pd, ci, fi).cpu().numpy()
        _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                                w.n_mag, ci, fi, want_counts=True, phase_overlap=po)
        band = check_counts_in_band(w, ci, fi, c32, want, phase_overlap=po,
                                    label=f"config {cfg}")
        assert np.all(gce.best_fields(b32)["flat_index"] >= 0)
        say(f"[fullsize] split config {cfg}: band {band}")
        p32.close()
        return
    p64 = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag)
    cube64 = p64.new_cube()
    _, b64 = p64.execute(t, m, P, Pd, out_ce=cube64)
    _, b32 = p32.execute(t, m, P, Pd)
    torch.cuda.synchronize()
    f64, f32 = gce.best_fields(b64), gce.best_fields(b32)
    at = cube64.view(w.n_curves, -1).gather(
        1, torch.from_numpy(f32["flat_index"]).cuda().view(-1, 1)).view(-1).cpu().numpy()
    del cube64
    tolerant = at - f64["ce_min"] <= 1e-5
    has = w.truth["inj_p"] >= 0
    found = has & (f64["period_index"] == w.truth["inj_p"]) & (
        f64["pdot_index"] == w.truth["inj_q"])
    strict = f64["flat_index"] == f32["flat_index"]
    c32 = p32.debug_counts(t, m, P, Pd, ci, fi).cpu().numpy()
    _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                            w.n_mag, ci, fi, want_counts=True)
    band = check_counts_in_band(w, ci, fi, c32, want, label=f"config {cfg}")
    say(f"[fullsize] split config {cfg}: best strict {strict.sum()}/{w.n_curves} "
        f"(signal recovered by FP64: {found.sum()}, of them strict "
        f"{np.sum(strict & found)}), tolerant {tolerant.sum()}; band {band}")
    assert np.all(strict[found])
    for c in np.flatnonzero(~tolerant):
        gap = at[c] - f64["ce_min"][c]
        bound = argmin_gap_bound(w, c, f32["flat_index"][c], f64["flat_index"][c])
        say(f"[fullsize] curve {c}: FP64 CE at the split minimum {gap:.3e} above the "
            f"FP64 minimum, band bound {bound:.3e}")
        assert gap <= bound, (c, gap, bound)
    p64.close()
    p32.close()
