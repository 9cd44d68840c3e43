"""Split-precision path (FP32 Pdot term and binning, FP64 entropy).

Its bins approximate the FP64 reference, so the checks are:
  * self-consistency: every CE value equals Eq. (4) of the histogram the
    split binning produces (debug hook, same device bin code), to FP32
    output rounding;
  * against the FP64 oracle, the error band (tests/split_band.py): a sampled
    trial's histogram equals the oracle's unless one of its epochs has an
    oracle phase within the split path's proven error bound of a bin edge,
    and then differs by at most those epochs;
  * the recovered minimum: identical to the oracle's for curves with a
    signal, within 1e-5 of the oracle's minimum CE otherwise.
Katz et al. 2020, Sec. 2.3, Eqs. (3)-(4).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import synth
from gce_testlib import say, upload
from split_band import check_counts_in_band

pytestmark = pytest.mark.gpu


def _split_run(w, tq=0):
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    precision=gce.PRECISION_SPLIT_FP32, trials_per_lane=tq)
    cube, best = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    torch.cuda.synchronize()
    return plan, (t, m, P, Pd), cube.cpu().numpy(), gce.best_fields(best)


def _self_consistency(plan, dev, w, gcube, n_sample, seed):
    rng = np.random.default_rng(seed)
    ci = rng.integers(0, w.n_curves, n_sample)
    fi = rng.integers(0, w.periods.size * w.pdots.size, n_sample)
    cnt = plan.debug_counts(*dev, ci, fi).cpu().numpy().astype(np.uint32)
    assert np.all(cnt.sum(axis=(1, 2)) == w.lengths[ci])
    h_own = np.array([oracle.entropy(c) for c in cnt])
    q, p = np.divmod(fi, w.periods.size)
    h_gpu = gcube[ci, q, p].astype(np.float64)
    # FP32 output rounding plus FP64 entropy rounding
    assert np.all(np.abs(h_gpu - h_own) <= 2.0 ** -23 * np.abs(h_own) + 1e-12)
    return ci, fi, cnt


@pytest.mark.parametrize("n_phase,n_mag,tq", [
    (10, 5, 0), (10, 5, 2), (10, 5, 4), (20, 10, 0), (20, 10, 8), (15, 5, 4),
    (50, 10, 2), (7, 3, 8), (1, 1, 0), (100, 5, 1),
])
def test_split_self_consistent_and_close(n_phase, n_mag, tq):
    w = synth.random_curves(60 + n_phase + tq, [1, 2, 63, 64, 65, 300, 1000], n_freq=150,
                            n_pdots=7, n_phase=n_phase, n_mag=n_mag, pdot_scale=5e-9)
    say(f"[split] nph={n_phase} nmag={n_mag} tq={tq}")
    plan, dev, gcube, bf = _split_run(w, tq)
    ci, fi, cnt = _self_consistency(plan, dev, w, gcube, 600, n_phase)
    _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, n_phase,
                            n_mag, ci, fi, want_counts=True)
    band = check_counts_in_band(w, ci, fi, cnt, want, label=f"nph={n_phase} tq={tq}")
    say(f"[split] band {band}")
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots,
                                 n_phase, n_mag)
    # statistics over the split path's own (float) CE values
    own = gcube.astype(np.float64).reshape(w.n_curves, -1)
    assert np.allclose(bf["ce_mean"], own.mean(axis=1), rtol=0, atol=1e-12)
    assert np.allclose(bf["ce_std"], own.std(axis=1), rtol=1e-9, atol=1e-12)
    # the minimum the split path picks is (near) the FP64 minimum
    for c in range(w.n_curves):
        q, p = divmod(int(bf["flat_index"][c]), w.periods.size)
        assert oc[c, q, p] <= obc[c] + 1e-5 or bf["flat_index"][c] == obf[c], c


def test_split_overlap_self_consistent():
    w = synth.random_curves(95, [2, 64, 300, 1000], n_freq=150, n_pdots=7, pdot_scale=5e-9)
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, 10, 5,
                    precision=gce.PRECISION_SPLIT_FP32, phase_overlap=True)
    cube, best = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    torch.cuda.synchronize()
    g = cube.cpu().numpy()
    rng = np.random.default_rng(3)
    ci = rng.integers(0, w.n_curves, 500)
    fi = rng.integers(0, w.periods.size * w.pdots.size, 500)
    cnt = plan.debug_counts(t, m, P, Pd, ci, fi).cpu().numpy().astype(np.uint32)
    assert np.all(cnt.sum(axis=(1, 2)) == 2 * w.lengths[ci])
    h_own = np.array([oracle.entropy(c) for c in cnt])
    q, p = np.divmod(fi, w.periods.size)
    assert np.all(np.abs(g[ci, q, p] - h_own) <= 2.0 ** -23 * np.abs(h_own) + 1e-12)
    _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 5, ci, fi,
                            want_counts=True, phase_overlap=True)
    band = check_counts_in_band(w, ci, fi, cnt, want, phase_overlap=True, label="overlap")
    say(f"[split] overlap band {band}")


@pytest.mark.parametrize("co", [1, 2])
def test_split_both_overlaps_in_band(co):
    """Overlapping phase and magnitude bins at once, one and two waves per
    unit: each CE value is Eq. (4) of its split histogram, which holds the
    oracle's entries (two phase bins per epoch, one or two magnitude rows),
    and the histogram differs from the oracle's only through band epochs."""
    w = synth.random_curves(96 + co, [3, 64, 257, 900], n_freq=150, n_pdots=5,
                            n_phase=20, n_mag=6, pdot_scale=5e-9)
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    precision=gce.PRECISION_SPLIT_FP32, phase_overlap=True,
                    mag_overlap=True, waves_per_unit=co, trials_per_lane=4)
    assert plan.info()["waves_per_unit"] == co
    cube, _ = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    torch.cuda.synchronize()
    g = cube.cpu().numpy()
    rng = np.random.default_rng(11 + co)
    ci = rng.integers(0, w.n_curves, 400)
    fi = rng.integers(0, w.periods.size * w.pdots.size, 400)
    cnt = plan.debug_counts(t, m, P, Pd, ci, fi).cpu().numpy().astype(np.uint32)
    _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                            w.n_mag, ci, fi, want_counts=True, phase_overlap=True,
                            mag_overlap=True)
    assert np.array_equal(cnt.sum(axis=(1, 2)), want.sum(axis=(1, 2)))
    h_own = np.array([oracle.entropy(c) for c in cnt])
    q, p = np.divmod(fi, w.periods.size)
    assert np.all(np.abs(g[ci, q, p] - h_own) <= 2.0 ** -23 * np.abs(h_own) + 1e-12)
    band = check_counts_in_band(w, ci, fi, cnt, want, phase_overlap=True, mag_overlap=True,
                                label=f"both overlaps co={co}")
    say(f"[split] both overlaps co={co} band {band}")
    plan.close()


def test_split_lds_limit_is_reported():
    # 128 phase bins: one trial pair's histogram and marginals fill 64 KiB of
    # LDS, as on the FP64 path; two pairs exceed it
    plan = gce.Plan(np.array([0, 10]), 5, 1, 128, 5, precision=gce.PRECISION_SPLIT_FP32,
                    trials_per_lane=1)
    assert plan.info()["lds_bytes_per_wave"] == 64 * 1024
    plan.close()
    with pytest.raises(gce.GceError) as ei:
        gce.Plan(np.array([0, 10]), 5, 8, 128, 5, precision=gce.PRECISION_SPLIT_FP32,
                 trials_per_lane=4)
    assert ei.value.status == -6


def test_split_c2_slice_agreement():
    """Eight curves of the batched workload, full 20,000 x 64 grid."""
    w = synth.make_config(2).subset(np.arange(8))
    say("[split] c2 slice")
    plan, dev, gcube, bf = _split_run(w)
    ci, fi, cnt = _self_consistency(plan, dev, w, gcube, 3000, 7)
    _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                            w.n_mag, ci, fi, want_counts=True)
    band = check_counts_in_band(w, ci, fi, cnt, want, label="c2 slice")
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots,
                                 w.n_phase, w.n_mag)
    dh = np.abs(gcube.astype(np.float64) - oc)
    frac_bad = float(np.mean(dh > 1e-5))
    say(f"[split] c2 slice: max|dH|={dh.max():.3e} frac(|dH|>1e-5)={frac_bad:.3e} "
        f"band {band} strict best {np.sum(bf['flat_index'] == obf)}/8")
    # a CE value moves only if an epoch of its trial lies in the band; the
    # union bound over the sampled trials bounds how often that happens
    assert frac_bad <= band["union_bound_mean"]
    # every curve of this workload carries an eclipse signal: same minimum
    assert np.array_equal(bf["flat_index"], obf)


def test_split_constant_and_invalid():
    w = synth.random_curves(70, [1, 40, 50], n_freq=70, n_pdots=3)
    w.mags[w.offsets[1]:w.offsets[2]] = 3.0
    w.mags[w.offsets[2] + 3] = np.inf
    plan, dev, gcube, bf = _split_run(w)
    assert np.all(gcube[0] == 0.0) and np.all(gcube[1] == 0.0)
    assert bf["flat_index"][0] == 0 and bf["flat_index"][1] == 0
    assert bf["flat_index"][2] == -1 and np.all(np.isnan(gcube[2]))


def test_split_random_shapes_self_consistent():
    """Seeded random shapes on the split path, every option drawn at once:
    each sampled CE value is Eq. (4) of the split path's own histogram (to
    float output rounding), histogram totals are the curve's entries, and the
    bins agree with the FP64 oracle's except for epochs in the error band."""
    rng = np.random.default_rng(6866)
    ran = 0
    for case in range(24):
        n_phase = int(rng.choice([1, 2, 7, 10, 15, 20, 33, 50, 64]))
        n_mag = int(rng.choice([1, 2, 5, 10, 17, 255]))
        tq = int(rng.choice([0, 1, 2, 4, 8]))
        placement = int(rng.choice([gce.TABLE_AUTO, gce.TABLE_GLOBAL, gce.TABLE_LDS]))
        po, mo = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
        lengths = [int(x) for x in rng.integers(1, 700, int(rng.integers(1, 6)))]
        w = synth.random_curves(2000 + case, lengths, n_freq=int(rng.integers(1, 120)),
                                n_pdots=int(rng.integers(1, 6)), n_phase=n_phase,
                                n_mag=n_mag, pdot_scale=5e-9)
        label = (f"case {case}: bins {n_phase}x{n_mag} tq={tq} table={placement} "
                 f"overlap={po}/{mo} N={lengths}")
        t, m, P, Pd = upload(w)
        try:
            plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, n_phase, n_mag,
                            precision=gce.PRECISION_SPLIT_FP32, trials_per_lane=tq,
                            phase_overlap=po, mag_overlap=mo, table_placement=placement)
        except gce.GceError as e:
            assert e.status == -6, (label, e)
            continue
        say(f"[split random] {label}")
        cube, best = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
        torch.cuda.synchronize()
        g = cube.cpu().numpy()
        n_tr = w.periods.size * w.pdots.size
        ci = rng.integers(0, w.n_curves, 96)
        fi = rng.integers(0, n_tr, 96)
        cnt = plan.debug_counts(t, m, P, Pd, ci, fi).cpu().numpy().astype(np.uint32)
        _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, n_phase,
                                n_mag, ci, fi, want_counts=True, phase_overlap=po,
                                mag_overlap=mo)
        assert np.array_equal(cnt.sum(axis=(1, 2)), want.sum(axis=(1, 2))), label
        h_own = np.array([oracle.entropy(c) for c in cnt])
        q, p = np.divmod(fi, w.periods.size)
        assert np.all(np.abs(g[ci, q, p] - h_own) <= 2.0 ** -23 * np.abs(h_own) + 1e-12), label
        check_counts_in_band(w, ci, fi, cnt, want, phase_overlap=po, mag_overlap=mo,
                             label=label)
        plan.close()
        ran += 1
    assert ran >= 15


def test_split_range_limits_mark_curves_invalid():
    """The split path forms x^2 = (t - t0)^2 / P^2 in FP32, so its plans take
    periods of at least 1e-6 d and spans of at most 1e10 d: a shorter period
    invalidates the grid (every curve), a longer span its curve, where the
    FP64 path accepts both.  Debug counts of valid split trials still total
    the curve's epochs."""
    w = synth.random_curves(71, [30, 40, 50], n_freq=16, n_pdots=2)
    wp = synth.Workload(w.name, w.times, w.mags, w.offsets, w.periods.copy(), w.pdots,
                        w.n_phase, w.n_mag)
    wp.periods[5] = 5e-7
    for prec, valid in ((gce.PRECISION_FP64, True), (gce.PRECISION_SPLIT_FP32, False)):
        t, m, P, Pd = upload(wp)
        plan = gce.Plan(wp.offsets, wp.periods.size, wp.pdots.size, wp.n_phase, wp.n_mag,
                        precision=prec)
        _, best = plan.execute(t, m, P, Pd)
        torch.cuda.synchronize()
        bf = gce.best_fields(best)
        assert np.all((bf["flat_index"] >= 0) == valid), (prec, bf["flat_index"])
        plan.close()
    ws = synth.Workload(w.name, w.times.copy(), w.mags, w.offsets, w.periods, w.pdots,
                        w.n_phase, w.n_mag)
    ws.times[ws.offsets[1]] -= 2e10   # curve 1 spans over 2e10 days
    for prec, want in ((gce.PRECISION_FP64, [True, True, True]),
                       (gce.PRECISION_SPLIT_FP32, [True, False, True])):
        t, m, P, Pd = upload(ws)
        plan = gce.Plan(ws.offsets, ws.periods.size, ws.pdots.size, ws.n_phase, ws.n_mag,
                        precision=prec)
        _, best = plan.execute(t, m, P, Pd)
        torch.cuda.synchronize()
        bf = gce.best_fields(best)
        assert (bf["flat_index"] >= 0).tolist() == want, (prec, bf["flat_index"])
        if prec == gce.PRECISION_SPLIT_FP32:
            ci = np.array([0, 2, 0, 2])
            fi = np.array([0, 5, 17, 31])
            cnt = plan.debug_counts(t, m, P, Pd, ci, fi).cpu().numpy()
            assert np.array_equal(cnt.sum(axis=(1, 2)), ws.lengths[ci])
        plan.close()
