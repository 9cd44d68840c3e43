"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

FP64 path contract: histogram counts bit-exact (debug-count hook), every CE
value within the derived tolerance, per-curve minima identical (or tied within
tolerance).  Katz et al. 2020, Sec. 2.3, Eqs. (3)-(4).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import synth
from gce_testlib import (say, to_dev, upload, ce_tolerance, run_gpu, assert_cube_close,
                         assert_best_valid, check_counts_exact)

pytestmark = pytest.mark.gpu


def _full_parity(w, label, trials_per_lane=0, counts_sample=400, seed=0,
                 phase_overlap=False, table_placement=0, mag_overlap=False):
    say(f"[parity] {label}: curves={w.n_curves} N={w.lengths.tolist()[:8]} "
        f"n_p={w.periods.size} n_pd={w.pdots.size} bins={w.n_phase}x{w.n_mag} "
        f"tq={trials_per_lane} overlap={phase_overlap}/{mag_overlap} table={table_placement}")
    plan, dev, cube, best = run_gpu(w, trials_per_lane=trials_per_lane,
                                    phase_overlap=phase_overlap,
                                    table_placement=table_placement,
                                    mag_overlap=mag_overlap)
    if table_placement:
        assert plan.info()["table_in_lds"] == int(table_placement == gce.TABLE_LDS)
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots,
                                 w.n_phase, w.n_mag, phase_overlap=phase_overlap,
                                 mag_overlap=mag_overlap)
    gc = cube.cpu().numpy()
    bf = gce.best_fields(best)
    cm = 2 if mag_overlap else 1
    assert_cube_close(gc, oc, w, label, count_mult=cm)
    assert_best_valid(bf["flat_index"], bf["ce_min"], obf, obc, oc, w, label, count_mult=cm)
    assert np.array_equal(bf["period_index"], bf["flat_index"] % w.periods.size)
    assert np.array_equal(bf["pdot_index"], bf["flat_index"] // w.periods.size)
    _check_statistics(bf, oc, w, label, count_mult=cm)
    rng = np.random.default_rng(seed)
    n_tr = w.periods.size * w.pdots.size
    ci = rng.integers(0, w.n_curves, counts_sample)
    fi = rng.integers(0, n_tr, counts_sample)
    ci = np.concatenate([ci, np.arange(w.n_curves)])
    fi = np.concatenate([fi, bf["flat_index"]])
    check_counts_exact(plan, dev, w, ci, fi, label)
    plan.close()


def _check_statistics(bf, oc, w, label, count_mult=1):
    """Eq. (5) inputs against the oracle's two-pass moments of its own cube:
    every CE value is within tol of the oracle's, so the mean and the
    population std are too (both are 1-Lipschitz in the max norm), plus
    summation rounding."""
    om, osd, orho = oracle.curve_statistics(oc)
    tol = ce_tolerance(np.abs(oc).reshape(w.n_curves, -1).max(axis=1), w.n_phase,
                       w.n_mag, count_mult * w.lengths)
    n = oc[0].size
    rnd = 4 * n * 2.0 ** -53 * np.abs(om) + 1e-15
    assert np.all(np.abs(bf["ce_mean"] - om) <= tol + rnd), label
    assert np.all(np.abs(bf["ce_std"] - osd) <= 2 * tol + rnd + 1e-12 * osd), label
    ok = osd > 1e-9
    rel = np.abs(bf["significance"][ok] - orho[ok]) / (1 + np.abs(orho[ok]))
    assert np.all(rel <= (4 * tol[ok] + rnd[ok]) / osd[ok] + 1e-9), label


def test_c1_single_curve_full():
    w = synth.make_config(1)
    _full_parity(w, "c1")
    # the injected period is recovered
    _, best = run_gpu(w, want_cube=False)[2:]
    assert gce.best_fields(best)["flat_index"][0] == w.truth["inj_p"][0]


EDGE_LENGTHS = [1, 2, 3, 63, 64, 65, 127, 300, 1000]


@pytest.mark.parametrize("n_phase,n_mag,tq", [
    (10, 5, 0), (10, 5, 1), (10, 5, 2), (10, 5, 4), (10, 5, 8),
    (15, 5, 0), (20, 10, 0), (20, 10, 8), (50, 10, 0), (50, 10, 4),
    (7, 3, 0), (7, 3, 8), (1, 1, 0), (2, 2, 0), (128, 5, 1), (33, 255, 2),
])
def test_ragged_small_grid(n_phase, n_mag, tq):
    w = synth.random_curves(20 + n_phase + 7 * tq, EDGE_LENGTHS, n_freq=150,
                            n_pdots=7, n_phase=n_phase, n_mag=n_mag, pdot_scale=5e-9)
    _full_parity(w, f"ragged nph={n_phase} nmag={n_mag}", trials_per_lane=tq)


@pytest.mark.parametrize("placement", [gce.TABLE_GLOBAL, gce.TABLE_LDS])
@pytest.mark.parametrize("n_phase,n_mag,tq", [
    (10, 5, 8), (50, 10, 4), (7, 3, 1), (20, 10, 2), (1, 1, 0),
])
def test_table_placement(n_phase, n_mag, tq, placement):
    """The c ln c table read from global memory or from a copy in each
    wave's LDS gives the same counts and CE values (curves up to 1,000
    epochs: the copy loop runs over several 64-lane strides and a tail)."""
    w = synth.random_curves(60 + n_phase + tq, EDGE_LENGTHS, n_freq=140,
                            n_pdots=5, n_phase=n_phase, n_mag=n_mag, pdot_scale=5e-9)
    _full_parity(w, f"table={placement} nph={n_phase}", trials_per_lane=tq,
                 table_placement=placement)
    _full_parity(w, f"table={placement} overlap nph={n_phase}", trials_per_lane=tq,
                 table_placement=placement, phase_overlap=True)


@pytest.mark.parametrize("precision", [gce.PRECISION_FP64, gce.PRECISION_SPLIT_FP32])
def test_table_placement_bitwise_equal(precision):
    """Both placements hold the same doubles and sum them in the same order,
    so every CE value and every minimum agrees bit for bit."""
    w = synth.random_curves(77, [1, 64, 65, 500, 1000], n_freq=200, n_pdots=9,
                            n_phase=50, n_mag=10, pdot_scale=5e-9)
    out = []
    for placement in (gce.TABLE_GLOBAL, gce.TABLE_LDS):
        plan, _, cube, best = run_gpu(w, precision=precision, table_placement=placement)
        out.append((cube, best))
        plan.close()
    assert torch.equal(out[0][0].view(torch.int32), out[1][0].view(torch.int32))
    assert torch.equal(out[0][1].view(torch.int64), out[1][1].view(torch.int64))


def test_single_pdot_and_single_period():
    w = synth.random_curves(31, [5, 70, 130], n_freq=1, n_pdots=1)
    _full_parity(w, "1x1 grid")
    w = synth.random_curves(32, [5, 70, 130], n_freq=65, n_pdots=1)
    _full_parity(w, "Pdot axis of one")


def test_dyadic_bin_edges_and_negative_phase():
    """Phases exactly on bin edges (dyadic inputs) and folds whose argument
    y = x - Pdot x^2 / 2 is negative, including -1 < y < 0 where y - floor(y)
    rounds: the GPU bins must equal the oracle's bit for bit."""
    rng = np.random.default_rng(40)
    ts, ms = [], []
    # dyadic epochs, power-of-two periods: exact phases, many on bin edges
    for _ in range(3):
        k = rng.integers(0, 1 << 12, 200)
        ts.append(10.0 + k / 64.0)
        ms.append(rng.integers(0, 9, 200) / 8.0)
    # y just below zero: x slightly beyond 1/a with a = Pdot/2 = 0.25, P = 1
    d = 4.0 + 10.0 ** rng.uniform(-15, -2, 300)
    ts.append(np.concatenate([[0.0], d]))
    ms.append(rng.uniform(size=301))
    off = np.zeros(len(ts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([x.size for x in ts])
    periods = np.array([0.25, 0.125, 0.0625, 1.0, 0.5, 1.0 / 3.0])
    pdots = np.array([0.0, 2.0 ** -12, -2.0 ** -12, 0.5, 0.9, -0.5])
    w = synth.Workload("edges", np.concatenate(ts), np.concatenate(ms), off, periods,
                       pdots, 8, 4)
    _full_parity(w, "dyadic edges", counts_sample=0)
    plan, dev, _, _ = run_gpu(w, want_cube=False)
    ci = np.repeat(np.arange(w.n_curves), periods.size * pdots.size)
    fi = np.tile(np.arange(periods.size * pdots.size), w.n_curves)
    check_counts_exact(plan, dev, w, ci, fi, "dyadic edges all trials")
    for nph in (10, 50):
        w2 = synth.Workload("edges", w.times, w.mags, off, periods, pdots, nph, 4)
        plan, dev, _, _ = run_gpu(w2, want_cube=False)
        check_counts_exact(plan, dev, w2, ci, fi, f"dyadic edges nph={nph}")


def test_constant_magnitudes_and_single_epoch():
    w = synth.random_curves(33, [1, 2, 50, 200], n_freq=70, n_pdots=3)
    w.mags[w.offsets[2]:w.offsets[3]] = 1.25        # constant curve
    plan, dev, cube, best = run_gpu(w)
    gc = cube.cpu().numpy()
    bf = gce.best_fields(best)
    for c in (0, 2):                                # N = 1 and constant
        assert np.all(gc[c] == 0.0), c
        assert bf["flat_index"][c] == 0 and bf["ce_min"][c] == 0.0
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 5)
    assert_cube_close(gc, oc, w, "constant")


@pytest.mark.parametrize("mag_overlap", [False, True])
def test_invalid_values_mark_curves(mag_overlap):
    w = synth.random_curves(34, [40, 50, 60], n_freq=70, n_pdots=3)
    mags = w.mags.copy()
    mags[w.offsets[1] + 7] = np.nan
    w_bad = synth.Workload("bad", w.times, mags, w.offsets, w.periods, w.pdots, 10, 5)
    plan, dev, cube, best = run_gpu(w_bad, mag_overlap=mag_overlap)
    gc = cube.cpu().numpy()
    bf = gce.best_fields(best)
    assert bf["flat_index"].tolist()[1] == -1 and math.isnan(bf["ce_min"][1])
    assert np.all(np.isnan(gc[1]))
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 5,
                                 mag_overlap=mag_overlap)
    keep = [0, 2]
    sub = w.subset(keep)
    assert_cube_close(gc[keep], oc[keep], sub, "valid curves beside a NaN curve",
                      count_mult=2 if mag_overlap else 1)
    if mag_overlap:
        assert_best_valid(bf["flat_index"][keep], bf["ce_min"][keep], obf[keep], obc[keep],
                          oc[keep], sub, "valid curves beside a NaN curve", count_mult=2)
        return
    assert np.array_equal(bf["flat_index"][keep], obf[keep])
    # a bad period invalidates every curve
    periods = w.periods.copy()
    periods[5] = -1.0
    t, m, P, Pd = upload(w)
    P = to_dev(periods)
    plan = gce.Plan(w.offsets, periods.size, w.pdots.size, 10, 5)
    cube2, best2 = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    torch.cuda.synchronize()
    assert np.all(gce.best_fields(best2)["flat_index"] == -1)
    assert torch.isnan(cube2).all().item()
    # a NaN Pdot too
    pdots = w.pdots.copy()
    pdots[1] = np.nan
    _, best3 = plan.execute(t, m, to_dev(w.periods), to_dev(pdots))
    torch.cuda.synchronize()
    assert np.all(gce.best_fields(best3)["flat_index"] == -1)


def test_best_only_equals_full_and_is_deterministic():
    w = synth.random_curves(35, [33, 600, 250, 1], n_freq=300, n_pdots=9)
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, 10, 5)
    c1, b1 = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    _, b2 = plan.execute(t, m, P, Pd)
    c3, b3 = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    torch.cuda.synchronize()
    # bitwise: the statistics fields hold NaN when statistics are off
    assert torch.equal(b1.view(torch.int64), b2.view(torch.int64))
    assert torch.equal(b1.view(torch.int64), b3.view(torch.int64))
    assert torch.equal(c1, c3)


def test_one_call_search_matches_plan():
    w = synth.random_curves(36, [80, 90], n_freq=100, n_pdots=4)
    t, m, P, Pd = upload(w)
    cube, best = gce.search(t, m, w.offsets, P, Pd, 10, 5)
    torch.cuda.synchronize()
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 5)
    assert_cube_close(cube.cpu().numpy(), oc, w, "gce_search")
    assert np.array_equal(gce.best_fields(best)["flat_index"], obf)


def test_graph_replay_matches_eager():
    w = synth.random_curves(37, [100, 500, 20], n_freq=200, n_pdots=8)
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, 10, 5)
    ref_c, ref_b = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    torch.cuda.synchronize()
    ref_c, ref_b = ref_c.clone(), ref_b.clone()
    cube, best = plan.new_cube(), plan.new_best()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.execute(t, m, P, Pd, out_ce=cube, out_best=best, stream=s)   # warm
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(t, m, P, Pd, out_ce=cube, out_best=best,
                     stream=torch.cuda.current_stream())
    for i in range(4):
        cube.fill_(-1.0)
        best.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(cube, ref_c), i
        assert torch.equal(best.view(torch.int64), ref_b.view(torch.int64)), i


def test_c2_slice_full_grid():
    """Eight curves of the batched workload over its full 20,000 x 64 grid."""
    w = synth.make_config(2).subset(np.arange(8))
    say("[parity] c2 slice: 8 curves, full grid")
    plan, dev, cube, best = run_gpu(w, want_cube=True)
    gc = cube.cpu().numpy()
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots,
                                 w.n_phase, w.n_mag)
    assert_cube_close(gc, oc, w, "c2 slice")
    bf = gce.best_fields(best)
    assert_best_valid(bf["flat_index"], bf["ce_min"], obf, obc, oc, w, "c2 slice")
    rng = np.random.default_rng(41)
    ci = rng.integers(0, w.n_curves, 2000)
    fi = rng.integers(0, w.periods.size * w.pdots.size, 2000)
    check_counts_exact(plan, dev, w, ci, fi, "c2 slice counts")


@pytest.mark.parametrize("axis", ["pdot", "period"])
def test_batches_merge_to_single_search(axis):
    """Searching parts of the grid and merging the per-curve results (Sec. 4)
    gives the single search's minimum and statistics."""
    w = synth.random_curves(38, [40, 300, 777, 5], n_freq=200, n_pdots=12)
    t, m, P, Pd = upload(w)
    whole = gce.Plan(w.offsets, w.periods.size, w.pdots.size, 10, 5)
    _, b = whole.execute(t, m, P, Pd)
    torch.cuda.synchronize()
    ref = gce.best_fields(b)
    acc, trials = None, 0
    if axis == "pdot":
        cuts = [(0, 0, w.periods.size, 0, 5), (0, 0, w.periods.size, 5, 7)]
    else:
        cuts = [(0, 0, 70, 0, 12), (0, 70, 130, 0, 12)]
    for _, pa, pn, qa, qn in cuts:
        plan = gce.Plan(w.offsets, pn, qn, 10, 5)
        _, bp = plan.execute(t, m, P[pa:pa + pn].contiguous(), Pd[qa:qa + qn].contiguous())
        torch.cuda.synchronize()
        acc = gce.merge_results(acc, trials, bp, w.periods.size, pa, pn, qa, qn)
        trials += pn * qn
    got = gce.best_fields(acc)
    for k in ("flat_index", "period_index", "pdot_index", "ce_min"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.allclose(got["ce_mean"], ref["ce_mean"], rtol=0, atol=1e-13)
    assert np.allclose(got["ce_std"], ref["ce_std"], rtol=1e-10, atol=1e-14)
    assert np.allclose(got["significance"], ref["significance"], rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("n_phase,n_mag,tq", [
    (10, 5, 0), (10, 5, 8), (50, 10, 0), (15, 5, 4), (7, 3, 2), (2, 2, 0), (1, 1, 0),
    (20, 10, 8), (1, 5, 0), (1, 5, 2),
])
def test_overlapping_phase_bins(n_phase, n_mag, tq):
    """50%-overlapping phase bins (Sec. 2.3): counts bit-exact and CE within
    tolerance of the oracle, which counts each epoch in the two bins whose
    spans contain its phase."""
    w = synth.random_curves(80 + n_phase + tq, EDGE_LENGTHS, n_freq=130, n_pdots=6,
                            n_phase=n_phase, n_mag=n_mag, pdot_scale=5e-9)
    _full_parity(w, f"overlap nph={n_phase}", trials_per_lane=tq, phase_overlap=True)


@pytest.mark.parametrize("n_phase,n_mag,tq,phase_overlap,placement", [
    (10, 5, 0, False, 0), (10, 5, 8, True, 0), (50, 10, 0, True, 0), (7, 3, 2, False, 0),
    (20, 10, 8, False, 0), (33, 255, 2, False, 0), (2, 2, 0, True, 0), (1, 5, 0, True, 0),
    (1, 5, 0, False, 0), (10, 1, 4, False, 0), (128, 5, 1, True, 0),
    (10, 5, 8, False, gce.TABLE_LDS), (50, 10, 2, True, gce.TABLE_LDS),
    (1, 5, 0, True, gce.TABLE_LDS), (10, 5, 2, False, gce.TABLE_GLOBAL),
])
def test_overlapping_magnitude_bins(n_phase, n_mag, tq, phase_overlap, placement):
    """50%-overlapping magnitude bins (Sec. 2.3), alone and with
    overlapping phase bins: an epoch is counted in each magnitude bin whose
    span holds it, probabilities are counts over the histogram total.
    Counts bit-exact, CE within tolerance, minima and statistics."""
    w = synth.random_curves(140 + n_phase + n_mag + tq, EDGE_LENGTHS, n_freq=130,
                            n_pdots=6, n_phase=n_phase, n_mag=n_mag, pdot_scale=5e-9)
    _full_parity(w, f"mag overlap nph={n_phase} nmag={n_mag}", trials_per_lane=tq,
                 phase_overlap=phase_overlap, table_placement=placement, mag_overlap=True)


@pytest.mark.parametrize("precision", [gce.PRECISION_FP64, gce.PRECISION_SPLIT_FP32])
def test_magnitude_overlap_largest_curves(precision):
    """Curves at the magnitude-overlap limit, 32,767 epochs, with the table in
    global memory (the counts reach 2N = 65,534), and 3,000 with it in LDS
    (counts in units of 8 reach 48,000; the table then fills most of the
    LDS, so one trial per lane).  The
    FP64 path against the oracle on sampled trials (counts bit-exact, CE in
    tolerance); the split path's CE against Eq. (4) of its own histograms,
    which must hold each curve's entries."""
    for n, placement, tq in ((32767, gce.TABLE_GLOBAL, 0), (3000, gce.TABLE_LDS, 1)):
        w = synth.random_curves(150 + n % 7, [n, 700], n_freq=70, n_pdots=3,
                                n_phase=10, n_mag=5, pdot_scale=5e-9)
        plan, dev, cube, best = run_gpu(w, precision=precision, table_placement=placement,
                                        trials_per_lane=tq, mag_overlap=True)
        say(f"[mag overlap limit] N={n} table={placement} prec={precision}")
        rng = np.random.default_rng(n)
        ids = rng.integers(0, w.periods.size * w.pdots.size, 40)
        for c in range(2):
            g = cube[c].reshape(-1).cpu().numpy()[ids].astype(np.float64)
            if precision == gce.PRECISION_FP64:
                h = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 5,
                                  np.full(ids.size, c), ids, mag_overlap=True)
                tol = ce_tolerance(h, 10, 5, 2 * w.lengths[c])
                assert np.all(np.abs(g - h) <= tol), (n, c)
                check_counts_exact(plan, dev, w, np.full(8, c), ids[:8], f"N={n} c={c}")
            else:
                cnt = plan.debug_counts(*dev, np.full(ids.size, c), ids)
                cnt = cnt.cpu().numpy().astype(np.uint32)
                _, a = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 5,
                                     [c], ids[:1], want_counts=True, mag_overlap=True)
                assert np.all(cnt.sum(axis=(1, 2)) == a.sum())   # the curve's entries
                h_own = np.array([oracle.entropy(x) for x in cnt])
                assert np.all(np.abs(g - h_own) <= 2.0 ** -23 * np.abs(h_own) + 1e-12), (n, c)
        plan.close()


def test_overlap_rejects_nothing_and_differs_from_disjoint():
    w = synth.random_curves(90, [300, 400], n_freq=80, n_pdots=2)
    _, _, c0, _ = run_gpu(w)
    _, _, c1, _ = run_gpu(w, phase_overlap=True)
    torch.cuda.synchronize()
    assert not torch.equal(c0, c1)


def test_autotune_picks_a_measured_tiling():
    w = synth.make_config(2).subset(np.arange(64))
    t, m, P, Pd = upload(w)
    tq, placement, ms = gce.autotune(t, m, w.offsets, P, Pd, w.n_phase, w.n_mag)
    say(f"[autotune] chose {tq}, table {placement}: {ms}")
    assert (tq, placement) in ms and ms[(tq, placement)] == min(ms.values())
    assert any(k[1] == gce.TABLE_LDS for k in ms) and any(k[1] == gce.TABLE_GLOBAL for k in ms)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag)
    info = plan.info()
    assert info["trials_per_lane"] == tq
    assert info["table_in_lds"] == int(placement == gce.TABLE_LDS)


def test_search_beyond_32bit_dispatch_grid():
    """More than 2^32 work-items of search waves (regression: a 1-D launch
    wrapped its 32-bit grid size and skipped the tail curves).  2 curves x
    65,536 Pdot values (one per lane) x 64,000 periods = 131M waves."""
    rng = np.random.default_rng(44)
    ts = [np.sort(rng.uniform(0, 100, 20)) for _ in range(2)]
    ms = [rng.normal(size=20) for _ in range(2)]
    off = np.array([0, 20, 40], dtype=np.int64)
    periods = 1.0 / np.linspace(1.0, 30.0, 64000)
    pdots = np.linspace(-1e-6, 1e-6, 65536)
    w = synth.Workload("wide", np.concatenate(ts), np.concatenate(ms), off, periods,
                       pdots, 10, 5)
    t, m, P, Pd = upload(w)
    plan = gce.Plan(off, periods.size, pdots.size, 10, 5, trials_per_lane=1)
    assert plan.info()["work_units"] * 64 > 2 ** 32
    _, best = plan.execute(t, m, P, Pd)
    torch.cuda.synchronize()
    bf = gce.best_fields(best)
    assert np.all(bf["flat_index"] >= 0)
    assert np.all(bf["ce_mean"] > 0) and np.all(np.isfinite(bf["ce_std"]))
    # the same search in two Pdot halves, merged: identical minima
    acc, n = None, 0
    for qa in (0, 32768):
        p2 = gce.Plan(off, periods.size, 32768, 10, 5, trials_per_lane=1)
        _, b2 = p2.execute(t, m, P, Pd[qa:qa + 32768].contiguous())
        torch.cuda.synchronize()
        acc = gce.merge_results(acc, n, b2, periods.size, 0, periods.size, qa, 32768)
        n += periods.size * 32768
        p2.close()
    got = gce.best_fields(acc)
    assert np.array_equal(got["flat_index"], bf["flat_index"])
    # and the minimum is the CE of its trial per the oracle
    h = oracle.trials(w.times, w.mags, off, periods, pdots, 10, 5, [0, 1],
                      bf["flat_index"])
    assert np.all(np.abs(h - bf["ce_min"]) <= 1e-13)


@pytest.mark.parametrize("overlap", [False, True])
def test_chunked_search_matches_one_launch(tmp_path, overlap):
    """Period-range chunks merged on the host (with a checkpoint, and a
    resume after an interruption) give the one-launch minimum exactly and
    its statistics to rounding."""
    from paper_2006_06866_amd import chunked
    w = synth.random_curves(120 + overlap, [64, 300, 1000], n_freq=900, n_pdots=6,
                            n_phase=20, n_mag=5, pdot_scale=5e-9)
    t, m, P, Pd = upload(w)
    # overlap: both overlapping phase and magnitude bins
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    phase_overlap=overlap, mag_overlap=overlap)
    _, best = plan.execute(t, m, P, Pd)
    torch.cuda.synchronize()
    want = gce.best_fields(best)
    plan.close()
    ck = str(tmp_path / "c.npz")
    seen = []

    class Stop(Exception):
        pass

    def stop_after_two(i, p0, p1, cube):
        seen.append((p0, p1))
        if len(seen) == 2:
            raise Stop

    with pytest.raises(Stop):
        chunked.search_chunked(t, m, w.offsets, P, Pd, w.n_phase, w.n_mag, 256,
                               checkpoint=ck, phase_overlap=overlap, mag_overlap=overlap,
                               on_range=stop_after_two)
    # the interrupted range ran but its callback raised before the save
    assert chunked.load_checkpoint(ck, chunked.fingerprint(
        [w.offsets, w.times, w.mags, w.periods, w.pdots], n_phase=w.n_phase,
        n_mag=w.n_mag, precision=0, phase_overlap=overlap, mag_overlap=overlap,
        chunk=256))[1] == 1
    seen.clear()
    acc = chunked.search_chunked(t, m, w.offsets, P, Pd, w.n_phase, w.n_mag, 256,
                                 checkpoint=ck, phase_overlap=overlap, mag_overlap=overlap,
                                 on_range=lambda i, p0, p1, c: seen.append((p0, p1)))
    assert seen == [(256, 512), (512, 768), (768, 900)]
    got = gce.best_fields(acc)
    for k in ("flat_index", "period_index", "pdot_index", "ce_min"):
        assert np.array_equal(got[k], want[k]), k
    assert np.allclose(got["ce_mean"], want["ce_mean"], rtol=0, atol=1e-13)
    assert np.allclose(got["ce_std"], want["ce_std"], rtol=1e-9, atol=1e-14)


def test_automatic_table_placement():
    """The automatic choice keeps the table in global memory for dense
    histograms, long curves or large LDS, and moves it to LDS for many cells
    per epoch (the paper-scale shape: 50 x 10 bins, ~500 epochs)."""
    def info(lengths, n_phase, n_mag, overlap=False, n_pd=32):
        off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
        p = gce.Plan(off, 1000, n_pd, n_phase, n_mag, phase_overlap=overlap)
        i = p.info()
        p.close()
        return i
    assert info([600] * 4, 10, 5)["table_in_lds"] == 0          # dense: c2-like
    assert info([500] * 4, 50, 10, True)["table_in_lds"] == 1   # paper scale
    assert info([3000] * 4, 50, 10)["table_in_lds"] == 0        # table over 8 KiB
    assert info([100] * 4, 128, 5, n_pd=1)["table_in_lds"] == 0  # LDS budget
    # ragged: the curves of at most 4 * 10 * 5 epochs get the LDS table
    assert info([3000, 700, 201, 200, 50, 1], 10, 5)["table_in_lds"] == 2
    assert info([200, 50, 1], 10, 5)["table_in_lds"] == 1       # all short


@pytest.mark.parametrize("precision", [gce.PRECISION_FP64, gce.PRECISION_SPLIT_FP32])
@pytest.mark.parametrize("phase_overlap,mag_overlap", [(False, False), (True, True)])
def test_length_split_matches_one_placement(precision, phase_overlap, mag_overlap):
    """A ragged batch searched in two launches (longer curves with the
    table in global memory, the shortest with it in LDS) gives bit for bit
    the cube and minima of the whole batch with the table in global memory
    (both placements hold the same doubles and add them in the same order),
    and the FP64 plan matches the oracle."""
    lengths = [1200, 650, 300, 201, 200, 199, 120, 64, 63, 2, 1]
    w = synth.random_curves(180 + precision + 2 * phase_overlap, lengths, n_freq=150,
                            n_pdots=6, n_phase=10, n_mag=5, pdot_scale=5e-9)
    split = run_gpu(w, precision=precision, phase_overlap=phase_overlap,
                    mag_overlap=mag_overlap)
    whole = run_gpu(w, precision=precision, phase_overlap=phase_overlap,
                    mag_overlap=mag_overlap, table_placement=gce.TABLE_GLOBAL)
    assert split[0].info()["table_in_lds"] == 2
    assert torch.equal(split[2], whole[2])
    assert torch.equal(split[3], whole[3])
    if precision == gce.PRECISION_FP64:
        oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 5,
                                     phase_overlap=phase_overlap, mag_overlap=mag_overlap)
        cm = 2 if mag_overlap else 1
        assert_cube_close(split[2].cpu().numpy(), oc, w, "length split", count_mult=cm)
        bf = gce.best_fields(split[3])
        assert_best_valid(bf["flat_index"], bf["ce_min"], obf, obc, oc, w, "length split",
                          count_mult=cm)
    split[0].close()
    whole[0].close()


@pytest.mark.parametrize("n_phase", [3, 10, 50, 128])
def test_fp64_bins_on_bin_edges_are_exact_floor(n_phase):
    """Phases on every bin edge k/n and one ulp either side (dt = phase with
    t0 = 0, P = 1, Pdot = 0, so the fold returns the phase unchanged): the
    FP64 path bins each at floor(phi * n) of the exact product, like the
    oracle; the rounded product would move many of them up a bin."""
    import math
    from fractions import Fraction
    phis = {0.0}
    for k in range(n_phase + 1):
        e = k / n_phase
        for v in (e, math.nextafter(e, 0.0), math.nextafter(e, 1.0)):
            if 0.0 <= v < 1.0:
                phis.add(v)
    t = np.array(sorted(phis))
    m = np.zeros_like(t)
    want = np.bincount([min(math.floor(Fraction(v) * n_phase), n_phase - 1) for v in t],
                       minlength=n_phase)
    if n_phase & (n_phase - 1):   # k/n inexact: some rounded products land on k
        assert not np.array_equal(want, np.bincount(
            np.minimum((t * n_phase).astype(int), n_phase - 1), minlength=n_phase))
    off = np.array([0, t.size], dtype=np.int64)
    w = synth.Workload("edges", t, m, off, np.array([1.0]), np.array([0.0]), n_phase, 1)
    plan = gce.Plan(off, 1, 1, n_phase, 1)
    got = plan.debug_counts(*upload(w), np.array([0]), np.array([0]))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().astype(np.int64).reshape(-1), want)
    assert np.array_equal(oracle.counts(t, m, 1.0, 0.0, n_phase, 1).reshape(-1), want)
    plan.close()
    # the search kernel over a few dyadic periods, against the oracle
    m2 = np.random.default_rng(n_phase).normal(size=t.size)
    w2 = synth.Workload("edges2", t, m2, off, np.array([1.0, 0.5, 0.25, 2.0, 4.0]),
                        np.array([0.0, 2.0 ** -30]), n_phase, 3)
    _full_parity(w2, f"edges n={n_phase}", counts_sample=20)


def test_tilings_agree():
    """Every tiling the plan or the autotuner may choose (1, 2, 4, 8 trials
    per lane x c ln c table in global memory or LDS) gives the same
    histograms (one bin code), CE values equal to rounding (sum orders
    differ between tilings), and the same minimum or one tied within it."""
    w = synth.random_curves(321, [64, 200, 600, 1000], n_freq=300, n_pdots=9,
                            n_phase=10, n_mag=5, pdot_scale=5e-9)
    ref = None
    rng = np.random.default_rng(3)
    ci = rng.integers(0, w.n_curves, 300)
    fi = rng.integers(0, w.periods.size * w.pdots.size, 300)
    for tq in (1, 2, 4, 8):
        for placement in (gce.TABLE_GLOBAL, gce.TABLE_LDS):
            plan, dev, cube, best = run_gpu(w, trials_per_lane=tq, table_placement=placement)
            got = (cube.cpu().numpy(), gce.best_fields(best),
                   plan.debug_counts(*dev, ci, fi).cpu().numpy())
            plan.close()
            if ref is None:
                ref = got
                continue
            n = w.lengths[:, None, None].astype(np.float64)
            tol = ce_tolerance(ref[0], w.n_phase, w.n_mag, n)
            assert np.all(np.abs(got[0] - ref[0]) <= tol), (tq, placement)
            assert np.array_equal(got[2], ref[2]), (tq, placement)
            for c in range(w.n_curves):
                f0, f1 = int(ref[1]["flat_index"][c]), int(got[1]["flat_index"][c])
                if f0 != f1:
                    q, p = divmod(f1, w.periods.size)
                    assert ref[0][c, q, p] <= ref[1]["ce_min"][c] + 2 * tol[c, 0, 0], (tq, placement, c)


@pytest.mark.parametrize("flags,phase_overlap,mag_overlap", [
    ([], False, False), (["--phase-overlap", "--mag-overlap"], True, True),
    (["--mag-overlap", "--table", "lds", "--trials-per-lane", "2"], False, True),
])
def test_file_search_program_matches_oracle(tmp_path, flags, phase_overlap, mag_overlap):
    """The C-ABI used from a native program (no Python in the search): inputs
    from raw files, results written to files, compared with the oracle."""
    import os
    import subprocess
    from paper_2006_06866_amd import build as gbuild
    w = synth.random_curves(170 + len(flags), EDGE_LENGTHS, n_freq=110, n_pdots=5,
                            n_phase=15, n_mag=5, pdot_scale=5e-9)
    d = str(tmp_path)
    w.times.astype("<f8").tofile(os.path.join(d, "times.f64"))
    w.mags.astype("<f8").tofile(os.path.join(d, "mags.f64"))
    np.asarray(w.offsets, dtype="<i8").tofile(os.path.join(d, "offsets.i64"))
    w.periods.astype("<f8").tofile(os.path.join(d, "periods.f64"))
    w.pdots.astype("<f8").tofile(os.path.join(d, "pdots.f64"))
    say(f"[file search] flags={flags}")
    r = subprocess.run([gbuild.FILE_SEARCH, d, "15", "5", "--cube", *flags],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    say(r.stdout.strip())
    cube = np.fromfile(os.path.join(d, "cube.f64"), dtype="<f8").reshape(
        w.n_curves, w.pdots.size, w.periods.size)
    bf = gce.best_fields(np.fromfile(os.path.join(d, "best.bin"), dtype=np.uint8))
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, 15, 5,
                                 phase_overlap=phase_overlap, mag_overlap=mag_overlap)
    cm = 2 if mag_overlap else 1
    assert_cube_close(cube, oc, w, "file search", count_mult=cm)
    assert_best_valid(bf["flat_index"], bf["ce_min"], obf, obc, oc, w, "file search",
                      count_mult=cm)


def test_file_search_program_split_with_fp64_confirmation(tmp_path):
    """The native program on the split path with 64 confirmed units per curve,
    more than this grid's curves have: every reported minimum is searched
    again in FP64, so it is the oracle's minimum (or ties it within the FP64
    tolerance) with an FP64 CE value; the float cube and the results are
    those of the same plan made through the Python binding, bit for bit."""
    import os
    import subprocess
    from paper_2006_06866_amd import build as gbuild
    w = synth.random_curves(181, EDGE_LENGTHS, n_freq=110, n_pdots=5, n_phase=15,
                            n_mag=5, pdot_scale=5e-9)
    d = str(tmp_path)
    w.times.astype("<f8").tofile(os.path.join(d, "times.f64"))
    w.mags.astype("<f8").tofile(os.path.join(d, "mags.f64"))
    np.asarray(w.offsets, dtype="<i8").tofile(os.path.join(d, "offsets.i64"))
    w.periods.astype("<f8").tofile(os.path.join(d, "periods.f64"))
    w.pdots.astype("<f8").tofile(os.path.join(d, "pdots.f64"))
    say("[file search] --split --refine-units 64")
    r = subprocess.run([gbuild.FILE_SEARCH, d, "15", "5", "--cube", "--split",
                        "--trials-per-lane", "4", "--refine-units", "64"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    cube = np.fromfile(os.path.join(d, "cube.f32"), dtype="<f4").reshape(
        w.n_curves, w.pdots.size, w.periods.size)
    assert not os.path.exists(os.path.join(d, "cube.f64"))
    raw = np.fromfile(os.path.join(d, "best.bin"), dtype=np.uint8)
    bf = gce.best_fields(raw)
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, 15, 5)
    # 110 periods x 5 Pdots at four trials per lane: 2 x 2 units per curve
    assert_best_valid(bf["flat_index"], bf["ce_min"], obf, obc, oc, w, "file search refine")
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, 15, 5,
                    precision=gce.PRECISION_SPLIT_FP32, trials_per_lane=4, refine_units=64)
    assert plan.info()["work_units"] == 4 * w.n_curves
    pc, pb = plan.execute(t, m, P, Pd, out_ce=plan.new_cube())
    torch.cuda.synchronize()
    assert np.array_equal(cube.view(np.int32), pc.cpu().numpy().view(np.int32))
    assert np.array_equal(raw, pb.cpu().numpy().view(np.uint8).ravel())
    plan.close()


def _aligned_curve_workload(n, n_phase, n_mag, seed):
    """A curve of n epochs at t = k / 8 d with two magnitude levels, plus a
    short noisy curve.  At P = 1/8 d and Pdot = 0 every epoch of the first
    curve folds to phase 0, so one phase bin holds all n epochs: the largest
    counts the 16-bit cells and the marginals can hold."""
    rng = np.random.default_rng(seed)
    k = np.arange(n, dtype=np.float64)
    t0 = k / 8.0
    m0 = (np.arange(n) % 2).astype(np.float64)
    t1 = np.sort(rng.uniform(0.0, 500.0, 37))
    m1 = rng.normal(size=37)
    periods = np.concatenate([[0.125], rng.uniform(0.05, 0.3, 40)])
    pdots = np.array([0.0, 3e-9])
    off = np.array([0, n, n + 37], dtype=np.int64)
    return synth.Workload("aligned", np.concatenate([t0, t1]), np.concatenate([m0, m1]),
                          off, periods, pdots, n_phase, n_mag)


@pytest.mark.parametrize("n,placement,tq", [
    (65535, gce.TABLE_GLOBAL, 0), (65535, gce.TABLE_GLOBAL, 8), (7000, gce.TABLE_LDS, 1),
])
def test_longest_curves_fill_the_counters(n, placement, tq):
    """Curves at the epoch limit (65,535; with the table in LDS, where counts
    are kept in units of 8, the longest that fits the LDS): one trial puts
    every epoch in one phase bin.  Counts bit-exact, CE within tolerance,
    the aligned trial's CE equal to the magnitude entropy."""
    w = _aligned_curve_workload(n, 10, 2, n)
    say(f"[longest] N={n} table={placement} tq={tq}")
    plan, dev, cube, best = run_gpu(w, trials_per_lane=tq, table_placement=placement)
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, 10, 2)
    gc = cube.cpu().numpy()
    assert_cube_close(gc, oc, w, f"N={n}")
    # phase bin 0 holds everything at (P = 1/8, Pdot = 0): H = H(magnitude)
    half = n // 2
    p1, p0 = half / n, (n - half) / n
    h_mag = -(p0 * math.log(p0) + p1 * math.log(p1))
    assert abs(gc[0, 0, 0] - h_mag) <= 1e-12
    ids = np.array([0, 1, 5, w.periods.size, w.periods.size + 7])
    check_counts_exact(plan, dev, w, np.zeros(ids.size, dtype=np.int64), ids, f"N={n}")
    cnt = plan.debug_counts(*dev, np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64))
    assert int(cnt[0, :, 0].sum().item()) == n
    plan.close()


def test_random_shapes_match_oracle():
    """Seeded random shapes across every option at once: phase and magnitude
    bin counts, trials per lane, table placement, both overlap kinds, ragged
    lengths and grid sizes that are not multiples of the tile.  Counts
    bit-exact on sampled trials, CE within tolerance, minima valid."""
    rng = np.random.default_rng(2006)
    ran = 0
    for case in range(40):
        n_phase = int(rng.choice([1, 2, 3, 7, 10, 15, 20, 33, 50, 64, 128]))
        n_mag = int(rng.choice([1, 2, 3, 5, 10, 17, 255]))
        tq = int(rng.choice([0, 1, 2, 4, 8]))
        placement = int(rng.choice([gce.TABLE_AUTO, gce.TABLE_GLOBAL, gce.TABLE_LDS]))
        po, mo = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
        lengths = [int(x) for x in rng.integers(1, 700, int(rng.integers(1, 6)))]
        w = synth.random_curves(1000 + case, lengths, n_freq=int(rng.integers(1, 150)),
                                n_pdots=int(rng.integers(1, 7)), n_phase=n_phase,
                                n_mag=n_mag, pdot_scale=5e-9)
        label = (f"case {case}: bins {n_phase}x{n_mag} tq={tq} table={placement} "
                 f"overlap={po}/{mo} N={lengths} grid={w.periods.size}x{w.pdots.size}")
        try:
            plan, dev, cube, best = run_gpu(w, trials_per_lane=tq, phase_overlap=po,
                                            table_placement=placement, mag_overlap=mo)
        except gce.GceError as e:
            # an explicit tiling that does not fit (LDS, no such variant) is
            # refused on the host; automatic choices always fit
            assert e.status == -6 and (tq != 0 or placement == gce.TABLE_LDS), (label, e)
            continue
        say(f"[random] {label}")
        oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots,
                                     n_phase, n_mag, phase_overlap=po, mag_overlap=mo)
        cm = 2 if mo else 1
        assert_cube_close(cube.cpu().numpy(), oc, w, label, count_mult=cm)
        bf = gce.best_fields(best)
        assert_best_valid(bf["flat_index"], bf["ce_min"], obf, obc, oc, w, label,
                          count_mult=cm)
        n_tr = w.periods.size * w.pdots.size
        ci = rng.integers(0, w.n_curves, 64)
        fi = rng.integers(0, n_tr, 64)
        check_counts_exact(plan, dev, w, ci, fi, label)
        plan.close()
        ran += 1
    assert ran >= 25


_TUNE_CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import synth
w = synth.make_config(2).subset(np.arange(48))
dev = torch.device("cuda:0")
t, m, P, Pd = (torch.from_numpy(a).to(dev) for a in (w.times, w.mags, w.periods, w.pdots))
out = {}
if sys.argv[2] == "tune":
    tq, pl, ms = gce.autotune(t, m, w.offsets, P, Pd, w.n_phase, w.n_mag,
                              phase_overlap=True, mag_overlap=True)
    out = {"tq": tq, "placement": pl}
else:
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    phase_overlap=True, mag_overlap=True, device=dev)
    out = plan.info()
    plan.close()
print(json.dumps(out), flush=True)
"""


def test_tune_cache_file_persists_overlap_choices(tmp_path):
    """gce_autotune with both overlap kinds appends its choice to the
    GCE_TUNE_CACHE file under the overlap bits 3; a later process creating an
    automatic plan of that shape class reads the file and uses the choice."""
    import json
    import os
    import subprocess
    import sys
    cache = str(tmp_path / "tune.txt")
    env = dict(os.environ, GCE_TUNE_CACHE=cache)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("[tune cache] autotune child")
    r1 = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root, "tune"], env=env,
                        capture_output=True, text=True, timeout=300)
    assert r1.returncode == 0, r1.stderr[-2000:]
    chosen = json.loads(r1.stdout.strip().splitlines()[-1])
    lines = open(cache).read().split("\n")
    rec = [l.split() for l in lines if l.strip()]
    assert len(rec) == 1 and rec[0][0] == "0" and rec[0][1] == "3", rec
    assert int(rec[0][6]) == chosen["tq"]
    assert int(rec[0][7]) == int(chosen["placement"] == gce.TABLE_LDS)
    # a choice the heuristics would not make, for the same shape class: the
    # plan can only take it from the file
    planted = (1, 0) if (chosen["tq"], chosen["placement"]) != (1, gce.TABLE_GLOBAL) else (2, 0)
    with open(cache, "w") as f:
        f.write(" ".join(rec[0][:6] + [str(planted[0]), str(planted[1])]) + "\n")
    say("[tune cache] plan child")
    r2 = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root, "plan"], env=env,
                        capture_output=True, text=True, timeout=300)
    assert r2.returncode == 0, r2.stderr[-2000:]
    info = json.loads(r2.stdout.strip().splitlines()[-1])
    assert (info["trials_per_lane"], info["table_in_lds"]) == planted


_TUNE_LONG_CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import synth
# nine curves of 300 epochs and one of 9,000: median length class 1 (< 512),
# like the planted tuned line, but a count bound above the 8191 that the
# table in LDS allows
w = synth.random_curves(41, [300] * 9 + [9000], n_freq=96, n_pdots=2)
dev = torch.device("cuda:0")
t, m, P, Pd = (torch.from_numpy(a).to(dev) for a in (w.times, w.mags, w.periods, w.pdots))
plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag, device=dev)
info = plan.info()
_, best = plan.execute(t, m, P, Pd)
torch.cuda.synchronize()
plan.close()
_, best2 = gce.search(t, m, w.offsets, P, Pd, w.n_phase, w.n_mag, want_cube=False)
torch.cuda.synchronize()
info["flat"] = gce.best_fields(best)["flat_index"].tolist()
info["flat_search"] = gce.best_fields(best2)["flat_index"].tolist()
print(json.dumps(info), flush=True)
"""


def test_tuned_table_in_lds_not_taken_when_the_batch_does_not_fit(tmp_path):
    """A tuned choice is per shape class (keyed by the median curve length):
    a batch of that class holding one curve too long for the table in LDS
    falls back to the heuristics instead of failing, through both the plan
    and gce_search."""
    import json
    import os
    import subprocess
    import sys
    from paper_2006_06866_amd import synth
    cache = tmp_path / "tune.txt"
    # precision 0, no overlap, 10 x 5 bins, 2 Pdots (class 1), median class 1,
    # 4 trials per lane, table in LDS
    cache.write_text("0 0 10 5 1 1 4 1\n")
    env = dict(os.environ, GCE_TUNE_CACHE=str(cache))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("[tune long] plan child")
    r = subprocess.run([sys.executable, "-c", _TUNE_LONG_CHILD, root], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    info = json.loads(r.stdout.strip().splitlines()[-1])
    assert info["table_in_lds"] != 1, info
    w = synth.random_curves(41, [300] * 9 + [9000], n_freq=96, n_pdots=2)
    _, obf, _ = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                              w.n_mag, want_cube=False)
    assert info["flat"] == obf.tolist()
    assert info["flat_search"] == obf.tolist()


def test_gce_search_on_two_streams_does_not_share_a_workspace():
    """Two gce_search calls of one shape enqueued back to back on two streams
    (no synchronisation between them) each return their own inputs' results:
    the cached plans are per stream."""
    import torch
    from paper_2006_06866_amd import synth
    wa = synth.make_config(2).subset(np.arange(32))
    wb = synth.make_config(2).subset(np.arange(32, 64))
    assert np.array_equal(wa.offsets, wb.offsets)
    da, db = upload(wa), upload(wb)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ref = []
    for d, w in ((da, wa), (db, wb)):   # sequential reference on the current stream
        _, b = gce.search(d[0], d[1], w.offsets, d[2], d[3], w.n_phase, w.n_mag,
                          want_cube=False)
        torch.cuda.synchronize()
        ref.append(gce.best_fields(b))
    torch.cuda.synchronize()
    say("[two streams] concurrent")
    for rep in range(3):
        _, ba = gce.search(da[0], da[1], wa.offsets, da[2], da[3], wa.n_phase, wa.n_mag,
                           want_cube=False, stream=sa)
        _, bb = gce.search(db[0], db[1], wb.offsets, db[2], db[3], wb.n_phase, wb.n_mag,
                           want_cube=False, stream=sb)
        torch.cuda.synchronize()
        for b, r in ((ba, ref[0]), (bb, ref[1])):
            f = gce.best_fields(b)
            assert np.array_equal(f["flat_index"], r["flat_index"]), rep
            assert np.array_equal(f["ce_min"], r["ce_min"]), rep


@pytest.mark.parametrize("n_mag,mag_overlap", [(10, False), (7, False), (50, False),
                                               (255, False), (10, True), (19, True)])
def test_magnitude_bins_on_bin_edges_are_exact_floor(n_mag, mag_overlap):
    """Normalised magnitudes on the doubles around every edge k / n (minimum
    0, maximum 1), including those whose rounded product u * n lands on the
    edge from below: the prepass bins each at the floor of the exact product,
    like the oracle (whole histograms compared, magnitude rows included)."""
    import math
    from fractions import Fraction
    n_sub = n_mag + 1 if mag_overlap else n_mag
    us = {0.0, 1.0}
    for k in range(1, n_sub):
        e = k / n_sub
        for v in (e, math.nextafter(e, 0.0), math.nextafter(e, 1.0),
                  math.nextafter(math.nextafter(e, 0.0), 0.0)):
            us.add(v)
    m = np.array(sorted(us))
    if not mag_overlap:   # the truncated rounded product would move some up
        exact = [min(math.floor(Fraction(v) * n_mag), n_mag - 1) for v in m]
        assert exact != [min(int(v * n_mag), n_mag - 1) for v in m]
    rng = np.random.default_rng(n_mag)
    t = np.sort(rng.uniform(0.0, 500.0, m.size))
    off = np.array([0, m.size], dtype=np.int64)
    w = synth.Workload("mag edges", t, rng.permutation(m), off,
                       synth.frequency_grid_periods(5.0, 50.0, 70), np.array([0.0, 1e-9]),
                       10, n_mag, mag_overlap=mag_overlap)
    _full_parity(w, f"magnitude edges n_mag={n_mag} overlap={mag_overlap}",
                 counts_sample=40, mag_overlap=mag_overlap)
