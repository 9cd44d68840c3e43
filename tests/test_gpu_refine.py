"""FP64 confirmation of the split path's minima (gce_opts.refine_units): the
split search ranks each curve's work units by their split minima, the FP64
search kernel of the same tiling searches the best few again, and the
reported minimum is the FP64 minimum over their trials.

Checked against the FP64 path, whose bins and CE values the other GPU tests
hold to the oracle: the reported flat index is the FP64 plan's wherever the
FP64 minimum lies in one of the confirmed units (on these workloads it
always does: the curves of the ragged and long-baseline workloads whose
split minimum differs from the FP64 one have their FP64 minimum in the unit
of the split minimum), and the reported CE is the FP64 value of that trial;
the cube keeps the split values and the moments the split ones.  A small
workload is checked against the oracle itself.  Katz et al. 2020, Sec. 2.3,
Eqs. (3)-(5).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import synth
from gce_testlib import say, upload, assert_best_valid, ce_tolerance

pytestmark = pytest.mark.gpu


def _plans(w, refine, tq=0, co=0, phase_overlap=False, mag_overlap=False, want_cube=True):
    d = upload(w)
    out = []
    for prec, k in ((gce.PRECISION_FP64, 0), (gce.PRECISION_SPLIT_FP32, 0),
                    (gce.PRECISION_SPLIT_FP32, refine)):
        plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                        precision=prec, trials_per_lane=tq, waves_per_unit=co,
                        phase_overlap=phase_overlap, mag_overlap=mag_overlap, refine_units=k)
        cube = plan.new_cube() if want_cube else None
        cube, best = plan.execute(*d, out_ce=cube)
        torch.cuda.synchronize()
        out.append((plan, None if cube is None else cube.cpu().numpy(), gce.best_fields(best)))
    return out


def _check_against_fp64(w, runs, label, strict=True):
    """strict: the confirmed minima are the FP64 plan's trials.  Always: the
    reported CE is the FP64 CE of the reported trial and no FP64 value is
    below it by more than the tolerance (the FP64 minimum); the cube and
    the moments stay the split path's."""
    (p64, c64, b64), (p32, c32, b32), (pr, cr, br) = runs
    assert pr.info()["refine_units"] > 0 and p32.info()["refine_units"] == 0
    assert pr.info()["trials_per_lane"] == p64.info()["trials_per_lane"]
    same = br["flat_index"] == b64["flat_index"]
    say(f"[refine] {label}: strict {int(same.sum())}/{w.n_curves} "
        f"(split alone {int((b32['flat_index'] == b64['flat_index']).sum())})")
    # histogram totals reach 4N with both overlap kinds
    tol = np.array([ce_tolerance(h, w.n_phase, w.n_mag, 4 * n) for h, n in
                    zip(b64["ce_min"], w.lengths)])
    if strict:
        assert np.all(same), (label, np.flatnonzero(~same)[:8])
        for f in ("period_index", "pdot_index"):
            assert np.array_equal(br[f], b64[f]), label
        # the FP64 value of the same trial
        assert np.all(np.abs(br["ce_min"] - b64["ce_min"]) <= tol), label
    assert np.all(br["flat_index"] >= 0), label
    assert np.all(br["ce_min"] >= b64["ce_min"] - tol), label
    if c64 is not None:
        h_at = c64.reshape(w.n_curves, -1)[np.arange(w.n_curves), br["flat_index"]]
        assert np.all(np.abs(h_at - br["ce_min"]) <= tol), label
    # the cube and the moments stay the split path's
    if cr is not None:
        assert np.array_equal(cr, c32), label
    assert np.array_equal(br["ce_mean"], b32["ce_mean"]), label
    assert np.array_equal(br["ce_std"], b32["ce_std"]), label
    sd = br["ce_std"]
    sig = np.divide(br["ce_mean"] - br["ce_min"], sd, out=np.zeros_like(sd), where=sd > 0)
    assert np.allclose(br["significance"], sig, rtol=1e-12, atol=1e-12), label
    for p, _, _ in runs:
        p.close()


def test_refine_ragged_curves_where_split_minima_differ():
    """The ragged workload's curves whose split minimum differs from the FP64
    one (near-equal CE values on short and pure-noise curves), with others
    around them: 10,000 P x 32 Pdot, 10 x 5 bins."""
    w4 = synth.make_config(4)
    ids = [284, 591, 693, 1385, 2746, 3972, 4346, 4961, 5125, 5314, 5320, 5333, 5563,
           0, 1, 2, 100, 4000, 8190, 8191]
    w = w4.subset(np.array(ids))
    _check_against_fp64(w, _plans(w, refine=4), "ragged subset")


def test_refine_long_baseline_curve():
    """The long-baseline workload's curve 19 (5,000 epochs, 100,000 P x 256
    Pdot, 20 x 10 bins), whose split minimum differs from the FP64 one by
    3e-5 in CE, and two others; minimum only."""
    w5 = synth.make_config(5)
    w = w5.subset(np.array([19, 0, 63]))
    _check_against_fp64(w, _plans(w, refine=2, want_cube=False), "long baseline subset")


@pytest.mark.parametrize("phase_overlap,mag_overlap", [(False, False), (True, False),
                                                       (False, True), (True, True)])
def test_refine_against_oracle(phase_overlap, mag_overlap):
    """A small ragged workload, both overlap kinds, one and two waves per
    unit: the confirmed minimum against the oracle's (the same trial, or one
    whose oracle CE ties the oracle minimum within the FP64 tolerance), its
    CE within that tolerance of the oracle's value."""
    w = synth.random_curves(77, [1, 30, 64, 65, 200, 700], n_freq=200, n_pdots=9,
                            n_phase=20, n_mag=5, pdot_scale=5e-9)
    for tq, co in ((4, 1), (4, 2), (1, 0)):
        say(f"[refine] oracle tq={tq} co={co} po={phase_overlap} mo={mag_overlap}")
        runs = _plans(w, refine=3, tq=tq, co=co, phase_overlap=phase_overlap,
                      mag_overlap=mag_overlap)
        oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots,
                                     w.n_phase, w.n_mag, phase_overlap=phase_overlap,
                                     mag_overlap=mag_overlap)
        br = runs[2][2]
        mult = (2 if phase_overlap else 1) * (2 if mag_overlap else 1)
        assert_best_valid(br["flat_index"], br["ce_min"], obf, obc, oc, w,
                          f"refine tq={tq} co={co}", count_mult=mult)
        _check_against_fp64(w, runs, f"random tq={tq} co={co}", strict=False)


def test_refine_paper_scale_slice():
    """Eight binaries of the paper-scale grid (5,183,995 P x 32 Pdot, 50 x 10
    bins, 50% phase overlap), minimum only: the confirmed minima are the FP64
    path's."""
    w6 = synth.make_config(6)
    w = w6.subset(np.arange(8))
    _check_against_fp64(w, _plans(w, refine=4, phase_overlap=True, want_cube=False),
                        "paper scale slice")


def test_refine_units_on_fp64_plans_change_nothing():
    w = synth.random_curves(78, [40, 300], n_freq=90, n_pdots=3)
    d = upload(w)
    bests = []
    for k in (0, 5):
        plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                        refine_units=k)
        assert plan.info()["refine_units"] == 0
        _, best = plan.execute(*d)
        bests.append(best.cpu().numpy())
        plan.close()
    assert np.array_equal(bests[0], bests[1])


def test_refined_split_graph_replay_matches_eager():
    """The whole split search with its FP64 confirmation captured once in a
    HIP graph: every replay (with eager work and synchronisations between
    them) gives the eager cube and minima bit for bit."""
    w = synth.random_curves(79, [100, 500, 20, 64], n_freq=200, n_pdots=8)
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, 10, 5,
                    precision=gce.PRECISION_SPLIT_FP32, refine_units=3)
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
    plan.close()


def test_refine_constant_and_invalid_curves():
    """A one-epoch curve, a constant curve and a curve with a non-finite
    magnitude beside a valid one: the confirmation leaves the invalid curve
    invalid (flat -1, NaN CE), reports flat 0 with CE 0 for the constant
    ones, and the FP64 plan's minimum for the valid one."""
    w = synth.random_curves(80, [1, 40, 50, 300], n_freq=70, n_pdots=3)
    w.mags[w.offsets[1]:w.offsets[2]] = 3.0
    w.mags[w.offsets[2] + 3] = np.inf
    runs = _plans(w, refine=2)
    b64, br = runs[0][2], runs[2][2]
    assert br["flat_index"][0] == 0 and br["flat_index"][1] == 0
    assert br["ce_min"][0] == 0.0 and br["ce_min"][1] == 0.0
    assert br["flat_index"][2] == -1 and np.isnan(br["ce_min"][2])
    assert br["flat_index"][3] == b64["flat_index"][3]
    assert abs(br["ce_min"][3] - b64["ce_min"][3]) <= 1e-14
    for p, _, _ in runs:
        p.close()


@pytest.mark.parametrize("k", [8, 64])
@pytest.mark.parametrize("co", [1, 2])
def test_refine_every_unit_of_a_curve(co, k):
    """k at least the units a curve has (8 here: 200 periods in four tiles of
    64 lanes, 5 Pdots in two groups of four): k = 8 takes every unit, k = 64
    (the largest accepted) takes them all and then repeats its last choice
    once the units run out.  Every unit is searched again in FP64, so the
    reported minima are the FP64 plan's trials with bit-identical CE values
    (the same kernel and tiling, the c ln c table read from global memory
    instead of LDS, which holds the same values).  k - 1 leaves one unit
    out: then only the FP64 value of the reported trial is required."""
    w = synth.random_curves(81, [1, 37, 64, 300, 900], n_freq=200, n_pdots=5,
                            pdot_scale=5e-9)
    runs = _plans(w, refine=k, tq=4, co=co)
    units = runs[2][0].info()["work_units"] // w.n_curves
    say(f"[refine] k={k} over {units} units per curve, co={co}")
    assert units == 8
    b64, br = runs[0][2], runs[2][2]
    assert np.array_equal(br["flat_index"], b64["flat_index"])
    assert np.array_equal(br["ce_min"].view(np.int64), b64["ce_min"].view(np.int64))
    _check_against_fp64(w, runs, f"k={k} co={co}")
    _check_against_fp64(w, _plans(w, refine=k - 1, tq=4, co=co), f"k={k - 1} co={co}",
                        strict=False)


@pytest.mark.parametrize("cfg", [2, 4, 5])
def test_refine_full_workloads(cfg):
    """The batched, ragged and long-baseline workloads at full size, minimum
    only: with four confirmed units per curve the split path's minima are
    the FP64 path's on every curve."""
    w = synth.make_config(cfg)
    say(f"[refine] full workload {cfg}: {w.n_curves} curves")
    _check_against_fp64(w, _plans(w, refine=4, want_cube=False), f"config {cfg}")


def test_refine_in_period_ranges():
    """The chunked driver with the split path and the FP64 confirmation over
    period ranges of a slice of the batched workload: the merged minima are
    the FP64 path's one-launch minima, the merged CE values FP64 ones."""
    from paper_2006_06866_amd import chunked
    w = synth.make_config(2).subset(np.arange(8))
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag)
    _, best = plan.execute(t, m, P, Pd)
    torch.cuda.synchronize()
    want = gce.best_fields(best)
    plan.close()
    acc = chunked.search_chunked(t, m, w.offsets, P, Pd, w.n_phase, w.n_mag, 6000,
                                 precision=gce.PRECISION_SPLIT_FP32, refine_units=4)
    got = gce.best_fields(acc)
    assert np.array_equal(got["flat_index"], want["flat_index"])
    tol = np.array([ce_tolerance(h, w.n_phase, w.n_mag, n) for h, n in
                    zip(want["ce_min"], w.lengths)])
    assert np.all(np.abs(got["ce_min"] - want["ce_min"]) <= tol)
