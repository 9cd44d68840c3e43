#!/usr/bin/env python3
"""Benchmark: conditional-entropy (P, Pdot) search on one MI355X.

One step = one whole search (grid set-up, per-curve preparation, the search
kernel writing the full CE cube, per-curve minimum) over the batched workload:
512 synthetic light curves x 600 epochs, 20,000 periods x 64 Pdots, 10 phase x
5 magnitude bins (Katz et al. 2020, Sec. 2.3).  `value` is the FP64 path
(bit-exact bins); the split-precision path (FP32 Pdot term and binning) is
timed the same way and compared with it: recovered minima, CE differences and
bin mismatches.  Inputs are resident in HBM before each timed region.  Prints
one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("point-trials/sec (1 MI355X), split-FP32 vs FP64 at equal best-(P,Pdot); "
          "% VALU peak")

# MI355X published peaks (AMD): FP64 vector 78.6 TFLOP/s and FP32 vector
# 157.3 TFLOP/s (FMA = 2).  Measured issue costs of a wave64 instruction on one
# SIMD: 4 cycles for FP64 arithmetic, conversions, fract and integer ops, 2
# cycles for v_fma_f32.  The VALU slot peak, one 4-cycle slot per SIMD:
# 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-slots/s.
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_VALU_TLANE = 256 * 64 * 2.4e9 / 1e12

WORKLOADS = {
    1: "c1: 1 curve x 200 epochs, 2,000 P x 1 Pdot, 10x5 bins",
    2: "c2: 512 curves x 600 epochs (3 yr nightly cadence, eclipses), "
       "20,000 P x 64 Pdot, 10x5 bins",
    4: "c4: 8,192 ragged curves (50-3,000 epochs), 10,000 P x 32 Pdot, 10x5 bins",
    5: "c5: 64 curves x 5,000 epochs (10 yr, 2 filters), 100,000 P x 256 Pdot, "
       "20x10 bins",
    6: "c6: paper scale: 135 binaries x 500 epochs (~10 yr), 5,183,995 P x 32 Pdot, "
       "50x10 bins with 50% phase overlap, minimum only",
}
TABLES = {"auto": 0, "global": 1, "lds": 2}


def flops_per_point_trial(precision, n_pd, n_phase, n_mag, mean_n, entries_per_point=1.0):
    """Algorithmic flops per point-trial (FMA = 2), the precision's own kind.

    FP64: per point and trial y = fma(-Pdot/2, x^2, x) (2), y - floor(y) (1),
    phase * n_phase (1); per point and period, shared by the n_pd trials,
    x = dt * (1/P) (1) and x^2 (1).  Split: the per-trial part in FP32, the
    same 4 flops.  Both: per trial the entropy sums, n_phase * (n_mag + 1)
    additions, a subtraction and a division, spread over the curve's points.
    With overlapping magnitude bins the per-point part is done once per
    histogram entry (entries_per_point per epoch).
    """
    return (4.0 + 2.0 / n_pd) * entries_per_point + (n_phase * (n_mag + 1) + 2) / mean_n


def valu_instr_per_point_trial(precision, tq, w, entries_per_point=1.0):
    """VALU issue slots the kernel's design takes per point-trial, in units
    of one wave64 instruction on one SIMD (4 cycles; measured on MI355X:
    v_fma_f64, v_add_f64, v_fract_f64, v_cvt_i32_f64, v_fract_f32 and
    v_lshl_add_u32 take 4 cycles, v_fma_f32 takes 2, i.e. half a slot).

    Fold and binning, per point-trial: FP64 fma, fract, the round-down fma
    that floors phase * n_phase, the histogram address (4 slots); split two
    FP32 fmas (Pdot term, rounding) at half a slot, fract and the address
    (3 slots).  Per epoch and lane, shared by the lane's tq Pdot trials:
    FP64 x and x^2 (2); split x and frac(x) in FP64, two conversions to
    float, the half-bin shift and x^2 in FP32 (5).

    Segment flush, per magnitude segment, phase bin and packed word (two
    trials): the marginal add, two table-offset extractions and two FP64
    adds, plus the neighbour add with overlapping bins.  A wave holds
    ceil(tq / 2) words per bin and folds n_mag segments per work unit, so
    over the workload this adds n_mag * n_phase * ceil(tq / 2) * k per wave
    against sum(N) * tq point-trials per lane.

    With overlapping magnitude bins an epoch is folded once per magnitude
    bin that holds it: the per-point part scales by the entries per epoch."""
    import numpy as np
    point = (4.0 + 2.0 / tq if precision == 0 else 3.0 + 5.0 / tq) * entries_per_point
    k = 5.0 + (1.0 if w.phase_overlap else 0.0)
    words = (tq + 1) // 2
    lengths = np.asarray(w.lengths, dtype=np.float64)
    flush = w.n_mag * w.n_phase * words * k * lengths.size / (tq * lengths.sum())
    return point + flush


def cpu_baseline(w, gpu_cube_rows, budget_s):
    """Time the oracle (as it stands) on whole curves of the same workload
    until about budget_s seconds of CPU work; compare its CE rows and minima
    with the GPU's FP64 rows on the same curves.  Where one curve's full grid
    would take more than half the budget (the paper-scale grid), every
    sampled curve is searched over the first periods of the grid instead,
    sized from a short probe, and there is no GPU row to compare."""
    import numpy as np
    import oracle
    from paper_2006_06866_amd import synth

    threads = oracle.max_threads()
    n_p = full_np = w.periods.size
    probe_p = min(n_p, 2048)
    probe = w.subset(np.arange(1))
    t0 = time.perf_counter()
    oracle.search(probe.times, probe.mags, probe.offsets, probe.periods[:probe_p],
                  probe.pdots, probe.n_phase, probe.n_mag, n_threads=threads,
                  want_cube=False, phase_overlap=w.phase_overlap,
                  mag_overlap=w.mag_overlap)
    per_period = (time.perf_counter() - t0) / probe_p
    sliced = per_period * n_p > 0.5 * budget_s
    if sliced:
        n_p = max(probe_p, int(0.25 * budget_s / per_period))
        w = synth.Workload(w.name, w.times, w.mags, w.offsets, w.periods[:n_p], w.pdots,
                           w.n_phase, w.n_mag, phase_overlap=w.phase_overlap,
                           mag_overlap=w.mag_overlap)
    done, spent, pt = 0, 0.0, 0
    max_err, best_agree, best_checked = 0.0, 0, 0
    per_curve = None
    while done < w.n_curves:
        if per_curve is not None and spent + 0.5 * per_curve > budget_s:
            break
        k = 1 if per_curve is None else max(1, min(w.n_curves - done,
                                                  int((budget_s - spent) / per_curve)))
        sub = w.subset(np.arange(done, done + k))
        g = None if sliced else gpu_cube_rows(done, done + k)
        t0 = time.perf_counter()
        oc, obf, obc = oracle.search(sub.times, sub.mags, sub.offsets, sub.periods,
                                     sub.pdots, sub.n_phase, sub.n_mag, n_threads=threads,
                                     want_cube=g is not None,
                                     phase_overlap=w.phase_overlap,
                                     mag_overlap=w.mag_overlap)
        spent += time.perf_counter() - t0
        pt += sub.point_trials
        per_curve = spent / (done + k)
        if g is not None and oc is not None:
            max_err = max(max_err, float(np.abs(g - oc).max()))
            best_agree += int(np.sum(g.reshape(k, -1).argmin(axis=1) == obf))
            best_checked += k
        done += k
    grid = (f"first {n_p} of {full_np} periods x {w.pdots.size} Pdots" if sliced
            else f"full {n_p} x {w.pdots.size} grid")
    # the same oracle on one thread: the first curve over a slice of the
    # periods sized to ~2 s from a short probe
    one = w.subset(np.arange(1))
    p1 = min(one.periods.size, 64)
    t0 = time.perf_counter()
    oracle.search(one.times, one.mags, one.offsets, one.periods[:p1], one.pdots,
                  one.n_phase, one.n_mag, n_threads=1, want_cube=False,
                  phase_overlap=w.phase_overlap, mag_overlap=w.mag_overlap)
    per = (time.perf_counter() - t0) / p1
    p1 = int(min(one.periods.size, max(p1, 2.0 / max(per, 1e-9))))
    t0 = time.perf_counter()
    oracle.search(one.times, one.mags, one.offsets, one.periods[:p1], one.pdots,
                  one.n_phase, one.n_mag, n_threads=1, want_cube=False,
                  phase_overlap=w.phase_overlap, mag_overlap=w.mag_overlap)
    t1 = time.perf_counter() - t0
    pt1 = int(one.offsets[-1]) * p1 * one.pdots.size
    return ({"value": pt / spent, "unit": "point-trials/s", "cores": threads,
             "kind": "oracle",
             "sample": f"{done} of {w.n_curves} curves, {grid}, {pt:.3g} point-trials "
                       f"in {spent:.1f} s",
             "value_1core": pt1 / t1,
             "sample_1core": f"curve 0, first {p1} periods x {one.pdots.size} Pdots, "
                             f"{pt1:.3g} point-trials in {t1:.1f} s on one thread"},
            {"curves_compared": best_checked, "max_abs_dH": max_err,
             "argmin_equal": f"{best_agree}/{best_checked}"})


def timed_leg(gce, torch, np, w, dev, inputs, precision, tq, steps, warmup, cube_on,
              graph=False, table=0):
    """Warm up, then time exactly `steps` whole searches.  With graph=True the
    search (all four kernels) is captured once in a HIP graph and the timed
    steps are graph replays; the search kernel's own duration then comes
    from a separate eager pass with events."""
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    precision=precision, trials_per_lane=tq,
                    phase_overlap=w.phase_overlap, table_placement=table,
                    mag_overlap=w.mag_overlap, device=dev)
    return _time_plan(torch, np, plan, inputs, steps, warmup, cube_on, graph)


def _time_plan(torch, np, plan, inputs, steps, warmup, cube_on, graph):
    dev = plan.device
    cube = plan.new_cube() if cube_on else None
    best = plan.new_best()
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        plan.execute(*inputs, out_ce=cube, out_best=best, stream=stream)
    torch.cuda.synchronize()
    if graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.execute(*inputs, out_ce=cube, out_best=best,
                         stream=torch.cuda.current_stream(dev))
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    plan.set_timing(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(*inputs, out_ce=cube, out_best=best, stream=stream)
    torch.cuda.synchronize()
    if not graph:
        elapsed = time.perf_counter() - t0
    kernel_ms = plan.search_times_ms()
    plan.set_timing(0)
    return plan, cube, best, elapsed, float(np.mean(kernel_ms)) / 1e3


SEARCH_SOURCES = ("gce_search.h", "gce_device.h")


def search_source_sha256(texts=None):
    """sha256 over the search kernel's code (the template and its device
    helpers, with // comments and blank lines dropped), which the committed
    counter summaries are tied to."""
    import hashlib
    h = hashlib.sha256()
    if texts is None:
        texts = []
        for name in SEARCH_SOURCES:
            with open(os.path.join(ROOT, "paper_2006_06866_amd", "csrc", name)) as f:
                texts.append(f.read())
    for text in texts:
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(config, precision, as_recorded=True):
    """HBM bytes per search launch from the committed rocprofv3 counter
    summary, or None when the kernel source has changed since it was taken
    or the run differs from the recorded one (as_recorded: the whole
    workload, default options)."""
    if not as_recorded:
        return None
    path = os.path.join(ROOT, "profiles", f"k_search_c{config}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        sha = search_source_sha256()
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    key = "k_search<fp64>" if precision == 0 else "k_search<split>"
    return rec.get("per_launch_bytes", {}).get(key)


def roofline(precision, w, kernel_s, config, tq, entries_per_point=1.0, as_recorded=True):
    """entries_per_point: histogram entries per epoch (above 1 only with
    overlapping magnitude bins, where an epoch is folded once per bin that
    holds it)."""
    pt = w.point_trials
    mean_n = float(w.lengths.mean())
    fpp = flops_per_point_trial(precision, w.pdots.size, w.n_phase, w.n_mag,
                                mean_n, entries_per_point)
    achieved = fpp * pt / kernel_s / 1e12
    peak = PEAK_FP64_TFLOPS if precision == 0 else PEAK_FP32_TFLOPS
    instr = valu_instr_per_point_trial(precision, tq, w, entries_per_point)
    return {
        "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": measured_traffic(config, precision, as_recorded),
        "kernel": "k_search<%s>" % ("fp64" if precision == 0 else "split"),
        "kernel_ms": kernel_s * 1e3, "flops_per_point_trial": fpp,
        "valu_instr_per_point_trial": instr,
        "valu_frac": instr * pt / kernel_s / 1e12 / PEAK_VALU_TLANE,
    }


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timing_sweep():
    """Sec. 2.3.2 timing figure axes on synthetic noise curves: for each
    (n_phase, N, search points, n_Pdot) the FP64 search kernel's time per
    light curve per search point, from HIP events over 3 executes of a plan
    holding enough curves for a measurable launch."""
    import numpy as np
    import torch
    import paper_2006_06866_amd as gce
    from paper_2006_06866_amd import synth

    dev = torch.device("cuda:0")
    rows = []
    for n_phase in (15, 50):
        for n in (100, 1000):
            for n_search in (10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7):
                for n_pd in (1, 32):
                    n_p = max(1, n_search // n_pd)
                    k = int(max(1, min(512, 2e10 // (n * n_p * n_pd))))
                    w = synth.random_curves(7 + n_phase + n, [n] * k, n_freq=n_p,
                                            n_pdots=n_pd, n_phase=n_phase, n_mag=10,
                                            pdot_scale=1e-12)
                    inputs = [torch.from_numpy(a).to(dev)
                              for a in (w.times, w.mags, w.periods, w.pdots)]
                    plan = gce.Plan(w.offsets, n_p, n_pd, n_phase, 10, device=dev)
                    best = plan.new_best()
                    plan.execute(*inputs, out_best=best)
                    plan.set_timing(3)
                    for _ in range(3):
                        plan.execute(*inputs, out_best=best)
                    torch.cuda.synchronize()
                    ms = float(np.median(plan.search_times_ms()))
                    info = plan.info()
                    plan.close()
                    rows.append({"n_phase": n_phase, "N": n, "search_points": n_p * n_pd,
                                 "n_pdot": n_pd, "curves": k,
                                 "trials_per_lane": info["trials_per_lane"],
                                 "table_in_lds": info["table_in_lds"], "kernel_ms": ms,
                                 "ns_per_curve_per_point": ms * 1e6 / (k * n_p * n_pd),
                                 "point_trials_per_s": k * n * n_p * n_pd / (ms * 1e-3)})
                    log(f"sweep {rows[-1]}")
    print(json.dumps({"sweep": rows, "kernel": "k_search<fp64>",
                      "data": "synthetic noise curves, uniform epochs"}), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cube", action="store_true", help="minimum only (no CE cube)")
    ap.add_argument("--trials-per-lane", type=int, default=0)
    ap.add_argument("--no-split", action="store_true", help="skip the split leg")
    ap.add_argument("--table", choices=["auto", "global", "lds"], default="auto",
                    help="where the search kernel reads its c ln c table")
    ap.add_argument("--mag-overlap", action="store_true",
                    help="50%%-overlapping magnitude bins in every leg")
    ap.add_argument("--chunk-periods", type=int, default=0, metavar="P",
                    help="also run the FP64 search in period ranges of P periods with a "
                         "checkpoint after each (the chunked driver) and report its time "
                         "and agreement with the single launch")
    ap.add_argument("--curves", type=int, default=0,
                    help="profiling aid: only the first CURVES curves of the workload")
    ap.add_argument("--graph", action="store_true",
                    help="time HIP-graph replays of the whole search")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU-baseline budget; 0 skips the oracle leg")
    ap.add_argument("--sweep", action="store_true",
                    help="time per light curve per search point over n_phase in {15, 50}, "
                         "N in {100, 1000}, 1e3..1e7 search points at n_Pdot 1 and 32 "
                         "(the axes of the paper's timing figure), one JSON line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (the "
                         "known-size kernel that scales HBM byte counters)")
    args = ap.parse_args()

    if args.sweep:
        raise SystemExit(timing_sweep())
    if args.copy_calibration > 0:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4,
                          "copies": 3}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this search runs on one GPU only; multi-GPU runs are not "
              "supported (each GPU would take its own share of the curves)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2006_06866_amd as gce
    from paper_2006_06866_amd import synth

    dev = torch.device("cuda:0")
    w = synth.make_config(args.config)
    if 0 < args.curves < w.n_curves:
        w = w.subset(range(args.curves))
    if args.mag_overlap:
        w.mag_overlap = True
    log(f"workload {WORKLOADS[args.config]}: {w.point_trials:.3g} point-trials")
    inputs = tuple(torch.from_numpy(a).to(dev) for a in (w.times, w.mags, w.periods, w.pdots))
    pt = w.point_trials
    # the paper-scale cube would be 179 GB: minimum and statistics only
    cube_on = not args.no_cube and args.config != 6

    plan64, cube64, best64, el64, k64 = timed_leg(
        gce, torch, np, w, dev, inputs, 0, args.trials_per_lane, args.steps,
        args.warmup, cube_on, args.graph, TABLES[args.table])
    log(f"fp64: {el64 / args.steps * 1e3:.2f} ms/step, kernel {k64 * 1e3:.2f} ms")
    # histogram entries per epoch: the total of one trial's histogram per
    # curve (it does not depend on the trial)
    entries = 1.0
    if w.mag_overlap:
        tot = plan64.debug_counts(*inputs, np.arange(w.n_curves),
                                  np.zeros(w.n_curves, dtype=np.int64)).sum().item()
        entries = float(tot) / float(w.offsets[-1]) / (2.0 if w.phase_overlap else 1.0)
    # the committed traffic record is of the whole workload with default options
    as_recorded = (args.curves <= 0 and not args.no_cube and not args.mag_overlap
                   and args.table == "auto" and args.trials_per_lane == 0)
    value = pt * args.steps / el64
    bf64 = gce.best_fields(best64)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "point-trials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el64 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.config] + (
                f" (first {w.n_curves} curves)" if 0 < args.curves else ""),
            "n_curves": w.n_curves, "points": int(w.offsets[-1]),
            "n_periods": int(w.periods.size), "n_pdots": int(w.pdots.size),
            "n_phase": w.n_phase, "n_mag": w.n_mag, "precision": "fp64",
            "cube": cube_on, "trials_per_lane": plan64.info()["trials_per_lane"],
            "table_in_lds": int(plan64.info()["table_in_lds"]),
            "timing": "hip-graph replay" if args.graph else "eager launches",
            "mag_overlap": bool(w.mag_overlap),
            "entries_per_epoch": entries,
        },
        "roofline": roofline(0, w, k64, args.config, plan64.info()["trials_per_lane"],
                             entries, as_recorded),
    }
    if "p_true" in w.truth:
        # injections off the grid (Sec. 3.1 criterion), and the same search
        # with Pdot = {0} beside it: what the Pdot axis buys
        from paper_2006_06866_amd import recovery
        ptrue = w.truth["p_true"]
        short = ptrue <= 10.0 * synth.MINUTE
        out["recovery_fp64"] = {"all": recovery.summary(bf64, w.periods, ptrue),
                                "p0_le_10min": recovery.summary(bf64, w.periods, ptrue, short)}
        plan0 = gce.Plan(w.offsets, w.periods.size, 1, w.n_phase, w.n_mag,
                         phase_overlap=w.phase_overlap, mag_overlap=w.mag_overlap,
                         device=dev)
        _, b0 = plan0.execute(inputs[0], inputs[1], inputs[2],
                              torch.zeros(1, dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        bf0 = gce.best_fields(b0)
        out["recovery_pdot0"] = {"all": recovery.summary(bf0, w.periods, ptrue),
                                 "p0_le_10min": recovery.summary(bf0, w.periods, ptrue, short)}
        plan0.close()
    else:
        has = w.truth["inj_p"] >= 0
        out["recovery_fp64"] = {
            "curves_with_injection": int(has.sum()),
            "injected_period_found": int(np.sum((bf64["period_index"] == w.truth["inj_p"]) & has)),
            "injected_period_and_pdot_found": int(np.sum(
                (bf64["period_index"] == w.truth["inj_p"]) &
                (bf64["pdot_index"] == w.truth["inj_q"]) & has)),
        }

    if args.chunk_periods > 0:
        # the period-range driver with a checkpoint after every range, timed
        # end to end (host merges and checkpoint writes included)
        import tempfile
        from paper_2006_06866_amd import chunked
        with tempfile.TemporaryDirectory(prefix="gce_chunk_") as d:
            t0 = time.perf_counter()
            acc = chunked.search_chunked(
                inputs[0], inputs[1], w.offsets, inputs[2], inputs[3], w.n_phase, w.n_mag,
                args.chunk_periods, checkpoint=os.path.join(d, "ck.npz"),
                phase_overlap=w.phase_overlap, mag_overlap=w.mag_overlap,
                table_placement=TABLES[args.table])
            el = time.perf_counter() - t0
        bc = gce.best_fields(acc)
        n_ranges = len(chunked.range_bounds(w.periods.size, args.chunk_periods))
        out["chunked"] = {
            "chunk_periods": args.chunk_periods, "ranges": n_ranges,
            "ms": el * 1e3, "one_launch_ms": el64 / args.steps * 1e3,
            "overhead": el / (el64 / args.steps) - 1.0,
            "best_equal": f"{int(np.sum(bc['flat_index'] == bf64['flat_index']))}/{w.n_curves}",
            "max_abs_dmean": float(np.nanmax(np.abs(bc["ce_mean"] - bf64["ce_mean"]))),
        }
        log(f"chunked: {n_ranges} ranges, {el * 1e3:.1f} ms")

    if not args.no_split:
        plan32, cube32, best32, el32, k32 = timed_leg(
            gce, torch, np, w, dev, inputs, 1, args.trials_per_lane, args.steps,
            args.warmup, cube_on, args.graph, TABLES[args.table])
        log(f"split: {el32 / args.steps * 1e3:.2f} ms/step, kernel {k32 * 1e3:.2f} ms")
        bf32 = gce.best_fields(best32)
        strict = int(np.sum(bf32["flat_index"] == bf64["flat_index"]))
        split = {
            "value": pt * args.steps / el32, "unit": "point-trials/s",
            "ms_per_step": el32 / args.steps * 1e3,
            "speedup_vs_fp64": el64 / el32,
            "trials_per_lane": plan32.info()["trials_per_lane"],
            "table_in_lds": int(plan32.info()["table_in_lds"]),
            "roofline": roofline(1, w, k32, args.config, plan32.info()["trials_per_lane"],
                                 entries, as_recorded),
            "best_equal_strict": f"{strict}/{w.n_curves}",
        }
        if cube_on:
            # tolerant agreement: the FP64 CE at the split minimum is within
            # 1e-5 of the FP64 minimum
            flat64 = cube64.view(w.n_curves, -1)
            h_at = flat64.gather(1, torch.from_numpy(bf32["flat_index"]).to(dev).view(-1, 1)).view(-1)
            hmin = torch.from_numpy(bf64["ce_min"]).to(dev)
            split["best_equal_tolerant_1e-5"] = (
                f"{int(((h_at - hmin) <= 1e-5).sum().item())}/{w.n_curves}")
            dh = (cube32.view(w.n_curves, -1).double() - flat64).abs()
            split["max_abs_dH"] = float(dh.max().item())
            split["frac_abs_dH_le_1e-5"] = float((dh <= 1e-5).double().mean().item())
            del dh
        # bin mismatches against the FP64 bins (which are bit-exact to the
        # reference) on sampled trials
        rng = np.random.default_rng(2006)
        ci = rng.integers(0, w.n_curves, 4096)
        fi = rng.integers(0, w.periods.size * w.pdots.size, 4096)
        c64 = plan64.debug_counts(*inputs, ci, fi).long()
        c32 = plan32.debug_counts(*inputs, ci, fi).long()
        moved = float((c64 - c32).abs().sum().item()) / 2
        split["count_mismatch_rate"] = moved / float(w.lengths[ci].sum())
        split["count_mismatch_sample"] = "4096 random trials"
        out["split"] = split
        plan32.close()
        del cube32

    if args.cpu_seconds > 0:
        def rows(a, b):
            return None if cube64 is None else cube64[a:b].cpu().numpy()
        cb, par = cpu_baseline(w, rows, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["parity"] = par
    print(json.dumps(out), flush=True)
    plan64.close()


if __name__ == "__main__":
    main()
