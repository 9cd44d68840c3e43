#!/usr/bin/env python3
"""Benchmark: conditional-entropy (P, Pdot) search on one MI355X.

One step = one whole search (grid set-up, per-curve preparation, the search
kernel writing the full CE cube, per-curve minimum) over the batched workload:
512 synthetic light curves x 600 epochs, 20,000 periods x 64 Pdots, 10 phase x
5 magnitude bins (Katz et al. 2020, Sec. 2.3).  The timed steps are replays of
the whole search captured once in a HIP graph (--eager: launches instead).
`value` is the FP64 path (bit-exact bins); the split-precision path (FP32 Pdot
term and binning) is timed the same way and compared with it: recovered
minima, CE differences and bin mismatches.  The ragged (8,192 curves) and
long-baseline (64 x 5,000 epochs, 20 x 10 bins) workloads run the same two
legs with fewer steps, under "workloads".  Inputs are resident in HBM before
each timed region.  Prints one JSON line.
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


# The defining expression of the fold and bin (Eq. (3), one point-trial):
# x = dt * (1/P), x^2, y = fma(-Pdot/2, x^2, x), floor(y), y - floor(y),
# phase * n_phase, conversion to an integer bin: 7 operations, 8 flops with
# the fma counted as 2.  The kernels compute x and x^2 once per (epoch,
# period) and reuse them along the Pdot axis, and fuse fract and the floored
# product, so they issue fewer instructions than these counts: the 7-lane-op
# rate can exceed the lane-op peak, and the flop rate is the fraction that
# stays below 1.
FLOPS_PER_POINT_TRIAL = 8.0
LANE_OPS_PER_POINT_TRIAL = 7.0


def valu_instr_per_point_trial(precision, tq, w, entries_per_point=1.0):
    """VALU issue slots the kernel's design takes per point-trial, in units
    of one wave64 instruction on one SIMD (4 cycles; measured on MI355X:
    v_fma_f64, v_add_f64, v_fract_f64, v_cvt_i32_f64, v_fract_f32 and
    v_lshl_add_u32 take 4 cycles, v_fma_f32 takes 2, i.e. half a slot).

    Fold and binning, per point-trial: FP64 fma, fract, the round-down fma
    that floors phase * n_phase, the histogram address (4 slots); split two
    FP32 fmas (Pdot term, rounding) at half a slot, fract and the address
    (3 slots).  Per epoch and lane, shared by the lane's tq Pdot trials:
    FP64 x and x^2 (2); split x and frac(x) in FP64, the conversion of
    frac(x) to float and x^2 = dt^2 (1/P)^2 in FP32 (3.5).

    Segment flush, per magnitude segment, phase bin and packed word (two
    trials): the marginal add, two table-offset extractions and two FP64
    adds, plus the neighbour add with overlapping bins.  A wave holds
    ceil(tq / 2) words per bin and folds n_mag segments per work unit, so
    over the workload this adds n_mag * n_phase * ceil(tq / 2) * k per wave
    against sum(N) * tq point-trials per lane.

    With overlapping magnitude bins an epoch is folded once per magnitude
    bin that holds it: the per-point part scales by the entries per epoch."""
    import numpy as np
    point = (4.0 + 2.0 / tq if precision == 0 else 3.0 + 3.5 / tq) * entries_per_point
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
              graph=False, table=0, refine=0):
    """Warm up, then time exactly `steps` whole searches.  With graph=True the
    search (all its kernels) is captured once in a HIP graph and the timed
    steps are graph replays; the search kernel's own duration then comes
    from a separate eager pass with events.  refine: the split path's FP64
    confirmation of each curve's `refine` best work units (part of the timed
    search)."""
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    precision=precision, trials_per_lane=tq,
                    phase_overlap=w.phase_overlap, table_placement=table,
                    mag_overlap=w.mag_overlap, refine_units=refine, device=dev)
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


SEARCH_SOURCES = ("gce_search.h", "gce_search_co.h", "gce_device.h")


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


def search_kernel_name(precision, n_phase, phase_overlap, info):
    """The search kernel a plan launches (its first launch, where a ragged
    batch is searched in two), as rocprofv3 names it."""
    nph = n_phase if n_phase in (10, 15, 20, 50) else 0
    base = "gce::k_search_co" if info["waves_per_unit"] == 2 else "gce::k_search"
    ll = 1 if info["table_in_lds"] == 1 else 0
    return (f"{base}<{precision}, {nph}, {info['trials_per_lane']}, {ll}, "
            f"{int(bool(phase_overlap))}>")


def measured_traffic(config, kernel, as_recorded=True):
    """HBM bytes per search launch from the committed rocprofv3 counter
    summary, or None when the kernel source has changed since it was taken,
    the run launches another kernel, or the run differs from the recorded
    one (as_recorded: the whole workload, default options)."""
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
    return rec.get("per_launch_bytes", {}).get(kernel)


def measured_counters(config, precision, kernel):
    """Counter-measured VALU busy of the search kernel on this workload from
    the committed rocprofv3 summary (SQ_INSTS_VALU x 4 cycles / (kernel
    cycles x 1024 SIMDs), with the fraction of 2-cycle FP32 fmas counted at
    half a slot), or None when the kernel source has changed since the
    counters were taken or the run launches another kernel."""
    path = os.path.join(ROOT, "profiles", "k_search_counters.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        sha = search_source_sha256()
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    key = f"c{config}_{'fp64' if precision == 0 else 'split'}"
    r = rec.get("kernels", {}).get(key)
    if r is None or r["kernel"] != kernel:
        return None
    kind = "fp64" if precision == 0 else "fp32"
    return {"valu_busy": r["valu_busy"], "waves_per_simd": r["waves_per_simd"],
            "valu_instr_per_point_trial": r["valu_instr_per_point_trial"],
            "lds_busy": r.get("lds_idx_active_per_cu_cycle"),
            "counted_tflops": r.get(f"counted_{kind}_tflops"), "kernel": r["kernel"],
            "workload": r["workload"], "record": "profiles/k_search_counters.json"}


def roofline(precision, w, kernel_s, config, info, entries_per_point=1.0, as_recorded=True):
    """The dominant kernel (the search) against the VALU peak of its
    precision.  `achieved` counts the defining expression's 8 flops per
    point-trial (FMA = 2) over the workload's point-trials in one launch,
    divided by the kernel's mean launch time.  entries_per_point: histogram
    entries per epoch (above 1 only with overlapping magnitude bins, where an
    epoch is folded once per bin that holds it)."""
    pt = w.point_trials
    rate = pt / kernel_s
    achieved = FLOPS_PER_POINT_TRIAL * rate / 1e12
    peak = PEAK_FP64_TFLOPS if precision == 0 else PEAK_FP32_TFLOPS
    slots = valu_instr_per_point_trial(precision, info["trials_per_lane"], w, entries_per_point)
    kernel = search_kernel_name(precision, w.n_phase, w.phase_overlap, info)
    return {
        "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": measured_traffic(config, kernel, as_recorded),
        "kernel": kernel,
        "kernel_ms": kernel_s * 1e3,
        "flops_per_point_trial": FLOPS_PER_POINT_TRIAL,
        "lane_ops_per_point_trial": LANE_OPS_PER_POINT_TRIAL,
        "frac_lane_ops": LANE_OPS_PER_POINT_TRIAL * rate / 1e12 / PEAK_VALU_TLANE,
        "valu_slots_per_point_trial": slots,
        "valu_frac_model": slots * rate / 1e12 / PEAK_VALU_TLANE,
        "valu_busy_counters": (measured_counters(config, precision, kernel)
                               if as_recorded else None),
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


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def split_vs_fp64(torch, np, gce, w, inputs, plan64, plan32, cube64, cube32, best64,
                  best32):
    """The split path's outputs against the FP64 path's, whose bins are
    bit-exact to the oracle's (the GPU tests check that on every workload):
    recovered minima, CE differences over the whole cube, bin mismatches on
    4,096 sampled trials."""
    bf64, bf32 = gce.best_fields(best64), gce.best_fields(best32)
    strict = bf32["flat_index"] == bf64["flat_index"]
    out = {"reference": "fp64 path (bins bit-exact to the oracle's)",
           "best_equal_strict": f"{int(strict.sum())}/{w.n_curves}"}
    ok = (bf64["flat_index"] >= 0) & (bf32["flat_index"] >= 0)
    if ok.any():
        out["max_abs_dH_reported_minimum"] = float(
            np.max(np.abs(bf32["ce_min"][ok] - bf64["ce_min"][ok])))
    if "inj_p" in w.truth:
        found = (np.asarray(w.truth["inj_p"]) >= 0) & (
            bf64["period_index"] == w.truth["inj_p"]) & (bf64["pdot_index"] == w.truth["inj_q"])
        out["best_equal_strict_where_fp64_recovers_signal"] = (
            f"{int(np.sum(strict & found))}/{int(found.sum())}")
    if cube64 is not None and cube32 is not None:
        flat64 = cube64.view(w.n_curves, -1)
        h_at = flat64.gather(1, torch.from_numpy(bf32["flat_index"]).to(flat64.device)
                             .view(-1, 1)).view(-1)
        hmin = torch.from_numpy(bf64["ce_min"]).to(flat64.device)
        out["best_equal_tolerant_1e-5"] = (
            f"{int(((h_at - hmin) <= 1e-5).sum().item())}/{w.n_curves}")
        flat32 = cube32.view(w.n_curves, -1)
        mx, ok, n = 0.0, 0, 0
        step = max(1, (1 << 28) // flat64.shape[1])
        for c0 in range(0, w.n_curves, step):
            dh = (flat32[c0:c0 + step].double() - flat64[c0:c0 + step]).abs()
            mx = max(mx, float(dh.max().item()))
            ok += int((dh <= 1e-5).sum().item())
            n += dh.numel()
            del dh
        out["max_abs_dH"] = mx
        out["frac_abs_dH_le_1e-5"] = ok / n
        # at the minima: the split CE at the FP64 minimum, and the split path's
        # own minimum against the FP64 CE at that trial
        f64i = torch.from_numpy(bf64["flat_index"]).to(flat64.device).view(-1, 1)
        at64 = flat32.gather(1, f64i).view(-1).double() - hmin
        at32 = torch.from_numpy(bf32["ce_min"]).to(flat64.device) - h_at
        dmin = torch.maximum(at64.abs(), at32.abs()).cpu().numpy()
        out["max_abs_dH_at_minima"] = float(dmin.max())
        if "inj_p" in w.truth:
            found = (np.asarray(w.truth["inj_p"]) >= 0) & (
                bf64["period_index"] == w.truth["inj_p"]) & (bf64["pdot_index"] == w.truth["inj_q"])
            if found.any():
                out["max_abs_dH_at_minima_where_fp64_recovers_signal"] = float(dmin[found].max())
    rng = np.random.default_rng(2006)
    ci = rng.integers(0, w.n_curves, 4096)
    fi = rng.integers(0, w.periods.size * w.pdots.size, 4096)
    c64 = plan64.debug_counts(*inputs, ci, fi).long()
    c32 = plan32.debug_counts(*inputs, ci, fi).long()
    moved = float((c64 - c32).abs().sum().item()) / 2
    out["count_mismatch_rate"] = moved / float(w.lengths[ci].sum())
    out["count_mismatch_sample"] = "4096 random trials"
    return out


def sample_trials(np, w, bf, n_curves_nb, n_random, seed):
    """Trials to check against the oracle: each of n_curves_nb curves' minimum
    and its +-2 neighbours in P and Pdot, plus n_random random trials."""
    rng = np.random.default_rng(seed)
    n_p, n_pd = w.periods.size, w.pdots.size
    ci = list(rng.integers(0, w.n_curves, n_random))
    fi = list(rng.integers(0, n_p * n_pd, n_random))
    for c in rng.choice(w.n_curves, size=min(n_curves_nb, w.n_curves), replace=False):
        if bf["flat_index"][c] < 0:
            continue
        q0, p0 = divmod(int(bf["flat_index"][c]), n_p)
        for dq in range(-2, 3):
            for dp in range(-2, 3):
                if 0 <= q0 + dq < n_pd and 0 <= p0 + dp < n_p:
                    ci.append(int(c))
                    fi.append((q0 + dq) * n_p + p0 + dp)
    return np.array(ci, dtype=np.int64), np.array(fi, dtype=np.int64)


def gather(torch, np, cube, w, ci, fi):
    q, p = np.divmod(fi, w.periods.size)
    d = cube.device
    idx = (torch.from_numpy(ci).to(d), torch.from_numpy(q).to(d), torch.from_numpy(p).to(d))
    return cube[idx].double().cpu().numpy()


def cpu_baseline_samples(np, w, ci, fi, g64, g32, bf64):
    """Part of the cpu_baseline (oracle) leg: the oracle's CE at sampled trials against the
    FP64 and split cubes there, and the FP64 minimum against every sampled
    trial of its curve."""
    import oracle
    h = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase, w.n_mag,
                      ci, fi, phase_overlap=w.phase_overlap, mag_overlap=w.mag_overlap)
    d64 = np.abs(g64 - h)
    beaten = int(np.sum(h < bf64["ce_min"][ci] - 1e-12))
    known = np.isfinite(g64)   # without a cube only the minima are known
    out = {"trials": int(ci.size), "fp64_values_compared": int(known.sum()),
           "fp64_max_abs_dH": float(d64[known].max()),
           "fp64_min_beaten_by_a_sample": beaten}
    if g32 is not None:
        d32 = np.abs(g32 - h)
        out["split_max_abs_dH"] = float(d32.max())
        out["split_frac_abs_dH_le_1e-5"] = float(np.mean(d32 <= 1e-5))
    return out


def run_workload(gce, torch, np, w, dev, config, steps, warmup, graph, cube_on, tq,
                 table, do_split, as_recorded, refine=0):
    """Both legs of one workload.  Returns (summary dict, FP64 leg state)."""
    inputs = tuple(torch.from_numpy(a).to(dev) for a in (w.times, w.mags, w.periods, w.pdots))
    pt = w.point_trials
    plan64, cube64, best64, el64, k64 = timed_leg(
        gce, torch, np, w, dev, inputs, 0, tq, steps, warmup, cube_on, graph, table)
    log(f"c{config} fp64: {el64 / steps * 1e3:.2f} ms/step, kernel {k64 * 1e3:.2f} ms")
    entries = 1.0
    if w.mag_overlap:
        tot = plan64.debug_counts(*inputs, np.arange(w.n_curves),
                                  np.zeros(w.n_curves, dtype=np.int64)).sum().item()
        entries = float(tot) / float(w.offsets[-1]) / (2.0 if w.phase_overlap else 1.0)
    res = {"value": pt * steps / el64, "unit": "point-trials/s",
           "ms_per_step": el64 / steps * 1e3, "steps": steps, "warmup": warmup,
           "trials_per_lane": plan64.info()["trials_per_lane"],
           "table_in_lds": int(plan64.info()["table_in_lds"]),
           "waves_per_unit": plan64.info()["waves_per_unit"],
           "entries_per_epoch": entries,
           "roofline": roofline(0, w, k64, config, plan64.info(), entries, as_recorded)}
    state = {"inputs": inputs, "plan64": plan64, "cube64": cube64, "best64": best64,
             "cube32": None, "el64": el64}
    if do_split:
        plan32, cube32, best32, el32, k32 = timed_leg(
            gce, torch, np, w, dev, inputs, 1, tq, steps, warmup, cube_on, graph, table,
            refine)
        log(f"c{config} split: {el32 / steps * 1e3:.2f} ms/step, kernel {k32 * 1e3:.2f} ms")
        split = {"value": pt * steps / el32, "unit": "point-trials/s",
                 "ms_per_step": el32 / steps * 1e3, "speedup_vs_fp64": el64 / el32,
                 "trials_per_lane": plan32.info()["trials_per_lane"],
                 "table_in_lds": int(plan32.info()["table_in_lds"]),
                 "waves_per_unit": plan32.info()["waves_per_unit"],
                 "refine_units": plan32.info()["refine_units"],
                 "roofline": roofline(1, w, k32, config, plan32.info(), entries,
                                      as_recorded)}
        if split["refine_units"]:
            split["reported_minimum"] = (
                f"FP64 minimum over each curve's {split['refine_units']} work units with "
                "the smallest split minima (split cube, split moments)")
        split.update(split_vs_fp64(torch, np, gce, w, inputs, plan64, plan32, cube64,
                                   cube32, best64, best32))
        res["split"] = split
        state["cube32"] = cube32
        plan32.close()
    return res, state


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cube", action="store_true", help="minimum only (no CE cube)")
    ap.add_argument("--trials-per-lane", type=int, default=0)
    ap.add_argument("--no-split", action="store_true", help="skip the split leg")
    ap.add_argument("--split-refine", type=int, default=4, metavar="K",
                    help="split leg: confirm each curve's minimum in FP64 over its K best "
                         "work units (0: the split minimum as found)")
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
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches instead of HIP-graph replays")
    ap.add_argument("--graph", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--extra", default="4,5,6",
                    help="further workloads run after the headline one, with --extra-steps "
                         "steps each (one for the paper-scale grid; '' for none)")
    ap.add_argument("--extra-steps", type=int, default=2)
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
    graph = not args.eager
    w = synth.make_config(args.config)
    if 0 < args.curves < w.n_curves:
        w = w.subset(range(args.curves))
    if args.mag_overlap:
        w.mag_overlap = True
    log(f"workload {WORKLOADS[args.config]}: {w.point_trials:.3g} point-trials")
    pt = w.point_trials
    # the paper-scale cube would be 179 GB: minimum and statistics only
    cube_on = not args.no_cube and args.config != 6
    # the committed traffic and counter records are of the whole workload
    # with default options
    as_recorded = (args.curves <= 0 and not args.no_cube and not args.mag_overlap
                   and args.table == "auto" and args.trials_per_lane == 0)
    head, st = run_workload(gce, torch, np, w, dev, args.config, args.steps, args.warmup,
                            graph, cube_on, args.trials_per_lane, TABLES[args.table],
                            not args.no_split, as_recorded, args.split_refine)
    plan64, cube64, best64, inputs = st["plan64"], st["cube64"], st["best64"], st["inputs"]
    el64 = st["el64"]
    bf64 = gce.best_fields(best64)

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "point-trials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
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
            "cube": cube_on, "trials_per_lane": head["trials_per_lane"],
            "table_in_lds": head["table_in_lds"],
            "timing": "hip-graph replay" if graph else "eager launches",
            "mag_overlap": bool(w.mag_overlap),
            "entries_per_epoch": head["entries_per_epoch"],
        },
        "roofline": head["roofline"],
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

    if "split" in head:
        out["split"] = head["split"]
    st["cube32"] = None
    torch.cuda.empty_cache()

    # oracle leg: the oracle timed on whole curves of the headline workload
    # (compared with the FP64 cube rows), and kept for the samples of the
    # further workloads below
    if args.cpu_seconds > 0:
        def rows(a, b):
            return None if cube64 is None else cube64[a:b].cpu().numpy()
        cb, par = cpu_baseline(w, rows, args.cpu_seconds)
        cb["cpu_model"] = cpu_model()
        out["cpu_baseline"] = cb
        out["parity"] = par
    plan64.close()
    del cube64, st
    torch.cuda.empty_cache()

    extras = [int(c) for c in args.extra.split(",") if c.strip()] if args.curves <= 0 else []
    workloads = {}
    for cfg in extras:
        if cfg == args.config or cfg not in WORKLOADS:
            continue
        we = synth.make_config(cfg)
        log(f"workload {WORKLOADS[cfg]}: {we.point_trials:.3g} point-trials")
        # the paper-scale grid: one step, minimum only (its cube would be 179 GB)
        cube_e = cfg != 6
        res, st = run_workload(gce, torch, np, we, dev, cfg,
                               args.extra_steps if cube_e else 1, 1, graph, cube_e, 0, 0,
                               not args.no_split, True, args.split_refine)
        res["workload"] = WORKLOADS[cfg]
        res["timing"] = "hip-graph replay" if graph else "eager launches"
        bfe = gce.best_fields(st["best64"])
        if "p_true" in we.truth:   # Sec. 3.1 recovery of the paper-scale injections
            from paper_2006_06866_amd import recovery
            res["recovery_fp64"] = recovery.summary(bfe, we.periods, we.truth["p_true"])
        ci, fi = sample_trials(np, we, bfe, 16, 256, 300 + cfg)
        if cube_e:
            g64 = gather(torch, np, st["cube64"], we, ci, fi)
            g32 = gather(torch, np, st["cube32"], we, ci, fi) if st["cube32"] is not None else None
        else:
            # no cube: the reported minimum at its own trial, NaN elsewhere
            g64 = np.where(fi == bfe["flat_index"][ci], bfe["ce_min"][ci], np.nan)
            g32 = None
        st["plan64"].close()
        del st
        torch.cuda.empty_cache()
        if args.cpu_seconds > 0:
            res["parity"] = cpu_baseline_samples(np, we, ci, fi, g64, g32, bfe)
        workloads[f"c{cfg}"] = res
    if workloads:
        out["workloads"] = workloads
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
