"""CPU checks of the benchmark's roofline bookkeeping: the FLOP-form
fraction of the defining expression, the VALU slot model, and the counter
and traffic records, which count only while the search kernel's code hashes
to the profiled code."""
import json
import math
import os

import numpy as np

import bench
from paper_2006_06866_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _info(tq, wpu=1, table=0):
    return {"trials_per_lane": tq, "waves_per_unit": wpu, "table_in_lds": table}


def test_search_kernel_names():
    """The kernel a plan launches, as the profiler names it: compiled bin
    counts or 0 (any count), trials, table in LDS (not for the first of two
    launches), bin kind; two waves per unit are k_search_co."""
    assert (bench.search_kernel_name(0, 10, False, _info(8, 2))
            == "gce::k_search_co<0, 10, 8, 0, 0>")
    assert (bench.search_kernel_name(1, 50, True, _info(2, 2, 1))
            == "gce::k_search_co<1, 50, 2, 1, 1>")
    assert bench.search_kernel_name(0, 64, False, _info(4, 1, 2)) == "gce::k_search<0, 0, 4, 0, 0>"


def test_roofline_flop_form_and_slot_model():
    w = synth.make_config(2)
    kernel_s = 0.0525
    r = bench.roofline(0, w, kernel_s, 2, _info(4), as_recorded=False)
    rate = w.point_trials / kernel_s
    assert r["flops_per_point_trial"] == 8.0 and r["lane_ops_per_point_trial"] == 7.0
    assert math.isclose(r["achieved"], 8.0 * rate / 1e12)
    assert math.isclose(r["frac"], r["achieved"] / 78.6)
    assert math.isclose(r["frac_lane_ops"], 7.0 * rate / (256 * 64 * 2.4e9))
    # FP64 at four trials per lane: 4 + 2/4 slots per point-trial plus the
    # segment flush, 5 segments x 10 bins x 2 words x 5 VALU per wave over
    # 600 epochs x 4 trials
    flush = 5 * 10 * 2 * 5.0 / (4 * 600)
    assert math.isclose(r["valu_slots_per_point_trial"], 4.5 + flush)
    s = bench.roofline(1, w, kernel_s, 2, _info(8, 2), as_recorded=False)
    assert math.isclose(s["frac"], s["achieved"] / 157.3)
    assert math.isclose(s["valu_slots_per_point_trial"], 3.0 + 3.5 / 8 + 5 * 10 * 4 * 5.0 / (8 * 600))
    assert r["traffic"] is None and r["valu_busy_counters"] is None


def test_records_count_only_for_the_profiled_code():
    with open(os.path.join(ROOT, "profiles", "k_search_counters.json")) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "profiles", "k_search_c2_traffic.json")) as f:
        tra = json.load(f)
    sha = bench.search_source_sha256()
    # comments and blank lines do not change the hash; code does
    texts = []
    for name in bench.SEARCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2006_06866_amd", "csrc", name)) as f:
            texts.append(f.read())
    assert bench.search_source_sha256([t + "\n// a note\n\n" for t in texts]) == sha
    assert bench.search_source_sha256([texts[0] + "\nint x;\n", *texts[1:]]) != sha
    k64 = rec["kernels"]["c2_fp64"]["kernel"]
    if rec["kernel_source_sha256"] == sha:
        c = bench.measured_counters(2, 0, k64)
        assert c is not None and 0.0 < c["valu_busy"] <= 1.05
        assert c["kernel"] == k64
    else:
        assert bench.measured_counters(2, 0, k64) is None
    # another kernel (tiling) than the recorded one: no record
    assert bench.measured_counters(2, 0, "gce::k_search<0, 10, 2, 0, 0>") is None
    if tra["kernel_source_sha256"] == sha:
        assert bench.measured_traffic(2, k64) == tra["per_launch_bytes"][k64]
    else:
        assert bench.measured_traffic(2, k64) is None
    assert bench.measured_traffic(2, "gce::k_search<0, 10, 2, 0, 0>") is None
    assert bench.measured_traffic(2, k64, as_recorded=False) is None
