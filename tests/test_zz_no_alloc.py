"""The allocation-free entry point gce_search_noalloc against gce_search,
through the C ABI: the same CE cube (within the FP64 tolerance) and minima on
consecutive calls of different sizes, with nothing allocated by the library
(its fixed device array holds the workspace)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import synth
from gce_testlib import say, upload, assert_cube_close, assert_best_valid

pytestmark = pytest.mark.gpu


def _outputs(w):
    cube = torch.empty((w.n_curves, w.pdots.size, w.periods.size), dtype=torch.float64,
                       device="cuda")
    best = torch.empty((w.n_curves, gce.BEST_WORDS), dtype=torch.float64, device="cuda")
    return cube, best


def _compare(w, label):
    d = upload(w)
    say(f"[no-alloc] {label}: curves={w.n_curves} n_p={w.periods.size} n_pd={w.pdots.size}")
    ref_cube, ref_best = gce.search(d[0], d[1], w.offsets, d[2], d[3], w.n_phase, w.n_mag)
    cube, best = _outputs(w)
    gce.search(d[0], d[1], w.offsets, d[2], d[3], w.n_phase, w.n_mag, out_ce=cube,
               out_best=best, no_alloc=True)
    torch.cuda.synchronize()
    rc, c = ref_cube.cpu().numpy(), cube.cpu().numpy()
    assert_cube_close(c, rc, w, label)
    bf, rf = gce.best_fields(best), gce.best_fields(ref_best)
    assert_best_valid(bf["flat_index"], bf["ce_min"], rf["flat_index"], rf["ce_min"], rc, w,
                      label)
    assert np.allclose(bf["ce_mean"], rf["ce_mean"], rtol=1e-12, atol=1e-14), label
    return c, bf


def test_noalloc_matches_gce_search_on_consecutive_calls():
    # a slice of the batched workload (12 x 600 epochs, 20,000 x 64 grid),
    # then a smaller ragged batch, then the first again
    w1 = synth.make_config(2).subset(np.arange(12))
    w2 = synth.random_curves(5, [37, 200, 5, 64], n_freq=70, n_pdots=3)
    _compare(w1, "c2 slice")
    c2, bf2 = _compare(w2, "small ragged")
    oc, obf, obc = oracle.search(w2.times, w2.mags, w2.offsets, w2.periods, w2.pdots,
                                 w2.n_phase, w2.n_mag)
    assert_cube_close(c2, oc, w2, "small ragged vs oracle")
    assert_best_valid(bf2["flat_index"], bf2["ce_min"], obf, obc, oc, w2, "oracle")
    _compare(w1, "c2 slice again")


def test_noalloc_allocates_nothing_and_bounds_its_shapes():
    """With allocation failure injected, gce_search fails (it would allocate
    a plan) while gce_search_noalloc still runs; a shape whose workspace
    exceeds the fixed array is refused with GCE_EWORKSPACE."""
    import os
    w = synth.random_curves(9, [120, 80], n_freq=100, n_pdots=2)
    d = upload(w)
    cube, best = _outputs(w)
    old = os.environ.get("GCE_FAIL_ALLOC")
    os.environ["GCE_FAIL_ALLOC"] = "1"
    try:
        with pytest.raises(gce.GceError) as ei:
            gce.search(d[0], d[1], w.offsets, d[2], d[3], w.n_phase, w.n_mag, out_ce=cube,
                       out_best=best)
        assert ei.value.status == -2
        gce.search(d[0], d[1], w.offsets, d[2], d[3], w.n_phase, w.n_mag, out_ce=cube,
                   out_best=best, no_alloc=True)
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["GCE_FAIL_ALLOC"]
        else:
            os.environ["GCE_FAIL_ALLOC"] = old
    oc, obf, obc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                                 w.n_mag)
    assert_cube_close(cube.cpu().numpy(), oc, w, "injected")
    bf = gce.best_fields(best)
    assert_best_valid(bf["flat_index"], bf["ce_min"], obf, obc, oc, w, "injected")
    c2 = synth.make_config(2)   # twice over: 2.6 M work units, beyond the array
    big = synth.Workload("c2 twice", np.concatenate([c2.times, c2.times]),
                         np.concatenate([c2.mags, c2.mags]),
                         np.concatenate([c2.offsets, c2.offsets[1:] + c2.offsets[-1]]),
                         c2.periods, c2.pdots, c2.n_phase, c2.n_mag)
    db = upload(big)
    with pytest.raises(gce.GceError) as ei:
        gce.search(db[0], db[1], big.offsets, db[2], db[3], big.n_phase, big.n_mag,
                   want_cube=False, no_alloc=True)
    assert ei.value.status == -4
