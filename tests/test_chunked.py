"""Period-range chunked search with checkpoint and resume (Sec. 3 grid size,
Sec. 4 batches combined).  The driver is exercised on the CPU with ranges
evaluated by the oracle; the GPU run of the same driver is in
test_gpu_parity.py."""
import os

import numpy as np
import pytest

import oracle
import paper_2006_06866_amd as gce
from paper_2006_06866_amd import build as gbuild
from paper_2006_06866_amd import chunked, synth
from gce_testlib import best_rows


def _ensure_built():
    if not os.path.exists(gce.LIB_PATH):
        gbuild.build()


def _workload():
    return synth.random_curves(12, [40, 65, 130], n_freq=53, n_pdots=3, pdot_scale=5e-9)


def _oracle_range(w, calls):
    def execute_range(p0, p1):
        calls.append((p0, p1))
        cube, _, _ = oracle.search(w.times, w.mags, w.offsets, w.periods[p0:p1], w.pdots,
                                   w.n_phase, w.n_mag)
        return best_rows(cube)
    return execute_range


def _whole(w):
    cube, bf, bc = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots,
                                 w.n_phase, w.n_mag)
    return gce.best_fields(best_rows(cube)), bf, bc


def _same(got, want):
    assert np.array_equal(got["flat_index"], want["flat_index"])
    assert np.array_equal(got["period_index"], want["period_index"])
    assert np.array_equal(got["pdot_index"], want["pdot_index"])
    assert np.array_equal(got["ce_min"], want["ce_min"])
    assert np.allclose(got["ce_mean"], want["ce_mean"], rtol=0, atol=1e-14)
    assert np.allclose(got["ce_std"], want["ce_std"], rtol=1e-11, atol=1e-15)


def test_range_bounds():
    assert chunked.range_bounds(10, 4) == [(0, 4), (4, 8), (8, 10)]
    assert chunked.range_bounds(8, 4) == [(0, 4), (4, 8)]
    assert chunked.range_bounds(3, 10) == [(0, 3)]
    with pytest.raises(ValueError):
        chunked.range_bounds(0, 4)


@pytest.mark.parametrize("chunk", [1, 7, 20, 53, 100])
def test_chunked_equals_whole_grid(chunk):
    _ensure_built()
    w = _workload()
    calls = []
    acc = chunked.run_ranges(w.periods.size, w.pdots.size, chunk, _oracle_range(w, calls),
                             gce.merge_results)
    want, bf, bc = _whole(w)
    _same(gce.best_fields(acc), want)
    assert np.array_equal(gce.best_fields(acc)["flat_index"], bf)
    assert len(calls) == -(-w.periods.size // chunk)


def test_resume_after_interruption(tmp_path):
    _ensure_built()
    w = _workload()
    ck = str(tmp_path / "run.ckpt.npz")
    fp = chunked.fingerprint([w.times, w.mags, w.offsets, w.periods, w.pdots], chunk=10)
    calls = []
    inner = _oracle_range(w, calls)

    class Interrupted(Exception):
        pass

    def flaky(p0, p1):
        if len(calls) == 3:
            raise Interrupted
        return inner(p0, p1)

    with pytest.raises(Interrupted):
        chunked.run_ranges(w.periods.size, w.pdots.size, 10, flaky, gce.merge_results,
                           ck, fp)
    acc3, nxt = chunked.load_checkpoint(ck, fp)
    assert nxt == 3 and calls == [(0, 10), (10, 20), (20, 30)]
    calls.clear()
    acc = chunked.run_ranges(w.periods.size, w.pdots.size, 10, inner, gce.merge_results,
                             ck, fp)
    assert calls == [(30, 40), (40, 50), (50, 53)]       # only the remaining ranges
    want, _, _ = _whole(w)
    _same(gce.best_fields(acc), want)
    # a finished checkpoint returns the result without running anything
    calls.clear()
    again = chunked.run_ranges(w.periods.size, w.pdots.size, 10, inner, gce.merge_results,
                               ck, fp)
    assert calls == [] and np.array_equal(again.view(np.int64), acc.view(np.int64))


def test_checkpoint_of_other_inputs_is_refused(tmp_path):
    _ensure_built()
    w = _workload()
    ck = str(tmp_path / "run.ckpt.npz")
    fp = chunked.fingerprint([w.times, w.mags], n_phase=10)
    chunked.run_ranges(w.periods.size, w.pdots.size, 25, _oracle_range(w, []),
                       gce.merge_results, ck, fp)
    other = chunked.fingerprint([w.times, w.mags], n_phase=11)
    with pytest.raises(ValueError, match="other inputs"):
        chunked.load_checkpoint(ck, other)
    assert chunked.load_checkpoint(str(tmp_path / "missing.npz"), fp) is None


def test_fingerprint_sees_every_input():
    a = np.arange(6, dtype=np.float64)
    base = chunked.fingerprint([a, a], k=1)
    assert base == chunked.fingerprint([a.copy(), a.copy()], k=1)
    b = a.copy()
    b[3] = np.nextafter(b[3], 10)
    assert chunked.fingerprint([a, b], k=1) != base
    assert chunked.fingerprint([a, a], k=2) != base
    assert chunked.fingerprint([a, a.reshape(2, 3)], k=1) != base
