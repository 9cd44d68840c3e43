"""Host-side merge of per-curve results over sub-grids (Sec. 4: batches keep
their minimum and statistics and are combined).  No GPU: the parts are built
from a CE array with numpy, merged through the C ABI, and compared with the
whole-array values."""
import numpy as np
import pytest

import paper_2006_06866_amd as gce
from gce_testlib import best_rows as _result
from paper_2006_06866_amd import build as gbuild
import os


def _ensure_built():
    if not os.path.exists(gce.LIB_PATH):
        gbuild.build()


@pytest.mark.parametrize("split_axis", ["pdot", "period", "both"])
def test_merge_equals_whole(split_axis):
    _ensure_built()
    rng = np.random.default_rng(5)
    nc, n_pd, n_p = 5, 12, 37
    cube = rng.normal(1.5, 0.05, (nc, n_pd, n_p))
    cube[1, 7, 3] = 0.9          # distinct minima
    cube[2, 0, 36] = 0.8
    cube[3, 4, 10] = cube[3, 9, 2] = 0.7   # tie: lower flat index (4*37+10) wins
    whole = gce.best_fields(_result(cube))
    q_cuts = [0, 5, 12] if split_axis in ("pdot", "both") else [0, 12]
    p_cuts = [0, 20, 37] if split_axis in ("period", "both") else [0, 37]
    acc, trials = None, 0
    for qa, qb in zip(q_cuts[:-1], q_cuts[1:]):
        for pa, pb in zip(p_cuts[:-1], p_cuts[1:]):
            part = _result(cube[:, qa:qb, pa:pb])
            acc = gce.merge_results(acc, trials, part, n_p, pa, pb - pa, qa, qb - qa)
            trials += (pb - pa) * (qb - qa)
    got = gce.best_fields(acc)
    assert np.array_equal(got["flat_index"], whole["flat_index"])
    assert np.array_equal(got["period_index"], whole["period_index"])
    assert np.array_equal(got["pdot_index"], whole["pdot_index"])
    assert np.array_equal(got["ce_min"], whole["ce_min"])
    assert np.allclose(got["ce_mean"], whole["ce_mean"], rtol=0, atol=1e-14)
    assert np.allclose(got["ce_std"], whole["ce_std"], rtol=1e-12, atol=0)
    assert np.allclose(got["significance"], whole["significance"], rtol=1e-10, atol=0)


def test_merge_keeps_invalid_and_rejects_bad_arguments():
    _ensure_built()
    cube = np.random.default_rng(6).normal(1.0, 0.1, (2, 3, 4))
    a = _result(cube)
    b = _result(cube).copy()
    raw = b.view(np.uint8).reshape(2, 48)
    raw[1, 0:8] = np.array([-1], dtype=np.int64).view(np.uint8)
    acc = gce.merge_results(a.copy(), 12, b, 4, 0, 4, 0, 3)
    f = gce.best_fields(acc)
    assert f["flat_index"][1] == -1 and np.isnan(f["ce_mean"][1])
    assert f["flat_index"][0] >= 0
    with pytest.raises(gce.GceError):
        gce.merge_results(a.copy(), 12, b, 4, 2, 4, 0, 3)   # periods beyond the grid
