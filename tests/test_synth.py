"""Synthetic workloads (stand-ins for the paper's light curves, Secs. 2.2
and 3): seeded generation is reproducible byte for byte, injections sit on
grid points, and an injected signal is the oracle's minimum where the noise
allows it."""
import numpy as np
import pytest

import oracle
from paper_2006_06866_amd import synth


def _arrays(w):
    return [w.times, w.mags, w.offsets, w.periods, w.pdots] + \
        [np.asarray(w.truth[k]) for k in sorted(w.truth)]


@pytest.mark.parametrize("cfg", [1, 2, 4, 5, 6])
def test_configs_reproduce_byte_for_byte(cfg):
    a, b = synth.make_config(cfg), synth.make_config(cfg)
    for x, y in zip(_arrays(a), _arrays(b)):
        assert x.dtype == y.dtype and x.tobytes() == y.tobytes()
    assert a.n_phase == b.n_phase and a.n_mag == b.n_mag


@pytest.mark.parametrize("cfg", [1, 2, 4, 5])
def test_injections_are_grid_points(cfg):
    """Injected (P, Pdot) are given as grid indices (the signals are drawn at
    exactly those grid values), within range; noise-only curves carry -1."""
    w = synth.make_config(cfg)
    ip, iq = np.asarray(w.truth["inj_p"]), np.asarray(w.truth["inj_q"])
    has = ip >= 0
    assert np.all((ip[has] < w.periods.size) & (iq[has] >= 0) & (iq[has] < w.pdots.size))
    assert np.all(iq[~has] == -1)
    # the grids are uniform in frequency and the Pdot grids symmetric
    f = 1.0 / w.periods
    assert np.allclose(np.diff(f), np.diff(f)[0], rtol=1e-9, atol=0)
    assert np.allclose(np.sort(w.pdots), -np.sort(w.pdots)[::-1])


def test_injected_signal_is_the_oracle_minimum():
    """Config 1 (a sinusoid snapped to grid point 666): the oracle's minimum
    is the injected trial.  Four curves of config 2 (eclipses at snapped
    (P, Pdot)): the minimum is at the injected period (most of its small
    Pdot values do not dephase a 3-yr curve measurably, so the Pdot index
    is not fixed by the data)."""
    w = synth.make_config(1)
    _, bf, _ = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                             w.n_mag, want_cube=False)
    assert bf[0] == w.truth["inj_p"][0] == 666
    w = synth.make_config(2).subset(np.arange(4))
    _, bf, _ = oracle.search(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                             w.n_mag, want_cube=False)
    assert np.array_equal(bf % w.periods.size, np.asarray(w.truth["inj_p"]))
