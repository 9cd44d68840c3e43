"""Recovery bookkeeping (Sec. 3.1 harmonics and 10% tolerance, Sec. 3.2
detection threshold) and the paper-scale workload's physics inputs."""
import math

import numpy as np

from paper_2006_06866_amd import recovery, synth


def test_harmonics_and_tolerance():
    t = np.full(8, 0.01)
    b = np.array([0.01, 0.0105, 0.02, 0.005, 0.01 / 3, 0.0025, 0.01 / 6, 0.0075])
    rec = recovery.recovered(b, t)
    assert rec.tolist() == [True, True, True, True, True, True, True, False]
    assert recovery.recovered([0.0111], [0.01]).tolist() == [False]
    assert recovery.harmonic_error([0.03], [0.01])[0] == 0.5   # 3x is not a listed harmonic


def test_detection_threshold():
    assert recovery.detected([9.99, 10.0, np.nan, 25.0]).tolist() == [False, True, False, True]


def test_summary_counts():
    periods = np.array([0.004, 0.005, 0.010, 0.020])
    fields = {"period_index": np.array([2, 3, 0, -1]),
              "significance": np.array([12.0, 30.0, 5.0, np.nan])}
    s = recovery.summary(fields, periods, np.array([0.01, 0.01, 0.01, 0.01]))
    assert s == {"curves": 4, "recovered_harmonic": 2, "recovered_fundamental": 1,
                 "detected_rho_ge_10": 2, "median_significance": 12.0}


def test_gw_period_derivative_matches_paper_numbers():
    """Eq. (1) at the 0.61 / 0.21 Msun masses gives the Pdot the paper quotes
    for the 7-min binary (-2.14e-11) and the ends of its 4..38 min catalogue
    (Sec. 3: -5.44e-11 at 4 min, of order -1.2e-12 at 38 min)."""
    mc = synth.chirp_mass(0.61, 0.21)
    assert abs(mc - 0.3032) < 5e-4
    assert abs(synth.pdot_gw(7 / 1440, mc) / -2.14e-11 - 1) < 0.005
    assert abs(synth.pdot_gw(4 / 1440, mc) / -5.44e-11 - 1) < 0.005
    assert 1.1e-12 < -synth.pdot_gw(38 / 1440, mc) < 1.35e-12


def test_paper_grid_size():
    """Sec. 3: 2/B .. 480 /d in steps of 1/(3B) is 5,183,995 frequencies for
    B = 3600 d."""
    p = synth.paper_grid()
    assert p.size == 5183995
    assert abs(1 / p[-1] - 480.0) < 1e-6 and abs(1 / p[0] - 2 / 3600) < 1e-15


def test_pdot_resolution_period_matches_paper():
    """Eqs. (6)-(7): the period below which a 10-yr search with n_b phase bins
    resolves the GW Pdot solves P = (n_b |Pdot(P)| / 2)^(1/2) t; for the
    0.61 / 0.21 Msun binary it is 33.2 min at n_b = 50 (the paper: P* of
    order 30-40 min) and 21.4 min at n_b = 10."""
    mc = synth.chirp_mass(0.61, 0.21)
    t = 10 * synth.YEAR
    for nb, want in ((50, 33.2), (10, 21.4)):
        p = 30 * synth.MINUTE
        for _ in range(200):       # a contraction: the map's slope is -5/6
            p = math.sqrt(0.5 * nb * abs(synth.pdot_gw(p, mc))) * t
        assert abs(p / synth.MINUTE - want) < 0.05
