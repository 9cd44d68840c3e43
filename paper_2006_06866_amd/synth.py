"""Seeded synthetic light curves and search grids.

These stand in for the paper's COSMIC / ``ellc`` / ZTF light curves (Katz et
al. 2020, Secs. 2.1-2.2), which are not available here.  Shapes, cadences and
value ranges follow the workloads the paper describes: sparse multi-year
cadence, detached-eclipse signals with two dips (secondary at half the primary
depth, the surface-brightness ratio of Sec. 2.2), sinusoids, pure noise,
periods of minutes and |Pdot| of 1e-13..1e-10 (Sec. 2.2, Sec. 3).

This module holds no part of the search method: injected signals use the
exact phase of a period that evolves linearly in time (Eq. (2)), i.e.
    phase(t) = integral_0^t dt' / (P0 + Pdot t') = ln(1 + Pdot t / P0) / Pdot,
not the quadratic fold that the search applies.  Both the oracle and the GPU
path consume these arrays unchanged.

Units: days for epochs and periods, Pdot dimensionless (s/s = d/d).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

SEED_ROOT = (2006, 6866)

KIND_NOISE, KIND_ECLIPSE, KIND_SINE = 0, 1, 2


def rng_for(*key: int) -> np.random.Generator:
    """Deterministic generator for a workload key."""
    return np.random.default_rng(np.random.SeedSequence([*SEED_ROOT, *key]))


@dataclass
class Workload:
    name: str
    times: np.ndarray          # f64 [sum N]
    mags: np.ndarray           # f64 [sum N]
    offsets: np.ndarray        # i64 [n_curves + 1]
    periods: np.ndarray        # f64 [n_p]
    pdots: np.ndarray          # f64 [n_pd]
    n_phase: int
    n_mag: int
    truth: Dict[str, np.ndarray] = field(default_factory=dict)
    phase_overlap: bool = False     # 50%-overlapping phase bins (Sec. 2.3)
    mag_overlap: bool = False       # 50%-overlapping magnitude bins (Sec. 2.3)

    @property
    def n_curves(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    @property
    def point_trials(self) -> int:
        return int(self.offsets[-1]) * int(self.periods.size) * int(self.pdots.size)

    def curve(self, c: int):
        a, b = int(self.offsets[c]), int(self.offsets[c + 1])
        return self.times[a:b], self.mags[a:b]

    def subset(self, curves) -> "Workload":
        """The same grid over a subset of the curves."""
        curves = np.asarray(curves, dtype=np.int64)
        ts, ms, lens = [], [], []
        for c in curves:
            t, m = self.curve(int(c))
            ts.append(t)
            ms.append(m)
            lens.append(t.size)
        off = np.zeros(len(lens) + 1, dtype=np.int64)
        off[1:] = np.cumsum(lens)
        truth = {k: v[curves] for k, v in self.truth.items()}
        return Workload(self.name + "[subset]", np.concatenate(ts),
                        np.concatenate(ms), off, self.periods, self.pdots,
                        self.n_phase, self.n_mag, truth, self.phase_overlap,
                        self.mag_overlap)


# ----------------------------------------------------------------------------
# grids (Sec. 3: uniform in frequency; Pdot log-spaced, here symmetric)
# ----------------------------------------------------------------------------
def frequency_grid_periods(f_min: float, f_max: float, n: int) -> np.ndarray:
    """Periods whose frequencies are uniform (inclusive) in [f_min, f_max]."""
    return 1.0 / np.linspace(f_min, f_max, n)


def symmetric_log_pdots(lo_exp: float, hi_exp: float, n_half: int) -> np.ndarray:
    """-logspace (descending magnitude) followed by +logspace: sorted order."""
    mags = np.logspace(lo_exp, hi_exp, n_half)
    return np.concatenate([-mags[::-1], mags])


# ----------------------------------------------------------------------------
# cadences
# ----------------------------------------------------------------------------
def uniform_epochs(rng, n: int, baseline: float) -> np.ndarray:
    return np.sort(rng.uniform(0.0, baseline, n))


def nightly_epochs(rng, n: int, baseline: float, max_per_night: int = 4) -> np.ndarray:
    """Clustered cadence: 1..max_per_night epochs on random distinct nights,
    each at night + 0.1 + U(0, 0.3) d; truncated to exactly n epochs."""
    n_nights_avail = max(1, int(baseline))
    mean_per = (1 + max_per_night) / 2.0
    n_nights = min(n_nights_avail, max(1, int(math.ceil(n / mean_per))))
    nights = np.sort(rng.choice(n_nights_avail, size=n_nights, replace=False))
    per = rng.integers(1, max_per_night + 1, size=n_nights)
    # too few nights for n epochs at this cadence: add epochs to random nights
    while per.sum() < n:
        per[rng.integers(0, n_nights)] += 1
    night_of = np.repeat(nights, per)[:n]
    return np.sort(night_of + 0.1 + rng.uniform(0.0, 0.3, n))


# ----------------------------------------------------------------------------
# signals
# ----------------------------------------------------------------------------
def true_phase(t: np.ndarray, p0: float, pdot: float, phi0: float) -> np.ndarray:
    """Cycles elapsed since t = 0 for P(t) = P0 + Pdot t (Eq. (2)), plus phi0."""
    if pdot == 0.0:
        return t / p0 + phi0
    return np.log1p(pdot * t / p0) / pdot + phi0


def _wrapped_distance(u: np.ndarray, centre: float) -> np.ndarray:
    d = np.mod(u - centre, 1.0)
    return np.minimum(d, 1.0 - d)


def eclipse_signal(cycles: np.ndarray, depth: float, width: float) -> np.ndarray:
    """Two Gaussian dips (fainter = larger magnitude) at phase 0 and 1/2, the
    secondary at half the primary depth."""
    u = np.mod(cycles, 1.0)
    g = lambda d: np.exp(-0.5 * (d / width) ** 2)
    return depth * g(_wrapped_distance(u, 0.0)) + 0.5 * depth * g(_wrapped_distance(u, 0.5))


def sine_signal(cycles: np.ndarray, amp: float) -> np.ndarray:
    return amp * np.sin(2.0 * np.pi * cycles)


def nearest_index(grid: np.ndarray, value: float) -> int:
    return int(np.argmin(np.abs(grid - value)))


def _pack(name, ts, ms, periods, pdots, n_phase, n_mag, truth) -> Workload:
    off = np.zeros(len(ts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in ts])
    tr = {k: np.asarray(v) for k, v in truth.items()}
    return Workload(name, np.concatenate(ts).astype(np.float64),
                    np.concatenate(ms).astype(np.float64), off,
                    np.ascontiguousarray(periods, dtype=np.float64),
                    np.ascontiguousarray(pdots, dtype=np.float64),
                    int(n_phase), int(n_mag), tr)


def _draw_injection(rng, periods, pdots, p_min_d, p_max_d, pd_lo, pd_hi,
                    signed=True):
    """Draw P log-uniform and |Pdot| log-uniform, snap both to grid points."""
    p = math.exp(rng.uniform(math.log(p_min_d), math.log(p_max_d)))
    ip = nearest_index(periods, p)
    if pdots.size == 1:
        return ip, 0
    mag = 10.0 ** rng.uniform(pd_lo, pd_hi)
    sgn = (1.0 if rng.uniform() < 0.5 else -1.0) if signed else -1.0
    iq = nearest_index(pdots, sgn * mag)
    return ip, iq


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
MINUTE = 1.0 / 1440.0
YEAR = 365.25


def config1() -> Workload:
    """1 curve, 200 epochs U[0, 1000) d, 0.3 sin + N(0, 0.05), P = 0.05 d
    snapped to a 2,000-frequency grid over [5, 50] 1/d, Pdot = {0}, 10x5."""
    rng = rng_for(1)
    periods = frequency_grid_periods(5.0, 50.0, 2000)
    pdots = np.array([0.0])
    ip = nearest_index(1.0 / periods, 20.0)
    t = uniform_epochs(rng, 200, 1000.0)
    phi0 = rng.uniform()
    m = sine_signal(true_phase(t, periods[ip], 0.0, phi0), 0.3) + rng.normal(0, 0.05, t.size)
    return _pack("c1_single_fp64", [t], [m], periods, pdots, 10, 5,
                 {"inj_p": [ip], "inj_q": [0], "kind": [KIND_SINE]})


def _eclipse_curve(rng, t, periods, pdots, ip, iq, sigma):
    depth = rng.uniform(0.2, 1.0)
    width = rng.uniform(0.02, 0.1)
    phi0 = rng.uniform()
    cyc = true_phase(t - t.min(), periods[ip], pdots[iq], phi0)
    return eclipse_signal(cyc, depth, width) + rng.normal(0.0, sigma, t.size)


def config2(n_curves: int = 512, n_points: int = 600, n_freq: int = 20000,
            n_pdot_half: int = 32) -> Workload:
    """Batched FP64: 512 x 600 epochs over 3 yr nightly cadence, eclipses,
    P log-uniform [5, 60] min, |Pdot| log-uniform [1e-13, 1e-10] with random
    sign; 20,000 frequencies in [24, 288] 1/d x 64 Pdots; 10x5 bins."""
    rng = rng_for(2)
    periods = frequency_grid_periods(24.0, 288.0, n_freq)
    pdots = symmetric_log_pdots(-13.0, -10.0, n_pdot_half)
    ts, ms, ips, iqs = [], [], [], []
    for _ in range(n_curves):
        t = nightly_epochs(rng, n_points, 3 * YEAR)
        ip, iq = _draw_injection(rng, periods, pdots, 5 * MINUTE, 60 * MINUTE, -13, -10)
        sigma = rng.uniform(0.02, 0.1)
        ts.append(t)
        ms.append(_eclipse_curve(rng, t, periods, pdots, ip, iq, sigma))
        ips.append(ip)
        iqs.append(iq)
    return _pack("c2_batched", ts, ms, periods, pdots, 10, 5,
                 {"inj_p": ips, "inj_q": iqs, "kind": [KIND_ECLIPSE] * n_curves})


def config4(n_curves: int = 8192, n_freq: int = 10000, n_pdot_half: int = 16) -> Workload:
    """Ragged: 8,192 curves, N = clip(round(lognormal(ln 300, 1)), 50, 3000),
    baselines U(1, 5) yr nightly cadence; 20% noise, 40% eclipse, 40% sine
    (A ~ U(0.05, 0.5)); 10,000 frequencies in [24, 288] 1/d x 32 Pdots; 10x5."""
    rng = rng_for(4)
    periods = frequency_grid_periods(24.0, 288.0, n_freq)
    pdots = symmetric_log_pdots(-13.0, -10.0, n_pdot_half)
    ts, ms, ips, iqs, kinds = [], [], [], [], []
    for _ in range(n_curves):
        n = int(np.clip(round(rng.lognormal(math.log(300.0), 1.0)), 50, 3000))
        t = nightly_epochs(rng, n, rng.uniform(1.0, 5.0) * YEAR)
        u = rng.uniform()
        sigma = rng.uniform(0.02, 0.1)
        if u < 0.2:
            kind, ip, iq = KIND_NOISE, -1, -1
            m = rng.normal(0.0, sigma, n)
        else:
            ip, iq = _draw_injection(rng, periods, pdots, 5 * MINUTE, 60 * MINUTE, -13, -10)
            if u < 0.6:
                kind = KIND_ECLIPSE
                m = _eclipse_curve(rng, t, periods, pdots, ip, iq, sigma)
            else:
                kind = KIND_SINE
                amp = rng.uniform(0.05, 0.5)
                cyc = true_phase(t - t.min(), periods[ip], pdots[iq], rng.uniform())
                m = sine_signal(cyc, amp) + rng.normal(0.0, sigma, n)
        ts.append(t)
        ms.append(m)
        ips.append(ip)
        iqs.append(iq)
        kinds.append(kind)
    return _pack("c4_ragged", ts, ms, periods, pdots, 10, 5,
                 {"inj_p": ips, "inj_q": iqs, "kind": kinds})


def _z_score(m: np.ndarray) -> np.ndarray:
    """Sec. 2.3 normalisation: subtract the median, divide by the std."""
    return (m - np.median(m)) / np.std(m)


def config5(n_curves: int = 64, n_points: int = 5000, n_freq: int = 100000,
            n_pdot_half: int = 128) -> Workload:
    """Long baseline, fine grid: 64 x 5,000 epochs U[0, 10 yr), two filters
    (g offset +0.3 mag, per-filter noise) merged by per-filter z-scores
    (Sec. 2.3), 50/50 eclipse/sine, P in [3, 30] min, |Pdot| <= 1e-10;
    100,000 frequencies in [48, 480] 1/d x 256 Pdots; 20 phase x 10 mag."""
    rng = rng_for(5)
    periods = frequency_grid_periods(48.0, 480.0, n_freq)
    pdots = symmetric_log_pdots(-13.0, -10.0, n_pdot_half)
    ts, ms, ips, iqs, kinds = [], [], [], [], []
    for c in range(n_curves):
        t = uniform_epochs(rng, n_points, 10 * YEAR)
        ip, iq = _draw_injection(rng, periods, pdots, 3 * MINUTE, 30 * MINUTE, -13, -10)
        cyc = true_phase(t - t.min(), periods[ip], pdots[iq], rng.uniform())
        if c % 2 == 0:
            kind = KIND_ECLIPSE
            clean = eclipse_signal(cyc, rng.uniform(0.2, 1.0), rng.uniform(0.02, 0.1))
        else:
            kind = KIND_SINE
            clean = sine_signal(cyc, rng.uniform(0.05, 0.5))
        is_g = rng.uniform(size=n_points) < 0.5
        sg, sr = rng.uniform(0.02, 0.1, 2)
        m = clean + np.where(is_g, 0.3, 0.0) + rng.normal(0.0, 1.0, n_points) * np.where(is_g, sg, sr)
        merged = np.empty_like(m)
        merged[is_g] = _z_score(m[is_g])
        merged[~is_g] = _z_score(m[~is_g])
        ts.append(t)
        ms.append(merged)
        ips.append(ip)
        iqs.append(iq)
        kinds.append(kind)
    return _pack("c5_long_baseline", ts, ms, periods, pdots, 20, 10,
                 {"inj_p": ips, "inj_q": iqs, "kind": kinds})


# ----------------------------------------------------------------------------
# paper-scale search (Sec. 3): 5,183,995 periods x 32 Pdot, 50 x 10 bins
# ----------------------------------------------------------------------------
G_SI = 6.67430e-11
C_SI = 299792458.0
MSUN_KG = 1.98847e30


def chirp_mass(m1: float, m2: float) -> float:
    return (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2


def pdot_gw(period_days: float, mchirp_msun: float) -> float:
    """Orbital decay by gravitational radiation (Eq. (1), Peters 1964):
    dP/dt = -(192 pi / 5) (2 pi G M_c / (c^3 P))^(5/3), dimensionless."""
    tc = G_SI * mchirp_msun * MSUN_KG / C_SI ** 3        # seconds
    x = 2.0 * math.pi * tc / (period_days * 86400.0)
    return -(192.0 * math.pi / 5.0) * x ** (5.0 / 3.0)


def gaussian_spacing_epochs(rng, n: int, mean_dt: float, sd_dt: float) -> np.ndarray:
    """Sec. 2.2: gaps between observations drawn from a Gaussian of mean dt."""
    gaps = np.clip(rng.normal(mean_dt, sd_dt, n - 1), 0.05, None)
    return np.concatenate([[0.0], np.cumsum(gaps)])


def paper_grid(baseline_days: float = 3600.0):
    """Sec. 3: frequencies from 2/B to 480 /d (3-min period) in steps of
    1/(3B); B = 3600 d gives the paper's 5,183,995 periods."""
    f_min, f_max, df = 2.0 / baseline_days, 480.0, 1.0 / (3.0 * baseline_days)
    n = int(math.floor((f_max - f_min) / df + 1e-9)) + 1
    return 1.0 / (f_min + df * np.arange(n))


def config6(n_burdge: int = 35, n_population: int = 100, n_pdots: int = 32,
            n_points: int = 500) -> Workload:
    """Paper-scale search: 35 'Burdge' binaries (P0 = 4..38 min, Pdot from
    Eq. (1) at the masses 0.61 / 0.21 Msun) and 100 population-like binaries
    (P0 log-uniform 5..40 min, chirp mass U(0.2, 0.5) Msun), ~500 epochs with
    7 +- 2 d Gaussian spacing (Sec. 2.2), eclipses, noise U(0.05, 0.2) mag;
    grid of Sec. 3 (5,183,995 periods) x 32 Pdot log-spaced in
    [-1e-10, -1e-12]; 50 phase x 10 magnitude bins.  Injections are not
    snapped to the grid: recovery is judged as in Sec. 3.1."""
    rng = rng_for(6)
    periods = paper_grid()
    pdots = -np.logspace(-12.0, -10.0, n_pdots)[::-1]
    ts, ms, p_true, pd_true, kinds = [], [], [], [], []
    mc_b = chirp_mass(0.61, 0.21)
    for i in range(n_burdge + n_population):
        if i < n_burdge:
            p0 = (4.0 + i) * MINUTE
            mc = mc_b
        else:
            p0 = math.exp(rng.uniform(math.log(5.0), math.log(40.0))) * MINUTE
            mc = rng.uniform(0.2, 0.5)
        pd = pdot_gw(p0, mc)
        t = gaussian_spacing_epochs(rng, n_points, 7.0, 2.0)
        cyc = true_phase(t, p0, pd, rng.uniform())
        m = eclipse_signal(cyc, rng.uniform(0.5, 1.0), rng.uniform(0.02, 0.05))
        m = 19.0 + m + rng.normal(0.0, rng.uniform(0.05, 0.2), t.size)
        ts.append(t)
        ms.append(m)
        p_true.append(p0)
        pd_true.append(pd)
        kinds.append(KIND_ECLIPSE)
    w = _pack("c6_paper_scale", ts, ms, periods, pdots, 50, 10,
              {"p_true": p_true, "pdot_true": pd_true, "kind": kinds,
               "inj_p": [-1] * len(ts), "inj_q": [-1] * len(ts)})
    w.phase_overlap = True
    return w


CONFIGS = {1: config1, 2: config2, 4: config4, 5: config5, 6: config6}


def make_config(k: int, **kw) -> Workload:
    """Workload of config k (3 is config 2's inputs on the split path)."""
    return CONFIGS[2 if k == 3 else k](**kw)


def random_curves(seed: int, lengths, baseline: float = 1000.0,
                  period_range=(0.02, 0.2), pdot_scale: float = 1e-9,
                  n_freq: int = 64, n_pdots: int = 4, n_phase: int = 10,
                  n_mag: int = 5, noise: float = 0.1,
                  pdots: Optional[np.ndarray] = None) -> Workload:
    """Small mixed workload for tests: curves of the given lengths with random
    uniform epochs, sinusoid/eclipse/noise magnitudes, and a small grid."""
    rng = rng_for(100, seed)
    f_lo, f_hi = 1.0 / period_range[1], 1.0 / period_range[0]
    periods = frequency_grid_periods(f_lo, f_hi, n_freq)
    if pdots is None:
        pdots = (np.linspace(-1.0, 1.0, n_pdots) * pdot_scale if n_pdots > 1
                 else np.array([0.0]))
    ts, ms, ips, iqs, kinds = [], [], [], [], []
    for n in lengths:
        n = int(n)
        t = uniform_epochs(rng, n, baseline) + rng.uniform(-50.0, 50.0)
        ip = int(rng.integers(0, periods.size))
        iq = int(rng.integers(0, pdots.size))
        kind = int(rng.integers(0, 3))
        cyc = true_phase(t - t.min(), periods[ip], pdots[iq], rng.uniform())
        if kind == KIND_NOISE:
            clean = np.zeros(n)
        elif kind == KIND_ECLIPSE:
            clean = eclipse_signal(cyc, rng.uniform(0.2, 1.0), rng.uniform(0.02, 0.1))
        else:
            clean = sine_signal(cyc, rng.uniform(0.05, 0.5))
        ts.append(t)
        ms.append(clean + rng.normal(0.0, noise, n))
        ips.append(ip)
        iqs.append(iq)
        kinds.append(kind)
    return _pack(f"random_{seed}", ts, ms, periods, pdots, n_phase, n_mag,
                 {"inj_p": ips, "inj_q": iqs, "kind": kinds})
