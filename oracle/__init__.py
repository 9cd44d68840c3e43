"""Plain FP64 CPU oracle for the conditional-entropy (P, Pdot) search.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  The
arithmetic lives in ``ce_oracle.c`` (Katz et al. 2020, Sec. 2.3, Eqs. (3) and
(4)); this module only builds that file with gcc and marshals numpy arrays.

Every entry point is pinned by the CPU tests in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ce_oracle.c")
# CE_ORACLE_LIB names another build of ce_oracle.c to load (the sanitizer
# test builds one with AddressSanitizer and UndefinedBehaviorSanitizer)
_LIB = os.environ.get("CE_ORACLE_LIB") or os.path.join(_HERE, "libce_oracle.so")

# -ffp-contract=off: no fused multiply-adds other than the explicit fma().
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile ce_oracle.c into libce_oracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u32 = ctypes.POINTER(ctypes.c_uint32)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.ce_oracle_mag_bins.argtypes = [_d, ctypes.c_int64, ctypes.c_int32, _i32]
        lib.ce_oracle_mag_bins2.argtypes = [_d, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_int32, _i32, _i32]
        lib.ce_oracle_fold_bin.argtypes = [ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int32]
        lib.ce_oracle_fold_bin.restype = ctypes.c_int32
        lib.ce_oracle_phases.argtypes = [_d, ctypes.c_int64, ctypes.c_double,
                                         ctypes.c_double, _d]
        lib.ce_oracle_entropy.argtypes = [_u32, ctypes.c_int32, ctypes.c_int32]
        lib.ce_oracle_entropy.restype = ctypes.c_double
        lib.ce_oracle_counts.argtypes = [_d, _d, ctypes.c_int64, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, _u32]
        search_args = [_d, _d, _i64, ctypes.c_int64, _d, ctypes.c_int64, _d,
                       ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                       _d, _i64, _d, ctypes.c_int32]
        lib.ce_oracle_search.argtypes = search_args
        lib.ce_oracle_search_ponly.argtypes = [_d, _d, _i64, ctypes.c_int64, _d,
                                               ctypes.c_int64, ctypes.c_int32,
                                               ctypes.c_int32, _d, _i64, _d,
                                               ctypes.c_int32]
        lib.ce_oracle_trials.argtypes = [_d, _d, _i64, ctypes.c_int64, _d,
                                         ctypes.c_int64, _d, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         _i64, _i64, ctypes.c_int64, _d, _u32,
                                         ctypes.c_int32]
        lib.ce_oracle_max_threads.restype = ctypes.c_int
        lib.ce_oracle_significance.argtypes = [_d, ctypes.c_int64, _d, _d, _d]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: Optional[np.ndarray], t):
    return None if a is None else a.ctypes.data_as(t)


def _check(rc: int, what: str) -> None:
    if rc < 0:
        raise ValueError(f"{what}: oracle rejected the arguments (rc={rc})")


def max_threads() -> int:
    return int(_load().ce_oracle_max_threads())


def mag_bins(mags, n_mag: int) -> np.ndarray:
    """Magnitude bin of every epoch of one curve (Sec. 2.3 normalisation)."""
    m = _f64(mags)
    out = np.empty(m.size, dtype=np.int32)
    rc = _load().ce_oracle_mag_bins(_p(m, _d), m.size, n_mag, _p(out, _i32))
    _check(rc, "mag_bins")
    if rc == 1:
        raise ValueError("mag_bins: non-finite magnitude")
    return out


def mag_bins_overlap(mags, n_mag: int):
    """50%-overlapping magnitude bins of one curve: (first, second) bin of
    every epoch, second = -1 where the epoch is in one bin only."""
    m = _f64(mags)
    a = np.empty(m.size, dtype=np.int32)
    b = np.empty(m.size, dtype=np.int32)
    rc = _load().ce_oracle_mag_bins2(_p(m, _d), m.size, n_mag, 1, _p(a, _i32),
                                     _p(b, _i32))
    _check(rc, "mag_bins_overlap")
    if rc == 1:
        raise ValueError("mag_bins_overlap: non-finite magnitude")
    return a, b


def _overlap_bits(phase_overlap: bool, mag_overlap: bool) -> int:
    return int(bool(phase_overlap)) | (int(bool(mag_overlap)) << 1)


def fold_bin(dt: float, period: float, pdot: float, n_phase: int) -> int:
    """Phase bin of one epoch offset dt under Eq. (3)."""
    return int(_load().ce_oracle_fold_bin(float(dt), float(period), float(pdot),
                                          int(n_phase)))


def phases(times, period: float, pdot: float) -> np.ndarray:
    """Eq. (3) phases of one curve's epochs under one (P, Pdot) trial (time
    origin: the curve's earliest epoch)."""
    t = _f64(times)
    out = np.empty(t.size)
    rc = _load().ce_oracle_phases(_p(t, _d), t.size, float(period), float(pdot),
                                  _p(out, _d))
    _check(rc, "phases")
    return out


def entropy(counts) -> float:
    """Eq. (4) of a [n_mag][n_phase] count table."""
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    if c.ndim != 2:
        raise ValueError("counts must be 2-D [n_mag][n_phase]")
    return float(_load().ce_oracle_entropy(_p(c, _u32), c.shape[0], c.shape[1]))


def counts(times, mags, period: float, pdot: float, n_phase: int,
           n_mag: int, phase_overlap: bool = False,
           mag_overlap: bool = False) -> np.ndarray:
    """[n_mag][n_phase] histogram of one curve at one (P, Pdot) trial
    (each epoch counted in two phase bins with 50%-overlapping phase bins,
    in one or two magnitude bins with 50%-overlapping magnitude bins)."""
    t, m = _f64(times), _f64(mags)
    if t.size != m.size:
        raise ValueError("times and mags differ in length")
    out = np.zeros((n_mag, n_phase), dtype=np.uint32)
    rc = _load().ce_oracle_counts(_p(t, _d), _p(m, _d), t.size, float(period),
                                  float(pdot), n_phase, n_mag,
                                  _overlap_bits(phase_overlap, mag_overlap), _p(out, _u32))
    _check(rc, "counts")
    if rc == 1:
        raise ValueError("counts: non-finite input")
    return out


def search(times, mags, offsets, periods, pdots, n_phase: int, n_mag: int,
           want_cube: bool = True, n_threads: int = 0, phase_overlap: bool = False,
           mag_overlap: bool = False):
    """Full grid search.  Returns (cube or None, best_flat, best_ce).

    cube is [n_curves][n_pdots][n_periods]; best_flat = q * n_periods + p.
    """
    t, m = _f64(times), _f64(mags)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    P, Pd = _f64(periods), _f64(pdots)
    nc = off.size - 1
    cube = np.empty((nc, Pd.size, P.size)) if want_cube else None
    bf = np.empty(nc, dtype=np.int64)
    bc = np.empty(nc)
    rc = _load().ce_oracle_search(_p(t, _d), _p(m, _d), _p(off, _i64), nc,
                                  _p(P, _d), P.size, _p(Pd, _d), Pd.size,
                                  n_phase, n_mag, _overlap_bits(phase_overlap, mag_overlap),
                                  _p(cube, _d),
                                  _p(bf, _i64), _p(bc, _d), n_threads)
    _check(rc, "search")
    return cube, bf, bc


def search_ponly(times, mags, offsets, periods, n_phase: int, n_mag: int,
                 want_cube: bool = True, n_threads: int = 0):
    """Classic P-only CE search.  Returns (cube [n_curves][n_periods] or None,
    best_flat, best_ce)."""
    t, m = _f64(times), _f64(mags)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    P = _f64(periods)
    nc = off.size - 1
    cube = np.empty((nc, P.size)) if want_cube else None
    bf = np.empty(nc, dtype=np.int64)
    bc = np.empty(nc)
    rc = _load().ce_oracle_search_ponly(_p(t, _d), _p(m, _d), _p(off, _i64), nc,
                                        _p(P, _d), P.size, n_phase, n_mag,
                                        _p(cube, _d), _p(bf, _i64), _p(bc, _d),
                                        n_threads)
    _check(rc, "search_ponly")
    return cube, bf, bc


def trials(times, mags, offsets, periods, pdots, n_phase: int, n_mag: int,
           curve_ids, flat_ids, want_counts: bool = False, n_threads: int = 0,
           phase_overlap: bool = False, mag_overlap: bool = False):
    """H_c (and optionally counts) of selected (curve, flat) trials."""
    t, m = _f64(times), _f64(mags)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    P, Pd = _f64(periods), _f64(pdots)
    ci = np.ascontiguousarray(curve_ids, dtype=np.int64)
    fi = np.ascontiguousarray(flat_ids, dtype=np.int64)
    if ci.size != fi.size:
        raise ValueError("curve_ids and flat_ids differ in length")
    ce = np.empty(ci.size)
    cnt = np.empty((ci.size, n_mag, n_phase), dtype=np.uint32) if want_counts else None
    rc = _load().ce_oracle_trials(_p(t, _d), _p(m, _d), _p(off, _i64),
                                  off.size - 1, _p(P, _d), P.size, _p(Pd, _d),
                                  Pd.size, n_phase, n_mag,
                                  _overlap_bits(phase_overlap, mag_overlap), _p(ci, _i64), _p(fi, _i64), ci.size, _p(ce, _d),
                                  _p(cnt, _u32), n_threads)
    _check(rc, "trials")
    return (ce, cnt) if want_counts else ce


def significance(values):
    """Eq. (5) inputs over one curve's CE values: (mean, population std,
    rho = (mean - min) / std, 0 when std = 0)."""
    v = _f64(values).ravel()
    mean, sd, rho = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = _load().ce_oracle_significance(_p(v, _d), v.size, ctypes.byref(mean),
                                        ctypes.byref(sd), ctypes.byref(rho))
    _check(rc, "significance")
    return mean.value, sd.value, rho.value


def curve_statistics(cube):
    """Per-curve (mean, std, rho) arrays of a [n_curves, ...] CE cube."""
    c = np.asarray(cube, dtype=np.float64).reshape(cube.shape[0], -1)
    out = np.array([significance(row) for row in c])
    return out[:, 0], out[:, 1], out[:, 2]
