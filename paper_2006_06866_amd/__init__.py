"""MI355X conditional-entropy (P, Pdot) period search.

Python binding of ``libgce.so`` (C ABI in ``include/gce.h``): argument
marshalling only.  Every step of the search runs in the library's HIP kernels
on a gfx950 GPU; there is no CPU fallback, and a missing library raises.
PyTorch supplies device memory and streams.

Katz et al. 2020, Sec. 2.3: quadratic phase fold (Eq. (3)), 2-D
(magnitude x phase) histogram, conditional entropy (Eq. (4)), per-curve
minimum over the (P, Pdot) grid.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # imported first: the library then shares torch's HIP runtime

__all__ = [
    "GceError", "Plan", "search", "best_fields", "merge_results", "autotune", "lib",
    "LIB_PATH",
    "PRECISION_FP64", "PRECISION_SPLIT_FP32", "TABLE_AUTO", "TABLE_GLOBAL", "TABLE_LDS",
]

# GCE_LIB names another build of the library to load (the host-sanitizer
# test builds one); it must exist like the default one
LIB_PATH = (os.environ.get("GCE_LIB")
            or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgce.so"))

PRECISION_FP64 = 0
PRECISION_SPLIT_FP32 = 1
# where the search kernel reads its c ln c table from
TABLE_AUTO, TABLE_GLOBAL, TABLE_LDS = 0, 1, 2

GCE_OK = 0
STATUS_NAMES = {0: "GCE_OK", -1: "GCE_EINVAL", -2: "GCE_ENOMEM", -3: "GCE_EHIP",
                -4: "GCE_EWORKSPACE", -5: "GCE_ENODEV", -6: "GCE_EUNSUPPORTED"}

# gce_best_t is 48 bytes: int64 flat, int32 p, int32 q, double min, mean,
# std, significance.
BEST_WORDS = 6


class GceError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {text}")
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("trials_per_lane", ctypes.c_int32),
                ("lds_bytes_per_wave", ctypes.c_int32), ("table_in_lds", ctypes.c_int32),
                ("work_units", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("waves_per_unit", ctypes.c_int32), ("refine_units", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("trials_per_lane", ctypes.c_int32),
                ("phase_overlap", ctypes.c_int32), ("table_placement", ctypes.c_int32),
                ("mag_overlap", ctypes.c_int32), ("waves_per_unit", ctypes.c_int32),
                ("refine_units", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def lib():
    """The loaded libgce.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.gce_version.restype = ctypes.c_char_p
        L.gce_status_string.restype = ctypes.c_char_p
        L.gce_status_string.argtypes = [ctypes.c_int]
        L.gce_search.argtypes = [_vp, _vp, ctypes.POINTER(_i64), _i64, _vp, _i64, _vp,
                                 _i64, _i32, _i32, _vp, _vp, _vp]
        L.gce_search_noalloc.argtypes = [_vp, _vp, ctypes.POINTER(_i64), _i64, _vp, _i64, _vp,
                                         _i64, _i32, _i32, _vp, _vp, _vp]
        L.gce_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_i64), _i64,
                                      _i64, _i64, _i32, _i32, ctypes.POINTER(_Opts), _i32]
        L.gce_plan_execute.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.gce_plan_debug_counts.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64,
                                            _vp, _vp]
        L.gce_plan_workspace_bytes.restype = ctypes.c_size_t
        L.gce_plan_workspace_bytes.argtypes = [_vp]
        L.gce_plan_destroy.argtypes = [_vp]
        L.gce_plan_set_timing.argtypes = [_vp, _i32]
        L.gce_plan_get_info.argtypes = [_vp, ctypes.POINTER(_Info)]
        L.gce_merge_results.argtypes = [_vp, _i64, _vp, _i64, _i64, _i64, _i64, _i64, _i64]
        L.gce_autotune.argtypes = [_vp, _vp, ctypes.POINTER(_i64), _i64, _vp, _i64, _vp, _i64,
                                   _i32, _i32, _i32, _i32, _i32, _i32, _vp, ctypes.POINTER(_i32),
                                   ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float)]
        L.gce_plan_search_times.argtypes = [_vp, ctypes.POINTER(ctypes.c_float), _i32,
                                            ctypes.POINTER(_i32)]
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != GCE_OK:
        raise GceError(rc, lib().gce_status_string(rc).decode())


def _host_offsets(offsets) -> np.ndarray:
    if isinstance(offsets, torch.Tensor):
        offsets = offsets.detach().cpu().numpy()
    return np.ascontiguousarray(offsets, dtype=np.int64)


def _dev_f64(x: torch.Tensor, name: str, device: torch.device) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or x.device != device:
        raise TypeError(f"{name} must be a torch tensor on {device}")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    return x


def _ptr(x: Optional[torch.Tensor]):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _stream_handle(stream, device) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return ctypes.c_void_p(h)


def best_fields(best: torch.Tensor) -> dict:
    """Split a [n_curves, 6] gce_best_t tensor (or a host array of the same
    bytes) into numpy fields."""
    if isinstance(best, torch.Tensor):
        best = best.detach().cpu().contiguous().numpy()
    raw = np.ascontiguousarray(best).view(np.uint8).reshape(-1, 8 * BEST_WORDS)
    return {
        "flat_index": raw[:, 0:8].copy().view(np.int64).ravel(),
        "period_index": raw[:, 8:12].copy().view(np.int32).ravel(),
        "pdot_index": raw[:, 12:16].copy().view(np.int32).ravel(),
        "ce_min": raw[:, 16:24].copy().view(np.float64).ravel(),
        "ce_mean": raw[:, 24:32].copy().view(np.float64).ravel(),
        "ce_std": raw[:, 32:40].copy().view(np.float64).ravel(),
        "significance": raw[:, 40:48].copy().view(np.float64).ravel(),
    }


class Plan:
    """A validated, scheduled and allocated search shape (gce_plan_t).

    offsets: host curve offsets [n_curves + 1]; precision: PRECISION_FP64
    (bit-exact bins) or PRECISION_SPLIT_FP32; trials_per_lane: 0 (automatic)
    or 1, 2, 4, 8; phase_overlap / mag_overlap: 50%-overlapping phase /
    magnitude bins (Sec. 2.3); table_placement: TABLE_AUTO, TABLE_GLOBAL or
    TABLE_LDS for the c ln c table; waves_per_unit: 0 (automatic), 1, or 2
    waves sharing one copy of a work unit's histograms; refine_units (split
    path): 0, or the number of each curve's best split work units searched
    again in FP64 for the reported minimum.  Options map one to one onto
    gce_opts.
    """

    def __init__(self, offsets, n_periods: int, n_pdots: int, n_phase: int,
                 n_mag: int, precision: int = PRECISION_FP64,
                 trials_per_lane: int = 0, phase_overlap: bool = False,
                 table_placement: int = TABLE_AUTO, mag_overlap: bool = False,
                 waves_per_unit: int = 0, refine_units: int = 0,
                 device: Optional[torch.device] = None):
        self._h = None
        self.offsets = _host_offsets(offsets)
        self.n_curves = int(self.offsets.size - 1)
        self.n_periods, self.n_pdots = int(n_periods), int(n_pdots)
        self.n_phase, self.n_mag = int(n_phase), int(n_mag)
        self.precision = int(precision)
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            idx = torch.cuda.current_device() if torch.cuda.is_available() else 0
            self.device = torch.device("cuda", idx)
        self.phase_overlap = bool(phase_overlap)
        self.mag_overlap = bool(mag_overlap)
        opts = _Opts(self.precision, int(trials_per_lane), int(self.phase_overlap),
                     int(table_placement), int(self.mag_overlap), int(waves_per_unit),
                     int(refine_units))
        h = ctypes.c_void_p()
        L = lib()
        _check(L.gce_plan_create(ctypes.byref(h),
                                 self.offsets.ctypes.data_as(ctypes.POINTER(_i64)),
                                 self.n_curves, self.n_periods, self.n_pdots,
                                 self.n_phase, self.n_mag, ctypes.byref(opts),
                                 self.device.index))
        self._h = h

    @property
    def workspace_bytes(self) -> int:
        return int(lib().gce_plan_workspace_bytes(self._h))

    def info(self) -> dict:
        """Tiling and resources the plan chose (gce_plan_get_info)."""
        i = _Info()
        _check(lib().gce_plan_get_info(self._h, ctypes.byref(i)))
        return {k: int(getattr(i, k)) for k, _ in _Info._fields_}

    def _inputs(self, times, mags, periods, pdots):
        d = self.device
        _dev_f64(times, "times", d)
        _dev_f64(mags, "mags", d)
        _dev_f64(periods, "periods", d)
        _dev_f64(pdots, "pdots", d)
        if times.numel() != self.offsets[-1] or mags.numel() != self.offsets[-1]:
            raise ValueError("times/mags length differs from the plan's offsets")
        if periods.numel() != self.n_periods or pdots.numel() != self.n_pdots:
            raise ValueError("grid size differs from the plan")

    def cube_dtype(self):
        return torch.float64 if self.precision == PRECISION_FP64 else torch.float32

    def new_cube(self) -> torch.Tensor:
        return torch.empty((self.n_curves, self.n_pdots, self.n_periods),
                           dtype=self.cube_dtype(), device=self.device)

    def new_best(self) -> torch.Tensor:
        return torch.empty((self.n_curves, BEST_WORDS), dtype=torch.float64,
                           device=self.device)

    def execute(self, times, mags, periods, pdots, out_ce=None, out_best=None,
                stream=None):
        """Enqueue the search; returns (out_ce or None, out_best)."""
        self._inputs(times, mags, periods, pdots)
        if out_ce is not None:
            if (out_ce.dtype != self.cube_dtype() or not out_ce.is_contiguous()
                    or out_ce.numel() != self.n_curves * self.n_pdots * self.n_periods
                    or out_ce.device != self.device):
                raise ValueError("out_ce has the wrong dtype, size or device")
        if out_best is None:
            out_best = self.new_best()
        elif (out_best.numel() != self.n_curves * BEST_WORDS or out_best.device != self.device
              or out_best.element_size() != 8 or not out_best.is_contiguous()):
            raise ValueError("out_best has the wrong size, element size, layout or device")
        _check(lib().gce_plan_execute(self._h, _ptr(times), _ptr(mags), _ptr(periods),
                                      _ptr(pdots), _ptr(out_ce), _ptr(out_best),
                                      _stream_handle(stream, self.device)))
        return out_ce, out_best

    def debug_counts(self, times, mags, periods, pdots, trial_curve, trial_flat,
                     stream=None) -> torch.Tensor:
        """[n_trials, n_mag, n_phase] uint32 histograms (returned as int32
        storage; the values are < 65536)."""
        self._inputs(times, mags, periods, pdots)
        tc = torch.as_tensor(trial_curve, dtype=torch.int64).to(self.device).contiguous()
        tf = torch.as_tensor(trial_flat, dtype=torch.int64).to(self.device).contiguous()
        if tc.numel() != tf.numel():
            raise ValueError("trial_curve and trial_flat differ in length")
        out = torch.empty((tc.numel(), self.n_mag, self.n_phase), dtype=torch.int32,
                          device=self.device)
        _check(lib().gce_plan_debug_counts(self._h, _ptr(times), _ptr(mags), _ptr(periods),
                                           _ptr(pdots), _ptr(tc), _ptr(tf), tc.numel(),
                                           _ptr(out), _stream_handle(stream, self.device)))
        return out

    def set_timing(self, capacity: int) -> None:
        """Record HIP events around the search kernel of the next executes."""
        _check(lib().gce_plan_set_timing(self._h, int(capacity)))

    def search_times_ms(self, max_n: int = 65536) -> np.ndarray:
        """Search-kernel durations (ms) of the most recent timed executes."""
        buf = (ctypes.c_float * max_n)()
        n = _i32(0)
        _check(lib().gce_plan_search_times(self._h, buf, max_n, ctypes.byref(n)))
        return np.frombuffer(buf, dtype=np.float32, count=n.value).astype(np.float64)

    def close(self) -> None:
        if self._h is not None and _lib is not None:
            _check(_lib.gce_plan_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(times: torch.Tensor, mags: torch.Tensor, offsets, periods: torch.Tensor,
             pdots: torch.Tensor, n_phase: int, n_mag: int,
             precision: int = PRECISION_FP64, phase_overlap: bool = False,
             mag_overlap: bool = False, stream=None):
    """Time the tilings (trials per lane x table placement) on a slice of this
    workload and remember the fastest for its shape class (gce_autotune).
    Returns (chosen trials per lane, chosen placement,
    {(trials, placement): kernel ms})."""
    device = times.device
    for name, x in (("times", times), ("mags", mags), ("periods", periods),
                    ("pdots", pdots)):
        _dev_f64(x, name, device)
    off = _host_offsets(offsets)
    tq, placement = _i32(0), _i32(0)
    ms = (ctypes.c_float * 8)()
    _check(lib().gce_autotune(_ptr(times), _ptr(mags),
                              off.ctypes.data_as(ctypes.POINTER(_i64)), off.size - 1,
                              _ptr(periods), periods.numel(), _ptr(pdots), pdots.numel(),
                              int(n_phase), int(n_mag), int(precision), int(phase_overlap),
                              int(mag_overlap), device.index or 0, _stream_handle(stream, device),
                              ctypes.byref(tq), ctypes.byref(placement), ms))
    keys = [(t, pl) for pl in (TABLE_GLOBAL, TABLE_LDS) for t in (1, 2, 4, 8)]
    return tq.value, placement.value, {k: float(v) for k, v in zip(keys, ms) if v >= 0}


def merge_results(acc: Optional[np.ndarray], acc_trials: int, part, n_periods: int,
                  part_p_offset: int, part_n_periods: int, part_q_offset: int,
                  part_n_pdots: int) -> np.ndarray:
    """Combine the per-curve results of a search over a sub-grid into a running
    result (gce_merge_results).  part: [n_curves, 6] tensor or array as
    returned by execute; acc: host array of the same shape or None.  Returns
    the updated host array."""
    if isinstance(part, torch.Tensor):
        part = part.detach().cpu().contiguous().numpy()
    part = np.ascontiguousarray(part, dtype=np.float64)
    if acc is None:
        acc = np.empty_like(part)
        acc_trials = 0
    _check(lib().gce_merge_results(acc.ctypes.data_as(_vp), int(acc_trials),
                                   part.ctypes.data_as(_vp), part.shape[0],
                                   int(n_periods), int(part_p_offset),
                                   int(part_n_periods), int(part_q_offset),
                                   int(part_n_pdots)))
    return acc


def search(times: torch.Tensor, mags: torch.Tensor, offsets, periods: torch.Tensor,
           pdots: torch.Tensor, n_phase: int, n_mag: int, want_cube: bool = True,
           stream=None, out_ce: Optional[torch.Tensor] = None,
           out_best: Optional[torch.Tensor] = None, no_alloc: bool = False):
    """One-call FP64 search through gce_search, or gce_search_noalloc with
    no_alloc=True (its workspace is the library's fixed device array; the
    library allocates nothing).  out_ce / out_best may be given (else they are
    allocated here, by torch).  Returns (cube or None, best)."""
    device = times.device
    for name, x in (("times", times), ("mags", mags), ("periods", periods),
                    ("pdots", pdots)):
        _dev_f64(x, name, device)
    off = _host_offsets(offsets)
    nc = off.size - 1
    cube = out_ce
    if cube is None and want_cube:
        cube = torch.empty((nc, pdots.numel(), periods.numel()), dtype=torch.float64,
                           device=device)
    if cube is not None and (cube.dtype != torch.float64 or not cube.is_contiguous()
                             or cube.numel() != nc * pdots.numel() * periods.numel()
                             or cube.device != device):
        raise ValueError("out_ce has the wrong dtype, size or device")
    best = out_best
    if best is None:
        best = torch.empty((nc, BEST_WORDS), dtype=torch.float64, device=device)
    elif (best.numel() != nc * BEST_WORDS or best.device != device
          or best.element_size() != 8 or not best.is_contiguous()):
        raise ValueError("out_best has the wrong size, element size, layout or device")
    entry = lib().gce_search_noalloc if no_alloc else lib().gce_search
    with torch.cuda.device(device):
        _check(entry(_ptr(times), _ptr(mags),
                                off.ctypes.data_as(ctypes.POINTER(_i64)), nc,
                                _ptr(periods), periods.numel(), _ptr(pdots),
                                pdots.numel(), int(n_phase), int(n_mag), _ptr(cube),
                                _ptr(best), _stream_handle(stream, device)))
    return cube, best
