"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad arguments on the host (no GPU compute here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2006_06866_amd as gce
from paper_2006_06866_amd import build as gbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gce.h")


def _ensure_built():
    if not os.path.exists(gce.LIB_PATH):
        gbuild.build()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*[\s\*]+([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n.startswith("gce_")))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("gce_search", "gce_plan_create", "gce_plan_execute",
                     "gce_plan_debug_counts", "gce_plan_destroy",
                     "gce_plan_workspace_bytes", "gce_status_string", "gce_version"):
        assert required in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(gce.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    _ensure_built()
    L = gce.lib()
    assert b"gfx950" in L.gce_version()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert len(L.gce_status_string(code)) > 0


@pytest.mark.parametrize("offsets,n_p,n_pd,n_phase,n_mag", [
    ([0, 5, 3], 10, 2, 10, 5),          # decreasing offsets
    ([0, 5, 5], 10, 2, 10, 5),          # empty curve
    ([1, 5, 9], 10, 2, 10, 5),          # offsets[0] != 0
    ([0, 70000], 10, 2, 10, 5),         # curve longer than 65535
    ([0, 5], 0, 2, 10, 5),              # no periods
    ([0, 5], 10, 0, 10, 5),             # no pdots
    ([0, 5], 10, 2, 0, 5),              # no phase bins
    ([0, 5], 10, 2, 129, 5),            # too many phase bins
    ([0, 5], 10, 2, 10, 0),             # no magnitude bins
    ([0, 5], 10, 2, 10, 256),           # too many magnitude bins
])
def test_bad_shapes_rejected_on_host(offsets, n_p, n_pd, n_phase, n_mag):
    _ensure_built()
    with pytest.raises(gce.GceError) as ei:
        gce.Plan(np.array(offsets), n_p, n_pd, n_phase, n_mag, device="cuda:0")
    assert ei.value.status == -1


def test_bad_options_rejected_on_host():
    _ensure_built()
    with pytest.raises(gce.GceError) as ei:
        gce.Plan(np.array([0, 5]), 10, 2, 10, 5, trials_per_lane=16, device="cuda:0")
    assert ei.value.status == -1
    with pytest.raises(gce.GceError) as ei:
        gce.Plan(np.array([0, 5]), 10, 2, 10, 5, precision=7, device="cuda:0")
    assert ei.value.status == -1
    with pytest.raises(gce.GceError) as ei:
        gce.Plan(np.array([0, 5]), 10, 2, 10, 5, table_placement=3, device="cuda:0")
    assert ei.value.status == -1


def test_null_plan_and_pointers_rejected():
    _ensure_built()
    L = gce.lib()
    assert L.gce_plan_execute(None, None, None, None, None, None, None, None) == -1
    assert L.gce_plan_destroy(None) == 0
    assert L.gce_plan_workspace_bytes(None) == 0
    off = np.array([0, 4], dtype=np.int64)
    rc = L.gce_search(None, None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1,
                      None, 3, None, 1, 10, 5, None, None, None)
    assert rc == -1


def test_valid_shape_needs_a_gfx950_device():
    """With no GPU the host checks pass and device selection fails cleanly."""
    _ensure_built()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(gce.GceError) as ei:
        gce.Plan(np.array([0, 5, 9]), 10, 2, 10, 5, device="cuda:0")
    assert ei.value.status == -5


def test_overlap_count_limits_rejected_on_host():
    """Overlapping bins count an epoch more than once; the 16-bit counts
    bound the longest curve (halved with overlapping magnitude bins, again
    for one overlapping phase bin, and at 8191 counts with the table in LDS)."""
    _ensure_built()
    cases = [
        (dict(mag_overlap=True), 10, 32768),
        (dict(mag_overlap=True, phase_overlap=True), 1, 16384),
        (dict(phase_overlap=True), 1, 32768),
        (dict(mag_overlap=True, table_placement=gce.TABLE_LDS), 10, 4096),
    ]
    for kw, n_phase, n in cases:
        with pytest.raises(gce.GceError) as ei:
            gce.Plan(np.array([0, n]), 10, 2, n_phase, 5, device="cuda:0", **kw)
        assert ei.value.status == -6, (kw, n_phase, n)
    L = gce.lib()
    off = np.array([0, 5], dtype=np.int64)
    h = ctypes.c_void_p()
    for bad in (gce._Opts(0, 0, 0, 0, 2), gce._Opts(0, 0, 0, 0, -1)):
        rc = L.gce_plan_create(ctypes.byref(h),
                               off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, 10,
                               2, 10, 5, ctypes.byref(bad), 0)
        assert rc == -1


def test_waves_per_unit_checked_on_host():
    """waves_per_unit is 0, 1 or 2 (else GCE_EINVAL); 2 needs a compiled
    two-wave kernel for the phase-bin count and trials per lane (else
    GCE_EUNSUPPORTED).  Both are refused before any device call."""
    _ensure_built()
    off = np.array([0, 5, 9])
    for bad in (-1, 3):
        with pytest.raises(gce.GceError) as ei:
            gce.Plan(off, 10, 8, 10, 5, waves_per_unit=bad, device="cuda:0")
        assert ei.value.status == -1, bad
    for n_phase, tq in ((15, 4), (10, 1), (10, 2), (33, 2), (20, 1)):
        with pytest.raises(gce.GceError) as ei:
            gce.Plan(off, 10, 8, n_phase, 5, trials_per_lane=tq, waves_per_unit=2,
                     device="cuda:0")
        assert ei.value.status == -6, (n_phase, tq)


def test_refine_units_checked_on_host():
    """refine_units is in [0, 64] (else GCE_EINVAL), refused before any
    device call, whatever the precision."""
    _ensure_built()
    off = np.array([0, 5, 9])
    for prec in (gce.PRECISION_FP64, gce.PRECISION_SPLIT_FP32):
        for bad in (-1, 65, 1 << 20):
            with pytest.raises(gce.GceError) as ei:
                gce.Plan(off, 10, 8, 10, 5, precision=prec, refine_units=bad, device="cuda:0")
            assert ei.value.status == -1, (prec, bad)


def _write_inputs(d, w):
    w.times.astype("<f8").tofile(os.path.join(d, "times.f64"))
    w.mags.astype("<f8").tofile(os.path.join(d, "mags.f64"))
    np.asarray(w.offsets, dtype="<i8").tofile(os.path.join(d, "offsets.i64"))
    w.periods.astype("<f8").tofile(os.path.join(d, "periods.f64"))
    w.pdots.astype("<f8").tofile(os.path.join(d, "pdots.f64"))


def test_file_search_program_rejects_bad_use_on_host(tmp_path):
    """The command-line program over raw files: usage, I/O and shape errors
    are reported before any GPU work."""
    import subprocess
    from paper_2006_06866_amd import synth
    if not os.path.exists(gbuild.FILE_SEARCH):
        gbuild.build()
    exe = gbuild.FILE_SEARCH
    assert subprocess.run([exe], capture_output=True).returncode == 2
    assert subprocess.run([exe, str(tmp_path), "10", "5", "--bogus"],
                          capture_output=True).returncode == 2
    r = subprocess.run([exe, str(tmp_path), "10", "5"], capture_output=True, text=True)
    assert r.returncode == 1 and "cannot open" in r.stderr
    w = synth.random_curves(3, [20, 30], n_freq=8, n_pdots=2)
    _write_inputs(str(tmp_path), w)
    r = subprocess.run([exe, str(tmp_path), "129", "5"], capture_output=True, text=True)
    assert r.returncode == 1 and "invalid argument" in r.stderr
    with open(os.path.join(str(tmp_path), "mags.f64"), "ab") as f:
        f.write(b"\0" * 8)   # one magnitude too many
    r = subprocess.run([exe, str(tmp_path), "10", "5"], capture_output=True, text=True)
    assert r.returncode == 1 and "inconsistent" in r.stderr


def test_injected_allocation_failure(monkeypatch):
    """GCE_FAIL_ALLOC=1 makes every allocating entry point return GCE_ENOMEM
    after its argument checks and before any device call; argument errors
    still come first."""
    _ensure_built()
    L = gce.lib()
    off = np.array([0, 5, 9], dtype=np.int64)
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    monkeypatch.setenv("GCE_FAIL_ALLOC", "1")
    with pytest.raises(gce.GceError) as ei:
        gce.Plan(off, 10, 2, 10, 5, device="cuda:0")
    assert ei.value.status == -2
    assert b"GCE_FAIL_ALLOC" in L.gce_status_string(-2)
    with pytest.raises(gce.GceError) as ei:   # a bad shape is still EINVAL
        gce.Plan(off, 10, 2, 129, 5, device="cuda:0")
    assert ei.value.status == -1
    dummy = ctypes.c_void_p(16)   # never dereferenced: the call fails first
    rc = L.gce_search(dummy, dummy, offp, 2, dummy, 10, dummy, 2, 10, 5, None, dummy, None)
    assert rc == -2
    tq, pl = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = L.gce_autotune(dummy, dummy, offp, 2, dummy, 10, dummy, 2, 10, 5, 0, 0, 0, 0, None,
                        ctypes.byref(tq), ctypes.byref(pl), None)
    assert rc == -2
    monkeypatch.setenv("GCE_FAIL_ALLOC", "0")
    import torch
    if not torch.cuda.is_available():   # without the injection: no device here
        with pytest.raises(gce.GceError) as ei:
            gce.Plan(off, 10, 2, 10, 5, device="cuda:0")
        assert ei.value.status == -5


def test_noalloc_entry_point_bounds_its_workspace_on_host():
    """gce_search_noalloc refuses shapes beyond its fixed device array with
    GCE_EWORKSPACE and bad arguments with GCE_EINVAL, before any device call."""
    _ensure_built()
    L = gce.lib()
    dummy = ctypes.c_void_p(16)   # never dereferenced: the calls fail first
    # 1,024 curves x 600 epochs, 20,000 x 64 trials: 2.6 M work units at
    # 8 trials per lane, beyond the array
    off = np.arange(0, 1025 * 600, 600, dtype=np.int64)
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = L.gce_search_noalloc(dummy, dummy, offp, 1024, dummy, 20000, dummy, 64, 10, 5, None,
                              dummy, None)
    assert rc == -4
    assert b"scratch" in L.gce_status_string(rc)
    rc = L.gce_search_noalloc(dummy, dummy, offp, 512, dummy, 20000, dummy, 64, 129, 5, None,
                              dummy, None)
    assert rc == -1
    rc = L.gce_search_noalloc(None, dummy, offp, 512, dummy, 100, dummy, 1, 10, 5, None,
                              dummy, None)
    assert rc == -1
