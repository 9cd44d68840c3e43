"""Period-range chunked search with checkpoint and resume.

A search over the paper's full grid (Sec. 3: 5,183,995 trial periods times
32 Pdot values per binary) runs long enough that it should survive an
interruption, and a CE cube over it does not fit in memory.  Sec. 4
describes the remedy the paper uses: run the grid in batches, keep each
batch's minimum, and combine the batches.

Here the period grid is cut into contiguous ranges.  Each range is one plan
execution over a view of the device period array; its per-curve result
(minimum and the moments behind Eq. (5)) is merged into a running result by
``gce_merge_results``, which takes the lexicographic minimum in full-grid
indices and merges the moments exactly.  After every range the running
result and the index of the next range go to a checkpoint file, written
beside the target and renamed over it, so the file always holds a complete
state.  A restarted run with the same inputs and options picks up after the
last completed range and ends with the result of an uninterrupted run; a
checkpoint of different inputs is refused.

The optional ``on_range`` callback receives each range's CE cube slice
(when ``want_cube`` is set) so a caller can write the cube out range by
range.
"""
from __future__ import annotations

import hashlib
import os
from typing import Callable, Optional

import numpy as np

CHECKPOINT_VERSION = 1


def range_bounds(n_periods: int, chunk: int):
    """[(p0, p1), ...] covering 0..n_periods in steps of chunk periods."""
    if n_periods < 1 or chunk < 1:
        raise ValueError("n_periods and chunk must be positive")
    return [(p0, min(p0 + chunk, n_periods)) for p0 in range(0, n_periods, chunk)]


def fingerprint(arrays, **scalars) -> str:
    """sha256 over the inputs (host arrays, raw bytes with dtype and shape)
    and the options that change the result."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str((a.dtype.str, a.shape)).encode())
        h.update(a.tobytes())
    for k in sorted(scalars):
        h.update(f"{k}={scalars[k]!r};".encode())
    return h.hexdigest()


def save_checkpoint(path: str, acc: np.ndarray, next_range: int, fp: str) -> None:
    """Write the running result atomically (temporary file, then rename)."""
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "wb") as f:
        np.savez(f, version=np.int64(CHECKPOINT_VERSION), acc=acc,
                 next_range=np.int64(next_range),
                 fingerprint=np.frombuffer(fp.encode(), dtype=np.uint8))
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def load_checkpoint(path: str, fp: str):
    """(acc, next_range) from a checkpoint of the same inputs, or None when
    there is no file.  A checkpoint of other inputs raises ValueError."""
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        if int(z["version"]) != CHECKPOINT_VERSION:
            raise ValueError(f"{path}: checkpoint version {int(z['version'])} "
                             f"is not {CHECKPOINT_VERSION}")
        if z["fingerprint"].tobytes().decode() != fp:
            raise ValueError(f"{path}: checkpoint belongs to other inputs or options")
        return np.array(z["acc"]), int(z["next_range"])


def run_ranges(n_periods: int, n_pdots: int, chunk: int,
               execute_range: Callable[[int, int], object],
               merge: Callable, checkpoint: Optional[str] = None, fp: str = "",
               on_range: Optional[Callable] = None) -> np.ndarray:
    """Drive the ranges: execute_range(p0, p1) returns the [n_curves, 6]
    result of periods p0..p1 (all Pdot values) and optionally a cube slice as
    (best, cube); merge is ``merge_results``.  Returns the merged host result."""
    bounds = range_bounds(n_periods, chunk)
    acc, start = None, 0
    if checkpoint:
        state = load_checkpoint(checkpoint, fp)
        if state is not None:
            acc, start = state
    for i in range(start, len(bounds)):
        p0, p1 = bounds[i]
        out = execute_range(p0, p1)
        best, cube = out if isinstance(out, tuple) else (out, None)
        acc = merge(acc, p0 * n_pdots, best, n_periods, p0, p1 - p0, 0, n_pdots)
        if on_range is not None:
            on_range(i, p0, p1, cube)
        if checkpoint:
            save_checkpoint(checkpoint, acc, i + 1, fp)
    if acc is None:   # the checkpoint already covered every range
        raise ValueError("no range left to run and no result: empty grid")
    return acc


def search_chunked(times, mags, offsets, periods, pdots, n_phase: int, n_mag: int,
                   chunk_periods: int, checkpoint: Optional[str] = None,
                   precision: int = 0, phase_overlap: bool = False,
                   trials_per_lane: int = 0, table_placement: int = 0,
                   mag_overlap: bool = False, refine_units: int = 0,
                   want_cube: bool = False, on_range: Optional[Callable] = None,
                   stream=None) -> np.ndarray:
    """Minimum and statistics of every curve over the full (P, Pdot) grid,
    computed range by range (chunk_periods periods at a time).

    times, mags, periods, pdots: float64 device tensors as for Plan.execute;
    offsets: host curve offsets.  Returns the merged [n_curves, 6] host
    array (read it with ``best_fields``).  With ``checkpoint`` set, progress
    is saved after every range and a rerun resumes from it.  refine_units
    (split path): each range's minima confirmed in FP64 over each curve's
    best work units of that range, as for Plan."""
    import torch
    from . import Plan, merge_results

    n_p, n_pd = int(periods.numel()), int(pdots.numel())
    fp = ""
    if checkpoint:
        host = [np.asarray(offsets, dtype=np.int64)] + [
            x.detach().cpu().numpy() for x in (times, mags, periods, pdots)]
        # a confirmation of the minima changes the results it checkpoints
        extra = {"refine": int(refine_units)} if refine_units else {}
        fp = fingerprint(host, n_phase=int(n_phase), n_mag=int(n_mag),
                         precision=int(precision), phase_overlap=bool(phase_overlap),
                         mag_overlap=bool(mag_overlap), chunk=int(chunk_periods), **extra)
    plans = {}

    def execute_range(p0, p1):
        n = p1 - p0
        if n not in plans:
            plans[n] = Plan(offsets, n, n_pd, n_phase, n_mag, precision=precision,
                            trials_per_lane=trials_per_lane, phase_overlap=phase_overlap,
                            table_placement=table_placement, mag_overlap=mag_overlap,
                            refine_units=refine_units, device=times.device)
        plan = plans[n]
        cube = plan.new_cube() if want_cube else None
        cube, best = plan.execute(times, mags, periods[p0:p1], pdots, out_ce=cube,
                                  stream=stream)
        s = stream if stream is not None else torch.cuda.current_stream(times.device)
        s.synchronize()
        return best, cube

    try:
        return run_ranges(n_p, n_pd, chunk_periods, execute_range, merge_results,
                          checkpoint, fp, on_range)
    finally:
        for plan in plans.values():
            plan.close()
