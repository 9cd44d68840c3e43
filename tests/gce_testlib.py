"""Shared helpers of the GPU tests: device upload, tolerances, sampling."""
import math
import sys

import numpy as np
import torch

import oracle
import paper_2006_06866_amd as gce


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).to("cuda")


def upload(w):
    return (to_dev(w.times), to_dev(w.mags), to_dev(w.periods), to_dev(w.pdots))


def ce_tolerance(h_ref, n_phase, n_mag, n_points):
    """|H_gpu - H_oracle| bound.

    The GPU forms N*H = sum_b c_b ln c_b - sum_jb c_jb ln c_jb: two sums of
    at most n_phase*(n_mag+1) table values, each sum bounded by N ln N, so
    its rounding is below (terms + 2) * 2^-53 * N ln N, i.e. a bound of
    (terms + 2) * 2^-53 * ln N on H, doubled for the table and the oracle's
    own rounding.  Plus 1e-12 relative, the agreement the method promises.
    """
    n = np.maximum(2.0 * np.asarray(n_points, dtype=np.float64), 2.0)
    terms = n_phase * (n_mag + 1) + 2
    return 1e-12 * np.abs(h_ref) + 2.0 * terms * 2.0 ** -53 * np.log(n)


def run_gpu(w, want_cube=True, trials_per_lane=0, stream=None, phase_overlap=False,
            precision=0, table_placement=0, mag_overlap=False, waves_per_unit=0):
    t, m, P, Pd = upload(w)
    plan = gce.Plan(w.offsets, w.periods.size, w.pdots.size, w.n_phase, w.n_mag,
                    trials_per_lane=trials_per_lane, phase_overlap=phase_overlap,
                    precision=precision, table_placement=table_placement,
                    mag_overlap=mag_overlap, waves_per_unit=waves_per_unit)
    cube = plan.new_cube() if want_cube else None
    cube, best = plan.execute(t, m, P, Pd, out_ce=cube, stream=stream)
    torch.cuda.synchronize()
    return plan, (t, m, P, Pd), cube, best


def assert_cube_close(gpu_cube, ora_cube, w, label="", count_mult=1):
    """count_mult: entries per epoch at most (2 with overlapping magnitude
    bins), which scales the N of the tolerance."""
    n = count_mult * w.lengths[:, None, None].astype(np.float64)
    tol = ce_tolerance(ora_cube, w.n_phase, w.n_mag, n)
    err = np.abs(gpu_cube - ora_cube)
    bad = ~(err <= tol)
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(
            f"{label}: {bad.sum()} of {bad.size} CE values out of tolerance; "
            f"first {idx.tolist()} gpu={gpu_cube[tuple(idx[0])]!r} "
            f"oracle={ora_cube[tuple(idx[0])]!r} max err={err.max():.3e}")


def assert_best_valid(bf_gpu, bc_gpu, bf_ora, bc_ora, ora_cube, w, label="", count_mult=1):
    """The GPU minimum must be the oracle's, or a trial whose oracle CE ties
    the oracle minimum within tolerance (near-equal CE values may order
    differently under the two exact-to-rounding formulas)."""
    n_p = w.periods.size
    for c in range(w.n_curves):
        tol = ce_tolerance(bc_ora[c], w.n_phase, w.n_mag, count_mult * w.lengths[c])
        assert abs(bc_gpu[c] - bc_ora[c]) <= tol, (label, c, bc_gpu[c], bc_ora[c])
        if bf_gpu[c] != bf_ora[c]:
            q, p = divmod(int(bf_gpu[c]), n_p)
            assert ora_cube[c, q, p] <= bc_ora[c] + 2 * tol, (label, c, bf_gpu[c], bf_ora[c])


def check_counts_exact(plan, dev_inputs, w, curve_ids, flat_ids, label=""):
    t, m, P, Pd = dev_inputs
    got = plan.debug_counts(t, m, P, Pd, curve_ids, flat_ids)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.uint32)
    ovl = getattr(plan, "phase_overlap", False)
    movl = getattr(plan, "mag_overlap", False)
    _, want = oracle.trials(w.times, w.mags, w.offsets, w.periods, w.pdots, w.n_phase,
                            w.n_mag, curve_ids, flat_ids, want_counts=True,
                            phase_overlap=ovl, mag_overlap=movl)
    if not np.array_equal(got, want):
        bad = np.argwhere(np.any(got != want, axis=(1, 2))).ravel()
        i = int(bad[0])
        raise AssertionError(f"{label}: {bad.size} of {len(curve_ids)} trial histograms differ; "
                             f"first trial curve={curve_ids[i]} flat={flat_ids[i]}\n"
                             f"gpu={got[i].tolist()}\noracle={want[i].tolist()}")
    mult = 2 if ovl else 1
    totals = got.sum(axis=(1, 2))
    if movl:   # N to 2N entries, the same for every trial of a curve
        n = w.lengths[np.asarray(curve_ids)]
        assert np.all((totals >= mult * n) & (totals <= 2 * mult * n))
    else:
        assert np.all(totals == mult * w.lengths[np.asarray(curve_ids)])


def best_rows(cube):
    """gce_best_t rows ([n_curves, 6] float64 words) of a [n_curves, n_pd, n_p]
    CE array: first minimum in flat order, population mean and std, rho."""
    nc = cube.shape[0]
    out = np.zeros((nc, gce.BEST_WORDS))
    raw = out.view(np.uint8).reshape(nc, 8 * gce.BEST_WORDS)
    for c in range(nc):
        flat = cube[c].ravel()
        f = int(np.argmin(flat))
        q, p = divmod(f, cube.shape[2])
        mu, sd = flat.mean(), flat.std()
        raw[c, 0:8] = np.array([f], dtype=np.int64).view(np.uint8)
        raw[c, 8:16] = np.array([p, q], dtype=np.int32).view(np.uint8)
        raw[c, 16:48] = np.array([flat[f], mu, sd, (mu - flat[f]) / sd if sd > 0 else 0.0]
                                 ).view(np.uint8)
    return out

