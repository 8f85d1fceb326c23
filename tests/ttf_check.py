"""Per-sample comparison of a GPU run-to-TTF result with the FP64 oracle's
(no arithmetic of the method here: only the comparison rules).

Tolerances: the t = 0 drop to 100 x the PCG tolerance (at least 1e-9); FP64
stepping, and FP32 samples that the library re-ran in FP64
because a worst drop came within the guard band of the failure threshold or
the time to failure was ill-conditioned (em_run_params.guard_band,
guard_ttf), are held to 1e-6 relative on TTF and final drop; other FP32
samples to 1e-3.  The integers are compared exactly: failure flag,
re-solve index, failed-segment set.  A sample whose oracle drop lies within
half the band of the threshold at some re-solve must have been re-run (the
FP32 drop error, measured below 1e-4 relative, is far inside half the band),
so no decision is left to FP32 where FP32 cannot resolve it."""
import math

import numpy as np

TOL_FP64 = 1e-6
TOL_FP32 = 1e-3


def near_threshold(ref, fail_frac, band):
    d = np.asarray(ref["drops"], np.float64)
    return band > 0 and np.min(np.abs(d - fail_frac)) < 0.5 * band * fail_frac


def check(r, ref, segs, prec, rn, label):
    band = float(rn.get("guard_band", 0.0)) if prec == 1 else 0.0
    if near_threshold(ref, rn["fail_frac"], band):
        assert r["redecided"] == 1, f"{label}: within half the guard band but not re-run in FP64"
    tol = TOL_FP64 if (prec == 0 or r["redecided"]) else TOL_FP32
    assert r["failed"] == ref["failed"], label
    # the t = 0 drop: an IR solve to the run's PCG tolerance (1e-11 with FP64
    # stepping, 1e-8 with FP32) against the oracle's direct solve
    rt = float(rn.get("cg_rtol", 0.0))
    rtol = rt if rt > 0 else (1e-11 if prec == 0 else 1e-8)
    tol_init = max(1e-9, 100.0 * rtol)
    assert abs(r["init_drop"] - ref["init_drop"]) <= tol_init * ref["init_drop"], label
    assert abs(r["final_drop"] - ref["final_drop"]) <= tol * ref["final_drop"], label
    assert r["outer_idx"] == ref["outer_idx"], label
    if ref["failed"]:
        assert abs(r["ttf_s"] - ref["ttf"]) <= tol * ref["ttf"], label
    else:
        assert math.isnan(r["ttf_s"]), label
    if segs is not None:
        assert np.array_equal(segs, ref["failed_segs"]), label
