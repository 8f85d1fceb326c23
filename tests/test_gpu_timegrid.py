"""Graded (non-uniform) time grid of em_run_to_ttf: aging interval k steps with
dt * g^k, the backward-Euler factors rebuilt at each step size (the paper's
non-uniform inner grid with per-step-size factors).  Against the FP64 oracle
on the same grid, FP64 and FP32, and the uniform step restored afterwards."""
import numpy as np
import pytest

import ttf_check

from paper_2604_10743_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def em():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_10743_amd as P
    return P


def _graded(rn, g):
    # the same ten-year horizon on a grid growing by g per interval
    n_int = rn["n_steps"] // rn["ir_every"]
    horizon = rn["dt"] * rn["n_steps"]
    dt0 = horizon / (rn["ir_every"] * sum(g ** k for k in range(n_int)))
    return dict(rn, dt=dt0, dt_growth=g)


@pytest.mark.parametrize("prec", [0, 1])
def test_graded_grid_matches_oracle(em, oracle_mod, prec):
    g, mat, rn, mc = synth.workload("mc_grid")
    rn = _graded(dict(rn, prec=prec), 1.25)
    S = 16
    mc = dict(mc, n_samples=S)
    print(f"graded grid prec {prec}", flush=True)
    B = em.Batch(g, mat, rn, mc)
    res = B.run_to_ttf()
    segs = {s: B.failed_segments(s) for s in range(0, S, 2)}
    B.close()
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    n_cmp = n_fail = 0
    for s in range(0, S, 2):
        ref = oracle_mod.run_sample(g, mat, rn, mc, s, topo=topo)
        r = res[s]
        n_cmp += 1
        n_fail += ref["failed"]
        ttf_check.check(r, ref, segs[s], prec, rn, s)
    assert n_cmp == 8 and n_fail >= 1


def test_uniform_step_restored_after_graded_run(em):
    g, mat, rn, mc = synth.workload("mc_grid")
    rn = _graded(dict(rn, prec=0), 1.5)
    mc = dict(mc, n_samples=2)
    A = em.Batch(g, mat, rn, mc)
    A.run_to_ttf()
    A.reset()
    A.ir_solve()
    A.stress_step(150)
    B = em.Batch(g, mat, rn, mc)
    B.ir_solve()
    B.stress_step(150)
    for s in range(2):
        assert np.array_equal(A.stress(s), B.stress(s))
    A.close()
    B.close()
    with pytest.raises(em.EmError):
        em.Batch(g, mat, dict(rn, dt_growth=-1.0), mc)


@pytest.mark.parametrize("prec", [0, 1])
def test_adaptive_grid_matches_oracle(em, oracle_mod, prec):
    """The adaptive grid (dt_adapt = 3: steps up to 8 dt between nucleations,
    back to dt after one) on one-sample batches, each a Monte Carlo sample of
    mc_grid picked by its index, against the oracle on the same rule: the
    failure decision, re-solve index, TTF, final drop and failed segments, at
    the precision's bar; fewer re-solves than the uniform grid's 20."""
    g, mat, rn, mc = synth.workload("mc_grid")
    rn = dict(rn, prec=prec, dt_adapt=3)
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    n_fail = 0
    for s in (0, 1, 2, 5):
        print(f"adaptive grid prec {prec} sample {s}", flush=True)
        B = em.Batch(g, mat, rn, dict(mc, n_samples=1, sample_ids=[s]))
        r = B.run_to_ttf()[0]
        segs = B.failed_segments(0)
        B.close()
        ref = oracle_mod.run_sample(g, mat, rn, mc, s, topo=topo)
        ttf_check.check(r, ref, segs, prec, rn, s)
        assert ref["outer_idx"] < 20 or ref["failed"]
        n_fail += ref["failed"]
    assert n_fail >= 1


def test_adaptive_grid_with_skipping_and_reduced_stepping(em):
    """The adaptive grid combined with steady-state skipping (exact within its
    band: the same results) and with reduced stepping (the same decisions,
    drops within the paper's 0.05 %), screen off, on a 16-sample batch."""
    g, mat, rn, mc = synth.workload("mc_grid")
    mc = dict(mc, n_samples=16)
    ra = dict(rn, prec=0, screen=0, dt_adapt=3)

    def go(over):
        B = em.Batch(g, mat, dict(ra, **over), mc)
        res = B.run_to_ttf()
        info = B.info()
        B.close()
        return res, info

    a, ia = go({})
    b, ib = go({"ss_tol": 1e-6})
    c, ic = go({"krylov_q": 6})
    assert ib["n_ss_skipped"] > 0 and ic["n_krylov_intervals"] > 0
    for s in range(16):
        for x, tol in ((b, 1e-6), (c, 5e-4)):
            assert a[s]["failed"] == x[s]["failed"] and a[s]["outer_idx"] == x[s]["outer_idx"], s
            assert abs(a[s]["final_drop"] - x[s]["final_drop"]) <= tol * a[s]["final_drop"], s
            if a[s]["failed"]:
                assert abs(a[s]["ttf_s"] - x[s]["ttf_s"]) <= tol * a[s]["ttf_s"], s
