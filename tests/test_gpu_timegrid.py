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
