"""The workgroup stepper of branched trees (heavy-path scans, one workgroup
per (tree, sample)) against the FP64 oracle and against the per-lane tree
kernel, on comb/stub trees of up to a few hundred branches: stress per tree,
nucleation events (including junction nodes), void records, Monte Carlo
samples, and the FP32 form."""
import numpy as np
import pytest

from cases import material, run
from paper_2604_10743_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def em():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_10743_amd as P
    return P


def _flush(msg):
    print(msg, flush=True)


def _per_tree_rel(a, b, tree_off):
    worst = 0.0
    for t in range(len(tree_off) - 1):
        sl = slice(tree_off[t], tree_off[t + 1])
        den = np.max(np.abs(b[sl]))
        if den > 0:
            worst = max(worst, np.max(np.abs(a[sl] - b[sl])) / den)
    return worst


def _events(ev, cols):
    if ev.size == 0:
        return ev.reshape(0, len(cols))
    e = ev[:, cols]
    return e[np.lexsort(e.T[::-1])]


def _degree(topo):
    deg = np.zeros(topo.n_stress, int)
    has_p = topo.parent >= 0
    deg[has_p] += 1
    np.add.at(deg, topo.parent[has_p], 1)
    return deg


def test_combs_fp64_vs_oracle(em, oracle_mod):
    g = synth.comb_trees(7001, n_trees=12)
    mat = material(sigma_crit=300e6)
    rn = run(prec=0, screen=0, max_voids_per_tree=4)
    _flush("combs fp64")
    B = em.Batch(g, mat, rn)
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    sim = oracle_mod.SampleSim(g, mat, rn, topo)
    sim.set_j(g.seg_j)
    done = 0
    for chunk in (1, 9, 90, 400, 1500):
        B.stress_step(chunk)
        sim.steps(chunk, done)
        done += chunk
        err = _per_tree_rel(B.stress(), sim.sigma(), topo.tree_off)
        assert err <= 1e-9, (done, err)
    ev_g = _events(B.events(), [1, 2, 3, 4])
    ev_o = _events(sim.events(), [0, 1, 2, 3])
    assert np.array_equal(ev_g, ev_o)
    deg = _degree(topo)
    n_junc = int(np.sum(deg[ev_o[:, 2]] >= 3))
    _flush(f"  {ev_o.shape[0]} nucleations, {n_junc} at junctions, stress err {err:.2e}")
    assert ev_o.shape[0] >= 12 and n_junc >= 1
    iv, dv = B.voids()
    iv_o, dv_o = sim.voids()
    assert np.array_equal(iv, iv_o)
    assert np.allclose(dv, dv_o, rtol=1e-9, atol=0)
    B.close()


def test_combs_branch_kernel_matches_lane_kernel(em):
    g = synth.comb_trees(7002, n_trees=40)
    mat = material(sigma_crit=300e6)
    out = {}
    for stepper in (0, 1):
        rn = run(prec=0, screen=0, stepper=stepper)
        _flush(f"combs stepper {stepper}")
        B = em.Batch(g, mat, rn)
        B.stress_step(600)
        out[stepper] = (B.stress(), _events(B.events(), [1, 2, 3, 4]), B.voids())
        topo = B.topology()
        B.close()
    assert _per_tree_rel(out[0][0], out[1][0], topo["tree_off"]) <= 1e-11
    assert np.array_equal(out[0][1], out[1][1]) and out[0][1].shape[0] > 0
    assert np.array_equal(out[0][2][0], out[1][2][0])
    assert np.allclose(out[0][2][1], out[1][2][1], rtol=1e-10, atol=0)


def test_combs_monte_carlo_fp64_vs_oracle(em, oracle_mod):
    g = synth.comb_trees(7003, n_trees=6)
    mat = material(sigma_crit=300e6)
    rn = run(prec=0, screen=0)
    mc = dict(n_samples=5, seed=77, cov_kappa=0.2, cov_scrit=0.2)
    _flush("combs mc fp64")
    B = em.Batch(g, mat, rn, mc)
    B.stress_step(300)
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    ev = B.events()
    for s in range(5):
        xk, xs = oracle_mod.sample_xi(g, mc, s, rn["T_ambient"])
        sim = oracle_mod.SampleSim(g, mat, rn, topo, xk, xs)
        sim.set_j(g.seg_j)
        sim.steps(300)
        assert _per_tree_rel(B.stress(s), sim.sigma(), topo.tree_off) <= 1e-9, s
        mine = _events(ev[ev[:, 0] == s], [1, 2, 3, 4])
        assert np.array_equal(mine, _events(sim.events(), [0, 1, 2, 3])), s
    B.close()


def test_combs_fp32_vs_oracle(em, oracle_mod):
    # FP32 storage of stress, factors and dt*f; the solve itself in FP64
    g = synth.comb_trees(7004, n_trees=20)
    mat = material(sigma_crit=1e12)           # no nucleation: compare the transient itself
    rn = run(prec=1, screen=0)
    _flush("combs fp32")
    B = em.Batch(g, mat, rn)
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    sim = oracle_mod.SampleSim(g, mat, rn, topo)
    sim.set_j(g.seg_j)
    B.stress_step(500)
    sim.steps(500)
    err = _per_tree_rel(B.stress(), sim.sigma(), topo.tree_off)
    _flush(f"  fp32 stress err {err:.2e}")
    assert err <= 1e-5
    B.close()
