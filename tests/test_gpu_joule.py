"""Joule-heating thermal pre-pass (Sec. III-A) on the GPU against the FP64
oracle: node temperatures after the pre-pass (P/G grid under a hotspot map,
via-free trees with prescribed currents, per-node temperature input), full
runs to time-to-failure with the pre-pass, the argument checks, and the
field's persistence across reset and snapshot/restore."""
import numpy as np
import pytest

import ttf_check

from cases import ladder_grid
from paper_2604_10743_amd import synth

pytestmark = pytest.mark.gpu

# a low-k dielectric (k_ILD 0.1 W/(m K)): Gamma = 12.6 um, so that the Joule
# rise of the synthetic grids' current densities reaches about a kelvin
LOWK = dict(k_ild=0.1)


@pytest.fixture(scope="module")
def em():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_10743_amd as P
    return P


@pytest.fixture(scope="module")
def thermal_mod():
    from oracle import thermal
    return thermal


def _oracle_T(oracle_mod, thermal_mod, g, mat, rn):
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    if g.seg_j is not None:
        j = g.seg_j
    else:
        _, _, j, _ = oracle_mod.ir_solve(g, g.res_R0.astype(np.float64))
    return thermal_mod.node_temperatures(g, mat, rn["T_ambient"], topo, j), j


def test_pg_grid_hotspot_map_node_temperatures(em, oracle_mod, thermal_mod):
    g, mat, rn, mc = synth.workload("mc_grid")
    mat = dict(mat, **LOWK)
    rn = dict(rn, joule=1, prec=0)
    print("joule: mc_grid node temperatures", flush=True)
    B = em.Batch(g, mat, rn, dict(mc, n_samples=4))
    T_gpu = B.node_state(0)[0]
    T3 = B.node_state(3)[0]
    B.close()
    T_o, j = _oracle_T(oracle_mod, thermal_mod, g, mat, rn)
    assert np.array_equal(T_gpu, T3)                        # one field for the batch
    assert np.max(np.abs(T_gpu - T_o)) <= 1e-8
    # the pre-pass changed the field: Joule rise and the free line ends
    A = em.Batch(g, mat, dict(rn, joule=0), dict(mc, n_samples=1))
    T_map = A.node_state(0)[0]
    A.close()
    print("max pre-pass rise over the map", float(np.max(T_gpu - T_map)), flush=True)
    assert np.max(T_gpu - T_map) > 0.3


def test_trees_only_and_node_temperature_input(em, oracle_mod, thermal_mod):
    # via-free straight trees with prescribed densities: every vertex free
    g, mat, rn, _ = synth.workload("tiny_trees")
    mat = dict(mat, **LOWK)
    rn = dict(rn, joule=1)
    print("joule: tiny_trees", flush=True)
    B = em.Batch(g, mat, rn)
    T_gpu = B.node_state(0)[0]
    B.close()
    T_o, _ = _oracle_T(oracle_mod, thermal_mod, g, mat, rn)
    assert np.max(np.abs(T_gpu - T_o)) <= 1e-8 and np.max(T_o) - rn["T_ambient"] > 1.0
    # per-node temperature input on a loaded chain from a pad (coupled mode,
    # no vias: every vertex free, T0 from the node values)
    gl = ladder_grid(40, sinks=np.full(40, 4e-5))
    gl.node_T = np.linspace(340.0, 372.0, gl.n_nodes)
    rl = synth.default_run(joule=1, T_ambient=300.0)
    print("joule: loaded line with node_T", flush=True)
    B = em.Batch(gl, mat, rl)
    T_gpu = B.node_state(0)[0]
    B.close()
    T_o, _ = _oracle_T(oracle_mod, thermal_mod, gl, mat, rl)
    assert np.max(np.abs(T_gpu - T_o)) <= 1e-8


@pytest.mark.parametrize("prec", [0, 1])
def test_run_to_ttf_with_prepass_matches_oracle(em, oracle_mod, prec):
    g, mat, rn, mc = synth.workload("mc_grid")
    mat = dict(mat, **LOWK)
    rn = dict(rn, joule=1, prec=prec)
    S = 16
    mc = dict(mc, n_samples=S)
    print(f"joule: mc_grid run prec {prec}", flush=True)
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


def test_bad_thermal_block_is_rejected(em):
    g, mat, rn, _ = synth.workload("tiny_trees")
    for bad in (dict(k_cu=0.0), dict(k_ild=-1.0), dict(t_ild=float("nan"))):
        with pytest.raises(em.EmError):
            em.Batch(g, dict(mat, **bad), dict(rn, joule=1))
    em.Batch(g, dict(mat, k_cu=0.0), dict(rn, joule=0)).close()   # not read without the pre-pass
    with pytest.raises(em.EmError):
        em.Batch(g, mat, dict(rn, joule=2))


def test_field_survives_reset_and_restore(em):
    g, mat, rn, mc = synth.workload("mc_grid")
    mat = dict(mat, **LOWK)
    rn = dict(rn, joule=1, prec=0)
    mc = dict(mc, n_samples=2)
    print("joule: reset and restore", flush=True)
    A = em.Batch(g, mat, rn, mc)
    T0 = A.node_state(0)[0]
    A.ir_solve()
    A.stress_step(300)
    snap = A.snapshot()
    A.reset()
    assert np.array_equal(A.node_state(0)[0], T0)
    A.restore(snap)
    A.stress_step(200)
    ref = [A.stress(s) for s in range(2)]
    B = em.Batch(g, mat, rn, mc)
    assert np.array_equal(B.node_state(1)[0], T0)
    B.restore(snap)
    B.stress_step(200)
    for s in range(2):
        assert np.array_equal(B.stress(s), ref[s])
    A.close()
    B.close()
