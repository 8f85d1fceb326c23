"""IR solve against the oracle's direct solve on a network built to exercise
the chain condensation: long chains between sparse vias, dangling chain ends,
a chain that leaves and re-enters one terminal through parallel vias, a ring
with no terminal, a pad-less island and a pad at a wire end, under per-sample
open and degraded resistors (em_set_seg_state)."""
import numpy as np
import pytest

from cases import UM, material
from paper_2604_10743_amd import synth
from paper_2604_10743_amd.synth import RHO_CU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def em():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_10743_amd as P
    return P


def _append(g, xy, layer, sink, res):
    """Append nodes (xy, layer, sink) and resistors (a, b, length, is_via)
    to grid g (node indices in res may refer to the new nodes)."""
    n0 = g.n_nodes
    g.xy = np.vstack([g.xy, np.asarray(xy, float)])
    g.layer = np.concatenate([g.layer, layer]).astype(np.int32)
    g.sink_I = np.concatenate([g.sink_I, sink])
    if g.node_T is not None:
        g.node_T = np.concatenate([g.node_T, np.full(len(layer), 330.0)])
    for a, b, L, via in res:
        w, h = (0.5 * UM, 0.2 * UM)
        g.res_a = np.append(g.res_a, a).astype(np.int32)
        g.res_b = np.append(g.res_b, b).astype(np.int32)
        g.res_len = np.append(g.res_len, 0.0 if via else L)
        g.res_w = np.append(g.res_w, w)
        g.res_h = np.append(g.res_h, h)
        g.res_is_via = np.append(g.res_is_via, 1 if via else 0).astype(np.uint8)
        g.res_R0 = np.append(g.res_R0, 0.5 if via else RHO_CU * L / (w * h))
    return n0


def _zoo():
    g = synth.pg_grid(11, n=24, via_every=8, pad_lattice=2, sink_scale=1.0, seg_range=(10, 23))
    i_sink = 2e-4
    # a chain from a grid node out through M1 node p and back to the same
    # grid node through two parallel vias to M2 node q: q -> p -> q
    t = int(np.nonzero(g.layer == 2)[0][5])
    x, y = g.xy[t]
    p = _append(g, [[x, y]], [1], [i_sink], [])
    _append(g, np.zeros((0, 2)), [], [], [(t, p, 0.0, True), (p, t, 0.0, True)])
    # a ring of four nodes with no pad and no terminal: M1 a-b, M2 c-d, vias
    r0 = _append(g, [[1 * UM, 1 * UM], [6 * UM, 1 * UM], [1 * UM, 1 * UM], [6 * UM, 1 * UM]], [1, 1, 2, 2],
                 [i_sink] * 4, [])
    _append(g, np.zeros((0, 2)), [], [], [(r0, r0 + 1, 5 * UM, False), (r0 + 2, r0 + 3, 5 * UM, False),
                                          (r0, r0 + 2, 0.0, True), (r0 + 1, r0 + 3, 0.0, True)])
    # a pad-less island: a two-node wire with a sink
    i0 = _append(g, [[2 * UM, 3 * UM], [9 * UM, 3 * UM]], [1, 1], [i_sink, 0.0], [])
    _append(g, np.zeros((0, 2)), [], [], [(i0, i0 + 1, 7 * UM, False)])
    # a pad at the end of a three-node M1 wire hanging from a grid M1 node
    m1 = int(np.nonzero(g.layer == 1)[0][40])
    x, y = g.xy[m1]
    w0 = _append(g, [[x, y + 2 * UM], [x, y + 4 * UM], [x, y + 6 * UM]], [1, 1, 1], [i_sink, i_sink, 0.0], [])
    _append(g, np.zeros((0, 2)), [], [], [(m1, w0, 2 * UM, False), (w0, w0 + 1, 2 * UM, False),
                                          (w0 + 1, w0 + 2, 2 * UM, False)])
    g.pad_node = np.append(g.pad_node, w0 + 2).astype(np.int32)
    return g


def _states(g, S, seed):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(S):
        dR = np.where(rng.random(g.n_res) < 0.2, rng.uniform(0.0, 3.0, g.n_res) * g.res_R0, 0.0)
        op = (rng.random(g.n_res) < (0.0 if s == 0 else 0.06)).astype(np.uint8)
        out.append((dR, op))
    return out


@pytest.mark.parametrize("precond,launch", [(0, 0), (1, 1), (1, 2), (1, 3), (2, 1), (2, 2), (2, 3)])
def test_condensed_network_with_opens_matches_direct_solve(em, oracle_mod, precond, launch):
    g = _zoo()
    S = 5
    print(f"ir zoo precond {precond} launch {launch}", flush=True)
    rn = synth.default_run(prec=0, T_ambient=330.0, cg_rtol=1e-14, cg_max_iter=200000,
                           ir_precond=precond, ir_launch=launch)
    B = em.Batch(g, material(), rn, dict(n_samples=S, seed=3, cov_kappa=0.2, cov_scrit=0.2))
    states = _states(g, S, 9)
    for s, (dR, op) in enumerate(states):
        B.set_seg_state(s, dR, op)
    drop = B.ir_solve()
    info = B.info()
    if precond == 2:
        assert info["ir_sys_nodes"] * 4 < g.n_nodes      # condensed
    else:
        assert info["ir_sys_nodes"] == g.n_nodes
    for s, (dR, op) in enumerate(states):
        u_o, I_o, j_o, d_o = oracle_mod.ir_solve(g, g.res_R0 + dR, op)
        u = B.voltages(s)
        assert np.max(np.abs(u - u_o)) <= 1e-10 * g.vdd, s
        assert abs(drop[s] - d_o) <= 1e-9 * max(d_o, 1e-3), s
        j = B.seg_j(s)
        assert np.max(np.abs(j - j_o)) <= 1e-6 * np.max(np.abs(j_o)), s
        # nodes without a conducting path to a pad (the ring, the island and
        # whatever the opens cut off) read 0 V
        dead = u_o == 0.0
        assert dead.sum() >= 6 and np.all(u[dead] == 0.0), s
    B.close()


def test_condensed_resolve_after_state_change(em, oracle_mod):
    # warm-started re-solves on the condensed system after the state changes
    g = _zoo()
    rn = synth.default_run(prec=0, T_ambient=330.0, cg_rtol=1e-14, cg_max_iter=200000)
    B = em.Batch(g, material(), rn)
    for k, (dR, op) in enumerate(_states(g, 3, 21)):
        B.set_seg_state(0, dR, op)
        d = B.ir_solve()[0]
        u_o, _, _, d_o = oracle_mod.ir_solve(g, g.res_R0 + dR, op)
        assert np.max(np.abs(B.voltages(0) - u_o)) <= 1e-10 * g.vdd, k
        assert abs(d - d_o) <= 1e-9 * max(d_o, 1e-3), k
    bad = np.zeros(g.n_res)
    bad[3] = -1.0
    with pytest.raises(em.EmError):
        B.set_seg_state(0, bad, np.zeros(g.n_res, np.uint8))
    B.close()


def test_single_pad_with_dangling_chains(em, oracle_mod):
    # one pad feeding open-ended wires: condensation would leave the pad
    # alone (no reduced edge), so the nodal system is solved; against the
    # direct solve and the ladder's closed form (node k sits below the pad by
    # R times the current still flowing past it)
    from cases import ladder_grid
    n, R = 40, 2.0
    sinks = np.linspace(1e-5, 5e-5, n)
    g = ladder_grid(n, R=R, sinks=sinks)
    print("ir single pad ladder", flush=True)
    B = em.Batch(g, material(), synth.default_run(prec=0, cg_rtol=1e-14, cg_max_iter=20000))
    drop = B.ir_solve()[0]
    u = B.voltages(0)
    info = B.info()
    B.close()
    assert info["ir_sys_nodes"] == g.n_nodes
    passing = np.cumsum(sinks[::-1])[::-1]                 # current through resistor k -> k+1
    u_cf = g.vdd - np.concatenate([[0.0], np.cumsum(R * passing)])
    u_o, _, _, d_o = oracle_mod.ir_solve(g, g.res_R0)
    assert np.max(np.abs(u_o - u_cf)) <= 1e-12
    assert np.max(np.abs(u - u_cf)) <= 1e-10 * g.vdd
    assert abs(drop - d_o) <= 1e-9 * d_o
