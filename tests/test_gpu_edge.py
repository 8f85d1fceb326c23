"""GPU edge cases against the oracle: ragged chain lengths around the lane
block and workgroup capacities (including chains too long for the resident
kernel), a zero-step run, nucleation disabled, a pad-less island in the IR
network, and argument errors."""
import math

import numpy as np
import pytest

from cases import UM, material, run, tree_from_edges
from paper_2604_10743_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def em():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_10743_amd as P
    return P


def _lines(seg_counts, L=5 * UM, j=3e10, T=378.0):
    """Independent straight lines with the given segment counts."""
    edges, xy, base = [], [], 0
    for t, S in enumerate(seg_counts):
        for k in range(S + 1):
            xy.append((k * L, t * 20 * UM))
        edges += [(base + k, base + k + 1) for k in range(S)]
        base += S + 1
    rng = np.random.default_rng(len(seg_counts))
    js = j * rng.uniform(0.5, 1.0, len(edges)) * np.where(rng.random(len(edges)) < 0.5, -1, 1)
    return tree_from_edges(base, edges, L, 0.5 * UM, 0.2 * UM, js, T=T, xy=np.array(xy))


def _per_tree_rel(a, b, off):
    w = 0.0
    for t in range(len(off) - 1):
        sl = slice(off[t], off[t + 1])
        w = max(w, np.max(np.abs(a[sl] - b[sl])) / max(np.max(np.abs(b[sl])), 1e-300))
    return w


@pytest.mark.parametrize("prec,N", [(0, 20), (0, 7), (0, 8), (1, 20), (1, 7)])
def test_ragged_chain_lengths(em, oracle_mod, prec, N):
    # node counts N*S + 1 straddle the 8-node lane block (N = 7, 8: 8 and 9
    # nodes per segment) and, with 205 and 410 segments at N = 20, the
    # capacity of the resident kernel's workgroup in FP64 (4096 nodes) and in
    # FP32 (8192): those chains take the generic tree kernel
    segs = [1, 2, 3, 205, 410] if N == 20 else [1, 2, 3, 9, 17]
    g = _lines(segs)
    mat = material(sigma_crit=1e12)
    rn = run(prec=prec, intervals_per_seg=N, dt=2e5, max_voids_per_tree=0)
    B = em.Batch(g, mat, rn)
    B.stress_step(60)
    topo = oracle_mod.topology(g, N)
    sim = oracle_mod.SampleSim(g, mat, dict(rn, prec=0), topo)
    sim.set_j(g.seg_j)
    sim.set_active(np.ones(topo.n_trees, np.uint8))
    sim.steps(60, 0)
    sg, so = B.stress(), sim.sigma()
    per = [_per_tree_rel(sg, so, topo.tree_off[t:t + 2]) for t in range(topo.n_trees)]
    nodes = np.diff(topo.tree_off)
    print(f"prec {prec} N {N}: nodes {nodes.tolist()}, errors {[f'{e:.1e}' for e in per]}")
    for n, e in zip(nodes, per):
        if prec == 0:
            assert e <= 1e-9
        else:
            # float factors: the error of each increment grows with the
            # conditioning of the step matrix of a long chain (~ its length
            # squared); measured 1.7e-7 (120 nodes), 8.2e-5 (4101 nodes,
            # resident kernel), 2.8e-4 (8201 nodes, generic kernel)
            assert e <= (1e-5 if n <= 1024 else 2e-4 if n <= 8192 else 5e-4), (n, e)


def test_zero_steps_and_no_nucleation(em):
    g, mat, rn, _ = synth.workload("tiny_mesh")
    B = em.Batch(g, mat, dict(rn, n_steps=0))
    r = B.run_to_ttf()[0]
    assert r["failed"] == 0 and math.isnan(r["ttf_s"]) and r["outer_idx"] == 0
    assert r["final_drop"] == r["init_drop"] and B.info()["node_steps"] == 0
    B.close()
    # a mortal workload with nucleation switched off records no event
    g = synth.two_layer_mesh(1001, nr=12, nc=12, sink_mu=math.log(490e-6), vdd=1.2, T_uniform=378.0)
    B = em.Batch(g, material(sigma_crit=150e6), run(prec=1, max_voids_per_tree=0))
    res = B.run_to_ttf()[0]
    assert B.info()["n_events"] == 0 and res["n_nucleated_trees"] == 0
    assert B.screen()[0].sum() > 0
    B.close()


def test_padless_island_reads_zero_volts(em, oracle_mod):
    # a 4x4 mesh plus a separate two-node wire with a sink and no pad: its
    # nodes have no path to a pad and read 0 V (worst drop 1)
    g = synth.two_layer_mesh(7, nr=4, nc=4, vdd=1.0, T_uniform=378.0)
    n0 = g.n_nodes
    g.xy = np.vstack([g.xy, [[1e-3, 1e-3], [1.01e-3, 1e-3]]])
    g.layer = np.concatenate([g.layer, [1, 1]]).astype(np.int32)
    g.res_a = np.concatenate([g.res_a, [n0]]).astype(np.int32)
    g.res_b = np.concatenate([g.res_b, [n0 + 1]]).astype(np.int32)
    for k, v in (("res_len", 10 * UM), ("res_w", 0.5 * UM), ("res_h", 0.2 * UM), ("res_R0", 1.0)):
        setattr(g, k, np.concatenate([getattr(g, k), [v]]))
    g.res_is_via = np.concatenate([g.res_is_via, [0]]).astype(np.uint8)
    g.sink_I = np.concatenate([g.sink_I, [1e-5, 0.0]])
    g.node_T = np.concatenate([g.node_T, [378.0, 378.0]])
    for pc in (0, 1, 2):
        B = em.Batch(g, material(), run(prec=0, ir_precond=pc, cg_rtol=1e-14, cg_max_iter=100000))
        drop = B.ir_solve()[0]
        u = B.voltages()
        u_o, _, _, d_o = oracle_mod.ir_solve(g, g.res_R0)
        assert u[n0] == 0.0 and u[n0 + 1] == 0.0
        assert drop == 1.0 and d_o == 1.0
        assert np.max(np.abs(u - u_o)) <= 1e-10
        B.close()


def test_argument_errors(em):
    g, mat, rn, _ = synth.workload("tiny_trees")
    bad = []
    bad.append((g, dict(mat, B=float("nan")), rn))
    bad.append((g, mat, dict(rn, dt=-1.0)))
    bad.append((g, mat, dict(rn, max_voids_per_tree=5)))
    bad.append((g, mat, dict(rn, ir_precond=3)))
    bad.append((g, mat, dict(rn, ir_launch=4)))
    bad.append((g, mat, dict(rn, intervals_per_seg=0)))
    for gg, mm, rr in bad:
        with pytest.raises(em.EmError) as ei:
            em.Batch(gg, mm, rr)
        assert ei.value.status == 1
    B = em.Batch(g, mat, rn)
    with pytest.raises(em.EmError):
        B.stress(5)                    # no such sample
    with pytest.raises(em.EmError) as ei:
        B.run_to_ttf()                 # trees-only batch has no IR coupling
    assert ei.value.status == 5
    B.close()


def _stressed():
    g = synth.two_layer_mesh(1001, nr=12, nc=12, sink_mu=math.log(490e-6), vdd=1.2, T_uniform=378.0)
    return g, material(sigma_crit=150e6)


@pytest.mark.parametrize("prec", [0, 1])
def test_snapshot_restore_continues_exactly(em, prec):
    g, mat = _stressed()
    rn = run(prec=prec)
    mc = dict(n_samples=3, seed=11, cov_kappa=0.2, cov_scrit=0.2)
    A = em.Batch(g, mat, rn, mc)
    A.ir_solve()
    A.stress_step(30)
    snap = A.snapshot()

    def cont(X):
        X.stress_step(40)
        X.ir_solve()
        X.stress_step(20)
        ev = X.events()
        ev = ev[np.lexsort(ev.T[::-1])]
        return ([X.stress(s) for s in range(3)], [X.voids(s) for s in range(3)],
                [X.seg_state(s) for s in range(3)], ev, X.info()["node_steps"])

    ra = cont(A)
    B = em.Batch(g, mat, rn, mc)
    B.restore(snap)
    rb = cont(B)
    assert len(ra[3]) > 0                      # voids appeared in the continued run
    for s in range(3):
        assert np.array_equal(ra[0][s], rb[0][s])
        assert np.array_equal(ra[1][s][0], rb[1][s][0]) and np.array_equal(ra[1][s][1], rb[1][s][1])
        assert np.array_equal(ra[2][s][0], rb[2][s][0]) and np.array_equal(ra[2][s][1], rb[2][s][1])
    assert np.array_equal(ra[3], rb[3]) and ra[4] == rb[4]
    # a snapshot belongs to a batch of the same shape
    C = em.Batch(*synth.workload("tiny_mesh")[:3])
    with pytest.raises(em.EmError):
        C.restore(snap)
    for X in (A, B, C):
        X.close()


def test_failed_segments_match_segment_state(em):
    g, mat = _stressed()
    B = em.Batch(g, mat, run(prec=0))
    r = B.run_to_ttf()[0]
    idx = B.failed_segments(0)
    dR, op = B.seg_state(0)
    want = np.nonzero((dR > 0) | (op != 0))[0]
    assert r["n_failed_segs"] > 0
    assert np.array_equal(idx, want) and len(idx) == r["n_failed_segs"]
    B.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_chain_workgroup_sizes_give_identical_results(em, prec):
    # instances never share a reduction, so the lanes per workgroup (how many
    # instances a workgroup holds, how many reduction levels it runs) change
    # no result bit.  The FP32 1024-lane form keeps no low part of the state
    # (no registers left for it): it agrees with the others to float rounding
    # of the state, with the same nucleation sites.
    g, mat, rn, _ = synth.workload("tiny_trees")
    mc = dict(n_samples=8, seed=5, cov_kappa=0.2, cov_scrit=0.2)
    # (lanes, register budget); the 128- and 168-VGPR forms run the same arithmetic
    sizes = (((256, 1), (512, 1), (256, 4), (512, 4), (256, 3), (512, 3), (64, 1), (128, 1), (64, 4), (128, 4),
              (1024, 1))
             if prec == 1 else ((256, 1), (512, 1), (64, 1), (128, 1)))
    out = []
    for w, occ in sizes:
        B = em.Batch(g, mat, dict(rn, prec=prec, chain_wg=w, chain_occ=occ), mc)
        B.stress_step(1000)
        ev = B.events()
        ev = ev[np.lexsort(ev.T[::-1])] if len(ev) else ev
        out.append(([B.stress(s) for s in range(8)], ev))
        B.close()
    assert len(out[0][1]) > 0
    n_exact = len(sizes) - 1 if prec == 1 else len(sizes)
    for st, ev in out[1:n_exact]:
        assert all(np.array_equal(a, b) for a, b in zip(st, out[0][0]))
        assert np.array_equal(ev, out[0][1])
    for st, ev in out[n_exact:]:
        for a, b in zip(st, out[0][0]):
            assert np.max(np.abs(a - b)) <= 1e-4 * np.max(np.abs(b))
        site = [0, 1, 3]                                   # sample, tree, node
        assert np.array_equal(np.unique(ev[:, site], axis=0), np.unique(out[0][1][:, site], axis=0))
        assert np.max(np.abs(ev[:, 2] - out[0][1][:, 2])) <= 20
    with pytest.raises(em.EmError):
        em.Batch(g, mat, dict(rn, prec=0, chain_wg=1024), mc)     # above the FP64 maximum
    for bad in (dict(prec=0, chain_wg=256, chain_occ=4), dict(prec=1, chain_wg=1024, chain_occ=4),
                dict(prec=1, chain_wg=256, chain_occ=2), dict(prec=1, chain_wg=128, chain_occ=3),
                dict(prec=0, chain_wg=256, chain_occ=3)):
        with pytest.raises(em.EmError):
            em.Batch(g, mat, dict(rn, **bad), mc)


def test_nine_node_blocks_match_oracle_and_pack(em, oracle_mod):
    # FP32 1024-lane chain kernel with 8- and 9-node lane blocks: chains of
    # 8201 nodes (912 lanes of 9 nodes; too long for 8-node blocks, which send
    # it to the generic kernel), 6001, 4601 (exactly 512 lanes) and short ones,
    # three samples each, against the FP64 oracle; the instances are packed
    # best-fit into no more workgroups than filling them in order would take
    segs = [410, 300, 230, 17, 3]
    g = _lines(segs)
    mat = material(sigma_crit=1e12)
    N = 20
    rn = run(prec=1, intervals_per_seg=N, dt=2e5, max_voids_per_tree=0)
    mc = dict(n_samples=3, seed=9, cov_kappa=0.2, cov_scrit=0.0)
    topo = oracle_mod.topology(g, N)
    nodes = np.diff(topo.tree_off)
    out = {}
    for m in (8, 9):
        print(f"chain_m {m}", flush=True)
        B = em.Batch(g, mat, dict(rn, chain_m=m), mc)
        B.stress_step(60)
        info = B.info()
        assert info["chain_m"] == m and info["chain_wg"] == 1024
        out[m] = [B.stress(s) for s in range(3)]
        B.close()
        lanes = [-(-int(n) // m) for n in nodes if -(-int(n) // m) <= 1024]
        nf, fill = 1, 0
        for L in sorted(lanes, reverse=True) * 3:
            if fill + L > 1024:
                nf, fill = nf + 1, 0
            fill += L
        assert -(-3 * sum(lanes) // 1024) <= info["n_chain_wg"] <= nf, (m, info["n_chain_wg"], nf)
    for s in range(3):
        xk, xs = oracle_mod.sample_xi(g, mc, s)
        sim = oracle_mod.SampleSim(g, mat, dict(rn, prec=0), topo, xk, xs)
        sim.set_j(g.seg_j)
        sim.set_active(np.ones(topo.n_trees, np.uint8))
        sim.steps(60, 0)
        so = sim.sigma()
        for m in (8, 9):
            per = [_per_tree_rel(out[m][s], so, topo.tree_off[t:t + 2]) for t in range(topo.n_trees)]
            print(f"sample {s} blocks {m}: errors {[f'{e:.1e}' for e in per]}", flush=True)
            for n, e in zip(nodes, per):
                # float state and factors: the error grows with the step
                # matrix's conditioning, about the chain length squared
                # (measured 8.2e-5 at 4101 nodes, 2.2e-4 at 6001)
                assert e <= max(1e-5, 1e-11 * float(n) ** 2), (m, s, n, e)
    for bad in (dict(chain_m=7), dict(chain_m=9, prec=0), dict(chain_m=9, chain_wg=512)):
        with pytest.raises(em.EmError):
            em.Batch(g, mat, dict(rn, **bad), mc)


def test_autotune_keeps_results_and_resets(em):
    g, mat, rn, mc = synth.workload("mc_grid")
    rn = dict(rn, prec=0)
    mc = dict(mc, n_samples=48)
    A = em.Batch(g, mat, rn, mc)
    ref = A.run_to_ttf()
    A.close()
    B = em.Batch(g, mat, rn, mc)
    t = B.autotune(20)
    print("autotune", t, flush=True)
    assert set(t["wg_ms"]) == {256, 512} and t["chain_wg"] in t["wg_ms"]      # FP64: up to 512 lanes
    assert t["ir_launch"] in (1, 2, 3) and t["ir_ms"][1] > 0 and t["ir_ms"][3] > 0 and t["ir_ms"][2] > 0
    assert t["amg_alpha"] in (1.4, 1.8, 2.2) and all(v > 0 for v in t["alpha_ms"].values())
    res = B.run_to_ttf()
    assert sum(r["failed"] for r in ref) > 0
    for a, b in zip(ref, res):
        assert a["failed"] == b["failed"] and a["n_failed_segs"] == b["n_failed_segs"]
        assert abs(a["final_drop"] - b["final_drop"]) <= 1e-9 * a["final_drop"]
        if a["failed"]:
            assert abs(a["ttf_s"] - b["ttf_s"]) <= 1e-8 * a["ttf_s"]
    B.stress_step(1)
    with pytest.raises(em.EmError):
        B.autotune(5)                      # not at t = 0
    B.close()
