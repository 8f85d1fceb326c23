"""Monte Carlo over resistivity, current loading and activation energy
(Sec. IV-F sampled inputs) on the GPU against the FP64 oracle: the draws, the
per-sample initial IR solve, full runs to time-to-failure (FP64 and FP32),
and the Joule pre-pass still taking the nominal network's currents."""
import numpy as np
import pytest

import ttf_check

from paper_2604_10743_amd import synth

pytestmark = pytest.mark.gpu

VAR = dict(cov_rho=0.1, cov_load=0.15)


@pytest.fixture(scope="module")
def em():
    import torch
    assert torch.cuda.is_available()
    import paper_2604_10743_amd as P
    return P


def test_draws_and_initial_drops(em, oracle_mod):
    g, mat, rn, mc = synth.workload("mc_grid")
    mc = dict(mc, n_samples=70, **VAR)
    rn = dict(rn, prec=0, cg_rtol=1e-13)
    print("mc inputs: draws and t=0 drops", flush=True)
    B = em.Batch(g, mat, rn, mc)
    drops = B.ir_solve()
    for s in (0, 1, 63, 69):
        xi_r, R0, sinks = oracle_mod.sample_inputs(g, mc, s)
        assert np.allclose(B.xi(s, 2), xi_r, rtol=1e-14, atol=0)
        with np.errstate(invalid="ignore", divide="ignore"):
            ld = np.where(g.sink_I != 0, sinks / g.sink_I, 1.0)
        assert np.allclose(B.xi(s, 3), ld, rtol=1e-14, atol=0)
        gs = synth.Grid(**{**g.__dict__, "sink_I": sinks})
        u_o, _, j_o, d_o = oracle_mod.ir_solve(gs, R0)
        assert abs(drops[s] - d_o) <= 1e-9 * d_o, s
        assert np.max(np.abs(B.voltages(s) - u_o)) <= 1e-9 * g.vdd, s
        assert np.max(np.abs(B.seg_j(s) - j_o)) <= 1e-7 * np.max(np.abs(j_o)), s
    assert np.std(drops) > 1e-3 * np.mean(drops)             # samples differ from t = 0
    B.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_run_to_ttf_matches_oracle(em, oracle_mod, prec):
    g, mat, rn, mc = synth.workload("mc_grid")
    S = 32
    mc = dict(mc, n_samples=S, **VAR)
    rn = dict(rn, prec=prec)
    print(f"mc inputs: run prec {prec}", flush=True)
    B = em.Batch(g, mat, rn, mc)
    res = B.run_to_ttf()
    segs = {s: B.failed_segments(s) for s in range(0, S, 4)}
    B.close()
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    n_cmp = n_fail = 0
    for s in range(0, S, 4):
        ref = oracle_mod.run_sample(g, mat, rn, mc, s, topo=topo)
        r = res[s]
        n_cmp += 1
        n_fail += ref["failed"]
        ttf_check.check(r, ref, segs[s], prec, rn, s)
    assert n_cmp >= 6 and n_fail >= 1


def test_prepass_uses_nominal_currents(em):
    g, mat, rn, mc = synth.workload("mc_grid")
    mat = dict(mat, k_ild=0.1)
    rn = dict(rn, joule=1, prec=0)
    print("mc inputs: pre-pass field", flush=True)
    A = em.Batch(g, mat, rn, dict(mc, n_samples=3))
    B = em.Batch(g, mat, rn, dict(mc, n_samples=3, **VAR))
    assert np.array_equal(A.node_state(0)[0], B.node_state(2)[0])
    d_a, d_b = A.ir_solve(), B.ir_solve()
    assert np.all(d_a == d_a[0]) and np.std(d_b) > 0      # the varied batch still varies
    A.close()
    B.close()


def test_bad_variation_is_rejected(em):
    g, mat, rn, mc = synth.workload("mc_grid")
    for bad in (dict(cov_rho=-0.1), dict(cov_load=float("nan"))):
        with pytest.raises(em.EmError):
            em.Batch(g, mat, rn, dict(mc, n_samples=2, **bad))


def test_trees_only_resistivity_variation_matches_oracle(em, oracle_mod):
    # prescribed currents: the sampled resistivity scales each segment's
    # electron-wind drive, so the screen and the stress differ per sample
    g, mat, rn, _ = synth.workload("tiny_trees")
    rn = dict(rn, screen=1)
    mc = dict(n_samples=6, seed=17, cov_kappa=0.2, cov_scrit=0.2, cov_rho=0.15, cov_load=0.0)
    print("mc inputs: trees-only resistivity", flush=True)
    B = em.Batch(g, mat, rn, mc)
    tm = B.screen()                               # applied: immortal instances are not stepped
    B.stress_step(rn["n_steps"])
    ev = B.events()
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    n_diff = 0
    for s in range(6):
        ref = oracle_mod.run_sample(g, mat, rn, mc, s, topo=topo)
        assert np.array_equal(tm[s], ref["tree_mortal"]), s
        n_diff += int(not np.array_equal(tm[s], tm[0]))
        got = B.stress(s)
        for t in range(topo.n_trees):
            i0, i1 = topo.tree_off[t], topo.tree_off[t + 1]
            scale = np.max(np.abs(ref["sigma"][i0:i1])) or 1.0
            assert np.max(np.abs(got[i0:i1] - ref["sigma"][i0:i1])) <= 1e-9 * scale, (s, t)
        mine = ev[ev[:, 0] == s][:, [1, 2, 3]]
        mine = mine[np.lexsort(mine.T[::-1])]
        theirs = np.asarray(ref["events"])[:, [0, 1, 2]]
        theirs = theirs[np.lexsort(theirs.T[::-1])]
        assert np.array_equal(mine, theirs), s
    B.close()
    assert n_diff >= 1                            # the verdicts differ between samples


def test_activation_energy_draws_and_runs_match_oracle(em, oracle_mod):
    # dEa ~ N(0, 0.01 eV) per wire segment under the hotspot map
    g, mat, rn, mc = synth.workload("mc_grid")
    S = 24
    mc = dict(mc, n_samples=S, sd_ea_eV=0.01)
    rn = dict(rn, prec=0)
    print("mc inputs: activation energy", flush=True)
    B = em.Batch(g, mat, rn, mc)
    for s in (0, 5, 23):
        xk, xs = oracle_mod.sample_xi(g, mc, s, T_amb=rn["T_ambient"])
        assert np.allclose(B.xi(s, 0), xk, rtol=1e-13, atol=0), s
        assert np.allclose(B.xi(s, 1), xs, rtol=1e-13, atol=0), s
    res = B.run_to_ttf()
    segs = {s: B.failed_segments(s) for s in range(0, S, 3)}
    B.close()
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    n_fail = 0
    for s in range(0, S, 3):
        ref = oracle_mod.run_sample(g, mat, rn, mc, s, topo=topo)
        r = res[s]
        n_fail += ref["failed"]
        assert r["failed"] == ref["failed"], s
        assert abs(r["final_drop"] - ref["final_drop"]) <= 1e-6 * ref["final_drop"], s
        if ref["failed"]:
            assert abs(r["ttf_s"] - ref["ttf"]) <= 1e-6 * ref["ttf"], s
            assert r["outer_idx"] == ref["outer_idx"], s
        assert np.array_equal(segs[s], ref["failed_segs"]), s
    assert n_fail >= 1


def test_die_temperature_offset_draws_and_runs_match_oracle(em, oracle_mod):
    # one die-temperature offset dT ~ N(0, 3 K) per sample under the hotspot map
    g, mat, rn, mc = synth.workload("mc_grid")
    S = 24
    mc = dict(mc, n_samples=S, sd_T_K=3.0)
    rn = dict(rn, prec=0)
    print("mc inputs: die temperature", flush=True)
    B = em.Batch(g, mat, rn, mc)
    for s in (0, 5, 23):
        xk, xs = oracle_mod.sample_xi(g, mc, s, T_amb=rn["T_ambient"], Ea_eV=mat["Ea_eV"])
        assert np.allclose(B.xi(s, 0), xk, rtol=1e-13, atol=0), s
        assert np.allclose(B.xi(s, 1), xs, rtol=1e-13, atol=0), s
    res = B.run_to_ttf()
    segs = {s: B.failed_segments(s) for s in range(0, S, 3)}
    B.close()
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    n_fail = 0
    for s in range(0, S, 3):
        ref = oracle_mod.run_sample(g, mat, rn, mc, s, topo=topo)
        r = res[s]
        n_fail += ref["failed"]
        assert r["failed"] == ref["failed"], s
        assert abs(r["final_drop"] - ref["final_drop"]) <= 1e-6 * ref["final_drop"], s
        if ref["failed"]:
            assert abs(r["ttf_s"] - ref["ttf"]) <= 1e-6 * ref["ttf"], s
            assert r["outer_idx"] == ref["outer_idx"], s
        assert np.array_equal(segs[s], ref["failed_segs"]), s
    assert n_fail >= 1


@pytest.mark.parametrize("screen", [1, 0])
def test_map_amplitude_draws_and_runs_match_oracle(em, oracle_mod, screen):
    # one thermal-map amplitude a (unit-mean lognormal, CoV 0.3) per sample:
    # the diffusivity factors at the segments' midpoints and the scaled
    # thermomigration drive of every edge, with the screen on (a per-sample
    # steady stress) and off
    g, mat, rn, mc = synth.workload("mc_grid")
    S = 24
    mc = dict(mc, n_samples=S, cov_map=0.3)
    rn = dict(rn, prec=0, screen=screen)
    print(f"mc inputs: map amplitude, screen {screen}", flush=True)
    B = em.Batch(g, mat, rn, mc)
    for s in (0, 5, 23):
        xk, xs = oracle_mod.sample_xi(g, mc, s, T_amb=rn["T_ambient"], Ea_eV=mat["Ea_eV"])
        assert np.allclose(B.xi(s, 0), xk, rtol=1e-13, atol=0), s
    res = B.run_to_ttf()
    picks = range(0, S, 6) if screen else (0, 12)
    segs = {s: B.failed_segments(s) for s in picks}
    B.close()
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    n_fail = 0
    for s in picks:
        ref = oracle_mod.run_sample(g, mat, rn, mc, s, topo=topo)
        r = res[s]
        n_fail += ref["failed"]
        assert r["failed"] == ref["failed"], s
        assert abs(r["final_drop"] - ref["final_drop"]) <= 1e-6 * ref["final_drop"], s
        if ref["failed"]:
            assert abs(r["ttf_s"] - ref["ttf"]) <= 1e-6 * ref["ttf"], s
            assert r["outer_idx"] == ref["outer_idx"], s
        assert np.array_equal(segs[s], ref["failed_segs"]), s
    if screen:
        assert n_fail >= 1
