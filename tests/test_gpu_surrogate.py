"""GPU parity of the learned screen against the CPU oracle: BF16 MFMA MLP
forward and backward, the Adam kernel, the feature kernel, nucleation-time
labels, and the exactness of lazy activation with catch-up replay."""
import math

import numpy as np
import pytest

from cases import UM, material, run
from paper_2604_10743_amd import synth

pytestmark = pytest.mark.gpu

# Tolerances.  Both sides form exact products of the same bfloat16 operands;
# they differ by float32 vs float64 accumulation (relative 256 x 2^-24 ~ 1.5e-5
# of the absolute sum per hidden unit, worst case) and, through that, by the
# rare operand that lands on the other side of a bfloat16 rounding boundary
# in the next layer (a change of 2^-8 of that one operand).  With unit-scale
# activations and He-scaled weights the output moves by at most ~2^-8 x |w4|
# x (a few flipped units); 2e-3 x (1 + |y|) bounds that with margin.
Y_TOL = 2e-3
G_TOL = 2e-2          # relative 2-norm error per parameter block
# Element-wise gradient bound.  Each gradient entry is a sum of products whose
# operands both sides round at the same points; they differ by float32 vs
# float64 accumulation (relative <= n 2^-24 ~ 2e-5 of the sum of |terms| for
# n = 300 rows) and by operands that round to the neighbouring bfloat16 value
# (2^-8 relative of that operand) because their float32 value moved across a
# rounding boundary -- in the entry's own sum or upstream, where the moved
# signal is itself bounded by the magnitude sums.  A few such flips per entry
# stay below 2^-6 of the entry's magnitude sum (oracle grad_magnitude), plus
# an absolute floor of 1e-6 of the largest gradient for entries whose terms
# all vanish.
G_ELEM = 2.0 ** -6


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2604_10743_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def SO():
    from oracle import surrogate_oracle as SO
    return SO


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 16)).astype(np.float32), rng.standard_normal(n).astype(np.float32)


@pytest.mark.parametrize("n", [1, 64, 300])
def test_mlp_forward_matches_oracle(P, SO, n):
    p = synth.init_mlp_params(7, out_bias=0.3)
    X, _ = _inputs(n, 1)
    m = P.MLP(p)
    y = m.forward(X).cpu().numpy().astype(np.float64)
    yo, _ = SO.forward(p.astype(np.float64), X.astype(np.float64))
    err = np.abs(y - yo)
    print(f"forward n={n}: max |dy| = {err.max():.3e}, max |y| = {np.abs(yo).max():.3f}")
    assert np.all(err <= Y_TOL * (1 + np.abs(yo)))
    m.close()


def test_mlp_grad_matches_oracle(P, SO):
    p = synth.init_mlp_params(8)
    X, t = _inputs(300, 2)
    m = P.MLP(p)
    loss, g = m.grad(X, t)
    lo, go = SO.loss_and_grad(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert abs(loss - lo) <= 1e-3 * lo
    mag = SO.grad_magnitude(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    floor = 1e-6 * np.max(np.abs(go))
    o = 0
    for name, shp in SO.SHAPES:
        k = int(np.prod(shp))
        a, b, mg = g[o:o + k].astype(np.float64), go[o:o + k], mag[o:o + k]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        ratio = np.abs(a - b) / (mg + floor)
        print(f"grad {name}: rel 2-norm err {rel:.2e}, max |dg| / magnitude {ratio.max():.2e}, "
              f"median |g| / magnitude {np.median(np.abs(b) / (mg + floor)):.2e}")
        assert rel <= G_TOL, name
        bad = np.nonzero(np.abs(a - b) > G_ELEM * mg + floor)[0]
        assert bad.size == 0, (name, bad[:8], a[bad[:8]], b[bad[:8]])
        o += k
    m.close()


def test_adam_kernel_matches_oracle_step(P, SO):
    import torch
    p0 = synth.init_mlp_params(9)
    X, t = _inputs(256, 3)
    m = P.MLP(p0)
    _, g = m.grad(X, t)                       # the gradient the step will use
    lr = 1e-3
    m.train_step(torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda"), lr)
    p1 = m.params().astype(np.float64)
    z = np.zeros_like(p1)
    pe, _, _ = SO.adam_step(p0.astype(np.float64), g.astype(np.float64), z, z, 1, lr)
    # float32 update of size <= lr on unit-scale parameters
    assert np.max(np.abs(p1 - pe)) <= 1e-6 + 1e-6 * np.max(np.abs(pe))
    m.close()


def test_training_reduces_loss(P):
    import torch
    rng = np.random.default_rng(4)
    X = rng.standard_normal((8192, 16)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 3] ** 2).astype(np.float32)
    Xd, td = torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda")
    m = P.MLP(synth.init_mlp_params(10))
    l0, _ = m.grad(X, t)
    from paper_2604_10743_amd import surrogate
    surrogate.train(m, Xd, td, steps=240, batch=1024, lr=1e-3)
    l1, _ = m.grad(X, t)
    print(f"training loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.05 * l0
    m.close()


def test_mlp_rejects_bad_arguments(P):
    m = P.MLP()
    with pytest.raises(P.EmError):
        m.set_params(np.zeros(10, np.float32))
    bad = synth.init_mlp_params(1)
    bad[5] = np.nan
    with pytest.raises(P.EmError):
        m.set_params(bad)
    m.close()


# ------------------------------------------------------------------ features
def _feature_grid():
    a = synth.straight_trees(41, n_trees=12)
    b = synth.random_branched_trees(42, n_trees=10, n_vertices=(3, 9))
    return a, b


@pytest.mark.parametrize("which", [0, 1])
def test_features_match_oracle(P, SO, oracle_mod, which):
    O = oracle_mod
    g = _feature_grid()[which]
    mat = material(sigma_crit=100e6)
    rn = run(prec=0)
    mc = dict(n_samples=3, seed=77, cov_kappa=0.2, cov_scrit=0.2)
    B = P.Batch(g, mat, rn, mc)
    X = B.features().cpu().numpy().reshape(B.n_trees, 3, 16)
    topo = O.topology(g, rn["intervals_per_seg"])
    for s in range(3):
        xk, xs = O.sample_xi(g, mc, s)
        sim = O.SampleSim(g, mat, rn, topo, xk, xs)
        sim.set_j(g.seg_j)
        _, _, ss = sim.screen()
        na = sim.node_arrays()
        F = SO.features(topo, g, mat, g.seg_j, xk, na["T"], ss, na["sc"])
        err = np.abs(X[:, s, :] - F)
        assert np.all(err <= 2e-6 * (1 + np.abs(F))), (s, np.unravel_index(err.argmax(), err.shape))
    B.close()


def test_first_nucleation_labels_match_oracle(P, oracle_mod):
    O = oracle_mod
    g = synth.straight_trees(43, n_trees=16, j_range=(2e10, 6e10))
    mat = material(sigma_crit=120e6)
    rn = run(prec=0, max_voids_per_tree=1)
    B = P.Batch(g, mat, rn)
    B.screen()
    B.stress_step(400)
    first = B.first_nucleation()[0]
    topo = O.topology(g, rn["intervals_per_seg"])
    sim = O.SampleSim(g, mat, rn, topo)
    sim.set_j(g.seg_j)
    tm, _, _ = sim.screen()
    sim.set_active(tm)
    sim.steps(400, 0)
    ev = sim.events()
    want = np.full(topo.n_trees, -1)
    for t, st, _, _ in ev:
        if want[t] < 0:
            want[t] = st
    assert (want >= 0).sum() >= 3
    assert np.array_equal(first, want)
    B.close()


# ---------------------------------------------------- lazy activation replay
def _coupled():
    g = synth.two_layer_mesh(1001, nr=12, nc=12, sink_mu=math.log(490e-6), vdd=1.2, T_uniform=378)
    return g, material(sigma_crit=150e6)


def _const_model(P, y):
    p = np.zeros(synth.init_mlp_params(0).size, np.float32)
    p[-1] = y
    return P.MLP(p)


def _result_key(B, res):
    ev = B.events()
    ev = ev[np.lexsort(ev.T[::-1])] if len(ev) else ev
    def nn(x):
        return None if math.isnan(x) else x
    return ([(r["failed"], nn(r["ttf_s"]), r["final_drop"], r["outer_idx"], r["n_nucleated_trees"],
              r["n_failed_segs"]) for r in res], ev.tolist())


@pytest.mark.parametrize("prec", [1, 0])
def test_lazy_activation_replay_is_exact(P, prec):
    # sparse-via grid at 330 K with 4 Monte Carlo samples: its first
    # nucleation falls after the first aging interval
    g, mat, _, mc = synth.workload("screen_mc")
    g = synth.sparse_via_grid(2103)
    mc = dict(mc, n_samples=4)
    rn = run(prec=prec, T_ambient=330.0)
    K, dt, m = rn["ir_every"], rn["dt"], 2.0
    B = P.Batch(g, mat, rn, mc)
    ref = B.run_to_ttf()
    key_ref = _result_key(B, ref)
    ns_ref = B.info()["node_steps"]
    ev = B.events()
    assert len(ev) > 0
    k_first = int(ev[:, 2].min()) // K            # interval of the first nucleation
    assert k_first >= 1, "workload nucleates in the first interval; replay untested"
    # every mortal tree predicted due in interval k_first: deferred at t = 0,
    # activated at the check at or before k_first and caught up before any nucleation
    th = m * (k_first + 0.5) * K * dt
    mdl = _const_model(P, math.log10(th / 1e8))
    B.reset()
    B.surrogate_screen(mdl, m)
    res = B.run_to_ttf()
    inf = B.info()
    print(f"prec {prec}: first nucleation interval {k_first}, deferred {inf['n_deferred']}, "
          f"activated {inf['n_activated']}, violations {inf['n_violations']}")
    assert inf["n_deferred"] > 0 and inf["n_activated"] == inf["n_deferred"]
    assert inf["n_late"] == 0 and inf["n_violations"] == 0
    assert _result_key(B, res) == key_ref
    assert inf["node_steps"] == ns_ref
    # activating after the first nucleation is a measured late activation: a
    # tree due at the first check after k_first is activated there
    k_late = 1
    while k_late <= k_first:
        k_late *= 4
    th2 = m * (k_late + 0.5) * K * dt
    mdl2 = _const_model(P, math.log10(th2 / 1e8))
    B.reset()
    B.surrogate_screen(mdl2, m)
    B.run_to_ttf()
    assert B.info()["n_late"] >= 1
    B.surrogate_screen(None)
    B.close()
    mdl.close()
    mdl2.close()


def test_never_due_trees_are_skipped_and_margin_checked(P):
    g, mat = _coupled()
    rn = run(prec=1)
    B = P.Batch(g, mat, rn)
    mdl = _const_model(P, 6.0)                    # 1e14 s: never due within the horizon
    with pytest.raises(P.EmError):
        B.surrogate_screen(mdl, 0.5)
    B.surrogate_screen(mdl, 2.0)
    res = B.run_to_ttf()
    inf = B.info()
    assert inf["n_deferred"] > 0 and inf["n_activated"] == 0
    assert inf["node_steps"] == 0                 # every mortal tree deferred, none stepped
    assert all(r["n_nucleated_trees"] == 0 for r in res)
    y, df = B.surrogate(0)
    assert np.all(np.abs(y - 6.0) < 1e-6) and df.sum() == inf["n_deferred"]
    B.close()
    mdl.close()


# ------------------------------------------------------ gain of a trained screen
def test_trained_screen_saves_steps_with_identical_results(P):
    # a model trained on ~480k labelled pairs of 24 random cold long-line
    # grids (fewer grids do not generalise to held-out ones), calibrated on
    # held-out grids, screening the cold long-line workload: the screened run
    # steps fewer nodes and fails every sample at the same TTF
    import torch
    from paper_2604_10743_amd import surrogate
    g, mat, rn, mc = synth.workload("screen_cold")
    mc = dict(mc, n_samples=64)
    lab = dict(rn, dt=rn["dt"] * 2.5)
    horizon = 4 * rn["n_steps"]
    X, y, _ = surrogate.training_set(11, 24, mat, lab, 1024, horizon, family="cold_lines")
    Xv, yv, _ = surrogate.training_set(12, 4, mat, lab, 256, horizon, family="cold_lines")
    assert X.shape[0] >= 200_000
    mdl = P.MLP(synth.init_mlp_params(1, out_bias=float(y.mean().item())))
    surrogate.train(mdl, X, y, 3000, batch=4096, lr=1e-3, lr_final=1e-4)
    surrogate.calibrate(mdl, Xv, yv, 0.98, y_cap=surrogate.label_cap(lab, horizon))
    B = P.Batch(g, mat, rn, mc)
    ref = B.run_to_ttf()
    ns_ref = B.info()["node_steps"]
    B.reset()
    B.surrogate_screen(mdl, 1.0)
    res = B.run_to_ttf()
    inf = B.info()
    B.close()
    mdl.close()
    torch.cuda.synchronize()
    print(f"node-steps {ns_ref} -> {inf['node_steps']}, deferred {inf['n_deferred']}, "
          f"activated {inf['n_activated']}, late {inf['n_late']}, violations {inf['n_violations']}, "
          f"re-run {inf['n_screen_rerun']}")

    def key(r):
        return (r["failed"], None if math.isnan(r["ttf_s"]) else r["ttf_s"], r["final_drop"],
                r["outer_idx"], r["n_failed_segs"])
    assert [key(r) for r in res] == [key(r) for r in ref]
    assert sum(r["failed"] for r in ref) >= len(ref) // 2
    # a violation's samples were re-run without the screen (their steps counted)
    rerun = [s for s, r in enumerate(res) if r["redecided"] == 2]
    assert len(rerun) == inf["n_screen_rerun"] and (inf["n_violations"] == 0) == (not rerun)
    assert inf["n_deferred"] > inf["n_activated"]
    assert inf["node_steps"] <= 0.85 * ns_ref
