"""Pins of the learned-screen oracle (CPU only).

Each pin checks the oracle against something other than itself: bfloat16
rounding against hand-worked bit patterns and torch's own conversion, GELU
against the normal-distribution table and its odd-part identity, the backward
pass against central finite differences, Adam against its closed-form first
two steps, and the features against closed forms on a straight line and a
hand-measured branched tree.
"""
import math

import numpy as np
import pytest

from cases import UM, line_grid, material, run, tree_from_edges
from oracle import surrogate_oracle as SO
from paper_2604_10743_amd import synth


# ---------------------------------------------------------------- bfloat16
def test_bf16_hand_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20,
                  -2.5, 3.0e-3, 0.0])
    # spacing of bfloat16 at 1 is 2^-7: ties go to the even mantissa
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -2.5, None, 0.0], dtype=object)
    got = SO.bf16(x)
    for k in (0, 1, 2, 3, 4, 6):
        assert got[k] == want[k], (k, got[k], want[k])
    # 3e-3 = 1.536 x 2^-9 -> mantissa 1.5390625 (nearest of 1.53125, 1.5390625)
    assert got[5] == 1.5390625 * 2.0 ** -9


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        (1.0 + np.arange(256) * 2.0 ** -15)])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(SO.bf16(x), ref)


# ------------------------------------------------------------------- GELU
def test_gelu_table_values_and_identity():
    # GELU(1) = Phi(1); Phi(1) = 0.841344746068543 (standard normal table)
    assert abs(SO.gelu(1.0) - 0.841344746068543) < 1e-15
    assert SO.gelu(0.0) == 0.0
    z = np.linspace(-6, 6, 97)
    # z Phi(z) - (-z) Phi(-z) = z (Phi(z) + Phi(-z)) = z
    assert np.allclose(SO.gelu(z) - SO.gelu(-z), z, atol=1e-14, rtol=0)
    h = 1e-5
    fd = (SO.gelu(z + h) - SO.gelu(z - h)) / (2 * h)
    assert np.allclose(SO.gelu_grad(z), fd, atol=1e-9, rtol=0)


# --------------------------------------------------------- MLP gradients
def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = {}
    for name, shp in SO.SHAPES:
        fan_in = shp[1] if len(shp) == 2 else SO.HID
        P[name] = rng.standard_normal(shp) * scale / math.sqrt(fan_in)
    return SO.pack(P)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(11)
    p = _params(3)
    X = rng.standard_normal((6, SO.NF))
    t = rng.standard_normal(6)
    loss, g = SO.loss_and_grad(p, X, t, rnd=None)
    # a few coordinates in every parameter block
    offs, o = [], 0
    for name, shp in SO.SHAPES:
        n = int(np.prod(shp))
        offs += list(o + rng.choice(n, size=min(n, 6), replace=False))
        o += n
    h = 1e-6
    for k in offs:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        lp = SO.loss_and_grad(pp, X, t, rnd=None)[0]
        lm = SO.loss_and_grad(pm, X, t, rnd=None)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_rounded_forward_is_forward_of_rounded_operands():
    # with every hidden-layer operand already a bfloat16 value, rounding must
    # change nothing in the first layer's pre-activation
    rng = np.random.default_rng(2)
    p = SO.bf16(_params(4))
    X = SO.bf16(rng.standard_normal((5, SO.NF)))
    y_r, c_r = SO.forward(p, X)
    y_n, c_n = SO.forward(p, X, rnd=None)
    assert np.array_equal(c_r["Z1"], c_n["Z1"])
    assert np.max(np.abs(y_r - y_n)) < 0.05 * (1 + np.max(np.abs(y_n)))


# ------------------------------------------------------------------- Adam
def test_adam_first_two_steps_closed_form():
    rng = np.random.default_rng(9)
    p0 = rng.standard_normal(50)
    g1, g2 = rng.standard_normal(50), rng.standard_normal(50)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    m = v = np.zeros(50)
    p1, m, v = SO.adam_step(p0, g1, m, v, 1, lr, b1, b2, eps)
    # step 1: bias correction gives mhat = g, vhat = g^2
    assert np.allclose(p1, p0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    p2, m, v = SO.adam_step(p1, g2, m, v, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(p2, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)


# --------------------------------------------------------------- features
def _oracle_features(O, grid, mat, rn):
    topo = O.topology(grid, rn["intervals_per_seg"])
    sim = O.SampleSim(grid, mat, rn, topo)
    sim.set_j(grid.seg_j)
    _, _, ss = sim.screen()
    na = sim.node_arrays()
    xi = np.ones(grid.n_res)
    return SO.features(topo, grid, mat, grid.seg_j, xi, na["T"], ss, na["sc"]), topo


def test_features_straight_line_closed_forms(oracle_mod):
    # segments of 10 and 13 um carrying the same j: the steady profile is
    # linear, sigma_T at x = 11.5 um (volume mean = midpoint value), peak at
    # the low-voltage end x = 23 um; the nearest node at or below sigma_T is
    # the 20-interval node at x = 10 + 2 x 0.65 = 11.3 um, so Lpk = 11.7 um
    j, T = 4e10, 378.0
    g = tree_from_edges(3, [(0, 1), (1, 2)], np.array([10, 13]) * UM, 0.5 * UM, 0.2 * UM, j, T=T)
    mat = material(sigma_crit=60e6)
    rn = run()
    F, topo = _oracle_features(oracle_mod, g, mat, rn)
    f = F[0]
    Lt = 23 * UM
    k = 2.22409e-14                         # Arrhenius value at 378 K (golden file)
    Sd = SO.E_CHG * mat["Z"] * mat["rho_cu"] * j / mat["Omega"]
    smax = mat["sigma_T"] + Sd * Lt / 2
    r = smax / mat["sigma_crit"]
    assert abs(f[0] - math.log10(23.0)) < 1e-12
    assert abs(f[1] - math.log10(23.0)) < 1e-12
    assert f[2] == 2 / 8 and f[3] == 0.0
    assert abs(f[4] - math.log10(j / 1e9)) < 1e-12 and abs(f[5] - math.log10(j / 1e9)) < 1e-12
    assert abs(f[6] - math.log10(k / 1e-15)) < 3e-6 and abs(f[7] - f[6]) < 1e-12
    assert abs(f[8] - r) < 1e-9 * r
    assert abs(f[9] - math.log10(r - 1)) < 1e-9
    assert abs(f[10] - (math.log10((11.7 * UM) ** 2 / (math.pi ** 2 * k)) - 8)) < 3e-6
    assert abs(f[11] - (T - 300) / 100) < 1e-12
    # early-time scales: the steady drive is Sd on every edge, all edges are
    # fast (one temperature); blocked-end time pi ds^2 / (4 kappa Sd^2) with
    # ds = sigma_crit - sigma_T, the whole line blocked builds Sd Lt / 2
    ds = mat["sigma_crit"] - mat["sigma_T"]
    t_blk = math.pi * ds ** 2 / (4 * k * Sd ** 2)
    assert abs(f[12] - (math.log10(t_blk) - 8)) < 3e-6
    assert abs(f[13] - f[6]) < 1e-12
    assert abs(f[14] - Sd * Lt / 2 / ds) < 1e-9 * f[14]
    assert abs(f[15] - (math.log10(Lt ** 2 / (math.pi ** 2 * k)) - 8)) < 3e-6


def test_features_uniform_line_peak_end():
    # pure-numpy check of the peak/neutral-point rule on a prescribed profile
    class Topo:
        pass
    t = Topo()
    t.N, t.n_trees, t.n_stress = 4, 1, 5
    t.tree_off = np.array([0, 5]); t.parent = np.array([-1, 0, 1, 2, 3]); t.seg = np.array([-1, 0, 0, 0, 0])
    g = Topo()
    g.res_len = np.array([8 * UM])
    mat = material()
    ss = np.array([5.0, 3.0, 0.0, -3.0, -5.0]) * 1e7     # sigma_T = 0: neutral node 2
    F = SO.features(t, g, mat, np.array([1e10]), np.ones(1), np.full(5, 350.0), ss, np.full(5, 4e7))
    k = SO.kappa0(350.0, mat)
    assert abs(F[0, 8] - 1.25) < 1e-12
    assert abs(F[0, 10] - (math.log10((4 * UM) ** 2 / (math.pi ** 2 * k)) - 8)) < 1e-12
    assert abs(F[0, 11] - 0.5) < 1e-12
    # edges of 2 um with stress steps 2, 3, 3, 2 x 1e7 Pa: steepest drive
    # 1.5e13 Pa/m, blocked-end time pi (4e7)^2 / (4 k 1.5e13^2); the whole
    # line is fast and builds (2 + 3 + 3 + 2) x 1e7 / 2 = 5e7 Pa = 1.25 ds
    assert abs(F[0, 12] - (math.log10(math.pi * 4e7 ** 2 / (4 * k * 1.5e13 ** 2)) - 8)) < 1e-12
    assert abs(F[0, 13] - math.log10(k / 1e-15)) < 1e-12
    assert abs(F[0, 14] - 1.25) < 1e-12
    assert abs(F[0, 15] - (math.log10((8 * UM) ** 2 / (math.pi ** 2 * k)) - 8)) < 1e-12


def test_features_fast_region_of_a_hot_end():
    # the same profile with node temperatures 350, 350, 400, 400, 400 K: edge
    # midpoints at 350, 375, 400, 400 K, so only the last two edges are within
    # a factor 4 of the largest diffusivity (the Arrhenius ratio at 375 K is
    # about 0.2); they span 4 um and build (3 + 2) x 1e7 / 2 Pa
    class Topo:
        pass
    t = Topo()
    t.N, t.n_trees, t.n_stress = 4, 1, 5
    t.tree_off = np.array([0, 5]); t.parent = np.array([-1, 0, 1, 2, 3]); t.seg = np.array([-1, 0, 0, 0, 0])
    g = Topo()
    g.res_len = np.array([8 * UM])
    mat = material()
    ss = np.array([5.0, 3.0, 0.0, -3.0, -5.0]) * 1e7
    T = np.array([350.0, 350.0, 400.0, 400.0, 400.0])
    k375, k400, k350 = SO.kappa0(375.0, mat), SO.kappa0(400.0, mat), SO.kappa0(350.0, mat)
    assert k375 < 0.25 * k400
    F = SO.features(t, g, mat, np.array([1e10]), np.ones(1), T, ss, np.full(5, 4e7))
    assert abs(F[0, 13] - math.log10(k400 / 1e-15)) < 1e-12
    assert abs(F[0, 14] - 2.5e7 / 4e7) < 1e-12
    assert abs(F[0, 15] - (math.log10((4 * UM) ** 2 / (math.pi ** 2 * k400)) - 8)) < 1e-12
    # blocked-end time: least of pi ds^2 / (4 kappa_e g_e^2) over the edges
    tb = min(math.pi * 4e7 ** 2 / (4 * ke * ge ** 2)
             for ke, ge in ((k350, 1e13), (k375, 1.5e13), (k400, 1.5e13), (k400, 1e13)))
    assert abs(F[0, 12] - (math.log10(tb) - 8)) < 1e-12


def test_features_branched_tree_hand_measures(oracle_mod):
    # vertex 0 - 1 - 2 with a branch 1 - 3 and 3 - 4: segment lengths 10, 20, 5, 7 um
    edges = [(0, 1), (1, 2), (1, 3), (3, 4)]
    Ls = np.array([10, 20, 5, 7]) * UM
    js = np.array([1e10, -3e10, 2e9, 0.0])
    g = tree_from_edges(5, edges, Ls, 0.5 * UM, 0.2 * UM, js)
    F, topo = _oracle_features(oracle_mod, g, material(), run())
    assert topo.n_trees == 1
    f = F[0]
    assert abs(f[0] - math.log10(42.0)) < 1e-12
    assert abs(f[1] - math.log10(30.0)) < 1e-12          # root 0 -> vertex 2
    assert f[2] == 4 / 8 and f[3] == 1 / 4                # vertex 1 has degree 3
    assert abs(f[4] - math.log10(3e10 / 1e9)) < 1e-12
    jm = (10 * 1e10 + 20 * 3e10 + 5 * 2e9 + 0) / 42
    assert abs(f[5] - math.log10(jm / 1e9)) < 1e-12


# ------------------------------------------------------- lazy activation
def test_activation_interval_hand_values():
    K, dt, m = 100, 1.0, 2.0                 # margin x t_{k+1} = 200 (k + 1)
    th = np.array([1.0, 200.0, 200.0001, 400.0, 1e4])
    assert list(SO.activation_interval(th, m, K, dt)) == [0, 0, 1, 1, 49]


def test_activation_check_schedule():
    # checks before intervals 1, 4, 16, 64, ...; each covers up to the next
    a = np.array([1, 2, 3, 4, 7, 15, 16, 63, 64, 200])
    assert list(SO.activation_check(a)) == [1, 1, 1, 4, 4, 4, 16, 16, 64, 64]
    # a check never comes after the interval it is for, nor before a quarter of it
    a = np.arange(1, 300)
    c = SO.activation_check(a)
    assert np.all(c <= a) and np.all(4 * c > a) and np.all((c & (c - 1)) == 0)
    assert np.all(np.isin(c, [1, 4, 16, 64, 256]))


def test_grad_magnitude_bounds_gradient():
    # the magnitude sums bound every gradient entry, with equality where all
    # terms share a sign: a single row through a network with non-negative
    # weights and inputs has no cancellation in the output-layer gradients
    from oracle import surrogate_oracle as SO
    rng = np.random.default_rng(5)
    p = synth.init_mlp_params(11)
    X, t = rng.standard_normal((64, 16)), rng.standard_normal(64)
    _, g = SO.loss_and_grad(p, X, t)
    mg = SO.grad_magnitude(p, X, t)
    assert np.all(mg >= np.abs(g) - 1e-15 * np.abs(g).max())
    p1 = np.abs(p)
    X1, t1 = np.abs(X[:1]), np.array([-50.0])
    _, g1 = SO.loss_and_grad(p1, X1, t1)
    m1 = SO.grad_magnitude(p1, X1, t1)
    o = sum(int(np.prod(s)) for n, s in SO.SHAPES if n not in ("w4", "b4"))
    assert np.allclose(m1[o:], np.abs(g1[o:]), rtol=1e-12, atol=0)
