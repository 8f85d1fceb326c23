"""Pins of the oracle's Joule-heating pre-pass (Sec. III-A, eqs. 2-4) against
the heat equation itself and textbook closed forms: the segment profile
solves k T'' + j^2 rho = k (T - T0)/Gamma^2 with its end values; the end
gradients are the profile's derivatives; a multi-segment line, solved through
the per-vertex flux balance, equals the single-wire solution over its whole
length (free end: cosh from the adiabatic end; both ends held: the sinh
form); a tree without vias sits at T0 + Tm everywhere; at a junction the heat
flux into its segments sums to zero."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import thermal as TH
from paper_2604_10743_amd.synth import Grid, RHO_CU, default_material

UM = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _mat(**over):
    m = default_material()
    m.update(over)
    return m


def _line(S, L, w, h, j, node_T, via_ends=(0,)):
    """Straight M1 line of S segments (nodes 0..S) with prescribed density j,
    and a via to an M2 node above each vertex listed in via_ends."""
    xy = [[k * L, 0.0] for k in range(S + 1)]
    layer = [1] * (S + 1)
    ra, rb = list(range(S)), list(range(1, S + 1))
    isv = [0] * S
    for v in via_ends:
        xy.append(list(xy[v]))
        layer.append(2)
        ra.append(v); rb.append(len(xy) - 1); isv.append(1)
    n_res = len(ra)
    nT = np.concatenate([node_T, np.full(len(xy) - S - 1, node_T[0])])
    lens = np.array([L] * S + [0.0] * (n_res - S))
    ww = np.full(n_res, w); hh = np.full(n_res, h)
    return Grid(xy=np.array(xy, float), layer=np.array(layer, np.int32),
                res_a=np.array(ra, np.int32), res_b=np.array(rb, np.int32), res_len=lens,
                res_w=ww, res_h=hh, res_is_via=np.array(isv, np.uint8),
                res_R0=np.where(lens > 0, RHO_CU * np.maximum(lens, 1e-12) / (ww * hh), 0.5),
                pad_node=np.zeros(0, np.int32), vdd=1.0, sink_I=np.zeros(len(xy)),
                node_T=nT, seg_j=np.concatenate([np.full(S, j), np.zeros(n_res - S)]))


def _stress_positions(grid, topo):
    """Distance of every stress node from node 0 along a straight line."""
    s = np.zeros(topo.n_stress)
    for i in range(topo.n_stress):
        if topo.vert[i] >= 0:
            s[i] = grid.xy[topo.vert[i], 0]
        else:
            e = topo.seg[i]
            s[i] = grid.xy[grid.res_a[e], 0] + topo.kpos[i] / topo.N * grid.res_len[e]
    return s


def test_profile_solves_heat_equation_and_meets_ends():
    mat = _mat()
    k = mat["k_cu"]
    for L, j, T0, T1, T2, t_cu in [(20 * UM, 5e10, 340.0, 352.0, 331.0, 0.2 * UM),
                                   (3 * UM, 2e11, 360.0, 360.0, 365.0, 0.4 * UM),
                                   (60 * UM, 1e10, 330.0, 338.0, 338.0, 0.2 * UM)]:
        G = TH.gamma(mat, t_cu)
        c = T0 + TH.joule_rise(mat, j, G)
        assert TH.profile(T1, T2, c, G, L, -L / 2) == pytest.approx(T1, abs=1e-10)
        assert TH.profile(T1, T2, c, G, L, L / 2) == pytest.approx(T2, abs=1e-10)
        dx = G * 1e-3       # truncation ~ T'''' dx^2 / 12, rounding ~ eps T / dx^2: both << scale
        x = np.linspace(-0.45 * L, 0.45 * L, 37)
        Tm_, T_, Tp_ = (TH.profile(T1, T2, c, G, L, x + s) for s in (-dx, 0.0, dx))
        d2 = (Tp_ - 2 * T_ + Tm_) / dx ** 2
        # k T'' + j^2 rho - k (T - T0)/Gamma^2 = 0
        resid = k * d2 + j * j * RHO_CU - k * (T_ - T0) / G ** 2
        scale = k * np.max(np.abs(T_ - T0)) / G ** 2 + j * j * RHO_CU
        assert np.max(np.abs(resid)) <= 1e-5 * scale


def test_gamma_hand_value():
    # eq. 2 with t_cu = t_ILD = 0.2 um, k_cu = 400, k_ILD = 1.4 W/(m K)
    assert TH.gamma(_mat(), 0.2 * UM) == pytest.approx(3.3806170189140663e-6, rel=1e-12)


def test_end_gradient_is_profile_derivative():
    mat = _mat()
    for L, c, T1, T2 in [(20 * UM, 345.0, 352.0, 331.0), (2 * UM, 340.5, 340.0, 341.0)]:
        G = TH.gamma(mat, 0.2 * UM)
        a_here, a_there, a0 = TH.end_gradient_coeffs(c, G, L)
        dx = L * 1e-5
        d_a = (TH.profile(T1, T2, c, G, L, -L / 2 + dx) - TH.profile(T1, T2, c, G, L, -L / 2 - dx)) / (2 * dx)
        d_b = (TH.profile(T1, T2, c, G, L, L / 2 + dx) - TH.profile(T1, T2, c, G, L, L / 2 - dx)) / (2 * dx)
        assert a_here * T1 + a_there * T2 + a0 == pytest.approx(d_a, rel=1e-6, abs=1e-3)
        assert a_here * T2 + a_there * T1 + a0 == pytest.approx(-d_b, rel=1e-6, abs=1e-3)


def test_line_with_free_end_is_single_wire_solution():
    mat = _mat()
    S, L, w, h, j = 7, 4 * UM, 0.5 * UM, 0.2 * UM, 8e10
    g = _line(S, L, w, h, j, np.full(S + 1, 350.0), via_ends=(0,))
    topo = O.topology(g, 20)
    T = TH.node_temperatures(g, mat, 300.0, topo, g.seg_j)
    G = TH.gamma(mat, h)
    c = 350.0 + TH.joule_rise(mat, j, G)
    s = _stress_positions(g, topo)
    Ltot = S * L
    # held at 350 K at s = 0 (via), adiabatic at s = Ltot
    exact = c + (350.0 - c) * np.cosh((Ltot - s) / G) / np.cosh(Ltot / G)
    assert np.max(np.abs(T - exact)) <= 1e-10 * 350.0
    assert T.max() - 350.0 > 0.8 * (c - 350.0)          # the free end heats up


def test_line_held_at_both_ends_is_single_wire_solution():
    mat = _mat()
    S, L, w, h, j = 5, 6 * UM, 1.0 * UM, 0.2 * UM, 6e10
    # alternating vertex values: every segment midpoint reads 350 K (uniform
    # T0), the two via ends read 340 K and 360 K
    nT = np.array([340.0 if k % 2 == 0 else 360.0 for k in range(S + 1)])
    g = _line(S, L, w, h, j, nT, via_ends=(0, S))
    topo = O.topology(g, 20)
    T = TH.node_temperatures(g, mat, 300.0, topo, g.seg_j)
    G = TH.gamma(mat, h)
    c = 350.0 + TH.joule_rise(mat, j, G)
    s = _stress_positions(g, topo)
    Ltot = S * L
    th1, th2 = 340.0 - c, 360.0 - c
    exact = c + (th1 * np.sinh((Ltot - s) / G) + th2 * np.sinh(s / G)) / np.sinh(Ltot / G)
    assert np.max(np.abs(T - exact)) <= 1e-10 * 350.0


def _star(j_arms, L_arms, w_arms, via_leaf=None):
    """Three M1 arms from hub node 0 to leaves 1..3 with their own length,
    width and density; optional via at one leaf."""
    xy = [[0.0, 0.0], [L_arms[0], 0.0], [-L_arms[1], 0.0], [0.0, L_arms[2]]]
    layer = [1, 1, 1, 1]
    ra, rb, isv = [0, 0, 0], [1, 2, 3], [0, 0, 0]
    lens = list(L_arms); ww = list(w_arms)
    if via_leaf is not None:
        xy.append(list(xy[via_leaf])); layer.append(2)
        ra.append(via_leaf); rb.append(4); isv.append(1); lens.append(0.0); ww.append(0.5 * UM)
    n = len(ra)
    hh = np.full(n, 0.2 * UM)
    lens = np.array(lens); ww = np.array(ww)
    return Grid(xy=np.array(xy, float), layer=np.array(layer, np.int32), res_a=np.array(ra, np.int32),
                res_b=np.array(rb, np.int32), res_len=lens, res_w=ww, res_h=hh,
                res_is_via=np.array(isv, np.uint8),
                res_R0=np.where(lens > 0, RHO_CU * np.maximum(lens, 1e-12) / (ww * hh), 0.5),
                pad_node=np.zeros(0, np.int32), vdd=1.0, sink_I=np.zeros(len(xy)),
                node_T=np.full(len(xy), 345.0), seg_j=np.concatenate([j_arms, np.zeros(n - 3)]))


def test_tree_without_via_sits_at_T0_plus_Tm():
    mat = _mat()
    g = _star(np.array([7e10, -7e10, 7e10]), [5 * UM, 9 * UM, 3 * UM], [0.5 * UM] * 3)
    topo = O.topology(g, 20)
    T = TH.node_temperatures(g, mat, 300.0, topo, g.seg_j)
    c = 345.0 + TH.joule_rise(mat, 7e10, TH.gamma(mat, 0.2 * UM))
    assert np.max(np.abs(T - c)) <= 1e-11 * c and c - 345.0 > 1.0


def test_junction_and_free_ends_balance_heat_flux():
    mat = _mat()
    g = _star(np.array([9e10, 3e10, -6e10]), [5 * UM, 9 * UM, 3 * UM], [0.5 * UM, 1.0 * UM, 0.3 * UM],
              via_leaf=2)
    topo = O.topology(g, 20)
    T = TH.node_temperatures(g, mat, 300.0, topo, g.seg_j)
    Tv = {int(topo.vert[i]): T[i] for i in range(topo.n_stress) if topo.vert[i] >= 0}
    assert Tv[2] == pytest.approx(345.0, abs=1e-12)            # the via leaf is held
    flux_hub, scale = 0.0, 0.0
    for e in range(3):
        L, w, h = g.res_len[e], g.res_w[e], g.res_h[e]
        G = TH.gamma(mat, h)
        c = 345.0 + TH.joule_rise(mat, g.seg_j[e], G)
        T1, T2 = Tv[int(g.res_a[e])], Tv[int(g.res_b[e])]
        dx = L * 1e-4
        # central differences of the profile (analytic past the ends)
        grad_in_a = (TH.profile(T1, T2, c, G, L, -L / 2 + dx) - TH.profile(T1, T2, c, G, L, -L / 2 - dx)) / (2 * dx)
        grad_b = (TH.profile(T1, T2, c, G, L, L / 2 + dx) - TH.profile(T1, T2, c, G, L, L / 2 - dx)) / (2 * dx)
        flux_hub += w * h * grad_in_a                          # every arm starts at the hub (res_a)
        scale += w * h * abs(grad_in_a)
        if int(g.res_b[e]) != 2:                               # free leaves are adiabatic
            assert abs(grad_b) <= 1e-6 * abs(grad_in_a)
    assert scale > 0 and abs(flux_hub) <= 1e-6 * scale
