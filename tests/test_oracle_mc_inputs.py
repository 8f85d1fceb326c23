"""Pins of the oracle's further Monte Carlo inputs (Sec. IV-F: resistivity
and current loading stamped into each sample's network): the draws' unit
mean and CoV, vias keep their resistance, the electron-wind drive and hence
the steady stress scale exactly with a segment's resistivity, the liner
formula's copper term takes the sampled resistivity, and a sample's pads
deliver exactly its own (scaled) sink currents."""
import math

import numpy as np
import pytest

from cases import material, run, tree_from_edges
from paper_2604_10743_amd import synth

UM = 1e-6


def test_param2_and_param3_draw_statistics(oracle_mod):
    for param in (2, 3):
        xi = oracle_mod.lognormal_xi(777, 5, 200000, param, 0.1)
        assert abs(xi.mean() - 1.0) < 4 * 0.1 / math.sqrt(xi.size)
        assert abs(xi.std() / xi.mean() - 0.1) < 0.002
        assert not np.allclose(xi[:100], oracle_mod.lognormal_xi(777, 5, 100, 0, 0.1))


def test_sampled_network_keeps_vias_and_scales_wires(oracle_mod):
    g = synth.pg_grid(11, n=24, via_every=8, pad_lattice=2, sink_scale=1.0, seg_range=(10, 23))
    mc = dict(seed=3, cov_kappa=0.2, cov_scrit=0.2, cov_rho=0.15, cov_load=0.1)
    xi_r, R0, sinks = oracle_mod.sample_inputs(g, mc, 4)
    wire = (g.res_is_via == 0) & (g.layer[g.res_a] == g.layer[g.res_b])
    assert np.all(xi_r[~wire] == 1.0) and np.all(R0[~wire] == g.res_R0[~wire])
    assert np.allclose(R0[wire] / g.res_R0[wire], xi_r[wire], rtol=1e-15)
    assert np.std(xi_r[wire]) > 0.05
    load = sinks[g.sink_I > 0] / g.sink_I[g.sink_I > 0]
    assert abs(np.std(load) / np.mean(load) - 0.1) < 0.03
    # the sample's pads deliver its own sink total (KCL on the sampled network)
    gs = synth.Grid(**{**g.__dict__, "sink_I": sinks})
    u, I, j, drop = oracle_mod.ir_solve(gs, R0)
    pads = set(int(p) for p in g.pad_node)
    pad_current = sum(I[r] * ((g.res_a[r] in pads) - (g.res_b[r] in pads)) for r in range(g.n_res))
    assert abs(pad_current - sinks.sum()) < 1e-10 * sinks.sum()
    # without the CoVs the sampled network is the nominal one
    xi0, R00, s00 = oracle_mod.sample_inputs(g, dict(mc, cov_rho=0.0, cov_load=0.0), 4)
    assert xi0 is None and np.array_equal(R00, g.res_R0) and np.array_equal(s00, g.sink_I)


def test_steady_stress_scales_with_segment_resistivity(oracle_mod):
    # uniform temperature (no thermomigration): sigma_ss - sigma_T is a sum
    # of dx * eZ rho xi_e j_e / Omega along the tree, so per-segment
    # multipliers act segment by segment; all equal to c scale it by c
    edges = [(0, 1), (1, 2), (1, 3), (3, 4)]
    g = tree_from_edges(5, edges, L=[10 * UM, 20 * UM, 15 * UM, 5 * UM], w=0.4 * UM, h=0.2 * UM,
                        j=[2e10, -1e10, 3e10, 1e10], T=378.0)
    N = 10
    topo = oracle_mod.topology(g, N)
    rn = run(intervals_per_seg=N)

    def sigma_ss(xi_r):
        sim = oracle_mod.SampleSim(g, material(), rn, topo, xi_r=xi_r)
        sim.set_j(g.seg_j)
        return sim.screen()[2]

    base = sigma_ss(None)
    assert np.max(np.abs(sigma_ss(np.full(g.n_res, 1.7)) - 1.7 * base)) <= 1e-12 * np.max(np.abs(base))
    # one segment's multiplier equals multiplying that segment's current density
    xi = np.ones(g.n_res); xi[2] = 1.3
    g2 = tree_from_edges(5, edges, L=[10 * UM, 20 * UM, 15 * UM, 5 * UM], w=0.4 * UM, h=0.2 * UM,
                         j=[2e10, -1e10, 3e10 * 1.3, 1e10], T=378.0)
    sim = oracle_mod.SampleSim(g2, material(), rn, topo)
    sim.set_j(g2.seg_j)
    assert np.max(np.abs(sigma_ss(xi) - sim.screen()[2])) <= 1e-12 * np.max(np.abs(base))


def test_liner_formula_takes_sampled_resistivity(oracle_mod):
    # eq. 17 with V_v - V_crit = (l - W) W H; copper term with rho_Cu xi
    import ctypes as C
    L = oracle_mod.lib()
    f = L.ora_late_dR
    f.restype = C.c_double
    f.argtypes = [C.c_double] * 6
    l, W, H, h_ta, rho_ta, rho = 3e-6, 0.5e-6, 0.2e-6, 5e-9, 2e-7, 2.25e-8
    for xi in (0.8, 1.0, 1.25):
        hand = (l - W) * (rho_ta / (h_ta * (2 * H + W)) - rho * xi / (W * H))
        assert abs(f(l, W, H, h_ta, rho_ta, rho * xi) - hand) <= 1e-12 * abs(hand)


def test_param4_normal_draw_statistics_and_counter(oracle_mod):
    # Box-Muller normals: moments and a Kolmogorov-Smirnov distance against
    # the normal CDF; the deviate is the one the lognormal of the same
    # counter maps (xi = exp(-s2/2 + sqrt(s2) z))
    z = oracle_mod.normal_z(4242, 9, 200000, 4)
    n = z.size
    assert abs(z.mean()) < 4 / math.sqrt(n) and abs(z.std() - 1.0) < 0.01
    zs = np.sort(z)
    cdf = 0.5 * (1.0 + np.array([math.erf(v / math.sqrt(2.0)) for v in zs[::50]]))
    emp = (np.arange(0, n, 50) + 1) / n
    assert np.max(np.abs(cdf - emp)) < 1.6 / math.sqrt(n) + 50 / n
    s2 = math.log(1.0 + 0.3 ** 2)
    xi = oracle_mod.lognormal_xi(4242, 9, 1000, 4, 0.3)
    assert np.allclose((np.log(xi) + 0.5 * s2) / math.sqrt(s2), z[:1000], rtol=0, atol=1e-12)


def test_activation_energy_offset_is_an_arrhenius_factor(oracle_mod):
    # D = D0 exp(-(Ea + dEa)/(k_B T)): the diffusivity multiplier changes by
    # exactly D(Ea + dEa)/D(Ea) per wire segment, vias untouched; at uniform T
    # the log-factor is normal with spread sd/(k_B T), mean exp((sd/k_B T)^2/2)
    g = synth.pg_grid(11, n=24, via_every=8, pad_lattice=2, sink_scale=1.0, seg_range=(10, 23))
    g = synth.Grid(**{**g.__dict__, "tmap": None, "node_T": None})
    wire = (g.res_is_via == 0) & (g.layer[g.res_a] == g.layer[g.res_b])
    kT = 1.380649e-23 * 350.0 / 1.602176634e-19
    sd = 0.6 * kT
    base = dict(seed=21, cov_kappa=0.2, cov_scrit=0.2)
    k0, s0 = oracle_mod.sample_xi(g, base, 3, T_amb=350.0)
    k1, s1 = oracle_mod.sample_xi(g, dict(base, sd_ea_eV=sd), 3, T_amb=350.0)
    assert np.array_equal(s0, s1) and np.array_equal(k0[~wire], k1[~wire])
    dEa = sd * oracle_mod.normal_z(21, 3, g.n_res, 4)[wire]
    D = lambda Ea: np.exp(-Ea / kT)                          # Arrhenius at 350 K, D0 = 1
    assert np.allclose(k1[wire] / k0[wire], D(0.85 + dEa) / D(0.85), rtol=1e-13)
    f = k1[wire] / k0[wire]
    assert abs(np.std(np.log(f)) - 0.6) < 0.08
    assert abs(np.mean(f) / math.exp(0.18) - 1.0) < 0.1


def test_activation_energy_factor_takes_the_midpoint_map_temperature(oracle_mod):
    # hot segments (a hotspot map) see a smaller spread in log D: k_B T log f
    # is -dEa whatever the temperature
    g, mat, rn, mc = synth.workload("mc_grid")
    assert g.tmap is not None
    from oracle import thermal
    sd = 0.01
    k0, _ = oracle_mod.sample_xi(g, mc, 2, T_amb=rn["T_ambient"])
    k1, _ = oracle_mod.sample_xi(g, dict(mc, sd_ea_eV=sd), 2, T_amb=rn["T_ambient"])
    wire = np.nonzero((g.res_is_via == 0) & (g.layer[g.res_a] == g.layer[g.res_b]))[0]
    T = np.array([thermal.midpoint_map_T(g, rn["T_ambient"], int(e)) for e in wire])
    assert np.ptp(T) > 5.0
    kB = 1.380649e-23 / 1.602176634e-19
    dEa = -kB * T * np.log(k1[wire] / k0[wire])
    assert np.allclose(dEa, sd * oracle_mod.normal_z(mc["seed"], 2, g.n_res, 4)[wire], rtol=0, atol=1e-15)


def test_die_temperature_offset_is_the_arrhenius_ratio(oracle_mod):
    # one offset dT ~ N(0, sd) per sample (param 5, counter index 0): at a
    # uniform map temperature every wire segment takes the same factor, the
    # ratio of the Arrhenius diffusivity kappa = D0 exp(-Ea/k_B T) B Omega /
    # (k_B T) at T + dT and at T; vias and sigma_crit untouched
    from oracle import surrogate_oracle as SO
    g = synth.pg_grid(11, n=24, via_every=8, pad_lattice=2, sink_scale=1.0, seg_range=(10, 23))
    g = synth.Grid(**{**g.__dict__, "tmap": None, "node_T": None})
    mat = synth.default_material()
    wire = (g.res_is_via == 0) & (g.layer[g.res_a] == g.layer[g.res_b])
    base = dict(seed=21, cov_kappa=0.2, cov_scrit=0.2)
    for s in (0, 3, 7):
        k0, s0 = oracle_mod.sample_xi(g, base, s, T_amb=350.0, Ea_eV=mat["Ea_eV"])
        k1, s1 = oracle_mod.sample_xi(g, dict(base, sd_T_K=3.0), s, T_amb=350.0, Ea_eV=mat["Ea_eV"])
        assert np.array_equal(s0, s1) and np.array_equal(k0[~wire], k1[~wire])
        f = k1[wire] / k0[wire]
        dT = 3.0 * oracle_mod.normal_z(21, s, 1, 5)[0]
        want = SO.kappa0(350.0 + dT, mat) / SO.kappa0(350.0, mat)
        assert np.allclose(f, want, rtol=1e-12), (s, dT)
        assert (want > 1.0) == (dT > 0.0)            # a hotter die diffuses faster
    # the offsets over many samples: mean 0, spread sd
    z = np.array([oracle_mod.normal_z(21, s, 1, 5)[0] for s in range(4000)])
    assert abs(z.mean()) < 4 / math.sqrt(z.size) and abs(z.std() - 1.0) < 0.04
    with pytest.raises(ValueError):
        oracle_mod.sample_xi(g, dict(base, sd_T_K=3.0), 0, T_amb=350.0)


def test_map_amplitude_drives_thermomigration_as_the_scaled_map(oracle_mod):
    """Param 6: the sample's amplitude a scales the map's rise above the
    ambient.  With no current, the zero-flux steady stress (the screen's,
    kappa-independent) is the path integral of the thermomigration drive
    alone; under map_a = a it must equal that of the same grid whose raster
    was scaled by hand, T_amb + a (T - T_amb) (node temperatures interpolate
    the raster linearly).  The amplitudes are unit-mean lognormal."""
    g, mat, rn, mc = synth.workload("mc_grid")
    T_amb = float(rn["T_ambient"])
    topo = oracle_mod.topology(g, rn["intervals_per_seg"])
    zero = np.zeros(g.n_res)
    for a in (0.7, 1.3):
        sim_a = oracle_mod.SampleSim(g, mat, rn, topo, map_a=a)
        sim_a.set_j(zero)
        _, _, ss_a = sim_a.screen()
        g2 = synth.Grid(**{**g.__dict__, "tmap": T_amb + a * (g.tmap - T_amb)})
        sim_b = oracle_mod.SampleSim(g2, mat, rn, topo)
        sim_b.set_j(zero)
        _, _, ss_b = sim_b.screen()
        scale = np.abs(ss_b - mat["sigma_T"]).max()
        assert scale > 1e5                                  # the map drives a real stress
        assert np.allclose(ss_a, ss_b, rtol=0, atol=1e-9 * scale), a
    # and not the unscaled map's
    sim_0 = oracle_mod.SampleSim(g, mat, rn, topo)
    sim_0.set_j(zero)
    _, _, ss_0 = sim_0.screen()
    assert np.abs(ss_0 - ss_a).max() > 0.1 * scale
    amps = np.array([oracle_mod.sample_map_amplitude(dict(mc, cov_map=0.2), s) for s in range(4000)])
    assert abs(amps.mean() - 1.0) < 0.02 and abs(amps.std() - 0.2) < 0.02 and amps.min() > 0
    assert oracle_mod.sample_map_amplitude(dict(mc, cov_map=0.0), 0) is None
