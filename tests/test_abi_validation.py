"""Argument checks of em_batch_create through the C ABI on the host: every
invalid input is refused with EM_ERR_ARG and a message before any device work
(validation and the wire-tree partition run on the host first), so these run
without a GPU.  The batch handle is returned even on failure (em_last_error)
and destroyed afterwards."""
import ctypes as C
import math

import numpy as np
import pytest

from cases import tree_from_edges
from paper_2604_10743_amd import _binding as Bd
from paper_2604_10743_amd import synth

UM = 1e-6


def _structs(grid, mat, run, mc):
    keep = []

    def ptr(a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dt)
        keep.append(a)
        return a.ctypes.data

    g = Bd.GridDesc(struct_size=C.sizeof(Bd.GridDesc))
    g.n_nodes = grid.n_nodes
    g.xy = ptr(grid.xy, np.float64)
    g.layer = ptr(grid.layer, np.int32)
    g.n_res = grid.n_res
    g.res_a = ptr(grid.res_a, np.int32); g.res_b = ptr(grid.res_b, np.int32)
    g.res_len = ptr(grid.res_len, np.float64); g.res_w = ptr(grid.res_w, np.float64)
    g.res_h = ptr(grid.res_h, np.float64); g.res_is_via = ptr(grid.res_is_via, np.uint8)
    g.res_R0 = ptr(grid.res_R0, np.float64)
    g.n_pads = len(grid.pad_node)
    g.pad_node = ptr(grid.pad_node, np.int32) if len(grid.pad_node) else None
    g.vdd = grid.vdd
    g.sink_I = ptr(grid.sink_I, np.float64)
    g.node_T = ptr(grid.node_T, np.float64)
    if grid.tmap is not None:
        g.tmap = ptr(grid.tmap, np.float64)
        g.tmap_ny, g.tmap_nx = grid.tmap.shape
        g.tmap_x0, g.tmap_y0, g.tmap_dx, g.tmap_dy = grid.tmap_x0, grid.tmap_y0, grid.tmap_dx, grid.tmap_dy
    g.seg_j = ptr(grid.seg_j, np.float64)
    m = Bd.Material(struct_size=C.sizeof(Bd.Material), **{k: float(v) for k, v in mat.items()})
    r = Bd.RunParams(struct_size=C.sizeof(Bd.RunParams))
    for k, v in run.items():
        setattr(r, k, v)
    mcp = None
    if mc is not None:
        mcp = Bd.MCParams(struct_size=C.sizeof(Bd.MCParams), **mc)
    return g, m, r, mcp, keep


def _create(g, m, r, mcp):
    L = Bd.lib()
    h = C.c_void_p()
    rc = L.em_batch_create(C.byref(g), C.byref(m), C.byref(r), C.byref(mcp) if mcp is not None else None,
                           None, None, C.byref(h))
    msg = L.em_last_error(h).decode() if h.value else ""
    if h.value:
        L.em_batch_destroy(h)
    return rc, msg


def _base():
    g = synth.two_layer_mesh(7, nr=6, nc=6)
    mat = synth.default_material()
    run = dict(synth.default_run())
    mc = dict(n_samples=4, seed=1, cov_kappa=0.2, cov_scrit=0.2, cov_rho=0.0, cov_load=0.0)
    return g, mat, run, mc


CASES = {
    "resistor node out of range": lambda g, m, r, mc: g.res_b.__setitem__(0, g.n_nodes),
    "R0 must be positive": lambda g, m, r, mc: g.res_R0.__setitem__(0, 0.0),
    "wire geometry": lambda g, m, r, mc: g.res_len.__setitem__(int(np.nonzero(g.res_is_via == 0)[0][0]), 0.0),
    "non-finite coordinates": lambda g, m, r, mc: g.xy.__setitem__((1, 0), math.nan),
    "vdd must be positive": lambda g, m, r, mc: setattr(g, "vdd", 0.0),
    "bad material": lambda g, m, r, mc: m.__setitem__("B", -1.0),
    "bad run parameters (intervals)": lambda g, m, r, mc: r.__setitem__("intervals_per_seg", 0),
    "bad run parameters (dt)": lambda g, m, r, mc: r.__setitem__("dt", -1.0),
    "bad run parameters (prec)": lambda g, m, r, mc: r.__setitem__("prec", 2),
    "bad run parameters (voids)": lambda g, m, r, mc: r.__setitem__("max_voids_per_tree", 5),
    "bad run parameters (precond)": lambda g, m, r, mc: r.__setitem__("ir_precond", 3),
    "bad run parameters (launch)": lambda g, m, r, mc: r.__setitem__("ir_launch", 4),
    "bad run parameters (joule)": lambda g, m, r, mc: r.__setitem__("joule", 2),
    "bad run parameters (growth)": lambda g, m, r, mc: r.__setitem__("dt_growth", math.inf),
    "bad run parameters (chain_m)": lambda g, m, r, mc: r.__setitem__("chain_m", 7),
    "bad run parameters (chain_m FP64)": lambda g, m, r, mc: (r.__setitem__("chain_m", 9), r.__setitem__("prec", 0)),
    "bad run parameters (chain_m lanes)": lambda g, m, r, mc: (r.__setitem__("chain_m", 9),
                                                              r.__setitem__("chain_wg", 512)),
    "Joule thermal block": lambda g, m, r, mc: (r.__setitem__("joule", 1), m.__setitem__("k_ild", 0.0)),
    "bad Monte Carlo (samples)": lambda g, m, r, mc: mc.__setitem__("n_samples", 0),
    "bad Monte Carlo (cov)": lambda g, m, r, mc: mc.__setitem__("cov_kappa", -0.1),
    "bad Monte Carlo (rho)": lambda g, m, r, mc: mc.__setitem__("cov_rho", math.nan),
    "bad Monte Carlo (Ea spread)": lambda g, m, r, mc: mc.__setitem__("sd_ea_eV", -0.01),
    "bad Monte Carlo (Ea spread, huge)": lambda g, m, r, mc: mc.__setitem__("sd_ea_eV", 2.0),
    "bad Monte Carlo (die temperature spread)": lambda g, m, r, mc: mc.__setitem__("sd_T_K", -1.0),
    "bad Monte Carlo (die temperature spread, huge)": lambda g, m, r, mc: mc.__setitem__("sd_T_K", 50.0),
    "bad Monte Carlo (map amplitude spread)": lambda g, m, r, mc: mc.__setitem__("cov_map", -0.1),
    "bad Monte Carlo (map amplitude spread, huge)": lambda g, m, r, mc: mc.__setitem__("cov_map", 1.5),
    "bad run parameters (multigrid scale)": lambda g, m, r, mc: r.__setitem__("amg_alpha", 0.5),
    "bad run parameters (steady-state tolerance)": lambda g, m, r, mc: r.__setitem__("ss_tol", -1e-6),
    "bad run parameters (steady-state tolerance, huge)": lambda g, m, r, mc: r.__setitem__("ss_tol", 0.05),
    "bad run parameters (Krylov order)": lambda g, m, r, mc: r.__setitem__("krylov_q", 9),
    "bad run parameters (Krylov order, negative)": lambda g, m, r, mc: r.__setitem__("krylov_q", -1),
    "bad run parameters (Krylov shift scale)": lambda g, m, r, mc: r.__setitem__("krylov_eta", -0.5),
    "reduced (Krylov) stepping and steady-state skipping are exclusive":
        lambda g, m, r, mc: r.update(krylov_q=4, ss_tol=1e-6),
    "bad run parameters (adaptive grid levels)": lambda g, m, r, mc: r.__setitem__("dt_adapt", 13),
    "the adaptive and the graded time grids are exclusive":
        lambda g, m, r, mc: r.update(dt_adapt=2, dt_growth=1.1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_invalid_input_is_refused(name):
    g, mat, run, mc = _base()
    CASES[name](g, mat, run, mc)
    rc, msg = _create(*_structs(g, mat, run, mc)[:4])
    assert rc == Bd.EM_ERR_ARG, (name, rc, msg)
    assert msg, name


def test_struct_size_mismatch_is_refused():
    g, mat, run, mc = _base()
    gs, m, r, mcp, keep = _structs(g, mat, run, mc)
    r.struct_size = C.sizeof(Bd.RunParams) - 8
    rc, msg = _create(gs, m, r, mcp)
    assert rc == Bd.EM_ERR_ARG and "struct_size" in msg


def test_netlist_without_wires_is_refused():
    g, mat, run, mc = _base()
    g.res_is_via[:] = 1                     # every resistor a via
    rc, msg = _create(*_structs(g, mat, run, mc)[:4])
    assert rc == Bd.EM_ERR_ARG and "wire" in msg


def test_wire_cycle_is_refused():
    # a same-layer loop is not a tree (Sec. IV-A: wire trees)
    g = tree_from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)], L=10 * UM, w=0.5 * UM, h=0.2 * UM, j=1e10)
    rc, msg = _create(*_structs(g, synth.default_material(), dict(synth.default_run()), None)[:4])
    assert rc == Bd.EM_ERR_ARG and "cycle" in msg
