"""Small hand-built inputs shared by the oracle pins and the GPU parity tests.

Only inputs live here (geometry, currents, temperatures); no stress, IR or
void arithmetic.
"""
import numpy as np

from paper_2604_10743_amd.synth import Grid, RHO_CU, default_material, default_run

UM = 1e-6


def line_grid(S=5, L=10 * UM, w=0.5 * UM, h=0.2 * UM, j=1e10, T=378.0, reverse=False):
    """One straight line of S equal segments, vertices 0..S left to right,
    every segment oriented left->right (or right->left with ``reverse``),
    uniform current density j along its a->b orientation."""
    n = S + 1
    xy = np.stack([np.arange(n) * L, np.zeros(n)], 1)
    a = np.arange(S, dtype=np.int32)
    b = a + 1
    if reverse:
        a, b = b, a
    return Grid(xy=xy, layer=np.ones(n, np.int32), res_a=a.astype(np.int32),
                res_b=b.astype(np.int32), res_len=np.full(S, L), res_w=np.full(S, w),
                res_h=np.full(S, h), res_is_via=np.zeros(S, np.uint8),
                res_R0=np.full(S, RHO_CU * L / (w * h)), pad_node=np.zeros(0, np.int32),
                vdd=1.0, sink_I=np.zeros(n), node_T=np.full(n, float(T)),
                seg_j=np.full(S, float(j)))


def tree_from_edges(n_vert, edges, L, w, h, j, T=378.0, xy=None, layer=None, vias=()):
    """Trees-only grid from explicit (a, b) edge list; optional extra via
    resistors (a, b) appended after the wires."""
    E = len(edges)
    a = [e[0] for e in edges] + [v[0] for v in vias]
    b = [e[1] for e in edges] + [v[1] for v in vias]
    nv = len(vias)
    L = np.concatenate([np.broadcast_to(np.asarray(L, float), (E,)), np.zeros(nv)])
    w = np.concatenate([np.broadcast_to(np.asarray(w, float), (E,)), np.full(nv, 0.5 * UM)])
    h = np.concatenate([np.broadcast_to(np.asarray(h, float), (E,)), np.full(nv, 0.2 * UM)])
    j = np.concatenate([np.broadcast_to(np.asarray(j, float), (E,)), np.zeros(nv)])
    if xy is None:
        xy = np.stack([np.arange(n_vert) * 10 * UM, np.zeros(n_vert)], 1)
    if layer is None:
        layer = np.ones(n_vert, np.int32)
    is_via = np.concatenate([np.zeros(E, np.uint8), np.ones(nv, np.uint8)])
    R0 = np.where(is_via == 1, 0.5, RHO_CU * np.maximum(L, 1e-12) / (w * h))
    return Grid(xy=np.asarray(xy, float), layer=np.asarray(layer, np.int32),
                res_a=np.array(a, np.int32), res_b=np.array(b, np.int32), res_len=L,
                res_w=w, res_h=h, res_is_via=is_via, res_R0=R0,
                pad_node=np.zeros(0, np.int32), vdd=1.0, sink_I=np.zeros(n_vert),
                node_T=np.full(n_vert, float(T)), seg_j=j)


def ladder_grid(n=10, R=2.0, sinks=None, vdd=1.0):
    """A chain of n resistors from one pad (node 0) with sinks on nodes 1..n."""
    if sinks is None:
        sinks = np.linspace(1e-3, 2e-3, n)
    L = 10 * UM
    w, h = 0.5 * UM, 0.2 * UM
    xy = np.stack([np.arange(n + 1) * L, np.zeros(n + 1)], 1)
    sink = np.concatenate([[0.0], sinks])
    return Grid(xy=xy, layer=np.ones(n + 1, np.int32), res_a=np.arange(n, dtype=np.int32),
                res_b=np.arange(1, n + 1, dtype=np.int32), res_len=np.full(n, L),
                res_w=np.full(n, w), res_h=np.full(n, h), res_is_via=np.zeros(n, np.uint8),
                res_R0=np.full(n, R), pad_node=np.array([0], np.int32), vdd=vdd,
                sink_I=sink, node_T=np.full(n + 1, 378.0))


def line_pad_load(S=4, L=25 * UM, w=0.5 * UM, h=0.2 * UM, I=4e-3, vdd=1.2, T=378.0):
    """A single wire of S equal segments from one pad (vertex 0) to one load
    drawing I at vertex S; one layer, no via.  The whole current runs through
    every segment whatever their resistances, so the worst drop is at the load:
    I (sum of segment resistances) / vdd."""
    n = S + 1
    xy = np.stack([np.arange(n) * L, np.zeros(n)], 1)
    sink = np.zeros(n)
    sink[-1] = I
    return Grid(xy=xy, layer=np.ones(n, np.int32), res_a=np.arange(S, dtype=np.int32),
                res_b=np.arange(1, n, dtype=np.int32), res_len=np.full(S, L), res_w=np.full(S, w),
                res_h=np.full(S, h), res_is_via=np.zeros(S, np.uint8),
                res_R0=np.full(S, RHO_CU * L / (w * h)), pad_node=np.array([0], np.int32), vdd=vdd,
                sink_I=sink, node_T=np.full(n, float(T)))


# Run settings of the outer-loop cases on line_pad_load (load current I): a
# crossing after several re-solves on a uniform and a graded grid, a censored
# run whose last interval is short, and a network already failed at t = 0.
OUTER_CASES = {
    "uniform": (dict(dt=1e3, ir_every=10, n_steps=200, fail_frac=0.10), 4e-3),
    "graded": (dict(dt=3e2, dt_growth=1.2, ir_every=10, n_steps=200, fail_frac=0.10), 4e-3),
    "censored_ragged": (dict(dt=1e3, ir_every=10, n_steps=195, fail_frac=0.5), 4e-3),
    "failed_at_t0": (dict(dt=1e3, ir_every=10, n_steps=200, fail_frac=0.10), 5e-3),
}


def pcg_rtol(rn):
    """The PCG tolerance a run dict asks for (0: the library's automatic
    choice by stepping precision, 1e-11 FP64 / 1e-8 FP32)."""
    r = float(rn.get("cg_rtol", 0.0))
    return r if r > 0 else (1e-11 if int(rn.get("prec", 0)) == 0 else 1e-8)


def material(**over):
    m = default_material()
    m.update(over)
    return m


def run(**over):
    return default_run(**over)
