"""FP64 CPU oracle for the coupled EM/TM stress + IR-drop path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package.  It shares no
code with the HIP path.  The per-tree arithmetic lives in ``em_oracle.c``
(scalar C loops); this module marshals arrays, performs the IR solve and runs
the outer aging loop, following EMSpice 3 (arXiv 2604.10743):

* IR solve (Sec. III-C, eq. 8): nodal analysis of the resistor network with
  ideal VDD pads and current-sink loads, solved by a sparse direct
  factorisation (a library primitive); open resistors conduct nothing and
  nodes cut off from every pad read 0 V.
* Outer loop (Fig. 2, Sec. IV-A/B): at each aging step the stress state is
  advanced with the currents of the last IR solve, void-induced resistance
  changes are written back, the IR problem is re-solved, and the network fails
  when the worst IR-drop reaches the failure fraction (Table I caption).
* Monte Carlo (Sec. IV-F): every sample re-runs the whole pipeline with
  unit-mean lognormal multipliers on diffusivity and critical stress.

Parity unpinned: nothing here reproduces a number of the paper's own designs
(the designs and thermal maps are not available).
"""
from __future__ import annotations

import ctypes as C
import math
import dataclasses
import os
import subprocess

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla

from . import krylov, thermal

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile em_oracle.c into liboracle.so (plain gcc, -O2, no fast-math)."""
    src = os.path.join(_HERE, "em_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99",
                               "-fno-fast-math", "-ffp-contract=off", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = C.CDLL(_SO)
        L = _lib
        L.ora_create.restype = C.c_void_p
        L.ora_lognormal_xi.restype = C.c_double
        L.ora_lognormal_xi.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_double]
        L.ora_fill_xi.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_double, C.c_void_p]
        L.ora_normal_z.restype = C.c_double
        L.ora_normal_z.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int]
        L.ora_fill_normal.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_void_p]
        for fn in ("ora_destroy", "ora_set_j", "ora_screen", "ora_set_active", "ora_steps",
                   "ora_get_sigma", "ora_set_sigma", "ora_get_node_arrays", "ora_get_seg_state",
                   "ora_get_voids", "ora_get_events", "ora_n_events", "ora_n_suppressed",
                   "ora_inject_void", "ora_set_dt"):
            getattr(L, fn).argtypes = None
    return _lib


class _Problem(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int), ("xy", C.c_void_p), ("layer", C.c_void_p),
        ("n_res", C.c_int), ("ra", C.c_void_p), ("rb", C.c_void_p),
        ("len", C.c_void_p), ("w", C.c_void_p), ("h", C.c_void_p), ("is_via", C.c_void_p),
        ("node_T", C.c_void_p), ("tnx", C.c_int), ("tny", C.c_int),
        ("tx0", C.c_double), ("ty0", C.c_double), ("tdx", C.c_double), ("tdy", C.c_double),
        ("tmap", C.c_void_p), ("T_amb", C.c_double),
        ("B", C.c_double), ("Omega", C.c_double), ("Z", C.c_double), ("rho", C.c_double),
        ("Ea_eV", C.c_double), ("D0", C.c_double), ("scrit", C.c_double), ("Q_eV", C.c_double),
        ("sigT", C.c_double), ("delta", C.c_double), ("rho_ta", C.c_double), ("h_ta", C.c_double),
        ("N", C.c_int), ("dt", C.c_double), ("max_voids", C.c_int),
        ("xi_k", C.c_void_p), ("xi_s", C.c_void_p), ("T_stress", C.c_void_p), ("xi_r", C.c_void_p),
        ("map_a", C.c_double),
    ]


def _pi(a):
    """Address as a plain int (for structure fields)."""
    return None if a is None else a.ctypes.data


def _p(a):
    """Address as a pointer argument (never truncated to a C int)."""
    return None if a is None else C.c_void_p(a.ctypes.data)


class _Keep:
    """Holds contiguous copies of every array the C side points to."""

    def __init__(self):
        self.arrs = []

    def __call__(self, a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        self.arrs.append(a)
        return a


def make_problem(grid, mat, run, xi_k=None, xi_s=None, T_stress=None, xi_r=None, map_a=None):
    keep = _Keep()
    P = _Problem()
    P.n_nodes = grid.n_nodes
    P.xy = _pi(keep(grid.xy, np.float64))
    P.layer = _pi(keep(grid.layer, np.int32))
    P.n_res = grid.n_res
    P.ra = _pi(keep(grid.res_a, np.int32)); P.rb = _pi(keep(grid.res_b, np.int32))
    P.len = _pi(keep(grid.res_len, np.float64)); P.w = _pi(keep(grid.res_w, np.float64))
    P.h = _pi(keep(grid.res_h, np.float64)); P.is_via = _pi(keep(grid.res_is_via, np.uint8))
    P.node_T = _pi(keep(grid.node_T, np.float64))
    if grid.tmap is not None:
        tm = keep(grid.tmap, np.float64)
        P.tmap = _pi(tm); P.tny, P.tnx = tm.shape
        P.tx0, P.ty0, P.tdx, P.tdy = grid.tmap_x0, grid.tmap_y0, grid.tmap_dx, grid.tmap_dy
    P.T_amb = float(run.get("T_ambient", 300.0))
    P.B = mat["B"]; P.Omega = mat["Omega"]; P.Z = mat["Z"]; P.rho = mat["rho_cu"]
    P.Ea_eV = mat["Ea_eV"]; P.D0 = mat["D0"]; P.scrit = mat["sigma_crit"]; P.Q_eV = mat["Q_eV"]
    P.sigT = mat["sigma_T"]; P.delta = mat["delta"]; P.rho_ta = mat["rho_ta"]; P.h_ta = mat["h_ta"]
    P.N = int(run["intervals_per_seg"]); P.dt = float(run["dt"])
    P.max_voids = int(run["max_voids_per_tree"])
    P.xi_k = _pi(keep(xi_k, np.float64)); P.xi_s = _pi(keep(xi_s, np.float64))
    P.T_stress = _pi(keep(T_stress, np.float64))
    P.xi_r = _pi(keep(xi_r, np.float64))
    P.map_a = float(map_a) if map_a else 0.0
    return P, keep


class Topology:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def topology(grid, N: int) -> Topology:
    """Wire trees, DFS pre-order stress-node numbering (Sec. IV-A)."""
    L = lib()
    P, keep = make_problem(grid, {k: 0.0 for k in ("B", "Omega", "Z", "rho_cu", "Ea_eV", "D0",
                                                   "sigma_crit", "Q_eV", "sigma_T", "delta",
                                                   "rho_ta", "h_ta")},
                           dict(intervals_per_seg=N, dt=0.0, max_voids_per_tree=0))
    cap_s = grid.n_res * N + grid.n_nodes + 1
    cap_t = grid.n_nodes + 1
    nt, ns = C.c_int(), C.c_int()
    off = np.zeros(cap_t + 1, np.int32)
    arr = {k: np.zeros(cap_s, np.int32) for k in ("parent", "seg", "dir", "vert", "kpos")}
    seg_tree = np.zeros(grid.n_res, np.int32)
    rc = L.ora_topology(C.byref(P), C.c_int(cap_t), C.c_int(cap_s), C.byref(nt), C.byref(ns),
                        _p(off), _p(arr["parent"]), _p(arr["seg"]), _p(arr["dir"]),
                        _p(arr["vert"]), _p(arr["kpos"]), _p(seg_tree))
    if rc != 0:
        raise ValueError("topology error %d (%s)" % (rc, "cycle" if rc == 1 else "capacity"))
    n = ns.value
    return Topology(n_trees=nt.value, n_stress=n, tree_off=off[:nt.value + 1].copy(),
                    parent=arr["parent"][:n].copy(), seg=arr["seg"][:n].copy(),
                    dir=arr["dir"][:n].copy(), vert=arr["vert"][:n].copy(),
                    kpos=arr["kpos"][:n].copy(), seg_tree=seg_tree, N=N)


def philox4x32_10(ctr, key):
    L = lib()
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    L.ora_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def lognormal_xi(seed: int, sample: int, n_seg: int, param: int, cov: float) -> np.ndarray:
    L = lib()
    out = np.zeros(n_seg)
    L.ora_fill_xi(C.c_uint64(seed), sample, n_seg, param, C.c_double(cov), _p(out))
    return out


def normal_z(seed: int, sample: int, n: int, param: int) -> np.ndarray:
    """Standard normal deviates of counters (0..n-1, sample, param, 0)."""
    L = lib()
    out = np.zeros(n)
    L.ora_fill_normal(C.c_uint64(seed), sample, n, param, _p(out))
    return out


class SampleSim:
    """One sample's stress/void state (wraps the C oracle)."""

    def __init__(self, grid, mat, run, topo: Topology, xi_k=None, xi_s=None, cap_events=1 << 16,
                 T_stress=None, xi_r=None, map_a=None):
        L = lib()
        self.grid, self.mat, self.run, self.topo = grid, mat, run, topo
        self.P, self.keep = make_problem(grid, mat, run, xi_k, xi_s, T_stress, xi_r, map_a)
        t = topo
        self._t = [np.ascontiguousarray(a, np.int32) for a in
                   (t.tree_off, t.parent, t.seg, t.dir, t.vert, t.kpos, t.seg_tree)]
        self.h = L.ora_create(C.byref(self.P), C.c_int(t.n_trees), C.c_int(t.n_stress),
                              *[_p(a) for a in self._t], C.c_int(cap_events))
        self.cap_events = cap_events

    def __del__(self):
        try:
            lib().ora_destroy(C.c_void_p(self.h))
        except Exception:
            pass

    @property
    def _h(self):
        return C.c_void_p(self.h)

    def set_j(self, jseg):
        j = np.ascontiguousarray(jseg, np.float64)
        lib().ora_set_j(self._h, _p(j))

    def screen(self):
        t = self.topo
        tm = np.zeros(t.n_trees, np.uint8)
        sm = np.zeros(self.grid.n_res, np.uint8)
        ss = np.zeros(t.n_stress)
        lib().ora_screen(self._h, _p(tm), _p(sm), _p(ss))
        return tm, sm, ss

    def set_active(self, active):
        a = np.ascontiguousarray(active, np.uint8)
        lib().ora_set_active(self._h, _p(a))

    def steps(self, n, step0=0):
        return lib().ora_steps(self._h, C.c_int(n), C.c_int(step0))

    def set_dt(self, dt):
        lib().ora_set_dt(self._h, C.c_double(dt))

    def sigma(self):
        s = np.zeros(self.topo.n_stress)
        lib().ora_get_sigma(self._h, _p(s))
        return s

    def set_sigma(self, s):
        s = np.ascontiguousarray(s, np.float64)
        lib().ora_set_sigma(self._h, _p(s))

    def node_arrays(self):
        n = self.topo.n_stress
        out = {k: np.zeros(n) for k in ("T", "V", "g", "f", "sc", "robsum")}
        lib().ora_get_node_arrays(self._h, *[_p(out[k]) for k in ("T", "V", "g", "f", "sc", "robsum")])
        return out

    def seg_state(self):
        dR = np.zeros(self.grid.n_res)
        op = np.zeros(self.grid.n_res, np.uint8)
        lib().ora_get_seg_state(self._h, _p(dR), _p(op))
        return dR, op

    def voids(self):
        n = lib().ora_get_voids(self._h, None, None)
        iv = np.zeros((max(n, 1), 6), np.int32)
        dv = np.zeros((max(n, 1), 2))
        lib().ora_get_voids(self._h, _p(iv), _p(dv))
        return iv[:n], dv[:n]

    def events(self):
        n = lib().ora_n_events(self._h)
        n = min(n, self.cap_events)
        e = np.zeros((max(n, 1), 4), np.int32)
        lib().ora_get_events(self._h, _p(e))
        return e[:n]

    def n_suppressed(self):
        return lib().ora_n_suppressed(self._h)

    def inject_void(self, tree, node, step=0):
        return lib().ora_inject_void(self._h, C.c_int(tree), C.c_int(node), C.c_int(step))


# ----------------------------------------------------------------------------
# IR solve (Sec. III-C): M u = P I with ideal pads
# ----------------------------------------------------------------------------
def ir_solve(grid, R, open_mask=None):
    """Nodal voltages, per-resistor currents and current densities, worst drop.

    R: per-resistor resistance (ohm); open_mask: resistors that conduct
    nothing (early failure).  Nodes with no conducting path to a pad are set
    to 0 V.  Returns (u, I, j, drop)."""
    n = grid.n_nodes
    G = 1.0 / np.asarray(R, np.float64)
    if open_mask is not None:
        G = np.where(np.asarray(open_mask) != 0, 0.0, G)
    a, b = grid.res_a.astype(np.int64), grid.res_b.astype(np.int64)
    cond = G > 0
    adj = sp.coo_matrix((np.ones(int(cond.sum())), (a[cond], b[cond])), shape=(n, n)).tocsr()
    _, lab = csg.connected_components(adj, directed=False)
    pad = np.zeros(n, bool)
    pad[grid.pad_node] = True
    live_labels = np.unique(lab[pad])
    live = np.isin(lab, live_labels)
    unk = live & ~pad
    idx = -np.ones(n, np.int64)
    idx[unk] = np.arange(int(unk.sum()))
    m = int(unk.sum())
    rows, cols, vals = [], [], []
    rhs = np.zeros(m)
    # KCL at every unknown node: sum_e G_e (u_i - u_j) = -sink_i
    np.add.at(rhs, idx[unk], -grid.sink_I[unk])
    for (p, q) in ((a, b), (b, a)):
        sel = cond & unk[p]
        ip = idx[p[sel]]
        rows.append(ip); cols.append(ip); vals.append(G[sel])
        other_unk = unk[q[sel]]
        rows.append(ip[other_unk]); cols.append(idx[q[sel]][other_unk]); vals.append(-G[sel][other_unk])
        other_pad = pad[q[sel]]
        np.add.at(rhs, ip[other_pad], G[sel][other_pad] * grid.vdd)
    A = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, m))
    u = np.zeros(n)
    u[pad] = grid.vdd
    if m:
        u[unk] = spla.spsolve(A, rhs, permc_spec="MMD_AT_PLUS_A")
    I = (u[a] - u[b]) * G
    j = I / (grid.res_w * grid.res_h)
    drop = float(np.max((grid.vdd - u) / grid.vdd))
    return u, I, j, drop


# ----------------------------------------------------------------------------
# Full pipeline for one sample
# ----------------------------------------------------------------------------
K_B_EV = 1.380649e-23 / 1.602176634e-19        # Boltzmann constant, eV/K


def sample_xi(grid, mc, sample, T_amb=300.0, Ea_eV=None):
    """Diffusivity and critical-stress multipliers of one sample, per segment.

    An activation-energy spread sd_ea_eV > 0 draws dEa ~ N(0, sd) per wire
    segment (param 4); the diffusivity D0 exp(-(Ea + dEa)/(k_B T)) then carries
    the extra factor exp(-dEa/(k_B T)), taken at the segment midpoint's map
    temperature and folded into the diffusivity multiplier.  A die-temperature
    spread sd_T_K > 0 draws one offset dT ~ N(0, sd) per sample (param 5,
    index 0): the map shifted by dT changes every wire segment's Arrhenius
    diffusivity D0 exp(-Ea/(k_B T)) B Omega/(k_B T) by the ratio of its values
    at T + dT and T (the same midpoint temperature), folded in likewise."""
    if mc is None:
        return None, None
    xi_k = lognormal_xi(mc["seed"], sample, grid.n_res, 0, mc["cov_kappa"])
    sd = float(mc.get("sd_ea_eV", 0.0))
    if sd > 0:
        wire = (grid.res_is_via == 0) & (grid.layer[grid.res_a] == grid.layer[grid.res_b])
        z = normal_z(mc["seed"], sample, grid.n_res, 4)
        for e in np.nonzero(wire)[0]:
            xi_k[e] *= np.exp(-sd * z[e] / (K_B_EV * thermal.midpoint_map_T(grid, T_amb, int(e))))
    sdT = float(mc.get("sd_T_K", 0.0))
    if sdT > 0:
        wire = (grid.res_is_via == 0) & (grid.layer[grid.res_a] == grid.layer[grid.res_b])
        if Ea_eV is None:
            raise ValueError("a die-temperature spread needs the material's activation energy")
        dT = sdT * float(normal_z(mc["seed"], sample, 1, 5)[0])
        Ea = float(Ea_eV)
        for e in np.nonzero(wire)[0]:
            T = thermal.midpoint_map_T(grid, T_amb, int(e))
            xi_k[e] *= np.exp(-Ea / (K_B_EV * (T + dT))) / (T + dT) / (np.exp(-Ea / (K_B_EV * T)) / T)
    a = sample_map_amplitude(mc, sample)
    if a is not None:
        wire = (grid.res_is_via == 0) & (grid.layer[grid.res_a] == grid.layer[grid.res_b])
        if Ea_eV is None:
            raise ValueError("a thermal-map amplitude spread needs the material's activation energy")
        Ea = float(Ea_eV)
        for e in np.nonzero(wire)[0]:
            T = thermal.midpoint_map_T(grid, T_amb, int(e))
            Ta = T_amb + a * (T - T_amb)
            xi_k[e] *= np.exp(-Ea / (K_B_EV * Ta)) / Ta / (np.exp(-Ea / (K_B_EV * T)) / T)
    return xi_k, lognormal_xi(mc["seed"], sample, grid.n_res, 1, mc["cov_scrit"])


def sample_map_amplitude(mc, sample):
    """The sample's thermal-map amplitude a (param 6, counter index 0): a
    unit-mean lognormal with CoV cov_map scaling the map's rise above the
    ambient, T_a = T_amb + a (T - T_amb).  Each wire segment's diffusivity
    takes the Arrhenius ratio at its midpoint map temperature (sample_xi);
    each edge's thermomigration drive (Q/(Omega T)) dT/dx that of the scaled
    field (the C oracle, from a).  None without the spread."""
    cov = float(mc.get("cov_map", 0.0)) if mc else 0.0
    if cov <= 0:
        return None
    return float(lognormal_xi(mc["seed"], sample, 1, 6, cov)[0])


def sample_inputs(grid, mc, sample):
    """The sampled network of one sample (Sec. IV-F: any input stamped into
    the per-sample netlist): resistivity multipliers per wire segment (param
    2; vias keep their resistance) and sink currents scaled per node by the
    loading multipliers (param 3).  Returns (xi_r or None, R0, sinks)."""
    R0 = grid.res_R0.astype(np.float64)
    sinks = None if grid.sink_I is None else np.asarray(grid.sink_I, np.float64)
    xi_r = None
    if mc is not None and mc.get("cov_rho", 0.0) > 0:
        wire = (grid.res_is_via == 0) & (grid.layer[grid.res_a] == grid.layer[grid.res_b])
        xi_r = np.where(wire, lognormal_xi(mc["seed"], sample, grid.n_res, 2, mc["cov_rho"]), 1.0)
        R0 = R0 * xi_r
    if mc is not None and mc.get("cov_load", 0.0) > 0 and grid.seg_j is None:
        sinks = sinks * lognormal_xi(mc["seed"], sample, grid.n_nodes, 3, mc["cov_load"])
    return xi_r, R0, sinks


def run_sample(grid, mat, run, mc=None, sample=0, topo=None, keep_sim=False, max_outer=None):
    """Screen -> (BE steps, void/dR, IR re-solve)* -> TTF for one sample.

    Returns a dict with ttf (NaN when censored), failed, outer_idx,
    init_drop, final_drop, failed_segs, n_nucleated_trees, events, sigma."""
    N = int(run["intervals_per_seg"])
    topo = topo or topology(grid, N)
    xi_k, xi_s = sample_xi(grid, mc, sample, float(run.get("T_ambient", 300.0)), mat["Ea_eV"])
    xi_r, R0, sinks = sample_inputs(grid, mc, sample)
    trees_only = grid.seg_j is not None
    gs = grid
    if not trees_only:
        gs = dataclasses.replace(grid, sink_I=sinks)        # this sample's loading
        u, I, j, d0 = ir_solve(gs, R0)
    T_stress = None
    if run.get("joule", 0):
        # one-time thermal pre-pass with the currents of the nominal network
        if trees_only:
            j_nom = grid.seg_j
        elif not (mc is not None and (mc.get("cov_rho", 0.0) > 0 or mc.get("cov_load", 0.0) > 0)):
            j_nom = j
        else:
            j_nom = ir_solve(grid, grid.res_R0.astype(np.float64))[2]
        T_stress = thermal.node_temperatures(grid, mat, float(run.get("T_ambient", 300.0)), topo, j_nom)
    sim = SampleSim(grid, mat, run, topo, xi_k, xi_s, T_stress=T_stress, xi_r=xi_r,
                    map_a=sample_map_amplitude(mc, sample))
    n_steps, K = int(run["n_steps"]), int(run["ir_every"])
    res = dict(sample=sample)
    # reduced (extended rational Krylov) stepping of long chains (Sec. IV-E)
    kq = int(run.get("krylov_q", 0))
    keta = float(run.get("krylov_eta", 0.0)) or 1.0
    bases = {}
    active = np.ones(topo.n_trees, np.uint8)

    def step_interval(nst, step0, dt):
        if kq > 0:
            krylov.interval(sim, topo, grid, bases, active, nst, step0, dt, kq, keta)
        else:
            sim.steps(nst, step0)
    if trees_only:
        sim.set_j(grid.seg_j)
        if run.get("screen", 0):
            tm, sm, _ = sim.screen()
            sim.set_active(tm)
            active[:] = tm
            res["tree_mortal"], res["seg_mortal"] = tm, sm
        step_interval(n_steps, 0, float(run["dt"]))
        res.update(ttf=float("nan"), failed=0, outer_idx=0, init_drop=float("nan"),
                   final_drop=float("nan"))
    else:
        sim.set_j(j)
        res["init_drop"] = d0
        res["u0"] = u
        if run.get("screen", 0):
            tm, sm, _ = sim.screen()
            sim.set_active(tm)
            active[:] = tm
            res["tree_mortal"], res["seg_mortal"] = tm, sm
        fail = float(run["fail_frac"])
        seg_prev = sim.seg_state()                   # the conductances of the last IR solve
        # time grid: interval k (ir_every steps) steps with dt * dt_growth^k
        growth = float(run.get("dt_growth", 0.0)) or 1.0
        t_now = 0.0
        t_prev, d_prev = 0.0, d0
        done = 0
        res.update(ttf=float("nan"), failed=0, outer_idx=0, final_drop=d0)
        drops = [d0]
        if d0 >= fail:
            res.update(ttf=0.0, failed=1)
        else:
            k = 0
            # adaptive grid (dt_adapt > 0): K steps of dt 2^m per interval, m
            # back to 0 after an interval in which a void nucleated and one
            # level up (to dt_adapt) after one without; the last interval's
            # steps shortened to end at the horizon n_steps dt
            amax = int(run.get("dt_adapt", 0))
            horizon = n_steps * float(run["dt"])
            m = 0
            times = []
            while (t_now < horizon * (1.0 - 1e-12)) if amax > 0 else (done < n_steps):
                if max_outer is not None and k >= max_outer:
                    break
                dt_k = float(run["dt"]) * growth ** k
                nst = min(K, n_steps - done)
                if amax > 0:
                    dt_k = math.ldexp(float(run["dt"]), m)
                    rem = horizon - t_now
                    nst = max(1, int(min(K, math.ceil(rem / dt_k - 1e-9))))
                    if nst * dt_k > rem:
                        dt_k = rem / nst
                k += 1
                n_ev = lib().ora_n_events(sim._h)
                sim.set_dt(dt_k)
                step_interval(nst, done, dt_k)
                if amax > 0:
                    m = 0 if lib().ora_n_events(sim._h) > n_ev else min(m + 1, amax)
                done += nst
                t_now += nst * dt_k
                times.append(t_now)
                dR, op = sim.seg_state()
                if np.any(dR != seg_prev[0]) or np.any(op != seg_prev[1]):
                    bases.clear()                       # new conductances: a new drive
                seg_prev = (dR.copy(), op.copy())
                u, I, j, dk = ir_solve(gs, R0 + dR, op)
                drops.append(dk)
                t = t_now
                res["final_drop"] = dk
                res["outer_idx"] = k
                if dk >= fail:
                    res["ttf"] = t_prev + (fail - d_prev) / (dk - d_prev) * (t - t_prev)
                    res["failed"] = 1
                    break
                sim.set_j(j)
                t_prev, d_prev = t, dk
        res["drops"] = np.array(drops)
        res["times"] = np.array(times) if d0 < fail else np.zeros(0)
        res["u"] = u
    dR, op = sim.seg_state()
    res["dR"], res["open"] = dR, op
    res["failed_segs"] = np.nonzero((dR > 0) | (op != 0))[0].astype(np.int32)
    ev = sim.events()
    res["events"] = ev
    res["n_nucleated_trees"] = int(np.unique(ev[:, 0]).size) if ev.size else 0
    res["sigma"] = sim.sigma()
    res["voids"] = sim.voids()
    res["n_suppressed"] = sim.n_suppressed()
    if keep_sim:
        res["sim"] = sim
    return res


def mc_summary(results):
    """Failed/censored counts and mean, sd, CoV over the uncensored TTFs
    (Sec. V-D statistics)."""
    ttf = np.array([r["ttf"] for r in results if r["failed"]])
    n_fail = int(ttf.size)
    out = dict(n_fail=n_fail, n_censored=len(results) - n_fail)
    if n_fail:
        out["mean"] = float(ttf.mean())
        out["sd"] = float(ttf.std(ddof=1)) if n_fail > 1 else 0.0
        out["cov"] = out["sd"] / out["mean"] if out["mean"] > 0 else float("nan")
    return out
