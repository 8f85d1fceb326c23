"""ctypes binding of libem.so (the C ABI declared in include/em.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory (its caching allocator, through
the em_allocator hook) and the stream.  Loading fails loudly if the library
has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libem.so")

EM_OK, EM_ERR_ARG, EM_ERR_OOM, EM_ERR_HIP, EM_ERR_NOCONV, EM_ERR_STATE, EM_ERR_OVERFLOW = range(7)
STATUS_NAMES = {0: "EM_OK", 1: "EM_ERR_ARG", 2: "EM_ERR_OOM", 3: "EM_ERR_HIP", 4: "EM_ERR_NOCONV",
                5: "EM_ERR_STATE", 6: "EM_ERR_OVERFLOW"}

# Every entry point declared in include/em.h.
API = ["em_batch_create", "em_batch_destroy", "em_get_info", "em_last_error", "em_ir_solve",
       "em_screen", "em_stress_step", "em_run_to_ttf", "em_get_topology", "em_get_stress",
       "em_set_stress", "em_get_voltages", "em_get_seg_j", "em_get_seg_state", "em_set_seg_state", "em_get_node_state",
       "em_get_events", "em_get_voids", "em_get_screen", "em_inject_void", "em_get_xi",
       "em_reset", "em_mlp_create", "em_mlp_destroy", "em_mlp_last_error", "em_mlp_num_params",
       "em_mlp_set_params", "em_mlp_get_params", "em_mlp_forward", "em_mlp_grad",
       "em_mlp_train_step", "em_features", "em_surrogate_screen", "em_get_surrogate",
       "em_first_nucleation", "em_get_failed_segments", "em_snapshot", "em_restore", "em_autotune",
       "em_mlp_forward_noalloc", "em_mlp_noalloc_max_rows"]


# Thermal block used when a material dict leaves it out (only read with joule=1):
# k_cu, k_ILD in W/(m K), t_ILD in m.
THERMAL_DEFAULTS = {"k_cu": 400.0, "k_ild": 1.4, "t_ild": 0.2e-6}
N_FEAT = 16        # learned-screen features per (tree, sample)


class EmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_nodes", C.c_int32), ("xy", C.c_void_p),
                ("layer", C.c_void_p), ("n_res", C.c_int32), ("res_a", C.c_void_p),
                ("res_b", C.c_void_p), ("res_len", C.c_void_p), ("res_w", C.c_void_p),
                ("res_h", C.c_void_p), ("res_is_via", C.c_void_p), ("res_R0", C.c_void_p),
                ("n_pads", C.c_int32), ("pad_node", C.c_void_p), ("vdd", C.c_double),
                ("sink_I", C.c_void_p), ("node_T", C.c_void_p), ("tmap_nx", C.c_int32),
                ("tmap_ny", C.c_int32), ("tmap_x0", C.c_double), ("tmap_y0", C.c_double),
                ("tmap_dx", C.c_double), ("tmap_dy", C.c_double), ("tmap", C.c_void_p),
                ("seg_j", C.c_void_p)]


class Material(C.Structure):
    _fields_ = [("struct_size", C.c_uint32)] + [(k, C.c_double) for k in (
        "B", "Omega", "Z", "rho_cu", "Ea_eV", "D0", "sigma_crit", "Q_eV", "sigma_T", "delta",
        "rho_ta", "h_ta", "k_cu", "k_ild", "t_ild")]


class RunParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("intervals_per_seg", C.c_int32), ("dt", C.c_double),
                ("n_steps", C.c_int32), ("ir_every", C.c_int32), ("fail_frac", C.c_double),
                ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int32), ("prec", C.c_int32),
                ("screen", C.c_int32), ("max_voids_per_tree", C.c_int32), ("T_ambient", C.c_double),
                ("stepper", C.c_int32), ("ir_precond", C.c_int32), ("ir_launch", C.c_int32),
                ("chain_wg", C.c_int32), ("chain_occ", C.c_int32), ("joule", C.c_int32),
                ("dt_growth", C.c_double), ("chain_m", C.c_int32), ("guard_band", C.c_double),
                ("guard_ttf", C.c_double), ("amg_alpha", C.c_double), ("ss_tol", C.c_double),
                ("krylov_q", C.c_int32), ("krylov_eta", C.c_double), ("dt_adapt", C.c_int32)]


class MCParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_samples", C.c_int32), ("seed", C.c_uint64),
                ("cov_kappa", C.c_double), ("cov_scrit", C.c_double), ("cov_rho", C.c_double),
                ("cov_load", C.c_double), ("sd_ea_eV", C.c_double), ("sd_T_K", C.c_double),
                ("sample_ids", C.c_void_p), ("cov_map", C.c_double)]


class TTFResult(C.Structure):
    _fields_ = [("ttf_s", C.c_double), ("final_drop", C.c_double), ("init_drop", C.c_double),
                ("failed", C.c_int32), ("outer_idx", C.c_int32), ("n_nucleated_trees", C.c_int32),
                ("n_failed_segs", C.c_int32), ("redecided", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n_trees", C.c_int32), ("n_stress", C.c_int32), ("n_samples", C.c_int32),
                ("n_nodes", C.c_int32), ("n_res", C.c_int32), ("max_tree_nodes", C.c_int32),
                ("prec", C.c_int32), ("trees_only", C.c_int32), ("n_events", C.c_int64),
                ("cg_iters_last", C.c_int32), ("n_outer_done", C.c_int32),
                ("node_steps", C.c_int64), ("step_launches", C.c_int64),
                ("step_kernel_ms", C.c_double), ("cg_iters_total", C.c_int64), ("ir_ms", C.c_double),
                ("n_deferred", C.c_int64), ("n_activated", C.c_int64), ("n_late", C.c_int64),
                ("n_violations", C.c_int64),
                ("surrogate_ms", C.c_double), ("ir_sys_nodes", C.c_int32), ("ir_sys_edges", C.c_int32),
                ("cg_sample_iters", C.c_int64), ("chain_m", C.c_int32), ("chain_wg", C.c_int32),
                ("n_chain_wg", C.c_int32), ("n_redecided", C.c_int32), ("n_void_capped", C.c_int64),
                ("n_screen_rerun", C.c_int32), ("n_ss_skipped", C.c_int64), ("n_ss_woken", C.c_int64),
                ("n_krylov_bases", C.c_int64), ("n_krylov_intervals", C.c_int64),
                ("n_krylov_fallbacks", C.c_int64), ("krylov_node_steps", C.c_int64)]


class TuneInfo(C.Structure):
    _fields_ = [("chain_wg", C.c_int32), ("chain_occ", C.c_int32), ("ir_launch", C.c_int32),
                ("n_wg", C.c_int32), ("wg", C.c_int32 * 12), ("occ", C.c_int32 * 12),
                ("wg_ms", C.c_double * 12), ("amg_alpha", C.c_double), ("alpha_ms", C.c_double * 3),
                ("ir_ms", C.c_double * 3)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


_lib = None
_live = weakref.WeakSet()        # batches and models still open


@atexit.register
def _close_all():
    """Release library objects before the interpreter tears down the modules
    their allocator callbacks use."""
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def lib():
    """Load libem.so; raises if it was not built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(or python -m paper_2604_10743_amd.build) first")
        L = C.CDLL(LIB_PATH)
        for name in API:
            getattr(L, name).restype = C.c_int
        for name in ("em_last_error", "em_mlp_last_error"):
            getattr(L, name).restype = C.c_char_p
            getattr(L, name).argtypes = [C.c_void_p]
        L.em_mlp_train_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                        C.c_void_p]
        L.em_surrogate_screen.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
        L.em_snapshot.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.em_restore.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _pint(a):
    return None if a is None else a.ctypes.data


class Batch:
    """One batch of (tree, sample) instances on the current GPU."""

    def __init__(self, grid, mat: dict, run: dict, mc: dict | None = None, stream=None,
                 torch_alloc: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the EM library runs only on the device")
        self._torch = torch
        L = lib()
        self._keep = []

        def keep(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a
        g = GridDesc()
        g.struct_size = C.sizeof(GridDesc)
        g.n_nodes = grid.n_nodes
        g.xy = _pint(keep(grid.xy, np.float64))
        g.layer = _pint(keep(grid.layer, np.int32))
        g.n_res = grid.n_res
        g.res_a = _pint(keep(grid.res_a, np.int32)); g.res_b = _pint(keep(grid.res_b, np.int32))
        g.res_len = _pint(keep(grid.res_len, np.float64)); g.res_w = _pint(keep(grid.res_w, np.float64))
        g.res_h = _pint(keep(grid.res_h, np.float64))
        g.res_is_via = _pint(keep(grid.res_is_via, np.uint8))
        g.res_R0 = _pint(keep(grid.res_R0, np.float64))
        g.n_pads = int(grid.pad_node.size)
        g.pad_node = _pint(keep(grid.pad_node, np.int32)) if grid.pad_node.size else None
        g.vdd = float(grid.vdd)
        g.sink_I = _pint(keep(grid.sink_I, np.float64))
        g.node_T = _pint(keep(grid.node_T, np.float64))
        if grid.tmap is not None:
            tm = keep(grid.tmap, np.float64)
            g.tmap = _pint(tm); g.tmap_ny, g.tmap_nx = tm.shape
            g.tmap_x0, g.tmap_y0 = grid.tmap_x0, grid.tmap_y0
            g.tmap_dx, g.tmap_dy = grid.tmap_dx, grid.tmap_dy
        g.seg_j = _pint(keep(grid.seg_j, np.float64))
        m = Material(struct_size=C.sizeof(Material), **{k: float(mat[k]) for k in (
            "B", "Omega", "Z", "rho_cu", "Ea_eV", "D0", "sigma_crit", "Q_eV", "sigma_T", "delta",
            "rho_ta", "h_ta")}, **{k: float(mat.get(k, v)) for k, v in THERMAL_DEFAULTS.items()})
        r = RunParams(struct_size=C.sizeof(RunParams),
                      intervals_per_seg=int(run["intervals_per_seg"]), dt=float(run["dt"]),
                      n_steps=int(run["n_steps"]), ir_every=int(run["ir_every"]),
                      fail_frac=float(run["fail_frac"]), cg_rtol=float(run["cg_rtol"]),
                      cg_max_iter=int(run["cg_max_iter"]), prec=int(run["prec"]),
                      screen=int(run["screen"]), max_voids_per_tree=int(run["max_voids_per_tree"]),
                      T_ambient=float(run["T_ambient"]), stepper=int(run.get("stepper", 0)),
                      ir_precond=int(run.get("ir_precond", 2)),
                      ir_launch=int(run.get("ir_launch", 0)), chain_wg=int(run.get("chain_wg", 0)),
                      chain_occ=int(run.get("chain_occ", 0)),
                      joule=int(run.get("joule", 0)), dt_growth=float(run.get("dt_growth", 0.0)),
                      chain_m=int(run.get("chain_m", 0)),
                      guard_band=float(run.get("guard_band", 0.0)),
                      guard_ttf=float(run.get("guard_ttf", 0.0)),
                      amg_alpha=float(run.get("amg_alpha", 0.0)),
                      ss_tol=float(run.get("ss_tol", 0.0)),
                      krylov_q=int(run.get("krylov_q", 0)), krylov_eta=float(run.get("krylov_eta", 0.0)),
                      dt_adapt=int(run.get("dt_adapt", 0)))
        mcp = None
        if mc is not None:
            mcp = MCParams(struct_size=C.sizeof(MCParams), n_samples=int(mc["n_samples"]),
                           seed=int(mc["seed"]), cov_kappa=float(mc["cov_kappa"]),
                           cov_scrit=float(mc["cov_scrit"]), cov_rho=float(mc.get("cov_rho", 0.0)),
                           cov_load=float(mc.get("cov_load", 0.0)), sd_ea_eV=float(mc.get("sd_ea_eV", 0.0)),
                           sd_T_K=float(mc.get("sd_T_K", 0.0)),
                           sample_ids=_pint(keep(mc.get("sample_ids"), np.int32)),
                           cov_map=float(mc.get("cov_map", 0.0)))
        self._alloc = None
        if torch_alloc:
            dev = torch.cuda.current_device()
            st = torch.cuda.current_stream()
            _alloc_fn = torch.cuda.caching_allocator_alloc
            _delete_fn = torch.cuda.caching_allocator_delete

            def _a(nbytes, ctx):
                return _alloc_fn(int(nbytes), dev, st)

            def _f(ptr, ctx):
                _delete_fn(int(ptr))
            self._alloc_fns = (ALLOC_FN(_a), FREE_FN(_f))
            self._alloc = Allocator(self._alloc_fns[0], self._alloc_fns[1], None)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self._h = C.c_void_p()
        rc = L.em_batch_create(C.byref(g), C.byref(m), C.byref(r),
                               C.byref(mcp) if mcp is not None else None,
                               C.byref(self._alloc) if self._alloc is not None else None,
                               C.c_void_p(stream), C.byref(self._h))
        if rc != EM_OK:
            msg = L.em_last_error(self._h).decode() if self._h else ""
            L.em_batch_destroy(self._h)
            self._h = None
            raise EmError(rc, msg)
        _live.add(self)
        self.grid = grid
        self.S = int(mc["n_samples"]) if mc else 1
        inf = self.info()
        self.n_trees, self.n_stress = inf["n_trees"], inf["n_stress"]
        self.n_res, self.n_nodes = grid.n_res, grid.n_nodes

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().em_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != EM_OK:
            raise EmError(rc, lib().em_last_error(self._h).decode())

    # -- entry points -----------------------------------------------------
    def info(self) -> dict:
        i = Info()
        self._chk(lib().em_get_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def ir_solve(self) -> np.ndarray:
        d = np.zeros(self.S)
        self._chk(lib().em_ir_solve(self._h, _ptr(d)))
        return d

    def screen(self) -> np.ndarray:
        out = np.zeros((self.S, self.n_trees), np.uint8)
        self._chk(lib().em_screen(self._h, _ptr(out)))
        return out

    def stress_step(self, n: int) -> int:
        ne = C.c_int32()
        self._chk(lib().em_stress_step(self._h, C.c_int32(n), C.byref(ne)))
        return ne.value

    def reset(self):
        self._chk(lib().em_reset(self._h))

    def run_to_ttf(self) -> list:
        res = (TTFResult * self.S)()
        self._chk(lib().em_run_to_ttf(self._h, res))
        return [{k: getattr(r, k) for k, _ in TTFResult._fields_} for r in res]

    # -- read-back ------------------------------------------------------------
    def topology(self) -> dict:
        t = dict(tree_off=np.zeros(self.n_trees + 1, np.int32),
                 **{k: np.zeros(self.n_stress, np.int32) for k in ("parent", "seg", "dir", "vert", "kpos")},
                 seg_tree=np.zeros(self.n_res, np.int32))
        self._chk(lib().em_get_topology(self._h, *[_ptr(t[k]) for k in (
            "tree_off", "parent", "seg", "dir", "vert", "kpos", "seg_tree")]))
        return t

    def stress(self, sample: int = 0) -> np.ndarray:
        s = np.zeros(self.n_stress)
        self._chk(lib().em_get_stress(self._h, C.c_int32(sample), _ptr(s)))
        return s

    def set_stress(self, sigma, sample: int = 0):
        s = np.ascontiguousarray(sigma, np.float64)
        self._chk(lib().em_set_stress(self._h, C.c_int32(sample), _ptr(s)))

    def voltages(self, sample: int = 0) -> np.ndarray:
        u = np.zeros(self.n_nodes)
        self._chk(lib().em_get_voltages(self._h, C.c_int32(sample), _ptr(u)))
        return u

    def seg_j(self, sample: int = 0) -> np.ndarray:
        j = np.zeros(self.n_res)
        self._chk(lib().em_get_seg_j(self._h, C.c_int32(sample), _ptr(j)))
        return j

    def seg_state(self, sample: int = 0):
        dR = np.zeros(self.n_res)
        op = np.zeros(self.n_res, np.uint8)
        self._chk(lib().em_get_seg_state(self._h, C.c_int32(sample), _ptr(dR), _ptr(op)))
        return dR, op

    def autotune(self, n_steps: int = 100) -> dict:
        t = TuneInfo()
        self._chk(lib().em_autotune(self._h, C.c_int32(n_steps), C.byref(t)))
        n = t.n_wg
        return {"chain_wg": t.chain_wg, "chain_occ": t.chain_occ, "ir_launch": t.ir_launch,
                "wg_ms": {int(t.wg[k]): float(t.wg_ms[k]) for k in range(n) if t.occ[k] == 1},
                "wg_ms_occ4": {int(t.wg[k]): float(t.wg_ms[k]) for k in range(n) if t.occ[k] == 4},
                "ir_ms": {1: float(t.ir_ms[0]), 3: float(t.ir_ms[1]), 2: float(t.ir_ms[2])},
                "amg_alpha": float(t.amg_alpha),
                "alpha_ms": {1.4: float(t.alpha_ms[0]), 1.8: float(t.alpha_ms[1]), 2.2: float(t.alpha_ms[2])}}

    def set_seg_state(self, sample: int, dR, open_):
        dR = np.ascontiguousarray(dR, np.float64)
        op = np.ascontiguousarray(open_, np.uint8)
        assert dR.shape == (self.n_res,) and op.shape == (self.n_res,)
        self._chk(lib().em_set_seg_state(self._h, C.c_int32(sample), _ptr(dR), _ptr(op)))

    def node_state(self, sample: int = 0):
        T = np.zeros(self.n_stress); V = np.zeros(self.n_stress); sc = np.zeros(self.n_stress)
        self._chk(lib().em_get_node_state(self._h, C.c_int32(sample), _ptr(T), _ptr(V), _ptr(sc)))
        return T, V, sc

    def events(self) -> np.ndarray:
        n_ev = self.info()["n_events"]
        cap = max(int(n_ev), 1)
        buf = np.zeros((cap, 5), np.int32)
        n = C.c_int32()
        self._chk(lib().em_get_events(self._h, _ptr(buf), C.c_int32(cap), C.byref(n)))
        return buf[:n.value]

    def voids(self, sample: int = 0):
        n = C.c_int32()
        self._chk(lib().em_get_voids(self._h, C.c_int32(sample), None, None, C.c_int32(0), C.byref(n)))
        cap = max(n.value, 1)
        iv = np.zeros((cap, 6), np.int32)
        dv = np.zeros((cap, 2))
        self._chk(lib().em_get_voids(self._h, C.c_int32(sample), _ptr(iv), _ptr(dv), C.c_int32(cap), C.byref(n)))
        return iv[:n.value], dv[:n.value]

    def screen_state(self, sample: int = 0):
        tm = np.zeros(self.n_trees, np.uint8)
        sm = np.zeros(self.n_res, np.uint8)
        ss = np.zeros(self.n_stress)
        self._chk(lib().em_get_screen(self._h, C.c_int32(sample), _ptr(tm), _ptr(sm), _ptr(ss)))
        return tm, sm, ss

    def inject_void(self, sample: int, tree: int, node: int):
        self._chk(lib().em_inject_void(self._h, C.c_int32(sample), C.c_int32(tree), C.c_int32(node)))

    def xi(self, sample: int = 0, param: int = 0) -> np.ndarray:
        x = np.zeros(self.info()["n_nodes"] if param == 3 else self.n_res)
        self._chk(lib().em_get_xi(self._h, C.c_int32(sample), C.c_int32(param), _ptr(x)))
        return x

    def failed_segments(self, sample: int = 0) -> np.ndarray:
        n = C.c_int32()
        self._chk(lib().em_get_failed_segments(self._h, C.c_int32(sample), None, C.c_int32(0), C.byref(n)))
        idx = np.zeros(max(n.value, 1), np.int32)
        self._chk(lib().em_get_failed_segments(self._h, C.c_int32(sample), _ptr(idx), C.c_int32(idx.size),
                                               C.byref(n)))
        return idx[:n.value]

    def snapshot(self) -> bytes:
        used = C.c_size_t()
        self._chk(lib().em_snapshot(self._h, None, 0, C.byref(used)))
        buf = (C.c_uint8 * used.value)()
        self._chk(lib().em_snapshot(self._h, buf, used.value, C.byref(used)))
        return bytes(buf)

    def restore(self, snap: bytes):
        buf = (C.c_uint8 * len(snap)).from_buffer_copy(snap)
        self._chk(lib().em_restore(self._h, buf, len(snap)))

    # -- learned screen ------------------------------------------------------
    def features(self):
        """[n_trees * n_samples][N_FEAT] float32 device tensor (row tree * S + sample)."""
        X = self._torch.empty((self.n_trees * self.S, N_FEAT), dtype=self._torch.float32, device="cuda")
        self._chk(lib().em_features(self._h, C.c_void_p(X.data_ptr())))
        return X

    def surrogate_screen(self, mlp, margin: float = 2.0) -> int:
        nd = C.c_int64()
        self._chk(lib().em_surrogate_screen(self._h, mlp._h if mlp is not None else None,
                                            C.c_double(margin), C.byref(nd)))
        self._mlp_ref = mlp
        return nd.value

    def surrogate(self, sample: int = 0):
        y = np.zeros(self.n_trees, np.float32)
        df = np.zeros(self.n_trees, np.uint8)
        self._chk(lib().em_get_surrogate(self._h, C.c_int32(sample), _ptr(y), _ptr(df)))
        return y, df

    def first_nucleation(self) -> np.ndarray:
        out = np.zeros((self.S, self.n_trees), np.int32)
        self._chk(lib().em_first_nucleation(self._h, _ptr(out)))
        return out


class MLP:
    """The learned-screen model (parameters, Adam state, activations on the GPU)."""

    def __init__(self, params=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the EM library runs only on the device")
        self._torch = torch
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._h = C.c_void_p()
        rc = L.em_mlp_create(C.c_void_p(stream), C.byref(self._h))
        if rc != EM_OK:
            L.em_mlp_destroy(self._h)
            self._h = None
            raise EmError(rc, "em_mlp_create failed")
        _live.add(self)
        self.n_params = L.em_mlp_num_params()
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "_h", None):
            lib().em_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != EM_OK:
            raise EmError(rc, lib().em_mlp_last_error(self._h).decode())

    def set_params(self, p):
        a = np.ascontiguousarray(p, np.float32)
        self._chk(lib().em_mlp_set_params(self._h, _ptr(a), C.c_int32(a.size)))

    def params(self) -> np.ndarray:
        a = np.zeros(self.n_params, np.float32)
        self._chk(lib().em_mlp_get_params(self._h, _ptr(a), C.c_int32(a.size)))
        return a

    def _dev(self, x):
        t = self._torch.as_tensor(x, dtype=self._torch.float32, device="cuda").contiguous()
        return t

    def forward(self, X):
        X = self._dev(X)
        n = X.shape[0]
        y = self._torch.empty(n, dtype=self._torch.float32, device="cuda")
        self._chk(lib().em_mlp_forward(self._h, C.c_void_p(X.data_ptr()), C.c_int32(n),
                                       C.c_void_p(y.data_ptr())))
        return y

    def forward_noalloc(self, X, y):
        """y[:n] = model(X) through the allocation-free entry point: X [n][N_FEAT]
        and y [>= n] are caller-owned float32 device tensors; the call
        allocates nothing and does not synchronise the model's stream."""
        n = int(X.shape[0])
        assert X.is_cuda and y.is_cuda and X.dtype == y.dtype == self._torch.float32 and y.numel() >= n
        assert X.is_contiguous() and y.is_contiguous() and tuple(X.shape[1:]) == (N_FEAT,)
        self._chk(lib().em_mlp_forward_noalloc(self._h, C.c_void_p(X.data_ptr()), C.c_int32(n),
                                               C.c_void_p(y.data_ptr())))

    @staticmethod
    def noalloc_max_rows() -> int:
        return int(lib().em_mlp_noalloc_max_rows())

    def grad(self, X, t):
        X, t = self._dev(X), self._dev(t)
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_float()
        self._chk(lib().em_mlp_grad(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(t.data_ptr()),
                                    C.c_int32(X.shape[0]), _ptr(g), C.byref(loss)))
        return loss.value, g

    def train_step(self, X, t, lr: float, want_loss: bool = False):
        """One Adam step on device tensors X [n][N_FEAT], t [n]."""
        loss = C.c_float()
        self._chk(lib().em_mlp_train_step(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(t.data_ptr()),
                                          C.c_int32(X.shape[0]), C.c_float(lr),
                                          C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
