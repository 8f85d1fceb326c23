"""Seeded synthetic power-grid inputs.

This module only *builds inputs*: node coordinates and layers, wire
resistors with their extracted geometry and nominal resistance, pads, sink
currents and thermal rasters.  It holds none of the stress, IR-drop, void or
Monte Carlo arithmetic of the method; both the HIP path and the CPU oracle
consume what it returns.  Every generator is deterministic in its seed.

Units are SI throughout (m, A, ohm, K).

The paper's own designs are SAED32 power grids extracted from a commercial
place-and-route flow (Section V); they are not available, so these grids
stand in for them with the shape statistics the paper reports (Table III:
tens to hundreds of trees, up to ~10^4 stress nodes per tree, initial worst
IR-drop a few percent of the supply; Section V-A: 0.95-1.2 V supply, base
temperature around 353 K, hotspots tens of kelvin above it).
"""
from __future__ import annotations

import copy
import dataclasses
from typing import Optional

import numpy as np

RHO_CU = 2.25e-8          # ohm*m, copper resistivity used for extraction
UM = 1e-6


@dataclasses.dataclass
class Grid:
    """An extracted P/G netlist plus its optional thermal raster.

    Resistors with ``res_is_via`` set (or joining two different layers) are
    vias; all others are wire segments on one layer.  ``seg_j`` (optional)
    prescribes a current density per resistor and switches the run to the
    trees-only mode (no IR coupling).
    """

    xy: np.ndarray            # (n_nodes, 2) float64, m
    layer: np.ndarray         # (n_nodes,) int32
    res_a: np.ndarray         # (n_res,) int32
    res_b: np.ndarray         # (n_res,) int32
    res_len: np.ndarray       # (n_res,) float64, m
    res_w: np.ndarray         # (n_res,) float64, m
    res_h: np.ndarray         # (n_res,) float64, m
    res_is_via: np.ndarray    # (n_res,) uint8
    res_R0: np.ndarray        # (n_res,) float64, ohm
    pad_node: np.ndarray      # (n_pads,) int32
    vdd: float
    sink_I: np.ndarray        # (n_nodes,) float64, A drawn at each node
    node_T: Optional[np.ndarray] = None     # (n_nodes,) K
    tmap: Optional[np.ndarray] = None       # (ny, nx) K raster, row-major
    tmap_x0: float = 0.0
    tmap_y0: float = 0.0
    tmap_dx: float = 1.0
    tmap_dy: float = 1.0
    seg_j: Optional[np.ndarray] = None      # (n_res,) A/m^2 along a->b
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_res(self) -> int:
        return int(self.res_a.shape[0])


def default_material() -> dict:
    """Cu constants of the tiny trees workload plus the values the paper
    leaves open (heat of transport, residual stress, void-interface
    thickness, Ta liner, the thermal block of the Joule pre-pass: bulk Cu and
    SiO2 conductivities, 0.2 um dielectric): SI units, activation energies in
    eV."""
    return dict(B=28e9, Omega=1.18e-29, Z=1.0, rho_cu=RHO_CU, Ea_eV=0.85,
                D0=7.56e-5, sigma_crit=400e6, Q_eV=0.1, sigma_T=0.0,
                delta=1e-9, rho_ta=2e-7, h_ta=5e-9, k_cu=400.0, k_ild=1.4, t_ild=0.2e-6)


def default_run(**over) -> dict:
    """Numerics: 20 intervals per segment, 2000 backward-Euler steps over
    ten years (a year of 365.25 days), IR re-solve every 100 steps, failure
    at 10 % worst IR-drop; FP32 runs re-run in FP64 the samples whose worst
    drop comes within 0.05 % of the threshold, or whose TTF a drop error of
    that size could move by more than 5e-3 relative (guard band): the FP32
    drop error is below 1e-4 relative, a fifth of the band, so a TTF
    unflagged by the second rule moves by at most 1e-3.  PCG tolerance
    automatic (0): a relative residual of 1e-11 with FP64 stepping, 1e-8
    with FP32."""
    horizon = 10 * 365.25 * 86400.0
    r = dict(intervals_per_seg=20, n_steps=2000, dt=horizon / 2000, ir_every=100,
             fail_frac=0.10, cg_rtol=0.0, cg_max_iter=20000, prec=0, screen=1,
             max_voids_per_tree=4, T_ambient=378.0, joule=0, guard_band=5e-4, guard_ttf=5e-3)
    r.update(over)
    return r


def _wire_R(L, w, h):
    return RHO_CU * L / (w * h)


def _empty_i32():
    return np.zeros(0, np.int32)


# ----------------------------------------------------------------------------
# Straight standalone trees with prescribed currents (trees-only mode)
# ----------------------------------------------------------------------------
def straight_trees(seed: int = 1001, n_trees: int = 200, seg_range=(2, 8),
                   L_range=(5 * UM, 50 * UM), w_range=(0.1 * UM, 1.0 * UM),
                   H=0.2 * UM, j_range=(1e9, 5e10)) -> Grid:
    """Independent straight lines of S ~ U{seg_range} segments; each segment
    has its own length, width and signed current density."""
    rng = np.random.default_rng(seed)
    xs, ys, ra, rb, L, W = [], [], [], [], [], []
    base = 0
    for t in range(n_trees):
        S = int(rng.integers(seg_range[0], seg_range[1] + 1))
        lens = rng.uniform(L_range[0], L_range[1], S)
        x = np.concatenate([[0.0], np.cumsum(lens)])
        xs.append(x)
        ys.append(np.full(S + 1, t * 20 * UM))
        ra.append(base + np.arange(S))
        rb.append(base + np.arange(1, S + 1))
        L.append(lens)
        W.append(rng.uniform(w_range[0], w_range[1], S))
        base += S + 1
    n = base
    res_len = np.concatenate(L)
    res_w = np.concatenate(W)
    nr = res_len.size
    mag = rng.uniform(j_range[0], j_range[1], nr)
    sign = np.where(rng.random(nr) < 0.5, -1.0, 1.0)
    res_h = np.full(nr, H)
    return Grid(xy=np.stack([np.concatenate(xs), np.concatenate(ys)], 1),
                layer=np.ones(n, np.int32),
                res_a=np.concatenate(ra).astype(np.int32),
                res_b=np.concatenate(rb).astype(np.int32),
                res_len=res_len, res_w=res_w, res_h=res_h,
                res_is_via=np.zeros(nr, np.uint8),
                res_R0=_wire_R(res_len, res_w, res_h),
                pad_node=_empty_i32(), vdd=1.0, sink_I=np.zeros(n),
                seg_j=mag * sign, name=f"straight_trees_{n_trees}_s{seed}")


def random_branched_trees(seed: int, n_trees: int, n_vertices=(2, 10),
                          L_range=(2 * UM, 20 * UM), w_range=(0.2 * UM, 1.0 * UM),
                          H=0.2 * UM, j_range=(1e8, 5e10), planar_jitter=True) -> Grid:
    """Random trees from uniform Pruefer sequences (trees-only mode).

    Vertex indices are shuffled so that roots and DFS orders are not the
    trivial ones; resistor orientation (a->b) is random.  Geometry lengths
    are drawn independently of the coordinates (an extracted netlist gives
    lengths; the coordinates only place the nodes on a thermal raster).
    """
    rng = np.random.default_rng(seed)
    xy_all, ra, rb, L, W = [], [], [], [], []
    base = 0
    for t in range(n_trees):
        nv = int(rng.integers(n_vertices[0], n_vertices[1] + 1))
        if nv == 2:
            edges = [(0, 1)]
        else:
            prufer = rng.integers(0, nv, nv - 2)
            degree = np.ones(nv, np.int64)
            for v in prufer:
                degree[v] += 1
            edges = []
            for v in prufer:
                leaf = int(np.nonzero(degree == 1)[0][0])
                edges.append((leaf, int(v)))
                degree[leaf] -= 1
                degree[v] -= 1
            u, w = np.nonzero(degree == 1)[0]
            edges.append((int(u), int(w)))
        perm = rng.permutation(nv)
        pos = rng.uniform(0, 100 * UM, (nv, 2)) + np.array([0.0, t * 200 * UM])
        xy_all.append(pos)
        order = rng.permutation(len(edges))
        for k in order:
            a, b = edges[k]
            a, b = int(perm[a]), int(perm[b])
            if rng.random() < 0.5:
                a, b = b, a
            ra.append(base + a)
            rb.append(base + b)
            L.append(rng.uniform(*L_range))
            W.append(rng.uniform(*w_range))
        base += nv
    nr = len(ra)
    res_len = np.array(L)
    res_w = np.array(W)
    res_h = np.full(nr, H)
    mag = rng.uniform(j_range[0], j_range[1], nr)
    sign = np.where(rng.random(nr) < 0.5, -1.0, 1.0)
    return Grid(xy=np.concatenate(xy_all), layer=np.ones(base, np.int32),
                res_a=np.array(ra, np.int32), res_b=np.array(rb, np.int32),
                res_len=res_len, res_w=res_w, res_h=res_h,
                res_is_via=np.zeros(nr, np.uint8), res_R0=_wire_R(res_len, res_w, res_h),
                pad_node=_empty_i32(), vdd=1.0, sink_I=np.zeros(base),
                seg_j=mag * sign, name=f"branched_{n_trees}_s{seed}")


def comb_trees(seed: int, n_trees: int = 200, trunk=(20, 100), p_tooth: float = 0.7, tooth=(1, 4),
               p_stub: float = 0.3, stub=(1, 2), L_range=(5 * UM, 20 * UM), w_range=(0.2 * UM, 1.0 * UM),
               H=0.2 * UM, j_range=(1e9, 5e10)) -> Grid:
    """Branched standalone trees with prescribed currents (trees-only mode):
    a trunk of U{trunk} segments along x; at each inner trunk vertex, with
    probability p_tooth, a tooth of U{tooth} segments along +-y; at each
    tooth vertex, with probability p_stub, a stub of U{stub} segments along
    x.  Up to a few hundred branches and several thousand FD nodes per tree
    at 20 intervals per segment (the paper's largest trees have 29-218
    branches).  Each segment has its own length, width and signed current
    density."""
    rng = np.random.default_rng(seed)
    xy, ra, rb, L, W = [], [], [], [], []
    base = 0
    for t in range(n_trees):
        pts = [(0.0, t * 2000 * UM)]

        def add(frm, dx, dy):
            lq = float(rng.uniform(*L_range))
            x0, y0 = pts[frm]
            pts.append((x0 + dx * lq, y0 + dy * lq))
            v = len(pts) - 1
            a, b = (frm, v) if rng.random() < 0.5 else (v, frm)
            ra.append(base + a); rb.append(base + b)
            L.append(lq); W.append(float(rng.uniform(*w_range)))
            return v

        T = int(rng.integers(trunk[0], trunk[1] + 1))
        cur = 0
        trunk_v = [0]
        for _ in range(T):
            cur = add(cur, 1.0, 0.0)
            trunk_v.append(cur)
        for v in trunk_v[1:-1]:
            if rng.random() >= p_tooth:
                continue
            dy = 1.0 if rng.random() < 0.5 else -1.0
            c = v
            for _ in range(int(rng.integers(tooth[0], tooth[1] + 1))):
                c = add(c, 0.0, dy)
                if rng.random() < p_stub:
                    s = c
                    for _ in range(int(rng.integers(stub[0], stub[1] + 1))):
                        s = add(s, 0.3, 0.0)
        xy.extend(pts)
        base += len(pts)
    nr = len(ra)
    res_len = np.array(L)
    res_w = np.array(W)
    res_h = np.full(nr, H)
    mag = rng.uniform(j_range[0], j_range[1], nr)
    sign = np.where(rng.random(nr) < 0.5, -1.0, 1.0)
    return Grid(xy=np.array(xy), layer=np.ones(base, np.int32),
                res_a=np.array(ra, np.int32), res_b=np.array(rb, np.int32),
                res_len=res_len, res_w=res_w, res_h=res_h,
                res_is_via=np.zeros(nr, np.uint8), res_R0=_wire_R(res_len, res_w, res_h),
                pad_node=_empty_i32(), vdd=1.0, sink_I=np.zeros(base),
                seg_j=mag * sign, name=f"combs_{n_trees}_s{seed}")


# ----------------------------------------------------------------------------
# Thermal rasters
# ----------------------------------------------------------------------------
def gaussian_hotspot_map(seed: int, extent_x: float, extent_y: float, base_K: float,
                         n_spots: int, amp_range, sig_range, res: float = 1 * UM):
    """Base temperature plus Gaussian hotspots on a regular raster.

    Returns (tmap[ny, nx], x0, y0, dx, dy)."""
    rng = np.random.default_rng(seed)
    nx = int(np.ceil(extent_x / res)) + 1
    ny = int(np.ceil(extent_y / res)) + 1
    x = np.arange(nx) * res
    y = np.arange(ny) * res
    T = np.full((ny, nx), float(base_K))
    for _ in range(n_spots):
        A = rng.uniform(*amp_range)
        s = rng.uniform(*sig_range)
        cx = rng.uniform(0, extent_x)
        cy = rng.uniform(0, extent_y)
        gx = np.exp(-0.5 * ((x - cx) / s) ** 2)
        gy = np.exp(-0.5 * ((y - cy) / s) ** 2)
        T += A * np.outer(gy, gx)
    return T, 0.0, 0.0, res, res


# ----------------------------------------------------------------------------
# Two-layer meshes (M1 horizontal rows, M2 vertical columns)
# ----------------------------------------------------------------------------
def two_layer_mesh(seed: int = 1001, nr: int = 32, nc: int = 32,
                   spacing=(5 * UM, 50 * UM), w1=0.5 * UM, w2=1.0 * UM, H=0.2 * UM,
                   R_via=0.5, vdd=1.0, sink_mu=None, sink_sigma=0.5,
                   cut_m1=False, cut_seg=(2, 8), T_uniform: Optional[float] = 378.0,
                   pads: str = "corners") -> Grid:
    """Small two-layer mesh with a via at every crossing and 4 pads on M2
    (at the corners, or spread along the top edge with ``pads="edge"``).  Row/column spacings are drawn from U[spacing]; node sinks are
    lognormal on M1.  With ``cut_m1`` every M1 row is cut into straight
    trees of U{cut_seg} segments separated by single missing segments.

    The default sink median puts the initial worst IR-drop near 6 % of the
    supply for seed 1001 (uncut, corner pads): a constant fixed once for this
    geometry."""
    rng = np.random.default_rng(seed)
    dy = rng.uniform(spacing[0], spacing[1], nr - 1)
    dx = rng.uniform(spacing[0], spacing[1], nc - 1)
    yr = np.concatenate([[0.0], np.cumsum(dy)])
    xc = np.concatenate([[0.0], np.cumsum(dx)])
    n1 = nr * nc
    idx1 = np.arange(n1).reshape(nr, nc)           # M1 node ids
    idx2 = n1 + np.arange(n1).reshape(nr, nc)      # M2 node ids
    X, Y = np.meshgrid(xc, yr)
    xy = np.concatenate([np.stack([X.ravel(), Y.ravel()], 1)] * 2)
    layer = np.concatenate([np.ones(n1, np.int32), np.full(n1, 2, np.int32)])
    ra, rb, L, W, Hh, via = [], [], [], [], [], []
    # M1 rows
    for r in range(nr):
        keep = np.ones(nc - 1, bool)
        if cut_m1:
            c = 0
            while c < nc - 1:
                S = int(rng.integers(cut_seg[0], cut_seg[1] + 1))
                c += S
                if c < nc - 1:
                    keep[c] = False
                    c += 1
        for c in range(nc - 1):
            if keep[c]:
                ra.append(idx1[r, c]); rb.append(idx1[r, c + 1])
                L.append(dx[c]); W.append(w1); Hh.append(H); via.append(0)
    # M2 columns
    for c in range(nc):
        for r in range(nr - 1):
            ra.append(idx2[r, c]); rb.append(idx2[r + 1, c])
            L.append(dy[r]); W.append(w2); Hh.append(H); via.append(0)
    # vias
    for r in range(nr):
        for c in range(nc):
            ra.append(idx1[r, c]); rb.append(idx2[r, c])
            L.append(0.0); W.append(w1); Hh.append(H); via.append(1)
    ra = np.array(ra, np.int32); rb = np.array(rb, np.int32)
    L = np.array(L); W = np.array(W); Hh = np.array(Hh); via = np.array(via, np.uint8)
    R0 = np.where(via == 1, R_via, _wire_R(np.maximum(L, 1e-12), W, Hh))
    if pads == "corners":
        pads = np.array([idx2[0, 0], idx2[0, nc - 1], idx2[nr - 1, 0], idx2[nr - 1, nc - 1]], np.int32)
    else:       # four pads spread along the top edge (one-sided delivery)
        cols = [(2 * k + 1) * nc // 8 for k in range(4)]
        pads = np.array([idx2[nr - 1, c] for c in cols], np.int32)
    if sink_mu is None:
        sink_mu = np.log(32.7e-6)
    sink = np.zeros(2 * n1)
    sink[:n1] = np.exp(rng.normal(sink_mu, sink_sigma, n1))
    g = Grid(xy=xy, layer=layer, res_a=ra, res_b=rb, res_len=L, res_w=W, res_h=Hh,
             res_is_via=via, res_R0=R0, pad_node=pads, vdd=vdd, sink_I=sink,
             name=f"mesh{nr}x{nc}{'_cut' if cut_m1 else ''}_s{seed}")
    if T_uniform is not None:
        g.node_T = np.full(2 * n1, float(T_uniform))
    return g


def pg_grid(seed: int = 2001, n: int = 400, pitch=5 * UM, w1=0.5 * UM, w2=1.0 * UM,
            H=0.2 * UM, via_every=4, R_via=0.5, pad_lattice=8, vdd=1.2,
            sink_mu=np.log(50e-6), sink_sigma=0.5, sink_scale=0.0651,
            seg_range=(100, 399), base_K=330.0, n_spots=6, amp_range=(15.0, 60.0),
            sig_range=(30 * UM, 80 * UM), raster=1 * UM, thermal=True,
            n_cols: Optional[int] = None, col_seg_range=None) -> Grid:
    """Two-layer n x n P/G grid: M1 rows and M2 columns at a fixed pitch
    (n rows by ``n_cols`` columns when given; column spans then come from
    ``col_seg_range``).

    Every line is one tree cut to a random contiguous span of U{seg_range}
    segments.  A via joins M1 and M2 at every crossing on a row or column
    whose index is a multiple of ``via_every`` (so every line carries a via
    at least every ``via_every`` nodes and the two layers form one network);
    VDD pads sit on M2 at a pad_lattice x pad_lattice lattice (snapped onto
    the nearest existing M2 node of that column); components that reach no
    pad are removed; lognormal sinks sit on
    every M1 node, scaled by ``sink_scale`` (the stated 50 uA median on this
    geometry gives a worst initial drop above 100 % of the supply; the
    default scale puts it near 8.5 % of a 1.2 V supply, inside the 5-9 %
    the paper's failing designs start from).  The thermal raster is the base
    temperature plus Gaussian hotspots at ``raster`` resolution.
    """
    rng = np.random.default_rng(seed)
    nc = n if n_cols is None else int(n_cols)
    csr = seg_range if col_seg_range is None else col_seg_range
    nseg_r, nseg_c = nc - 1, n - 1          # segments of a full row / column
    span_r = rng.integers(seg_range[0], min(seg_range[1], nseg_r) + 1, n)
    off_r = np.array([rng.integers(0, nseg_r - s + 1) for s in span_r])
    span_c = rng.integers(csr[0], min(csr[1], nseg_c) + 1, nc)
    off_c = np.array([rng.integers(0, nseg_c - s + 1) for s in span_c])
    # node ids: allocate only existing nodes
    id1 = -np.ones((n, nc), np.int64)
    id2 = -np.ones((n, nc), np.int64)
    xy, layer = [], []
    cnt = 0
    for r in range(n):
        for c in range(off_r[r], off_r[r] + span_r[r] + 1):
            id1[r, c] = cnt; cnt += 1
            xy.append((c * pitch, r * pitch)); layer.append(1)
    for c in range(nc):
        for r in range(off_c[c], off_c[c] + span_c[c] + 1):
            id2[r, c] = cnt; cnt += 1
            xy.append((c * pitch, r * pitch)); layer.append(2)
    ra, rb, L, W, via = [], [], [], [], []
    for r in range(n):
        for c in range(off_r[r], off_r[r] + span_r[r]):
            ra.append(id1[r, c]); rb.append(id1[r, c + 1]); L.append(pitch); W.append(w1); via.append(0)
    for c in range(nc):
        for r in range(off_c[c], off_c[c] + span_c[c]):
            ra.append(id2[r, c]); rb.append(id2[r + 1, c]); L.append(pitch); W.append(w2); via.append(0)
    rr, cc = np.nonzero((id1 >= 0) & (id2 >= 0))
    sel = ((rr % via_every) == 0) | ((cc % via_every) == 0)
    for r, c in zip(rr[sel], cc[sel]):
        ra.append(id1[r, c]); rb.append(id2[r, c]); L.append(0.0); W.append(w1); via.append(1)
    ra = np.array(ra, np.int32); rb = np.array(rb, np.int32)
    L = np.array(L); W = np.array(W); via = np.array(via, np.uint8)
    Hh = np.full(L.size, H)
    R0 = np.where(via == 1, R_via, _wire_R(np.maximum(L, 1e-12), W, Hh))
    # pads on M2
    step, cstep = n // pad_lattice, nc // pad_lattice
    pads = []
    for a in range(pad_lattice):
        for b in range(pad_lattice):
            r = step // 2 + a * step
            c = cstep // 2 + b * cstep
            r = int(np.clip(r, off_c[c], off_c[c] + span_c[c]))
            pads.append(id2[r, c])
    pads = np.unique(np.array(pads, np.int32))
    # component labelling (plain union-find over all resistors) to keep the
    # nodal system non-singular: sinks only where a pad is reachable
    parent = np.arange(cnt)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for a, b in zip(ra, rb):
        fa, fb = find(a), find(b)
        if fa != fb:
            parent[fa] = fb
    roots = np.array([find(i) for i in range(cnt)])
    live_roots = set(roots[pads].tolist())
    live = np.array([rt in live_roots for rt in roots])
    # drop pad-less components entirely (nodes and their resistors)
    remap = -np.ones(cnt, np.int64)
    remap[live] = np.arange(int(live.sum()))
    keep_r = live[ra] & live[rb]
    ra = remap[ra[keep_r]].astype(np.int32); rb = remap[rb[keep_r]].astype(np.int32)
    L, W, Hh, via, R0 = L[keep_r], W[keep_r], Hh[keep_r], via[keep_r], R0[keep_r]
    pads = remap[pads].astype(np.int32)
    xy = np.array(xy, float)[live]
    layer = np.array(layer, np.int32)[live]
    cnt = int(live.sum())
    sink = np.zeros(cnt)
    m1 = layer == 1
    sink[m1] = sink_scale * np.exp(rng.normal(sink_mu, sink_sigma, int(m1.sum())))
    g = Grid(xy=xy, layer=layer, res_a=ra, res_b=rb, res_len=L, res_w=W,
             res_h=Hh, res_is_via=via, res_R0=R0, pad_node=pads, vdd=vdd, sink_I=sink,
             name=f"pg{n}x{nc}_s{seed}")
    if thermal:
        tm, x0, y0, dxr, dyr = gaussian_hotspot_map(seed + 7, (nc - 1) * pitch, (n - 1) * pitch,
                                                   base_K, n_spots, amp_range, sig_range, raster)
        g.tmap, g.tmap_x0, g.tmap_y0, g.tmap_dx, g.tmap_dy = tm, x0, y0, dxr, dyr
    else:
        g.node_T = np.full(cnt, base_K)
    return g


def _cut_runs(rng, n_seg: int, span) -> np.ndarray:
    """Keep-mask over a line of n_seg segments cut into pieces of U{span}
    segments separated by single missing segments."""
    keep = np.ones(n_seg, bool)
    c = 0
    while c < n_seg:
        c += int(rng.integers(span[0], span[1] + 1))
        if c < n_seg:
            keep[c] = False
            c += 1
    return keep


FULLCHIP_SINK_SCALE = 3.23


def fullchip_grid(seed: int = 5001, n: int = 2000, pitch=1 * UM, e12: int = 4, e34: int = 20,
                  w=(0.4 * UM, 0.6 * UM, 0.6 * UM, 1.0 * UM), H=(0.2 * UM, 0.2 * UM, 0.2 * UM, 0.2 * UM),
                  cut12=(2, 8), cut34=(40, 99), R_via=(0.5, 0.5, 0.25), pad_lattice=4, via12_every=1,
                  via23_every=1, via34_every=4, vdd=1.0,
                  sink_mu=np.log(1e-6), sink_sigma=0.5, sink_scale=1.0, base_K=340.0, n_spots=12,
                  amp_range=(20.0, 70.0), sig_range=(60 * UM, 200 * UM), raster=4 * UM) -> Grid:
    """Four-layer P/G grid on an n x n routing grid of ``pitch`` tracks (a
    2 mm die at the defaults): M1 rows and M2 columns on every e12-th track,
    M3 rows and M4 columns on every e34-th track, each with a node at every
    crossing of its own layer pair.  M1 and M2 stripes are cut into short
    trees of U{cut12} segments, M3 and M4 stripes into lines of U{cut34}
    segments, by single missing segments.  Vias: M1-M2 at the crossings on
    a row or column index that is a multiple of via12_every; M2-M3 at the M3
    nodes on a row or column index that is a multiple of via23_every; M3-M4
    at the M3 nodes whose row and column indices are both multiples of
    via34_every.  VDD pads on M4 at a
    pad_lattice x pad_lattice lattice; lognormal sinks on every M1 node;
    thermal raster = base + n_spots Gaussian hotspots.  Built with array
    operations (about 5e5 nodes and 7e5 resistors at the defaults)."""
    rng = np.random.default_rng(seed)
    m, m3 = n // e12, n // e34
    r34 = e34 // e12                               # M2 nodes per M3 node spacing
    n12, n34 = m * m, m3 * m3
    base = np.array([0, n12, 2 * n12, 2 * n12 + n34, 2 * n12 + 2 * n34])
    ii, jj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    II, JJ = np.meshgrid(np.arange(m3), np.arange(m3), indexing="ij")
    xy12 = np.stack([jj.ravel() * e12 * pitch, ii.ravel() * e12 * pitch], 1)
    xy34 = np.stack([JJ.ravel() * e34 * pitch, II.ravel() * e34 * pitch], 1)
    xy = np.concatenate([xy12, xy12, xy34, xy34])
    layer = np.concatenate([np.full(n12, 1), np.full(n12, 2), np.full(n34, 3), np.full(n34, 4)]).astype(np.int32)
    ra, rb, L, W, Hh, via, R = [], [], [], [], [], [], []

    def wires(lay, mm, horizontal, span, spacing):
        keep = np.stack([_cut_runs(rng, mm - 1, span) for _ in range(mm)])      # [line][segment]
        li, sj = np.nonzero(keep)
        if horizontal:
            a, b = li * mm + sj, li * mm + sj + 1
        else:
            a, b = sj * mm + li, (sj + 1) * mm + li
        k = lay - 1
        ra.append(base[k] + a); rb.append(base[k] + b)
        L.append(np.full(a.size, spacing)); W.append(np.full(a.size, w[k])); Hh.append(np.full(a.size, H[k]))
        via.append(np.zeros(a.size, np.uint8))
        R.append(RHO_CU * spacing / (w[k] * H[k]) * np.ones(a.size))

    wires(1, m, True, cut12, e12 * pitch)
    wires(2, m, False, cut12, e12 * pitch)
    wires(3, m3, True, cut34, e34 * pitch)
    wires(4, m3, False, cut34, e34 * pitch)

    def vias(a, b, rv):
        ra.append(a); rb.append(b)
        L.append(np.zeros(a.size)); W.append(np.full(a.size, w[0])); Hh.append(np.full(a.size, H[0]))
        via.append(np.ones(a.size, np.uint8)); R.append(np.full(a.size, rv))

    v12 = np.nonzero(((ii.ravel() % via12_every) == 0) | ((jj.ravel() % via12_every) == 0))[0]
    vias(base[0] + v12, base[1] + v12, R_via[0])
    v23 = np.nonzero(((II.ravel() % via23_every) == 0) | ((JJ.ravel() % via23_every) == 0))[0]
    m2_at_m3 = (II.ravel()[v23] * r34) * m + JJ.ravel()[v23] * r34
    vias(base[1] + m2_at_m3, base[2] + v23, R_via[1])
    v34 = ((II.ravel() % via34_every) == 0) & ((JJ.ravel() % via34_every) == 0)
    vias(base[2] + np.nonzero(v34)[0], base[3] + np.nonzero(v34)[0], R_via[2])
    ra = np.concatenate(ra).astype(np.int32); rb = np.concatenate(rb).astype(np.int32)
    L = np.concatenate(L); W = np.concatenate(W); Hh = np.concatenate(Hh)
    via = np.concatenate(via); R0 = np.concatenate(R)
    # pads on a lattice of M4 nodes that carry an M3-M4 via (indices rounded
    # to multiples of via34_every), so that every pad feeds the grid
    step = m3 // pad_lattice
    pi = step // 2 + step * np.arange(pad_lattice)
    pi = np.minimum(via34_every * np.round(pi / via34_every).astype(np.int64), (m3 - 1) // via34_every * via34_every)
    pads = np.unique(base[3] + (pi[:, None] * m3 + pi[None, :]).ravel()).astype(np.int32)
    sink = np.zeros(xy.shape[0])
    sink[:n12] = sink_scale * np.exp(rng.normal(sink_mu, sink_sigma, n12))
    # keep only the components that reach a pad (sparse M3-M4 vias leave M4
    # pieces without one)
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    nn = xy.shape[0]
    _, lab = connected_components(sp.coo_matrix((np.ones(ra.size), (ra, rb)), shape=(nn, nn)), directed=False)
    live = np.isin(lab, np.unique(lab[pads]))
    remap = -np.ones(nn, np.int64)
    remap[live] = np.arange(int(live.sum()))
    kr = live[ra] & live[rb]
    ra, rb = remap[ra[kr]].astype(np.int32), remap[rb[kr]].astype(np.int32)
    L, W, Hh, via, R0 = L[kr], W[kr], Hh[kr], via[kr], R0[kr]
    xy, layer, sink = xy[live], layer[live], sink[live]
    pads = remap[pads].astype(np.int32)
    g = Grid(xy=xy, layer=layer, res_a=ra, res_b=rb, res_len=L, res_w=W, res_h=Hh,
             res_is_via=via, res_R0=R0, pad_node=pads, vdd=vdd, sink_I=sink,
             name=f"fullchip{n}_s{seed}")
    ext = (n - 1) * pitch
    tm, x0, y0, dxr, dyr = gaussian_hotspot_map(seed + 7, ext, ext, base_K, n_spots, amp_range, sig_range, raster)
    g.tmap, g.tmap_x0, g.tmap_y0, g.tmap_dx, g.tmap_dy = tm, x0, y0, dxr, dyr
    return g


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
def workload(name: str):
    """Return (grid, material, run, mc) for a named workload.

    tiny_trees      200 straight trees, prescribed currents, 378 K, FP64
    tiny_mesh       32x32 two-layer mesh with 4 corner pads (IR solve)
    pg400           400x400 two-layer grid, ~800 line trees, thermal map
    mc_mesh         32x32 mesh with cut M1 rows, 1024 Monte Carlo samples
    mc_grid         96x96 sparse-via grid (via every 32 nodes, 16 pads), 330 K +
                    hotspots, 1024 Monte Carlo samples, FP32: worst initial drop 7 %,
                    about 40 % of the samples fail within the 10-year horizon
    screen_cold     64 x 257 long-line grid at 310 K with two +70..100 K hotspots,
                    256 samples, FP32: every sample fails within years through the hot
                    lines while most steady-state-mortal lines would nucleate decades
                    later (the learned screen's workload)
    screen_mc       200x200 sparse-via grid (via every 64 nodes), 330 K + hotspots,
                    64 Monte Carlo samples: mortal trees with nucleation times
                    spread over years and failures within the horizon
    combs           200 comb/stub trees (trunks of 20-100 segments with teeth and
                    stubs: up to a few hundred branches per tree), prescribed
                    currents, 378 K, FP32, screen off
    long_lines      24 x 257 two-layer grid whose 24 M1 rows are lines of 212-256
                    segments (4241-5121 stress nodes: the chain kernel's 1024-lane
                    form), short M2 straps, via every 32 nodes, 330 K + hotspots,
                    64 samples, FP32: early and late failures after 3-5 re-solves
                    and censored samples with voids
    """
    mat = default_material()
    if name == "tiny_trees":
        return straight_trees(1001), mat, default_run(prec=0, screen=0), None
    if name == "tiny_mesh":
        return two_layer_mesh(1001), mat, default_run(prec=0), None
    if name == "pg400":
        return pg_grid(2001), mat, default_run(prec=1, T_ambient=330.0), None
    if name == "pg400_fp64":
        return pg_grid(2001), mat, default_run(prec=0, T_ambient=330.0), None
    if name == "mc_mesh":
        return (two_layer_mesh(3001, cut_m1=True, vdd=1.2, sink_mu=np.log(32e-6)), mat,
                default_run(prec=1),
                dict(n_samples=1024, seed=3001, cov_kappa=0.2, cov_scrit=0.2))
    if name == "mc_grid":
        g = pg_grid(4001, n=96, via_every=32, pad_lattice=4, sink_scale=0.06618,
                    seg_range=(48, 95), base_K=330.0)
        return (g, mat, default_run(prec=1, T_ambient=330.0),
                dict(n_samples=1024, seed=3001, cov_kappa=0.2, cov_scrit=0.2))
    if name == "combs":
        return comb_trees(7001), mat, default_run(prec=1, screen=0), None
    if name == "fullchip":
        g = fullchip_grid(5001, sink_scale=FULLCHIP_SINK_SCALE)
        return (g, mat, default_run(prec=1, T_ambient=340.0, ir_every=50, joule=1),
                dict(n_samples=256, seed=5001, cov_kappa=0.2, cov_scrit=0.2))
    if name == "long_lines":
        g = line_grid_family(6001)
        return (g, mat, default_run(prec=1, T_ambient=330.0),
                dict(n_samples=64, seed=6001, cov_kappa=0.2, cov_scrit=0.2))
    if name == "screen_cold":
        return (cold_line_grid(6101, sink_scale=0.107), mat,
                default_run(prec=1, T_ambient=310.0),
                dict(n_samples=256, seed=6101, cov_kappa=0.2, cov_scrit=0.2))
    if name == "screen_mc":
        return (sparse_via_grid(2101), mat, default_run(prec=1, T_ambient=330.0),
                dict(n_samples=64, seed=5, cov_kappa=0.2, cov_scrit=0.2))
    raise KeyError(name)


# ----------------------------------------------------------------------------
# Learned-screen inputs: initial parameters and training grids
# ----------------------------------------------------------------------------
MLP_SHAPES = [(256, 16), (256,), (256, 256), (256,), (256, 256), (256,), (256,), (1,)]


def init_mlp_params(seed: int, out_bias: float = 0.0) -> np.ndarray:
    """Seeded initial parameters of the 16-256-256-256-1 screen model in its
    flat layout (W1, b1, W2, b2, W3, b3, w4, b4): weights N(0, 2/fan_in)
    (He scaling for rectifier-like units), biases zero, output bias
    ``out_bias``."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, shp in enumerate(MLP_SHAPES):
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp) * np.sqrt(2.0 / shp[1]))
        elif k == 6:
            parts.append(rng.standard_normal(shp) * np.sqrt(1.0 / 256))
        elif k == 7:
            parts.append(np.array([out_bias]))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def sparse_via_grid(seed: int, n: int = 200, via_every: int = 64, sink_scale: float = 0.012,
                    base_K: float = 330.0) -> Grid:
    """The P/G grid family of :func:`pg_grid` with sparse vias (one every
    ``via_every`` nodes along a line), so that M1 lines carry one-directional
    current over long spans: the regime where many trees are steady-state
    mortal and their nucleation times spread over years at 330 K."""
    return pg_grid(seed, n=n, via_every=via_every, sink_scale=sink_scale, base_K=base_K)


def screen_training_grids(seed: int, n_grids: int, n: int = 200, j_scale=(0.8, 1.5)):
    """Random sparse-via grids for learned-screen labels: via spacing 48 or
    64 nodes, sink scale drawn per grid so that the initial worst drop stays
    roughly within 5-9 % of the supply, new thermal map per grid.  Returns
    (grid, factor) pairs; the labels hold each grid's t = 0 currents fixed,
    multiplied by ``factor`` ~ U[j_scale] to widen the range of stress
    margins seen in training."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_grids):
        ve = int(rng.choice([48, 64]))
        lo, hi = (0.014, 0.022) if ve == 48 else (0.008, 0.013)
        g = sparse_via_grid(int(rng.integers(1, 2 ** 31)), n=n, via_every=ve,
                            sink_scale=float(rng.uniform(lo, hi)))
        out.append((g, float(rng.uniform(*j_scale))))
    return out


def line_grid_family(seed: int, sink_scale: float = 0.16, via_every: int = 32, rows: int = 24,
                     base_K: float = 330.0, n_spots: int = 6, amp_range=(15.0, 60.0),
                     sig_range=(30 * UM, 80 * UM)) -> Grid:
    """The long-line P/G grid family: ``rows`` M1 rows of 212-256 segments
    (lines of 4241-5121 FD nodes) strapped by M2 columns spanning about half
    the rows, a via every ``via_every`` nodes, 16 pads, a thermal map of
    base_K plus n_spots Gaussian hotspots."""
    return pg_grid(seed, n=rows, n_cols=257, seg_range=(212, 256),
                   col_seg_range=(rows // 2, rows - 1), via_every=via_every, pad_lattice=4,
                   sink_scale=sink_scale, base_K=base_K, n_spots=n_spots, amp_range=amp_range,
                   sig_range=sig_range)


def cold_line_grid(seed: int, sink_scale: float = 0.05) -> Grid:
    """Long-line grid of 64 rows at a cold base temperature (310 K) with two
    strong hotspots (+70..100 K): lines through a hotspot nucleate and fail
    within years, while many steady-state-mortal lines in the cold part would
    need decades (the regime where a nucleation-time screen pays)."""
    return line_grid_family(seed, sink_scale=sink_scale, rows=64, base_K=310.0, n_spots=2,
                            amp_range=(70.0, 100.0), sig_range=(60 * UM, 120 * UM))


def line_training_grids(seed: int, n_grids: int, j_scale=(0.8, 1.5), cold: bool = False):
    """Random long-line grids for learned-screen labels (the 24-row family, or
    with ``cold`` the 64-row cold grids with two hotspots; sink scale drawn so
    that the initial drop spans about 6-9 %, new line spans, sinks and thermal
    map per grid), each with a current factor ~ U[j_scale] for the fixed-j
    label runs.  Returns (grid, factor) pairs."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_grids):
        sd = int(rng.integers(1, 2 ** 31))
        g = (cold_line_grid(sd, float(rng.uniform(0.08, 0.12))) if cold
             else line_grid_family(sd, float(rng.uniform(0.12, 0.18))))
        out.append((g, float(rng.uniform(*j_scale))))
    return out


def hotspot_map_at(extent_x: float, extent_y: float, base_K: float, centers, amp_K: float,
                   sigma: float, res: float = 1 * UM):
    """Base temperature plus equal Gaussian hotspots (amplitude amp_K, width
    sigma) at the given (x, y) centres, on a regular raster.  Returns
    (tmap[ny, nx], x0, y0, dx, dy)."""
    nx = int(np.ceil(extent_x / res)) + 1
    ny = int(np.ceil(extent_y / res)) + 1
    x = np.arange(nx) * res
    y = np.arange(ny) * res
    T = np.full((ny, nx), float(base_K))
    for cx, cy in centers:
        T += amp_K * np.outer(np.exp(-0.5 * ((y - cy) / sigma) ** 2), np.exp(-0.5 * ((x - cx) / sigma) ** 2))
    return T, 0.0, 0.0, res, res


def hotspot_centers(g: Grid, seg_j: np.ndarray, k: int, min_sep: float, highest: bool = True):
    """Midpoints of the k wire segments of highest (or lowest) |j| that lie
    at least min_sep apart (greedy in |j| order)."""
    wire = g.res_is_via == 0
    key = np.where(wire, np.abs(seg_j), -np.inf if highest else np.inf)
    order = np.argsort(-key if highest else key, kind="stable")
    mid = 0.5 * (g.xy[g.res_a] + g.xy[g.res_b])
    out = []
    for e in order:
        if not wire[e]:
            break
        c = mid[e]
        if all(np.hypot(*(c - h)) >= min_sep for h in out):
            out.append(c)
            if len(out) == k:
                break
    return out


def thermal_variants(g: Grid, hot_centers, cold_centers, mean_K: float, amp_K: float, sigma: float,
                     hotter_K: float = 0.0):
    """Copies of grid g under thermal maps of one die-average temperature
    (the raster mean): 'uniform'; 'hot_on_high_j', hotspots at hot_centers
    (e.g. over the wires of highest current density); 'hot_on_low_j', the
    same hotspots at cold_centers; and 'hot_on_low_j_hotter', the latter
    raised by hotter_K on average.  The paper's thermal observations compare
    lifetimes under maps of equal and of different average temperature."""
    ext_x = float(g.xy[:, 0].max())
    ext_y = float(g.xy[:, 1].max())
    out = {}
    for name, centers, shift in (("uniform", [], 0.0), ("hot_on_high_j", hot_centers, 0.0),
                                 ("hot_on_low_j", cold_centers, 0.0),
                                 ("hot_on_low_j_hotter", cold_centers, hotter_K)):
        if name == "hot_on_low_j_hotter" and hotter_K == 0.0:
            continue
        T, x0, y0, dx, dy = hotspot_map_at(ext_x, ext_y, 0.0, centers, amp_K, sigma)
        T = T - T.mean() + mean_K + shift
        h = copy.deepcopy(g)
        h.node_T = None
        h.tmap, h.tmap_x0, h.tmap_y0, h.tmap_dx, h.tmap_dy = T, x0, y0, dx, dy
        h.name = f"{g.name}_{name}"
        out[name] = h
    return out


def seeded_current_density(g: Grid, seed: int, lo: float = 1e9, hi: float = 5e10) -> np.ndarray:
    """Per-resistor current density +-U[lo, hi] A/m^2 with equiprobable sign
    (zero on vias): prescribed currents of the tiny-trees kind for any grid."""
    rng = np.random.default_rng(seed)
    j = rng.uniform(lo, hi, g.n_res) * np.where(rng.random(g.n_res) < 0.5, -1.0, 1.0)
    return np.where(g.res_is_via != 0, 0.0, j)


def with_prescribed_j(g: Grid, seg_j: np.ndarray) -> Grid:
    """A copy of ``g`` in trees-only mode with the given per-resistor current
    densities held fixed."""
    return dataclasses.replace(g, seg_j=np.asarray(seg_j, np.float64).copy(),
                               name=g.name + "_fixed_j")
