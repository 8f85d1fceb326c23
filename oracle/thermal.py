"""Joule-heating thermal pre-pass of the FP64 oracle (Sec. III-A, eqs. 1-4).

TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package.  It shares no
code with the HIP path.

What it computes, in the paper's notation:

* Eq. 3, stationary heat balance along a wire with Joule source j^2 rho and
  exchange with the surroundings at T0 through the thermal characteristic
  length Gamma (eq. 2: Gamma^2 = t_cu t_ILD k_cu / k_ILD).  The exchange is
  read as a loss towards T0 (the printed signs, and the cosine/sine form of
  eq. 4, would make the profile oscillate and cannot meet both end
  temperatures; eq. 4 as printed does not satisfy T(-L/2) = T1): the profile
  is the hyperbolic one, with the symmetric Joule rise Tm = j^2 rho Gamma^2 /
  k_cu and the antisymmetric part (T2 - T1)/2 that eq. 4 names.
* Per-tree end conditions: tree vertices with a via take the map
  temperature; every other vertex (junctions, free wire ends) is solved from
  heat-flux balance over the segments that meet there (tridiagonal blocks
  for a line, a tree-shaped system for a tree).  Written here as one dense
  linear system per tree, solved by a library routine.
* T0 of a segment is the map temperature at its midpoint (the uniform
  ambient without thermal data): the map stands for the die temperature
  around the wire.

Profile of one segment with end temperatures T1 at x = -L/2 (res_a) and T2 at
x = +L/2 (res_b), h = L / (2 Gamma), c = T0 + Tm:

    T(x) = c + (Tbar - c) cosh(x/Gamma)/cosh(h) + (T2 - T1)/2 sinh(x/Gamma)/sinh(h)

and the gradient pointing into the segment at the res_a end, from
differentiating it,

    T'(-L/2) = [ -(Tbar - c) tanh(h) + (T2 - T1)/2 coth(h) ] / Gamma

(by symmetry the same expression with the ends swapped at the res_b end).
"""
from __future__ import annotations

import numpy as np


def map_T_xy(grid, T_amb, x, y):
    """Map temperature at points (x, y): the raster sampled bilinearly with
    edge clamping; without a raster the uniform ambient."""
    if grid.tmap is None:
        return np.full(np.shape(x), float(T_amb))
    M = np.asarray(grid.tmap, np.float64)
    ny, nx = M.shape
    fx = np.clip((np.asarray(x) - grid.tmap_x0) / grid.tmap_dx, 0.0, nx - 1)
    fy = np.clip((np.asarray(y) - grid.tmap_y0) / grid.tmap_dy, 0.0, ny - 1)
    ix = np.clip(np.floor(fx).astype(int), 0, max(nx - 2, 0))
    iy = np.clip(np.floor(fy).astype(int), 0, max(ny - 2, 0))
    tx, ty = fx - ix, fy - iy
    ix1 = ix + 1 if nx > 1 else ix
    iy1 = iy + 1 if ny > 1 else iy
    lo = (1 - tx) * M[iy, ix] + tx * M[iy, ix1]
    hi = (1 - tx) * M[iy1, ix] + tx * M[iy1, ix1]
    return (1 - ty) * lo + ty * hi


def vertex_map_T(grid, T_amb, v):
    """Map temperature at grid node v (raster, else node_T, else ambient)."""
    if grid.tmap is not None:
        return float(map_T_xy(grid, T_amb, grid.xy[v, 0], grid.xy[v, 1]))
    if grid.node_T is not None:
        return float(grid.node_T[v])
    return float(T_amb)


def midpoint_map_T(grid, T_amb, e):
    """Map temperature at the midpoint of segment e (node_T: the mean of its
    end values, the straight line between them)."""
    a, b = int(grid.res_a[e]), int(grid.res_b[e])
    if grid.tmap is not None:
        m = 0.5 * (grid.xy[a] + grid.xy[b])
        return float(map_T_xy(grid, T_amb, m[0], m[1]))
    if grid.node_T is not None:
        return 0.5 * (float(grid.node_T[a]) + float(grid.node_T[b]))
    return float(T_amb)


def gamma(mat, t_cu):
    """Thermal characteristic length, eq. 2."""
    return np.sqrt(t_cu * mat["t_ild"] * mat["k_cu"] / mat["k_ild"])


def joule_rise(mat, j, G):
    """Symmetric (Joule-heating) rise Tm = j^2 rho Gamma^2 / k_cu (eq. 4)."""
    return j * j * mat["rho_cu"] * G * G / mat["k_cu"]


def profile(T1, T2, c, G, L, x):
    """Steady segment temperature at x in [-L/2, L/2]."""
    h = L / (2.0 * G)
    Tbar = 0.5 * (T1 + T2)
    return c + (Tbar - c) * np.cosh(x / G) / np.cosh(h) + 0.5 * (T2 - T1) * np.sinh(x / G) / np.sinh(h)


def end_gradient_coeffs(c, G, L):
    """Gradient into the segment at an end, as a_here T_here + a_there
    T_there + a0 (differentiated profile)."""
    h = L / (2.0 * G)
    t, ct = np.tanh(h), 1.0 / np.tanh(h)
    return (-0.5 * t - 0.5 * ct) / G, (-0.5 * t + 0.5 * ct) / G, c * t / G


def has_via(grid):
    """Grid nodes touched by a resistor that is not a wire segment."""
    wire = (grid.res_is_via == 0) & (grid.layer[grid.res_a] == grid.layer[grid.res_b])
    out = np.zeros(grid.n_nodes, bool)
    out[grid.res_a[~wire]] = True
    out[grid.res_b[~wire]] = True
    return out


def node_temperatures(grid, mat, T_amb, topo, jseg):
    """Temperature at every stress node (DFS order of `topo`) from the
    per-tree vertex solve and the per-segment profile."""
    jseg = np.asarray(jseg, np.float64)
    via = has_via(grid)
    N = topo.N
    T = np.zeros(topo.n_stress)
    seg_G, seg_c = {}, {}

    def seg_par(e):
        if e not in seg_G:
            G = float(gamma(mat, grid.res_h[e]))
            seg_G[e] = G
            seg_c[e] = midpoint_map_T(grid, T_amb, e) + float(joule_rise(mat, jseg[e], G))
        return seg_G[e], seg_c[e]

    for t in range(topo.n_trees):
        o0, o1 = int(topo.tree_off[t]), int(topo.tree_off[t + 1])
        vnodes = [i for i in range(o0, o1) if topo.vert[i] >= 0]
        idx = {int(topo.vert[i]): k for k, i in enumerate(vnodes)}
        n = len(vnodes)
        A = np.zeros((n, n))
        rhs = np.zeros(n)
        segs = sorted({int(topo.seg[i]) for i in range(o0 + 1, o1)})
        for e in segs:
            G, c = seg_par(e)
            L = float(grid.res_len[e])
            area = float(grid.res_w[e] * grid.res_h[e])
            a_here, a_there, a0 = end_gradient_coeffs(c, G, L)
            ends = (int(grid.res_a[e]), int(grid.res_b[e]))
            for here, there in (ends, ends[::-1]):
                k, m = idx[here], idx[there]
                # heat-flux balance at `here`: sum over its segments of
                # area x (gradient into the segment) = 0
                A[k, k] += area * a_here
                A[k, m] += area * a_there
                rhs[k] -= area * a0
        for v, k in idx.items():
            if via[v]:
                A[k, :] = 0.0
                A[k, k] = 1.0
                rhs[k] = vertex_map_T(grid, T_amb, v)
        Tv = np.linalg.solve(A, rhs)
        for k, i in enumerate(vnodes):
            T[i] = Tv[k]
        for i in range(o0, o1):
            if topo.vert[i] >= 0:
                continue
            e = int(topo.seg[i])
            G, c = seg_par(e)
            L = float(grid.res_len[e])
            T1 = Tv[idx[int(grid.res_a[e])]]
            T2 = Tv[idx[int(grid.res_b[e])]]
            x = (topo.kpos[i] / N - 0.5) * L
            T[i] = profile(T1, T2, c, G, L, x)
    return T
