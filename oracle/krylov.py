"""Extended rational Krylov reduction of one tree's stress system: the plain,
slow FP64 reference (EMSpice 3, arXiv 2604.10743, Sec. IV-E, Alg. 1,
eqs. 21-27).

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's CPU
leg; never by the product package.  Shares no code with the HIP path.

A tree's finite-difference system between two IR solves is

    C s'(t) = A s(t) + f,        s(0) = s0                          (eq. 21)

with C = diag(V) the node volumes, A = -L the negated Laplacian of the edge
conductances g (edge (parent(i), i) carries g_i = a kappa / dx), and f the
constant drive (electron wind and thermomigration, Sec. III-A).

* Shifted moments (eq. 24): with K = s0 C - A and R = K^-1,
  m_0 = R (s0 C s0_vec + f), m_1 = R (C s0_vec - C m_0), m_k = -R C m_(k-1).
* Basis (Alg. 1): starting block [R C s0, R f]; blocks V_(j+1) from
  R C V_j by block Gram-Schmidt against every earlier block and a thin QR;
  stop when a new block's norm collapses.
* Reduced model (eq. 25): A_h = V^T A V, C_h = V^T C V, f_h = V^T f,
  stepped by backward Euler from V^T s0 and lifted as V z.
* Shift time (eq. 26): t_s = eta L_max^2 / (pi^2 kappa); s0 = 1 / t_s.
* Selection (eq. 27): the reduced path is used when n >= max(3q, 30).

Readings (where the paper leaves a choice): the thin QR is a column-by-column
Gram-Schmidt with one re-orthogonalisation pass; a column whose norm after
orthogonalisation falls below eps times its norm before is dropped (a rank
deficiency of the block), and the iteration stops when a whole block is
dropped -- the block-norm breakdown test of Alg. 1 made scale-free.  A
library sparse LU factors K (as the paper does).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

EPS = 1e-10


def tree_matrices(parent, V, g):
    """C (vector of node volumes) and A = -L (sparse) of one tree; parent[i]
    is the local index of node i's parent (-1 at the root), g[i] the
    conductance of the edge (parent(i), i)."""
    n = len(V)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for i in range(n):
        p = parent[i]
        if p < 0:
            continue
        rows += [i, p]
        cols += [p, i]
        vals += [g[i], g[i]]
        diag[i] -= g[i]
        diag[p] -= g[i]
    A = sp.csr_matrix((vals + list(diag), (rows + list(range(n)), cols + list(range(n)))), shape=(n, n))
    return np.asarray(V, np.float64), A


def shift_time(L_max, kappa, eta=1.0):
    """eq. 26: the slowest blocked-line mode's time constant, scaled by eta."""
    return eta * L_max ** 2 / (np.pi ** 2 * kappa)


def krylov_selected(n, q):
    """eq. 27: the reduced path only for trees of at least max(3q, 30) nodes."""
    return n >= max(3 * q, 30)


def _resolvent(Cv, A, s0):
    K = (s0 * sp.diags(Cv) - A).tocsc()
    return spla.splu(K)


def shifted_moments(Cv, A, f, x0, s0, k_max):
    """The full system's shifted moments m_0 .. m_(k_max-1) (eq. 24)."""
    lu = _resolvent(Cv, A, s0)
    m = [lu.solve(s0 * Cv * x0 + f)]
    if k_max > 1:
        m.append(lu.solve(Cv * x0 - Cv * m[0]))
    for _ in range(2, k_max):
        m.append(-lu.solve(Cv * m[-1]))
    return m


def _add_columns(basis, W, eps):
    """Orthonormalise the columns of W against basis and each other (two
    Gram-Schmidt passes); returns the accepted columns."""
    out = []
    for c in range(W.shape[1]):
        w = W[:, c].copy()
        n0 = np.linalg.norm(w)
        if n0 == 0.0:
            continue
        for _ in range(2):
            for v in basis + out:
                w -= v * (v @ w)
        nw = np.linalg.norm(w)
        if nw > eps * n0:
            out.append(w / nw)
    return out


def reduce(Cv, A, f, x0, s0, q, eps=EPS):
    """Alg. 1: orthonormal basis V (n x r, r <= 2q) and the reduced matrices."""
    lu = _resolvent(Cv, A, s0)
    F0 = np.column_stack([lu.solve(Cv * x0), lu.solve(f)])
    basis = _add_columns([], F0, eps)
    block = list(basis)
    for _ in range(1, q):
        if not block:
            break
        W = np.column_stack([lu.solve(Cv * v) for v in block])
        block = _add_columns(basis, W, eps)
        basis += block
    V = np.column_stack(basis)
    Ah = V.T @ (A @ V)
    Ch = V.T @ (Cv[:, None] * V)
    fh = V.T @ f
    return V, Ah, Ch, fh


def reduced_be(V, Ah, Ch, fh, x0, dt, n_steps):
    """Backward Euler on the reduced system from V^T x0; returns the reduced
    states z_1 .. z_n_steps (rows) -- lift with V z."""
    M = Ch - dt * Ah
    z = V.T @ x0
    out = np.zeros((n_steps, len(z)))
    for k in range(n_steps):
        z = np.linalg.solve(M, Ch @ z + dt * fh)
        out[k] = z
    return out


def full_be(Cv, A, f, x0, dt, n_steps):
    """Backward Euler on the full system (for comparison); rows are states."""
    lu = spla.splu((sp.diags(Cv) - dt * A).tocsc())
    x = np.array(x0, np.float64)
    out = np.zeros((n_steps, len(x)))
    for k in range(n_steps):
        x = lu.solve(Cv * x + dt * f)
        out[k] = x
    return out


# ----------------------------------------------------------------------------
# The reduced path inside the aging loop (one sample)
# ----------------------------------------------------------------------------
class ChainBasis:
    """A chain's reduced model and its present reduced state."""

    def __init__(self, V, Ah, Ch, fh, z):
        self.V, self.Ah, self.Ch, self.fh, self.z = V, Ah, Ch, fh, z


def chain_shift(g, V, dx):
    """s0 = 1 / t_s with t_s = L^2 / (pi^2 kappa) (eq. 26; the caller scales
    by eta): L the chain's length, kappa = sum g dx^2 / sum V its volume-
    weighted diffusivity (g dx = a kappa on every edge)."""
    L = float(np.sum(dx))
    kappa = float(np.sum(g * dx * dx) / np.sum(V))
    return np.pi ** 2 * kappa / L ** 2


def interval(sim, topo, grid, bases, active, n_steps, step0, dt, q, eta):
    """One aging interval of one sample with the reduced path: every active
    chain of at least max(3q, 30) nodes without voids builds (or keeps) its
    basis and steps the reduced model; the interval is kept in reduced form
    when max_i(s_end,i - sigma_crit,i + |V_i|_2 max_k |z_k - z_end|_2) < 0
    (the lifted states cannot reach a critical stress), else the chain is stepped exactly
    and its basis dropped.  The other trees are stepped exactly.  bases maps
    tree -> ChainBasis and persists across intervals."""
    arr = sim.node_arrays()
    sig = sim.sigma()
    iv, _ = sim.voids()
    has_void = set(int(t) for t in iv[:, 0]) if len(iv) else set()
    exact = np.array(active, np.uint8).copy()
    N = topo.N
    for t in range(topo.n_trees):
        i0, i1 = int(topo.tree_off[t]), int(topo.tree_off[t + 1])
        n = i1 - i0
        chain = all(topo.parent[i] == i - 1 for i in range(i0 + 1, i1))
        if not active[t] or t in has_void or not chain or not krylov_selected(n, q):
            bases.pop(t, None)
            continue
        V = arr["V"][i0:i1]
        g = arr["g"][i0:i1].copy()
        g[0] = 0.0
        f = arr["f"][i0:i1]
        if t not in bases:
            dx = grid.res_len[topo.seg[i0 + 1:i1]] / N
            s0 = chain_shift(g[1:], V, dx) / eta
            Cv, A = tree_matrices(np.arange(-1, n - 1), V, g)
            Vb, Ah, Ch, fh = reduce(Cv, A, f, sig[i0:i1], s0, q)
            bases[t] = ChainBasis(Vb, Ah, Ch, fh, Vb.T @ sig[i0:i1])
        b = bases[t]
        M = b.Ch - dt * b.Ah
        zs = [b.z]
        z = b.z
        for _ in range(n_steps):
            z = np.linalg.solve(M, b.Ch @ z + dt * b.fh)
            zs.append(z)
        ze = zs[-1]
        dist = max(float(np.linalg.norm(zk - ze)) for zk in zs)
        s_end = b.V @ ze
        rown = np.sqrt(np.sum(b.V * b.V, axis=1))      # node i moves by at most |V_i| dist
        if np.max(s_end - arr["sc"][i0:i1] + rown * dist) < 0.0:
            sig[i0:i1] = s_end
            b.z = ze
            exact[t] = 0
        else:
            bases.pop(t)
    sim.set_sigma(sig)
    sim.set_active(exact)
    sim.steps(n_steps, step0)
    sim.set_active(np.array(active, np.uint8))
