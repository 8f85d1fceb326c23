"""The steady-state skipping criterion (em_run_params.ss_tol).  Between two
IR solves an instance without voids steps C s' = f - A s by backward Euler
(Sec. II's stress equation with blocked ends: A the Laplacian of positive
edge conductances g, C = diag(V)).  Each step maps the distance e = s - s_inf
to the steady state by (C + dt A)^-1 C, a nonnegative matrix with unit row
sums, so every later e lies componentwise within [min e_n, max e_n].  On a
tree e is known up to a constant from the residual: across the edge above a
subtree, g (e_child - e_parent) is the sum of A e = A s - f over the
subtree.  Hence, with P the potential so obtained (P = e_n + const):

    every later state s_m satisfies  s_n,i - (P_i - min P) <= s_m,i
                                     <= s_n,i + (max P - P_i).

Checked on random chains and branched trees by stepping to the steady state
in FP64 with random step sizes; the bound is attained by the steady state
itself, and an estimate that ignores the residual's subtree structure (a
plain max-norm of the residual) is shown to fail."""
import numpy as np


def laplacian(n, edges, g):
    A = np.zeros((n, n))
    for (a, b), w in zip(edges, g):
        A[a, a] += w
        A[b, b] += w
        A[a, b] -= w
        A[b, a] -= w
    return A


def random_tree(rng, n, chain):
    if chain:
        return [(i - 1, i) for i in range(1, n)]
    return [(int(rng.integers(0, i)), i) for i in range(1, n)]


def potential(n, edges, g, V, f, s):
    """P = e + const from the residual, by subtree sums (edges are
    (parent, child) with parent < child, so children come later).  The
    forcing's total is removed in proportion to V first, as the stepping's
    content projection does."""
    A = laplacian(n, edges, g)
    fp = f - V * f.sum() / V.sum()
    w = A @ s - fp
    sub = w.copy()
    for (a, b) in reversed(edges):
        sub[a] += sub[b]
    P = np.zeros(n)
    for (a, b), ge in zip(edges, g):
        P[b] = P[a] + sub[b] / ge
    return P


def chain_potential(g, V, f, s):
    """The chain form the check kernel uses: prefix sums of the residual
    r = f' - A s (node i's edge to i - 1 carries the sum over nodes < i)."""
    n = len(s)
    fp = f - V * f.sum() / V.sum()
    r = fp.copy()
    r[1:] += g * (s[:-1] - s[1:])
    r[:-1] += g * (s[1:] - s[:-1])
    pre = np.concatenate([[0.0], np.cumsum(r)[:-1]])      # sum over nodes < i
    P = np.zeros(n)
    P[1:] = np.cumsum(pre[1:] / g)
    return P


def case(rng, chain):
    n = int(rng.integers(2, 48))
    edges = random_tree(rng, n, chain)
    g = rng.lognormal(0.0, 1.0, n - 1)
    V = rng.lognormal(0.0, 0.6, n)
    f = rng.normal(size=n)
    f -= f.sum() / n
    A = laplacian(n, edges, g)
    s = rng.normal(size=n) * 3.0
    C = np.diag(V)
    for _ in range(int(rng.integers(0, 6))):        # a state along a trajectory
        dt = float(rng.lognormal(-1.0, 1.5))
        s = np.linalg.solve(C + dt * A, C @ s + dt * f)
    return n, edges, g, V, f, A, s


def later_states(rng, A, V, f, s):
    C = np.diag(V)
    out = []
    for _ in range(60):
        dt = float(rng.lognormal(0.0, 2.0))
        s = np.linalg.solve(C + dt * A, C @ s + dt * f)
        out.append(s)
    M = np.vstack([A, V[None, :]])                  # the steady state of the same content
    out.append(np.linalg.lstsq(M, np.concatenate([f, [V @ s]]), rcond=None)[0])
    return out


def test_bound_holds_on_chains_and_trees():
    rng = np.random.default_rng(20261203)
    ratios = []
    for trial in range(300):
        n, edges, g, V, f, A, s = case(rng, chain=trial % 2 == 0)
        P = potential(n, edges, g, V, f, s)
        up = P.max() - P
        dn = P - P.min()
        later = later_states(rng, A, V, f, s)
        for x in later:
            d = x - s
            assert np.all(d <= up + 1e-9 * (1 + np.abs(s))), trial
            assert np.all(-d <= dn + 1e-9 * (1 + np.abs(s))), trial
        spread = max(float(np.max(np.abs(x - s))) for x in later)
        osc = P.max() - P.min()
        if spread > 1e-9:
            ratios.append(osc / spread)
    assert len(ratios) > 200
    # the oscillation is at most twice the largest move (the steady state
    # lies inside the band), so the criterion is tight
    assert max(ratios) <= 2.0 + 1e-6
    print(f"osc(P) / largest later move: median {np.median(ratios):.2f}, max {np.max(ratios):.2f}")


def test_chain_prefix_form_equals_subtree_form():
    rng = np.random.default_rng(3)
    for _ in range(50):
        n, edges, g, V, f, A, s = case(rng, chain=True)
        f = f + rng.normal() * 1e-3 * V                # a forcing whose total is not zero
        P1 = potential(n, edges, g, V, f, s)
        P2 = chain_potential(g, V, f, s)
        assert np.allclose(P1, P2, rtol=1e-10, atol=1e-10 * (1 + np.abs(P1).max()))


def test_residual_max_norm_alone_is_not_a_bound():
    """Scaling the residual's max-norm by the largest 1/(g) (no subtree sums)
    underestimates the move on long chains: the structure is needed."""
    rng = np.random.default_rng(5)
    hit = False
    for _ in range(100):
        n, edges, g, V, f, A, s = case(rng, chain=True)
        naive = np.max(np.abs(A @ s - f)) * np.max(1.0 / g)
        spread = max(float(np.max(np.abs(x - s))) for x in later_states(rng, A, V, f, s))
        if spread > naive * 1.01:
            hit = True
            break
    assert hit


def test_bound_vanishes_at_the_steady_state():
    rng = np.random.default_rng(11)
    n, edges, g, V, f, A, s = case(rng, chain=True)
    ss = later_states(rng, A, V, f, s)[-1]
    P = potential(n, edges, g, V, f, ss)
    assert P.max() - P.min() < 1e-8 * (1 + np.max(np.abs(ss)))
