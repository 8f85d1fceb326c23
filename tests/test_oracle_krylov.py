"""Pins of the extended rational Krylov reference (Sec. IV-E, Alg. 1,
eqs. 21-27) against what the mathematics fixes: the Galerkin projection onto
the block rational Krylov space matches the full system's first q shifted
moments (eq. 24); a basis that spans the whole space reproduces full
backward Euler; eq. 26's time constant is that of the discrete line's slowest
mode; eq. 27's threshold; and the paper's accuracy statement (under 1 %
nucleation-time error at eta = 1, q = 4-6) on a blocked line."""
import numpy as np
import scipy.sparse as sp

from oracle import krylov as K


def line(n, rng, L=100e-6, kappa=1e-14, a=1e-13, wind=5e8):
    dx = L / (n - 1)
    parent = np.arange(-1, n - 1)
    g = np.full(n, a * kappa / dx) * rng.lognormal(0.0, 0.2, n)
    g[0] = 0.0
    V = np.full(n, a * dx)
    V[0] *= 0.5
    V[-1] *= 0.5
    # the wind's flux phi = g dx S enters a node and leaves its parent
    f = np.zeros(n)
    for i in range(1, n):
        phi = g[i] * dx * wind
        f[i] += phi
        f[i - 1] -= phi
    Cv, A = K.tree_matrices(parent, V, g)
    return Cv, A, f, dx


def reduced_moments(Ah, Ch, fh, z0, s0, k_max):
    Kh = s0 * Ch - Ah
    m = [np.linalg.solve(Kh, s0 * Ch @ z0 + fh)]
    if k_max > 1:
        m.append(np.linalg.solve(Kh, Ch @ z0 - Ch @ m[0]))
    for _ in range(2, k_max):
        m.append(-np.linalg.solve(Kh, Ch @ m[-1]))
    return m


def test_reduced_model_matches_the_first_q_shifted_moments():
    """From a zero initial state the space is K_q(R C, R f) and the Galerkin
    model matches m_0 .. m_(q-1) exactly; the moment after them is no longer
    matched (so a dropped or mis-built block fails here)."""
    rng = np.random.default_rng(1)
    Cv, A, f, dx = line(400, rng)
    x0 = np.zeros(400)
    s0 = 1.0 / 2e6
    for q in (3, 5, 6):
        V, Ah, Ch, fh = K.reduce(Cv, A, f, x0, s0, q)
        assert V.shape[1] == q                   # the zero column of the starting block dropped
        full = K.shifted_moments(Cv, A, f, x0, s0, q + 2)
        red = reduced_moments(Ah, Ch, fh, V.T @ x0, s0, q + 2)
        for k in range(q):
            err = np.linalg.norm(V @ red[k] - full[k]) / np.linalg.norm(full[k])
            assert err < 1e-7, (q, k, err)            # K's condition number is ~1e6 here
        err = np.linalg.norm(V @ red[q + 1] - full[q + 1]) / np.linalg.norm(full[q + 1])
        assert err > 1e-5, (q, err)


def test_a_uniform_initial_state_lies_in_the_space():
    """R C 1 = 1 / s0 (A 1 = 0): a uniform thermal stress is reproduced by the
    projection, and its direction adds no further block (dropped as dependent)."""
    rng = np.random.default_rng(5)
    Cv, A, f, dx = line(300, rng)
    x0 = np.full(300, 3e7)
    V, Ah, Ch, fh = K.reduce(Cv, A, f, x0, 1.0 / 2e6, 4)
    assert V.shape[1] == 1 + 4
    assert np.allclose(V @ (V.T @ x0), x0, rtol=1e-8)


def test_a_spanning_basis_reproduces_full_backward_euler():
    rng = np.random.default_rng(2)
    n = 12
    Cv, A, f, dx = line(n, rng)
    x0 = rng.normal(size=n) * 1e7
    V, Ah, Ch, fh = K.reduce(Cv, A, f, x0, 1.0 / 1e5, q=n)
    assert V.shape[1] == n
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-12)
    dt = 3e4
    z = K.reduced_be(V, Ah, Ch, fh, x0, dt, 50)
    ref = K.full_be(Cv, A, f, x0, dt, 50)
    assert np.allclose(z @ V.T, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_shift_time_is_the_slowest_line_mode():
    rng = np.random.default_rng(3)
    n, L, kappa = 401, 80e-6, 2e-14
    dx = L / (n - 1)
    V = np.full(n, dx)
    V[0] *= 0.5
    V[-1] *= 0.5
    g = np.full(n, kappa / dx)
    g[0] = 0.0
    Cv, A = K.tree_matrices(np.arange(-1, n - 1), V, g)
    lam = np.sort(np.linalg.eigvals(np.linalg.solve(np.diag(Cv), -A.toarray())).real)
    tau = K.shift_time(L, kappa, 1.0)
    assert abs(1.0 / lam[1] - tau) / tau < 1e-4
    assert abs(K.shift_time(L, kappa, 2.5) - 2.5 * tau) <= 1e-12 * tau


def test_selection_threshold():
    assert not K.krylov_selected(29, 4)
    assert K.krylov_selected(30, 4)
    assert not K.krylov_selected(35, 12)
    assert K.krylov_selected(36, 12)


def test_nucleation_time_within_one_percent_at_eta_one():
    """A blocked line under electron wind from the thermal stress: the
    reduced model's nucleation step (first step with the peak at sigma_crit)
    against full backward Euler."""
    rng = np.random.default_rng(4)
    n, L, kappa = 300, 100e-6, 1e-14
    Cv, A, f, dx = line(n, rng, L=L, kappa=kappa)
    x0 = np.full(n, 3e7)
    dt, steps = 1e3, 3000                            # tau = L^2 / (pi^2 kappa) is ~100 steps
    ref = K.full_be(Cv, A, f, x0, dt, steps)
    peak = ref.max(axis=1)
    scrit = 0.6 * peak[-1] + 0.4 * peak[0]         # crossed in the transient
    k_ref = int(np.argmax(peak >= scrit))
    assert 10 < k_ref < steps - 10
    s0 = 1.0 / K.shift_time(L, kappa, 1.0)
    errs = []
    for q in (4, 5, 6):
        V, Ah, Ch, fh = K.reduce(Cv, A, f, x0, s0, q)
        z = K.reduced_be(V, Ah, Ch, fh, x0, dt, steps)
        k = int(np.argmax((z @ V.T).max(axis=1) >= scrit))
        errs.append(abs(k - k_ref) / k_ref)
    assert max(errs) < 0.01, errs
