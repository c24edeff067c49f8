"""Pins of the oracle's eigen-solvers, Chebyshev filter, Lanczos bound and ChFSI (no GPU)."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, eig as E, chebyshev as Ch, chfsi as C, lanczos as Lz

from test_oracle_operator import laplace_eigs


# ----------------------------------------------------------------------------- eigen-solvers
def test_jacobi_bruteforce_matches_closed_form():
    A = O.assemble(si.laplace_operator(5)).toarray()
    w, V = E.jacobi_eigh(A)
    np.testing.assert_allclose(w, laplace_eigs(5), rtol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(25), atol=1e-13)
    np.testing.assert_allclose(A @ V, V * w, atol=1e-11 * w[-1])


def test_dense_smallest_matches_jacobi_on_random_operator():
    op = si.divk_operator(6, 4, 17)
    A = O.assemble(op)
    wj, Vj = E.jacobi_eigh(A.toarray())
    w, V = E.smallest_eigenpairs(A, 10, method="dense")
    np.testing.assert_allclose(w, wj[:10], rtol=1e-12)
    assert np.max(E.subspace_sines(V, Vj[:, :10])) < 1e-10


@pytest.mark.slow
def test_shift_invert_matches_closed_form_at_n_10000():
    A = O.assemble(si.laplace_operator(100))
    w, V = E.smallest_eigenpairs(A, 100, method="shift_invert")
    np.testing.assert_allclose(w, laplace_eigs(100)[:100], rtol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(100), atol=1e-12)


def test_shift_invert_matches_dense_on_random_operator():
    A = O.assemble(si.operator(si.CONFIGS[1], 2))
    w1, V1 = E.smallest_eigenpairs(A, 16, method="dense")
    w2, V2 = E.smallest_eigenpairs(A, 16, method="shift_invert")
    np.testing.assert_allclose(w2, w1, rtol=1e-12)
    for a, b in E.clusters(w1):
        if b >= 16:
            break
        assert np.max(E.subspace_sines(V1[:, a:b], V2[:, a:b])) < 1e-9


def test_canonical_sign():
    V = np.array([[0.1, -3.0], [-2.0, 3.0], [1.0, 0.5]])
    S = E.canonical_sign(V)
    np.testing.assert_array_equal(S[:, 0], -V[:, 0])
    np.testing.assert_array_equal(S[:, 1], -V[:, 1])   # tie |-3| = |3| goes to index 0


# ----------------------------------------------------------------------------- Chebyshev
def test_cheb_closed_form_vs_recurrence_and_low_degrees():
    t = np.linspace(-3, 3, 601)
    for m in range(0, 25):
        np.testing.assert_allclose(Ch.cheb(m, t), Ch.cheb_recurrence(m, t),
                                   rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(Ch.cheb(2, t), 2 * t * t - 1, atol=1e-12)
    np.testing.assert_allclose(Ch.cheb(3, t), 4 * t ** 3 - 3 * t, rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("m", [1, 2, 7, 20])
def test_filter_on_exact_sine_modes(m):
    """p_m(A) v = C_m((mu-c)/e) / C_m((lambda-c)/e) v on the closed-form eigenvectors."""
    N = 16
    h = 1.0 / (N + 1)
    x = (np.arange(N) + 1.0) * h
    A = O.assemble(si.laplace_operator(N))
    modes = [(1, 1), (1, 2), (3, 2), (7, 9), (16, 16)]
    Y0 = np.stack([np.outer(np.sin(j * np.pi * x), np.sin(i * np.pi * x)).ravel()
                   for i, j in modes], axis=1)
    mu = np.array([4 / h ** 2 * (np.sin(i * np.pi * h / 2) ** 2 + np.sin(j * np.pi * h / 2) ** 2)
                   for i, j in modes])
    lam, alpha, beta = mu[0], mu[2] * 1.01, 8.0 / h ** 2
    c, e = (alpha + beta) / 2, (beta - alpha) / 2
    Y = Ch.filter_block(A, Y0, m, lam, c, e)
    np.testing.assert_allclose(Y, Y0 * Ch.filter_gain(mu, m, lam, c, e), rtol=1e-10, atol=1e-12)
    assert abs(Ch.filter_gain(mu[:1], m, lam, c, e)[0] - 1.0) < 1e-12


def test_filter_on_random_operator_eigenvectors():
    A = O.assemble(si.operator(si.CONFIGS[1], 0))
    w, V = np.linalg.eigh(A.toarray())
    sel = [0, 3, 30, 200, 1023]
    lam, alpha, beta = w[0], w[40], w[-1] * 1.05
    c, e = (alpha + beta) / 2, (beta - alpha) / 2
    Y = Ch.filter_block(A, V[:, sel], 20, lam, c, e)
    g = Ch.filter_gain(w[sel], 20, lam, c, e)
    np.testing.assert_allclose(Y, V[:, sel] * g, atol=1e-9 * np.max(np.abs(g)))
    assert g[0] == pytest.approx(1.0, abs=1e-12)
    assert abs(g[-1]) <= 1.0 / abs(Ch.cheb(20, np.array([(lam - c) / e]))[0]) * (1 + 1e-12)


# ----------------------------------------------------------------------------- Lanczos
def test_lanczos_bounds_bracket_lambda_max():
    N = 20
    A = O.assemble(si.laplace_operator(N))
    lmax = laplace_eigs(N)[-1]
    lo, hi, ub = Lz.lanczos_bounds(A, 20, np.random.default_rng(0).standard_normal(N * N))
    assert hi <= lmax * (1 + 1e-12) and ub >= lmax and lo >= laplace_eigs(N)[0] * (1 - 1e-12)
    assert Lz.gershgorin_upper(A) >= lmax


def test_lanczos_full_length_recovers_extremes():
    A = O.assemble(si.divk_operator(4, 4, 9))
    w = np.linalg.eigvalsh(A.toarray())
    lo, hi, _ = Lz.lanczos_bounds(A, 16, np.random.default_rng(1).standard_normal(16))
    assert lo == pytest.approx(w[0], rel=1e-9) and hi == pytest.approx(w[-1], rel=1e-9)


def test_upper_bound_is_min_of_both():
    A = O.assemble(si.operator(si.CONFIGS[1], 4))
    ub = Lz.upper_bound(A, 20, seed=2)
    assert ub >= np.linalg.eigvalsh(A.toarray())[-1]
    assert ub <= Lz.gershgorin_upper(A)


# ----------------------------------------------------------------------------- ChFSI
def _check_solution(A, res, L, tol):
    n = A.shape[0]
    V, lam = res.evecs, res.evals
    np.testing.assert_allclose(V.T @ V, np.eye(L), atol=1e-12)
    R = A @ V - V * lam
    rel = np.linalg.norm(R, axis=0) / np.linalg.norm(A @ V, axis=0)
    assert np.all(rel <= tol * 1.0000001)
    assert np.all(np.diff(lam) >= 0)


@pytest.mark.parametrize("tol", [1e-8, 1e-12])
def test_chfsi_matches_dense_eigensolver(tol):
    A = O.assemble(si.operator(si.CONFIGS[1], 5))
    L = 16
    r = C.chfsi(A, L, 24, 20, tol, seed=11)
    assert r.converged
    w, V = E.smallest_eigenpairs(A, L + 8)
    _check_solution(A, r, L, tol)
    np.testing.assert_allclose(r.evals, w[:L], rtol=1e-10)
    # subspace angle per cluster (relative gap 1e-2); a cluster straddling L is skipped
    for a, b in E.clusters(w):
        if b > L:
            break
        s = np.max(E.subspace_sines(r.evecs[:, a:b], V[:, a:b]))
        assert s <= (1e-6 if tol < 1e-10 else 1e-6 * 100), (a, b, s)


def test_chfsi_laplacian_closed_form_at_cluster_boundary():
    A = O.assemble(si.laplace_operator(32))
    r = C.chfsi(A, 15, 24, 20, 1e-10, seed=1)     # lambda_16 = lambda_17, so stop at L = 15
    np.testing.assert_allclose(r.evals, laplace_eigs(32)[:15], rtol=1e-10)


def test_identical_operator_warm_start_converges_at_once():
    """App. E.7: re-solving the same operator (0% perturbation) needs almost no work."""
    A = O.assemble(si.operator(si.CONFIGS[1], 7))
    r = C.chfsi(A, 16, 24, 20, 1e-8, seed=3)
    r2 = C.chfsi(A, 16, 24, 20, 1e-8, X0=r.X_next, theta0=r.theta_next)
    assert r2.iterations == 1 and r2.converged
    np.testing.assert_allclose(r2.evals, r.evals, rtol=1e-12)


def test_max_iter_reports_unconverged():
    A = O.assemble(si.operator(si.CONFIGS[1], 8))
    r = C.chfsi(A, 16, 24, 20, 1e-8, seed=3, max_iter=1)
    assert not r.converged and r.iterations == 1 and r.evals.shape == (16,)


def test_invalid_sizes_rejected():
    A = O.assemble(si.laplace_operator(4))
    with pytest.raises(ValueError):
        C.chfsi(A, 8, 8, 10, 1e-8)
    with pytest.raises(ValueError):
        C.chfsi(A, 8, 17, 10, 1e-8)


# ------------------------------------------------------------- stopping rule: the L smallest
def test_wanted_locked_rule():
    assert not C.wanted_locked([1.0, 2.0], [5.0], 3)               # fewer than L locked
    assert C.wanted_locked([1.0, 2.0, 3.0], [5.0], 3)
    assert not C.wanted_locked([1.0, 2.0, 6.0], [5.0], 3)          # 5 < 6: a pair may be missing
    assert C.wanted_locked([1.0, 2.0, 6.0, 4.0], [5.0], 3)
    assert C.wanted_locked([1.0, 2.0, 6.0], [], 3)                 # nothing left unconverged
    assert C.wanted_locked([1.0, 5.0, 2.0], [5.0], 3)              # equal value counts


def planted_late_pairs():
    """A diagonal operator whose two smallest eigenvectors are present in the warm-start block
    only as small admixtures of two guard columns, while exact eigenvectors of larger values
    (with lambda = 12 missing) converge at once: the two small pairs are found after three
    larger ones were locked."""
    import scipy.sparse as sp
    lam = np.array([1.0, 2.0] + list(np.arange(10.0, 48.0)))
    A = sp.diags(lam).tocsr()

    def e(v):
        x = np.zeros(lam.size)
        x[int(np.nonzero(lam == v)[0][0])] = 1.0
        return x
    u1 = e(14.0) + 1e-3 * e(1.0)
    u2 = e(15.0) + 1e-7 * e(2.0)
    X0 = np.stack([e(10.0), e(11.0), e(13.0), u1 / np.linalg.norm(u1),
                   u2 / np.linalg.norm(u2), e(16.0)], axis=1)
    th0 = np.array([x @ (A @ x) for x in X0.T])
    return A, X0, th0


def test_chfsi_returns_the_L_smallest_when_pairs_enter_late():
    A, X0, th0 = planted_late_pairs()
    r = C.chfsi(A, 4, 6, 2, 1e-10, X0=X0, theta0=th0, beta=60.0, max_iter=200)
    assert r.converged
    np.testing.assert_allclose(r.evals, [1.0, 2.0, 10.0, 11.0], rtol=1e-12)
    # stopping as soon as L pairs are locked, and returning the first L of them, would give
    # 1, 10, 11, 13 here: lambda = 2 is still unconverged below the locked 13 at that point
    old = C.wanted_locked
    try:
        C.wanted_locked = lambda locked, active, L: len(locked) >= L
        bad = C.chfsi(A, 4, 6, 2, 1e-10, X0=X0, theta0=th0, beta=60.0, max_iter=200)
    finally:
        C.wanted_locked = old
    assert not np.allclose(bad.evals, [1.0, 2.0, 10.0, 11.0])
