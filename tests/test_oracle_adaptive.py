"""Pins of the per-vector adaptive filter degree (no GPU)."""
import numpy as np
import scipy.sparse as sp

import scsf_inputs as si
from oracle import operator as O, eig as E, chebyshev as Ch, chfsi as C


def ritz_residual(A, x):
    th = x @ (A @ x) / (x @ x)
    w = A @ x
    return th, np.linalg.norm(w - th * x) / np.linalg.norm(w)


def test_degree_is_the_smallest_that_reaches_tol():
    """Diagonal operator, damped interval [10, 100], one wanted eigenvalue at 1 and an
    unwanted component at the interval's edge (|C_m| = 1 there): the predicted degree brings
    the residual to within a factor 2 of tol, one degree less does not reach tol."""
    spec = np.array([1.0, 10.0, 40.0, 100.0])
    A = sp.diags(spec).tocsr()
    alpha, beta = 10.0, 100.0
    c, e = (alpha + beta) / 2, (beta - alpha) / 2
    # the residual model is asymptotic: small contamination, Ritz value at the eigenvalue
    for delta, tol in ((1e-2, 1e-8), (1e-4, 1e-10), (1e-3, 1e-6)):
        x = np.array([1.0, delta, 0.0, 0.0])
        th, res = ritz_residual(A, x)
        m = int(Ch.adaptive_degrees([th], [res], tol, c, e, m_max=200)[0])
        y = Ch.filter_block(A, x[:, None], m, th, c, e)[:, 0]
        assert ritz_residual(A, y)[1] <= 2.05 * tol, (delta, tol, m)
        y1 = Ch.filter_block(A, x[:, None], m - 1, th, c, e)[:, 0]
        assert ritz_residual(A, y1)[1] > tol, (delta, tol, m)


def test_degree_clamps():
    c, e = 55.0, 45.0
    d = Ch.adaptive_degrees([1.0, 1.0, 50.0], [1e-12, 1.0, 1e-3], 1e-8, c, e, m_max=20, m_min=2)
    assert list(d) == [2, 20, 20] or (d[0] == 2 and d[2] == 20)
    assert d[1] <= 20


def test_adaptive_chfsi_reaches_dense_eigenpairs_in_fewer_iterations():
    """Degrees in [m, 2m] from the residuals: the same eigenpairs and fewer outer iterations;
    the filter work stays within a quarter of the plain iteration's (on these small blocks
    the guard vectors take the upper bound; on 24-wide blocks it was equal)."""
    its = {False: 0, True: 0}
    work = {False: 0, True: 0}
    for seed in (23, 29, 31):
        op = si.divk_operator(14, 4, seed)
        A = O.assemble(op)
        w, V = E.smallest_eigenpairs(A, 12, method="dense")
        for adaptive in (False, True):
            r = C.chfsi(A, 6, 10, 20, 1e-10, seed=3, adaptive=adaptive)
            assert r.converged
            np.testing.assert_allclose(r.evals, w[:6], rtol=1e-10)
            assert np.max(E.subspace_sines(r.evecs, V[:, :6])) < 1e-7
            its[adaptive] += r.iterations
            work[adaptive] += r.filter_matvecs
    assert its[True] < its[False]
    assert work[True] < 1.25 * work[False]
    seq = C.scsf_sequence([O.assemble(si.divk_operator(14, 4, s)) for s in (23, 24)], 6, 10, 20,
                          1e-10, adaptive=True)
    assert all(r.converged for r in seq.values())
