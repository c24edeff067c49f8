"""Pins of the thin-plate vibration family (no GPU): the assembled K against a pointwise
finite-difference definition, the closed-form spectrum of the constant plate, the standard
form against the generalized eigenproblem, and ChFSI on the standard form."""
import numpy as np
import pytest
import scipy.linalg

import scsf_inputs as si
from oracle import operator as O, eig as E, chfsi as C


def pointwise_plate(op, u):
    """(del_h^2 (D del_h^2 u))_p by loops: del_h^2 w at node p is
    (4 w_p - w_W - w_E - w_S - w_N) / h^2 with w = 0 beyond the boundary."""
    N = op.N
    h = 1.0 / (N + 1)
    U = u.reshape(N, N)

    def lap(W):
        out = np.zeros_like(W)
        for iy in range(N):
            for ix in range(N):
                s = 4 * W[iy, ix]
                for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                    y, x = iy + dy, ix + dx
                    if 0 <= y < N and 0 <= x < N:
                        s -= W[y, x]
                out[iy, ix] = s / (h * h)
        return out
    return lap(op.D * lap(U)).ravel()


def test_plate_matrix_matches_pointwise_definition():
    op = si.plate_operator(6, 4, 11)
    K, M = O.assemble_plate_pair(op)
    rng = np.random.default_rng(0)
    for _ in range(3):
        u = rng.standard_normal(op.n)
        np.testing.assert_allclose(K @ u, pointwise_plate(op, u), rtol=1e-12,
                                   atol=1e-12 * np.abs(K @ u).max())
    np.testing.assert_array_equal(M.diagonal(), op.rho.ravel())
    assert abs(K - K.T).max() == 0.0


def test_constant_plate_closed_form_spectrum():
    """D = d, rho = r: K = d L^2, M = r I, so lambda = (d / r) mu^2 with
    mu = 4/h^2 (sin^2(i pi h / 2) + sin^2(j pi h / 2))."""
    N, d, r = 12, 2.5, 0.8
    op = si.Plate(N=N, D=np.full((N, N), d), rho=np.full((N, N), r), field=np.zeros((2, N, N)))
    h = 1.0 / (N + 1)
    s = np.sin(np.arange(1, N + 1) * np.pi * h / 2) ** 2
    mu = (4 / h ** 2 * (s[:, None] + s[None, :])).ravel()
    lam = np.sort((d / r) * mu ** 2)
    w = np.linalg.eigvalsh(O.assemble_plate(op).toarray())
    np.testing.assert_allclose(w, lam, rtol=1e-11)


def test_standard_form_matches_generalized_problem():
    op = si.plate_operator(9, 4, 3)
    K, M = O.assemble_plate_pair(op)
    wg, Ug = scipy.linalg.eigh(K.toarray(), M.toarray())
    A = O.assemble_plate(op)
    w, Y = np.linalg.eigh(A.toarray())
    np.testing.assert_allclose(w, wg, rtol=1e-10)
    U = Y / np.sqrt(op.rho.ravel())[:, None]          # u = M^{-1/2} y
    np.testing.assert_allclose(U.T @ M @ U, np.eye(op.n), atol=1e-10)
    R = K @ U[:, :8] - (M @ U[:, :8]) * w[:8]
    assert np.abs(R).max() <= 1e-9 * np.abs(K @ U[:, :8]).max()
    # energy identity u^T K u = sum_p D_p (L u)_p^2 > 0
    u = np.random.default_rng(1).standard_normal(op.n)
    Lu = O.dirichlet_laplacian(op.N) @ u
    assert u @ (K @ u) == pytest.approx(np.sum(op.D.ravel() * Lu ** 2), rel=1e-12)


def test_chfsi_on_the_plate_standard_form():
    op = si.plate_operator(14, 4, 5)
    A = O.assemble_plate(op)
    w, V = E.smallest_eigenpairs(A, 14, method="dense")
    r = C.chfsi(A, 8, 14, 20, 1e-8, seed=2, max_iter=2000)
    assert r.converged
    np.testing.assert_allclose(r.evals, w[:8], rtol=1e-10)
