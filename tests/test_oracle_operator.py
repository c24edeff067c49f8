"""Pins of the oracle's operator assembly (no GPU)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import scsf_inputs as si
from oracle import operator as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def laplace_eigs(N):
    """(4/h^2)(sin^2(i pi h/2) + sin^2(j pi h/2)), i, j = 1..N, ascending."""
    h = 1.0 / (N + 1)
    s = np.sin(np.arange(1, N + 1) * np.pi * h / 2.0) ** 2
    return np.sort((4.0 / h ** 2 * (s[:, None] + s[None, :])).ravel())


def test_worked_example_2x2():
    """Section 2.1 eq. (eq_p): k == 1 on a 2x2 grid, unit spacing, row-major order."""
    M = np.loadtxt(os.path.join(GOLDEN, "eq_p_2x2.txt"))
    A = O.assemble(si.laplace_operator(2)).toarray()
    h = 1.0 / 3.0
    # the paper's k Laplace u carries the opposite sign of -div(K grad u) and no 1/h^2
    np.testing.assert_array_equal(-A * h * h, M)
    np.testing.assert_allclose(np.linalg.eigvalsh(M), [-6.0, -4.0, -4.0, -2.0], atol=1e-14)


def test_kronecker_sum_of_1d_matrix():
    """K == 1 gives (T (x) I + I (x) T)/h^2 with T = tridiag(-1, 2, -1), the 1-D central
    difference matrix of App. C taken with the sign of -d^2/dx^2."""
    N = 7
    h = 1.0 / (N + 1)
    T = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    ref = (np.kron(T, np.eye(N)) + np.kron(np.eye(N), T)) / h ** 2
    np.testing.assert_allclose(O.assemble(si.laplace_operator(N)).toarray(), ref, rtol=1e-15)


@pytest.mark.parametrize("N", [5, 12, 32])
def test_laplacian_closed_form_spectrum(N):
    A = O.assemble(si.laplace_operator(N)).toarray()
    np.testing.assert_allclose(np.linalg.eigvalsh(A), laplace_eigs(N), rtol=1e-12)


def test_laplacian_sine_eigenvectors():
    N = 9
    h = 1.0 / (N + 1)
    x = (np.arange(N) + 1.0) * h
    A = O.assemble(si.laplace_operator(N))
    for i, j in [(1, 1), (2, 5), (9, 3)]:
        v = np.outer(np.sin(j * np.pi * x), np.sin(i * np.pi * x)).ravel()   # [iy, ix]
        lam = 4 / h ** 2 * (np.sin(i * np.pi * h / 2) ** 2 + np.sin(j * np.pi * h / 2) ** 2)
        np.testing.assert_allclose(A @ v, lam * v, rtol=1e-12, atol=1e-9 * lam)


def test_random_k_is_spd_and_courant_fischer():
    """A(K) = sum_f K_f a_f a_f^T / h^2, so Kmin lam_j(Lap) <= lam_j(A) <= Kmax lam_j(Lap)."""
    op = si.operator(si.CONFIGS[1], 3)
    A = O.assemble(op)
    assert abs(A - A.T).max() == 0.0
    h2 = (1.0 / (op.N + 1)) ** 2
    kmin = min(op.wx.min(), op.wy.min()) * h2
    kmax = max(op.wx.max(), op.wy.max()) * h2
    lam = np.linalg.eigvalsh(A.toarray())
    lap = laplace_eigs(op.N)
    assert lam[0] > 0
    assert np.all(lam >= kmin * lap * (1 - 1e-12))
    assert np.all(lam <= kmax * lap * (1 + 1e-12))


def test_potential_family_bounds():
    op = si.potential_operator(16, 8, 5)
    assert op.v.min() == 0.0 and abs(op.v.max() - 100.0) < 1e-12
    lam = np.linalg.eigvalsh(O.assemble(op).toarray())
    lap = laplace_eigs(16)
    assert np.all(lam >= lap - 1e-9) and np.all(lam <= lap + 100.0 + 1e-9)


def test_face_sum_quadratic_form():
    """u^T A u = sum over faces w_f (u_a - u_b)^2 (+ boundary faces w_f u_a^2), the energy the
    conservative difference scheme discretises."""
    op = si.operator(si.CONFIGS[1], 1)
    N = op.N
    rng = np.random.default_rng(0)
    U = rng.standard_normal((N, N))
    Up = np.pad(U, 1)                       # zero Dirichlet frame
    ex = np.sum(op.wx * (Up[1:-1, 1:] - Up[1:-1, :-1]) ** 2)
    ey = np.sum(op.wy * (Up[1:, 1:-1] - Up[:-1, 1:-1]) ** 2)
    u = U.ravel()
    assert abs(u @ (O.assemble(op) @ u) - (ex + ey)) <= 1e-12 * (ex + ey)


def q1_laplace_eigs(N):
    h = 1.0 / (N + 1)
    c = np.cos(np.arange(1, N + 1) * np.pi * h)
    lam = (8 - 2 * c[:, None] - 2 * c[None, :] - 4 * c[:, None] * c[None, :]) / (3 * h * h)
    return np.sort(lam.ravel())


def test_q1_isotropic_closed_form():
    N = 10
    op = si.aniso_operator(N, 4, 0)
    op.cell[:] = [1.0, 0.0, 1.0]
    np.testing.assert_allclose(np.linalg.eigvalsh(O.assemble(op).toarray()), q1_laplace_eigs(N),
                               rtol=1e-12)


def test_q1_energy_by_gauss_quadrature():
    """u^T A u h^2 = sum over cells of the integral of grad(u_h)^T K grad(u_h) for the bilinear
    interpolant u_h, evaluated here by 2x2 Gauss quadrature (exact for these integrands)."""
    N = 6
    op = si.aniso_operator(N, 4, 11)
    h = 1.0 / (N + 1)
    rng = np.random.default_rng(1)
    U = np.pad(rng.standard_normal((N, N)), 1)
    g = 0.5 + np.array([-1, 1]) / (2 * np.sqrt(3))
    energy = 0.0
    for cy in range(N + 1):
        for cx in range(N + 1):
            u00, u10 = U[cy, cx], U[cy, cx + 1]          # (x,y) corners in cell coordinates
            u01, u11 = U[cy + 1, cx], U[cy + 1, cx + 1]
            k11, k12, k22 = op.cell[cy, cx]
            K = np.array([[k11, k12], [k12, k22]])
            for xi in g:
                for eta in g:
                    gx = ((u10 - u00) * (1 - eta) + (u11 - u01) * eta) / h
                    gy = ((u01 - u00) * (1 - xi) + (u11 - u10) * xi) / h
                    gr = np.array([gx, gy])
                    energy += 0.25 * h * h * gr @ K @ gr
    u = U[1:-1, 1:-1].ravel()
    A = O.assemble(op)
    assert abs(A - A.T).max() < 1e-9 * abs(A).max()
    assert abs(u @ (A @ u) * h * h - energy) <= 1e-12 * energy


def test_q1_random_tensor_bounds():
    """Each cell tensor satisfies 0.1 I <= K <= 10 I, hence 0.1 lam_j(Q1 Lap) <= lam_j(A) <= 10 lam_j."""
    op = si.aniso_operator(12, 8, 3)
    lam = np.linalg.eigvalsh(O.assemble(op).toarray())
    ref = q1_laplace_eigs(12)
    assert np.all(lam >= 0.1 * ref * (1 - 1e-12)) and np.all(lam <= 10.0 * ref * (1 + 1e-12))
