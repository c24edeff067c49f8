"""Pins of the smallest-magnitude ChFSI (no GPU): a shifted Laplacian with its closed-form
spectrum, an indefinite Helmholtz operator against the dense eigensolver, and the positive
definite case where it must agree with the plain method."""
import numpy as np
import pytest
import scipy.sparse as sp

import scsf_inputs as si
from oracle import operator as O, chfsi as C, magnitude as Mg


def by_magnitude(w):
    return w[np.argsort(np.abs(w), kind="stable")]


def test_shifted_laplacian_closed_form():
    """A = L - c I: eigenvalues mu_ij - c; the smallest |.| straddle zero."""
    N = 14
    h = 1.0 / (N + 1)
    s = np.sin(np.arange(1, N + 1) * np.pi * h / 2) ** 2
    mu = (4 / h ** 2 * (s[:, None] + s[None, :])).ravel()
    c = 0.5 * (np.sort(mu)[20] + np.sort(mu)[21]) + 3.3       # no two |mu - c| equal
    A = (O.assemble(si.laplace_operator(N)) - c * sp.identity(N * N)).tocsr()
    r = Mg.chfsi_magnitude(A, 12, 20, 20, 1e-10, seed=1)
    assert r.converged
    ref = by_magnitude(mu - c)[:12]
    np.testing.assert_allclose(r.evals, ref, rtol=1e-10)
    assert np.any(ref < 0) and np.any(ref > 0)


def test_helmholtz_against_dense():
    op = si.helmholtz_operator(16, 8, 7)
    A = O.assemble(op)
    w, V = np.linalg.eigh(A.toarray())
    assert w[0] < 0 < w[-1]                                    # indefinite
    order = np.argsort(np.abs(w), kind="stable")
    r = Mg.chfsi_magnitude(A, 10, 16, 20, 1e-9, seed=2)
    assert r.converged
    np.testing.assert_allclose(r.evals, w[order[:10]], rtol=1e-10, atol=1e-10 * np.abs(w).max())
    X = r.evecs
    R = A @ X - X * r.evals
    assert np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(A @ X, axis=0)) <= 1e-9 * (1 + 1e-6)
    # each vector in the eigenspace of its eigenvalue (gaps here are well above 1e-6)
    for j in range(10):
        v = V[:, order[j]]
        assert abs(abs(v @ X[:, j]) - 1.0) < 1e-8


def test_positive_definite_case_matches_the_plain_method():
    op = si.operator(si.CONFIGS[1], 0)
    A = O.assemble(op)
    a = Mg.chfsi_magnitude(A, 8, 16, 20, 1e-9, seed=3)
    b = C.chfsi(A, 8, 16, 20, 1e-9, seed=3)
    np.testing.assert_allclose(a.evals, b.evals, rtol=1e-10)


def test_gershgorin_interval_contains_the_spectrum():
    A = O.assemble(si.helmholtz_operator(12, 8, 3))
    lo, hi = Mg.gershgorin_interval(A)
    w = np.linalg.eigvalsh(A.toarray())
    assert lo <= w[0] and w[-1] <= hi
