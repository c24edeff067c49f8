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


def test_lower_end_route_on_helmholtz_against_dense():
    """A Helmholtz operator with a short negative spectrum: the L + 1 algebraically smallest
    pairs contain the L smallest in magnitude, and the certificate says so."""
    op = si.helmholtz_operator(20, 8, 7)                     # 9 negative eigenvalues
    A = O.assemble(op)
    w, V = np.linalg.eigh(A.toarray())
    L = 30
    assert w[0] < 0 < w[L] and abs(w[0]) <= w[L]             # indefinite, certificate true
    r, ok = Mg.smallest_magnitude_lower_end(A, L, 40, 20, 1e-10, seed=4)
    assert ok
    ref = by_magnitude(w)[:L]
    np.testing.assert_allclose(r.evals, ref, rtol=1e-10, atol=1e-10 * np.abs(w).max())
    X = r.evecs
    rel = np.linalg.norm(A @ X - X * r.evals, axis=0) / np.linalg.norm(A @ X, axis=0)
    assert rel.max() <= 1e-10 * (1 + 1e-6)


def test_lower_end_route_refuses_a_deep_negative_spectrum():
    """L - c I with c in the middle of the wanted window: the L + 1 lowest eigenvalues are all
    negative and far from zero, so the certificate fails (the squared filter is needed), and
    the dense spectrum confirms that the lower end does not hold the smallest magnitudes."""
    N = 14
    h = 1.0 / (N + 1)
    s = np.sin(np.arange(1, N + 1) * np.pi * h / 2) ** 2
    mu = np.sort((4 / h ** 2 * (s[:, None] + s[None, :])).ravel())
    c = mu[40] + 1.7
    A = (O.assemble(si.laplace_operator(N)) - c * sp.identity(N * N)).tocsr()
    r, ok = Mg.smallest_magnitude_lower_end(A, 8, 16, 20, 1e-10, seed=5)
    assert not ok
    assert not np.allclose(np.sort(r.evals), np.sort(by_magnitude(mu - c)[:8]))


def test_lower_end_gives_up_early_when_no_certificate_can_come():
    """A Helmholtz operator with 46 negative eigenvalues and L = 12, k = 20: the block holds
    only negative values, the top pairs of the block never converge, so only the early exit
    ends the lower-end route (uncertified, within a few outer iterations, not at max_iter)."""
    A = O.assemble(si.helmholtz_operator(24, 8, 54))
    w = np.linalg.eigvalsh(A.toarray())
    assert np.count_nonzero(w < 0) > 20
    r, ok = Mg.smallest_magnitude_lower_end(A, 12, 20, 20, 1e-9, seed=2, max_iter=200)
    assert not ok and r.iterations < 20


def test_magnitude_hopeless_rule():
    """The give-up rule of the lower-end route against hand-made blocks, and never on a
    certified state (random blocks)."""
    assert C.magnitude_hopeless([], [-5.0, -4.0, -3.0], 1)          # every |theta| > max
    assert not C.magnitude_hopeless([-1.0], [2.0, 3.0], 3)           # |-1|, 2, 3 <= 3
    assert C.magnitude_hopeless([-9.0, -1.0], [2.0, 3.0], 4)         # |-9| > 3: only three
    rng = np.random.default_rng(4)
    for _ in range(2000):
        L = int(rng.integers(1, 6))
        thl = np.sort(rng.normal(0.0, 3.0, int(rng.integers(0, 9))))
        tha = np.sort(rng.normal(1.0, 3.0, int(rng.integers(0, 9))))
        if C.magnitude_certified(thl, tha, L):
            assert not C.magnitude_hopeless(thl, tha, L)


def test_smallest_magnitude_definition_dense_and_shift_invert_agree():
    """The plain definition (eigenvalues nearest 0) by dense eigh and by shift-invert about 0,
    on an indefinite Helmholtz operator and on a shifted Laplacian's closed form."""
    from oracle import eig as E
    A = O.assemble(si.helmholtz_operator(24, 8, 9))
    w1, V1 = E.smallest_magnitude_eigenpairs(A, 20, method="dense")
    w2, V2 = E.smallest_magnitude_eigenpairs(A, 20, method="shift_invert")
    np.testing.assert_allclose(w2, w1, rtol=1e-11, atol=1e-9)
    assert np.any(w1 < 0) and np.all(np.diff(np.abs(w1)) >= 0)
    assert np.max(E.subspace_sines(V1, V2)) < 1e-8
    N = 14
    h = 1.0 / (N + 1)
    s = np.sin(np.arange(1, N + 1) * np.pi * h / 2) ** 2
    mu = (4 / h ** 2 * (s[:, None] + s[None, :])).ravel()
    c = np.sort(mu)[25] + 2.9
    B = (O.assemble(si.laplace_operator(N)) - c * sp.identity(N * N)).tocsr()
    w3, _ = E.smallest_magnitude_eigenpairs(B, 10, method="shift_invert")
    np.testing.assert_allclose(w3, by_magnitude(mu - c)[:10], rtol=1e-10, atol=1e-9)


def test_magnitude_certificate_with_a_large_negative_outlier():
    """Eigenvalues -10, -1, 1, 2, 3, ...: the L = 3 of smallest magnitude (-1, 1, 2) are not the
    3 algebraically smallest, but the 4 lowest hold 3 with |lambda| <= lambda_4 = 2."""
    lam = np.array([-10.0, -1.0] + list(np.arange(1.0, 59.0)))
    A = sp.diags(lam).tocsr()
    assert C.magnitude_certified([-10.0, -1.0, 1.0, 2.0], [3.0], 3)
    assert not C.magnitude_certified([-10.0, -1.0, 1.0], [2.0], 3)
    assert not C.magnitude_certified([-10.0, -9.0, -8.0, -7.0], [], 3)
    r, ok = Mg.smallest_magnitude_lower_end(A, 3, 8, 20, 1e-10, seed=6)
    assert ok
    np.testing.assert_allclose(r.evals, [-1.0, 1.0, 2.0], rtol=1e-12)


def test_smallest_eigenpairs_of_an_indefinite_operator():
    """The L algebraically smallest of an indefinite operator by shift-invert (about the
    Gershgorin lower end) equal the dense ones; about 0 they would be the nearest to 0."""
    from oracle import eig as E
    A = O.assemble(si.helmholtz_operator(24, 8, 5))
    w = np.linalg.eigvalsh(A.toarray())
    assert w[0] < 0 and (w < 0).sum() > 20
    w2, V2 = E.smallest_eigenpairs(A, 20, method="shift_invert")
    np.testing.assert_allclose(w2, w[:20], rtol=1e-11, atol=1e-9)
    R = A @ V2 - V2 * w2
    assert np.max(np.linalg.norm(R, axis=0)) < 1e-8 * np.abs(w).max()
