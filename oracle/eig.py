"""The result SCSF reaches: the L algebraically smallest eigenpairs (oracle).

Eq. (eq_basic) of Section 2.1 asks, for each matrix, for L eigenpairs ordered by |lambda|; the
operators here are symmetric positive definite so this is the L smallest.  The method is an
acceleration that does not change the result at the requested precision (Section 4.1), so the
plain definition -- a full symmetric eigendecomposition -- is the reference:

* n <= 4096: dense `numpy.linalg.eigh`;
* larger n: ARPACK shift-invert (`scipy.sparse.linalg.eigsh(sigma=s)`) run to machine
  tolerance, which returns the eigenvalues nearest s: s = 0 when the Gershgorin interval is
  nonnegative (then the nearest to 0 are the smallest), else s = the Gershgorin lower end
  (every eigenvalue lies above it, so the nearest are again the smallest; an indefinite
  operator needs this).

`jacobi_eigh` is the textbook cyclic Jacobi method, used as a brute-force cross-check on
tiny matrices.  `canonical_sign` fixes the sign of eigenvectors: the entry of largest
magnitude is made positive (ties go to the lowest index).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def canonical_sign(V: np.ndarray) -> np.ndarray:
    V = np.array(V, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(V), axis=0)
    s = np.sign(V[idx, np.arange(V.shape[1])])
    s[s == 0] = 1.0
    return V * s


def smallest_eigenpairs(A, L: int, method: str = "auto"):
    """(lambda[0:L] ascending, V n x L orthonormal) of a symmetric matrix A."""
    n = A.shape[0]
    if method == "auto":
        method = "dense" if n <= 4096 else "shift_invert"
    if method == "dense":
        M = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
        w, V = np.linalg.eigh(M)
        return w[:L].copy(), canonical_sign(V[:, :L])
    if method == "shift_invert":
        As = sp.csc_matrix(A)
        d = As.diagonal()
        lo = float(np.min(d - (np.asarray(abs(As).sum(axis=1)).ravel() - np.abs(d))))
        sigma = 0.0 if lo >= 0.0 else lo - 1e-3 * abs(lo)
        w, V = sla.eigsh(As, k=L, sigma=sigma, which="LM", tol=0)
        order = np.argsort(w)
        return w[order], canonical_sign(V[:, order])
    raise ValueError(method)


def smallest_magnitude_eigenpairs(A, L: int, method: str = "auto"):
    """(lambda[0:L] ordered by |lambda|, V n x L) of a symmetric, possibly indefinite matrix:
    the L eigenvalues nearest 0 (the smallest in absolute value, as the Helmholtz experiments
    ask).  Dense `eigh` sorted by |lambda| up to n = 4096, else ARPACK shift-invert about 0,
    whose largest |1 / (lambda - 0)| are exactly those."""
    n = A.shape[0]
    if method == "auto":
        method = "dense" if n <= 4096 else "shift_invert"
    if method == "dense":
        M = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
        w, V = np.linalg.eigh(M)
    elif method == "shift_invert":
        w, V = sla.eigsh(sp.csc_matrix(A), k=L, sigma=0.0, which="LM", tol=0)
    else:
        raise ValueError(method)
    order = np.argsort(np.abs(w), kind="stable")[:L]
    return w[order], canonical_sign(V[:, order])


def jacobi_eigh(S: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Cyclic-by-row Jacobi for a small symmetric matrix; returns ascending (w, V)."""
    A = np.array(S, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    scale = np.linalg.norm(A)
    for _ in range(max_sweeps):
        off = np.linalg.norm(A - np.diag(np.diag(A)))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0.0:
                    continue
                # rotation angle that annihilates A[p, q]
                if abs(apq) <= 1e-300 * max(abs(A[p, p]), abs(A[q, q]), 1.0):
                    continue
                zeta = (A[q, q] - A[p, p]) / (2.0 * apq)
                if abs(zeta) > 1e150:                    # t ~ 1/(2 zeta) without overflow
                    t = 1.0 / (2.0 * zeta)
                else:
                    t = np.sign(zeta) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta)) if zeta != 0 else 1.0
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                J = np.array([[c, s], [-s, c]])
                A[[p, q], :] = J.T @ A[[p, q], :]
                A[:, [p, q]] = A[:, [p, q]] @ J
                V[:, [p, q]] = V[:, [p, q]] @ J
    w = np.diag(A).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def subspace_sines(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Sines of the principal angles between span(U) and span(V) (both orthonormal, same
    width): the singular values of (I - U U^T) V, accurate also for tiny angles."""
    return np.sort(np.linalg.svd(V - U @ (U.T @ V), compute_uv=False))


def clusters(w: np.ndarray, rel_gap: float = 1e-2):
    """Maximal runs of ascending eigenvalues whose consecutive relative gaps are < rel_gap."""
    out, start = [], 0
    for j in range(1, len(w) + 1):
        if j == len(w) or (w[j] - w[j - 1]) >= rel_gap * abs(w[j - 1]):
            out.append((start, j))
            start = j
    return out
