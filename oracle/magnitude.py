"""ChFSI for the eigenvalues of smallest magnitude of a symmetric, possibly indefinite operator
(oracle): the Helmholtz family of App. D.2, whose experiments ask for the L eigenvalues
smallest in absolute value (Section 4).

Reading: Algorithm 1 amplifies the low end of the spectrum of the operator it is given, so
the filter runs on B = A^2 (its low end is the spectrum of A near zero) while Rayleigh-Ritz,
the residual test and locking stay with A, the Ritz pairs ordered by |theta|:
  repeat
    filter the active block with the degree-m Chebyshev polynomial of B = A^2 on
      [alpha_B, beta_B], alpha_B = max active theta^2, beta_B >= max lambda(A)^2,
      normalised at lambda_B = min theta^2
    orthonormalise [locked | V0] (Householder QR)
    G = Q_a^T A Q_a, G W = W Theta, order the pairs by |theta|, V0 <- Q_a W
    lock the longest prefix with ||A v - theta v|| <= tol ||A v||
beta_B is the square of the larger end of A's Gershgorin interval.

Squaring the operator squares its spread, so the squared filter converges slowly at working
sizes.  When the negative part of the spectrum is short (the Helmholtz operators of App. D.2
at n = 6400 have tens of negative eigenvalues above -k^2 and their 200 smallest in magnitude
reach far into the positive part), the wanted pairs sit at the lower end of the spectrum and
the plain method finds them (`smallest_magnitude_lower_end`): Algorithm 3 at the lower end,
going on until the q algebraically smallest converged pairs lambda_1 <= ... <= lambda_q hold
L with |lambda| <= lambda_q; those L are then the L smallest in magnitude overall (every
eigenvalue outside the q is >= lambda_q).  When the block runs out of pairs before that
certificate holds, the squared filter is the route.
"""
from __future__ import annotations

import numpy as np

from .chebyshev import filter_block
from .chfsi import Result, _gaussian, chfsi
from .eig import canonical_sign


def gershgorin_interval(A):
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    return float(np.min(d - off)), float(np.max(d + off))


def _ritz_by_magnitude(A, Q):
    AQ = A @ Q
    G = Q.T @ AQ
    theta, Z = np.linalg.eigh(0.5 * (G + G.T))
    order = np.argsort(np.abs(theta), kind="stable")
    return theta[order], Q @ Z[:, order], AQ @ Z[:, order]


def chfsi_magnitude(A, L: int, k: int, m: int, tol: float, X0=None, theta0=None,
                    seed: int = 0, max_iter: int = 500) -> Result:
    n = A.shape[0]
    if not (0 < L < k <= n):
        raise ValueError("need 0 < L < k <= n")
    lo, hi = gershgorin_interval(A)
    beta = max(abs(lo), abs(hi)) ** 2
    A2 = A @ A
    if X0 is None:
        Q, _ = np.linalg.qr(_gaussian(n, k, seed))
        theta, X, _ = _ritz_by_magnitude(A, Q)
    else:
        X = np.array(X0, dtype=np.float64, copy=True)
        theta = np.array(theta0, dtype=np.float64, copy=True)
    Vl = np.zeros((n, 0))
    thl = np.zeros(0)
    matvecs, it = 0, 0
    while it < max_iter and thl.size < L:
        it += 1
        lam = (thl[0] if thl.size else theta[0]) ** 2
        alpha = float(np.max(theta ** 2))
        c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
        Y = filter_block(A2, X, m, lam, c, e)
        matvecs += 2 * m * X.shape[1]
        Q, _ = np.linalg.qr(np.hstack([Vl, Y]))
        theta, X, W = _ritz_by_magnitude(A, Q[:, Vl.shape[1]:])
        res = np.linalg.norm(W - X * theta, axis=0) / np.linalg.norm(W, axis=0)
        j = 0
        while j < theta.size and res[j] <= tol:
            j += 1
        Vl = np.hstack([Vl, X[:, :j]])
        thl = np.concatenate([thl, theta[:j]])
        X, theta = X[:, j:], theta[j:]
    allV = np.hstack([Vl, X])
    allth = np.concatenate([thl, theta])
    order = np.argsort(np.abs(allth[:L]), kind="stable")
    return Result(evals=allth[:L][order], evecs=canonical_sign(allV[:, :L][:, order]),
                  X_next=allV, theta_next=allth, iterations=it, converged=thl.size >= L,
                  filter_matvecs=matvecs, beta=float(beta))


def smallest_magnitude_lower_end(A, L: int, k: int, m: int, tol: float, X0=None, theta0=None,
                                 seed: int = 0, max_iter: int = 200):
    """(Result with the L pairs of smallest |lambda|, ordered by |lambda|, certified) from the
    plain method at the lower end of the spectrum (`chfsi(magnitude=True)`): it goes on until
    the q algebraically smallest converged pairs contain L with |lambda| <= lambda_q.
    certified is False when the block ran out of pairs (or iterations) first."""
    if not (0 < L < k <= A.shape[0]):
        raise ValueError("need 0 < L < k <= n")
    r = chfsi(A, L, k, m, tol, X0=X0, theta0=theta0, seed=seed, max_iter=max_iter,
              magnitude=True)
    return r, bool(r.converged)
