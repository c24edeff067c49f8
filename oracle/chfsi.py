"""Chebyshev filtered subspace iteration with locking, and the warm-started sequence (oracle).

Algorithm 3 (Section 3.2), taken step by step:
  repeat
    filter the active block:                 V0 <- C_m(V0)                (Algorithm 1)
    orthonormalise [locked | V0] by Householder QR
    Rayleigh quotient on the active part:    G = Q_a^T A Q_a
    solve G W = W Theta, rotate:             V0 <- Q_a W
    lock converged pairs
  until the number of locked pairs >= L
Warm start (Section 3.2, Fig. 2 g): the block and the Ritz values come from the previous
problem of the sorted sequence; the first problem starts from a random block.

Readings (ambiguous or silent passages):
* the damped interval is [alpha, beta] with alpha the largest current Ritz value of the block
  and beta an upper bound of the spectrum; lambda is the smallest current Ritz value
  (Section 2.2 places the *other* eigenvalues in [alpha, beta]); c = (alpha+beta)/2,
  e = (beta-alpha)/2;
* a cold start first runs one QR + Rayleigh-Ritz on the random block to obtain Ritz values;
* G is formed on the active columns only, and the rotated Ritz vectors replace V0;
* convergence uses the relative residual ||A v - theta v|| / ||A v|| (App. D.5 error metric);
  the longest converged ascending prefix of the active Ritz pairs is locked;
* "until L pairs are locked" is read as: until at least L locked values lie at or below the
  smallest unconverged Ritz value (`wanted_locked`), and the L smallest locked pairs are
  returned.  A Ritz value of the block orthogonal to the locked vectors that lies below a
  locked one means a wanted pair entered the block after larger ones were locked;
* all k final Ritz pairs (locked and active) are handed to the next problem; between
  operators on grids of different sides the vectors are moved by bilinear interpolation
  (transfer.py) and the Ritz values are kept (the operators are scaled by 1/h^2, so the low
  eigenvalues hardly depend on the side);
* after `max_iter` outer iterations the best pairs so far are returned, flagged unconverged.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .chebyshev import adaptive_degrees, filter_block
from .eig import canonical_sign
from . import lanczos, transfer


@dataclasses.dataclass
class Result:
    evals: np.ndarray            # (L,) ascending
    evecs: np.ndarray            # (n, L), canonical sign
    X_next: np.ndarray           # (n, k) all Ritz vectors (locked first)
    theta_next: np.ndarray       # (k,)
    iterations: int
    converged: bool
    filter_matvecs: int          # number of single-vector products inside the filter
    beta: float


def _gaussian(n: int, k: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).standard_normal((n, k))


def wanted_locked(theta_locked, theta_active, L: int) -> bool:
    """True when at least L locked values are <= the smallest unconverged active Ritz value
    (all locked values count when no active value is left)."""
    theta_locked = np.asarray(theta_locked, dtype=np.float64)
    if theta_locked.size < L:
        return False
    if len(theta_active) == 0:
        return True
    return int(np.count_nonzero(theta_locked <= np.min(theta_active))) >= L


def lowest_locked(theta_locked, theta_active):
    """The locked values at or below every unconverged Ritz value: by the argument of
    `wanted_locked`, the q algebraically smallest eigenvalues (q = their count)."""
    theta_locked = np.asarray(theta_locked, dtype=np.float64)
    if len(theta_active) == 0:
        return theta_locked
    return theta_locked[theta_locked <= np.min(theta_active)]


def magnitude_certified(theta_locked, theta_active, L: int) -> bool:
    """True when the q algebraically smallest eigenvalues (`lowest_locked`) contain the L of
    smallest magnitude: at least L of them have |lambda| <= lambda_q, their largest (every
    eigenvalue outside them is >= lambda_q)."""
    low = lowest_locked(theta_locked, theta_active)
    if low.size < L:
        return False
    return int(np.count_nonzero(np.abs(low) <= np.max(low))) >= L


def magnitude_hopeless(theta_locked, theta_active, L: int) -> bool:
    """True when the block cannot reach `magnitude_certified`: fewer than L of all its values
    (locked and active) have |theta| <= the largest of them.  A certified state has at least L
    such values (the L it certifies lie at or below lambda_q <= that largest value), so this
    never stops a solve that is certified now; the Ritz values of a converging block only
    drift down, which shrinks that count further.  Giving up only sends the solve to the
    squared filter (the general route for the |lambda| order of eq. eq_basic on the
    indefinite operators of App. D.2), so the rule decides speed, never the result."""
    allv = np.concatenate([np.asarray(theta_locked, dtype=np.float64),
                           np.asarray(theta_active, dtype=np.float64)])
    if allv.size == 0:
        return True
    return int(np.count_nonzero(np.abs(allv) <= np.max(allv))) < L


def chfsi(A, L: int, k: int, m: int, tol: float, X0=None, theta0=None, beta=None,
          seed: int = 0, max_iter: int = 200, lanczos_steps: int = 20,
          adaptive: bool = False, magnitude: bool = False) -> Result:
    """adaptive: after the first outer iteration every active vector is filtered with the
    degree its residual calls for (chebyshev.adaptive_degrees), between m and min(2m, 64):
    vectors near convergence keep m, slow ones get up to twice as many steps.
    magnitude: the L pairs of smallest |lambda| from the lower end of the spectrum: the solve
    goes on until `magnitude_certified`, or gives up uncertified when the block has no
    unconverged pair left or, after an outer iteration, `magnitude_hopeless` holds; it returns,
    ordered by |lambda|, the L of smallest magnitude among the lowest locked pairs;
    `converged` reports the certificate."""
    n = A.shape[0]
    if not (0 < L < k <= n):
        raise ValueError("need 0 < L < k <= n")
    if beta is None:
        beta = lanczos.upper_bound(A, lanczos_steps, seed=seed + 1)
    if X0 is None:
        Q, _ = np.linalg.qr(_gaussian(n, k, seed))
        G = Q.T @ (A @ Q)
        theta, Z = np.linalg.eigh(0.5 * (G + G.T))
        X = Q @ Z
    else:
        X = np.array(X0, dtype=np.float64, copy=True)
        theta = np.array(theta0, dtype=np.float64, copy=True)

    Vl = np.zeros((n, 0))
    thl = np.zeros(0)
    matvecs = 0
    it = 0
    res_act = None                       # residuals of the active Ritz pairs (last iteration)
    def finished():
        if magnitude:
            return (magnitude_certified(thl, theta, L) or theta.size == 0
                    or (it > 0 and magnitude_hopeless(thl, theta, L)))
        return wanted_locked(thl, theta, L)

    while it < max_iter and not finished():
        it += 1
        lam = thl[0] if thl.size else theta[0]
        alpha = theta[-1]
        c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
        if adaptive and res_act is not None:
            deg = adaptive_degrees(theta, res_act, tol, c, e, m_max=max(m, min(2 * m, 64)),
                                   m_min=m)
            Y = np.empty_like(X)
            for d in np.unique(deg):
                cols = np.nonzero(deg == d)[0]
                Y[:, cols] = filter_block(A, X[:, cols], int(d), lam, c, e)
            matvecs += int(deg.sum())
        else:
            Y = filter_block(A, X, m, lam, c, e)
            matvecs += m * X.shape[1]
        Q, _ = np.linalg.qr(np.hstack([Vl, Y]))
        Qa = Q[:, Vl.shape[1]:]
        AQ = A @ Qa
        G = Qa.T @ AQ
        theta, Z = np.linalg.eigh(0.5 * (G + G.T))
        X = Qa @ Z
        W = AQ @ Z
        res = np.linalg.norm(W - X * theta, axis=0) / np.linalg.norm(W, axis=0)
        j = 0
        while j < theta.size and res[j] <= tol:
            j += 1
        Vl = np.hstack([Vl, X[:, :j]])
        thl = np.concatenate([thl, theta[:j]])
        X, theta = X[:, j:], theta[j:]
        res_act = res[j:]

    allV = np.hstack([Vl, X])
    allth = np.concatenate([thl, theta])
    if magnitude:                        # the L smallest in |lambda| of the lowest locked pairs
        low = np.nonzero(thl <= (np.min(theta) if theta.size else np.inf))[0]
        cand = low if low.size >= L else np.arange(max(L, thl.size))
        order = cand[np.argsort(np.abs(allth[cand]), kind="stable")[:L]]
        conv = magnitude_certified(thl, theta, L)
    else:
        nsel = max(L, thl.size)          # the L smallest of the locked pairs
        order = np.argsort(allth[:nsel], kind="stable")[:L]
        conv = wanted_locked(thl, theta, L)
    return Result(evals=allth[order], evecs=canonical_sign(allV[:, order]),
                  X_next=allV, theta_next=allth, iterations=it, converged=conv,
                  filter_matvecs=matvecs, beta=float(beta))


def scsf_sequence(mats, L: int, k: int, m: int, tol: float, order=None, warm: bool = True,
                  seed: int = 0, max_iter: int = 200, adaptive: bool = False):
    """Solve the matrices in `order`, each warm-started from the previous one (Algorithm 3)."""
    order = list(range(len(mats))) if order is None else list(order)
    out = {}
    prev = None
    prev_n = None
    for i in order:
        n = mats[i].shape[0]
        if warm and prev is not None:
            X0 = prev.X_next
            if n != prev_n:
                # operators on square grids of different sides: the fields move by bilinear
                # interpolation (zero Dirichlet boundary) before the warm start
                N0, N1 = math.isqrt(prev_n), math.isqrt(n)
                if N0 * N0 != prev_n or N1 * N1 != n:
                    raise ValueError("warm start across sizes needs square grids")
                X0 = transfer.interpolate_block(X0, N0, N1)
            r = chfsi(mats[i], L, k, m, tol, X0=X0, theta0=prev.theta_next,
                      seed=seed, max_iter=max_iter, adaptive=adaptive)
        else:
            r = chfsi(mats[i], L, k, m, tol, seed=seed, max_iter=max_iter, adaptive=adaptive)
        out[i] = r
        prev = r
        prev_n = n
    return out
