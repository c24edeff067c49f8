"""Upper bound of the spectrum for the filter window (oracle).

Section 2.2 takes beta, the upper end of the damped interval, as an estimate of the top of the
spectrum; the ChFSI solver the paper builds on (and the commented-out step of Algorithm 3)
obtains it from a few Lanczos steps (Zhou & Li 2011): with T_s the s x s Lanczos tridiagonal
matrix and beta_s = ||f_s|| the norm of the last residual, theta_max(T_s) + beta_s bounds
lambda_max in practice.  Gershgorin's max row sum is a rigorous bound.  The window uses the
smaller of the two.
"""
from __future__ import annotations

import numpy as np


def gershgorin_upper(A) -> float:
    d = A.diagonal()
    absA = abs(A)
    off = np.asarray(absA.sum(axis=1)).ravel() - np.abs(d)
    return float(np.max(d + off))


def lanczos(A, steps: int, v0: np.ndarray):
    """Plain Lanczos (no reorthogonalisation). Returns (alpha[s], beta[s]); beta[-1] = ||f_s||."""
    v = np.asarray(v0, dtype=np.float64) / np.linalg.norm(v0)
    v_old = np.zeros_like(v)
    b_old = 0.0
    alpha, beta = [], []
    for _ in range(steps):
        w = A @ v - b_old * v_old
        a = float(v @ w)
        w = w - a * v
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if b == 0.0:
            break
        v_old, v, b_old = v, w / b, b
    return np.array(alpha), np.array(beta)


def tridiag_eigvals(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    s = len(alpha)
    T = np.diag(alpha) + np.diag(beta[: s - 1], 1) + np.diag(beta[: s - 1], -1)
    return np.linalg.eigvalsh(T)


def lanczos_bounds(A, steps: int, v0: np.ndarray):
    """(theta_min(T_s), theta_max(T_s), theta_max + beta_s)."""
    a, b = lanczos(A, steps, v0)
    th = tridiag_eigvals(a, b)
    return float(th[0]), float(th[-1]), float(th[-1] + abs(b[-1]))


def upper_bound(A, steps: int = 20, v0: np.ndarray | None = None, seed: int = 0) -> float:
    if v0 is None:
        v0 = np.random.Generator(np.random.PCG64(seed)).standard_normal(A.shape[0])
    _, _, ub = lanczos_bounds(A, steps, v0)
    return min(gershgorin_upper(A), ub)
