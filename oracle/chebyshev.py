"""Chebyshev polynomials and the scaled Chebyshev filter (oracle).

Section 2.2 defines C_m(t) = cos(m arccos t) on [-1, 1] with the three-term recurrence
C_{m+1}(t) = 2 t C_m(t) - C_{m-1}(t); outside [-1, 1] the same polynomial equals
cosh(m arccosh|t|) sgn(t)^m.

Algorithm 1 applies the recurrence to a block: with the shifted and scaled matrix
A' = (A - cI)/e (c, e the centre and half-width of the damped interval [alpha, beta]),
sigma_1 = e/(lambda - c) and sigma_{i+1} = 1/(2/sigma_1 - sigma_i),
    Y_1     = sigma_1 A' Y_0
    Y_{i+1} = 2 sigma_{i+1} A' Y_i - sigma_{i+1} sigma_i Y_{i-1}.
The printed algorithm writes Y_i in the last term and splits the columns by a per-column
degree; the reading used here is the standard scaled recurrence (last term Y_{i-1}, one
degree for every column), which makes Y_m = C_m(A') Y_0 / C_m((lambda - c)/e).
"""
from __future__ import annotations

import numpy as np


def cheb(m: int, t):
    """C_m(t) from the trigonometric / hyperbolic closed form."""
    t = np.asarray(t, dtype=np.float64)
    inside = np.abs(t) <= 1.0
    out = np.empty_like(t)
    out[inside] = np.cos(m * np.arccos(t[inside]))
    ta = np.abs(t[~inside])
    out[~inside] = np.cosh(m * np.arccosh(ta)) * np.sign(t[~inside]) ** m
    return out


def cheb_recurrence(m: int, t):
    """C_m(t) by the three-term recurrence (used to cross-check `cheb`)."""
    t = np.asarray(t, dtype=np.float64)
    c0, c1 = np.ones_like(t), t.copy()
    if m == 0:
        return c0
    for _ in range(m - 1):
        c0, c1 = c1, 2.0 * t * c1 - c0
    return c1


def filter_block(A, Y0: np.ndarray, m: int, lam: float, c: float, e: float) -> np.ndarray:
    """Y_m of Algorithm 1 (scaled recurrence, uniform degree m >= 1)."""
    def Ap(Y):                       # A' Y = (A - cI) Y / e
        return (A @ Y - c * Y) / e

    sigma1 = e / (lam - c)
    Yprev = np.array(Y0, dtype=np.float64, copy=True)
    Y = sigma1 * Ap(Yprev)
    sigma = sigma1
    for _ in range(1, m):
        sigma_next = 1.0 / (2.0 / sigma1 - sigma)
        Ynext = 2.0 * sigma_next * Ap(Y) - sigma_next * sigma * Yprev
        Yprev, Y, sigma = Y, Ynext, sigma_next
    return Y


def filter_gain(mu, m: int, lam: float, c: float, e: float):
    """Scalar factor the filter applies to an eigenvector of eigenvalue mu."""
    return cheb(m, (np.asarray(mu, dtype=np.float64) - c) / e) / cheb(m, np.array([(lam - c) / e]))[0]


def adaptive_degrees(theta, res, tol: float, c: float, e: float, m_max: int, m_min: int = 1):
    """Per-vector filter degree of the optimized filter the paper cites for Algorithm 1
    (per-column degrees) and leaves out of Algorithm 3: each non-converged vector gets the
    degree its residual and Ritz value call for.

    A Ritz value theta below the damped interval [c - e, c + e] (t = (theta - c)/e < -1) is
    amplified by |C_m(t)| ~ |rho|^m / 2 against the interval, |rho| = |t| + sqrt(t^2 - 1), so
    a residual res falls to tol after m = ceil(ln(res / tol) / ln|rho|) steps.  The degree is
    clamped to [m_min, m_max]; a Ritz value inside the interval (|t| <= 1) gets m_max.
    """
    theta = np.asarray(theta, dtype=np.float64)
    res = np.asarray(res, dtype=np.float64)
    t = (theta - c) / e
    out = np.full(theta.shape, m_max, dtype=np.int64)
    grow = np.abs(t) > 1.0
    rho = np.abs(t[grow]) + np.sqrt(t[grow] ** 2 - 1.0)
    need = np.log(np.maximum(res[grow], tol) / tol) / np.log(rho)
    out[grow] = np.ceil(need - 1e-12).astype(np.int64)
    return np.clip(out, m_min, m_max)
