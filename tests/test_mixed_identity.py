"""CPU check of the residual form used by the mixed-precision filter (no GPU).

For a Ritz pair (theta, x) with residual r = A x - theta x, the scaled Chebyshev polynomials p_i
of Algorithm 1 satisfy p_m(A) x = p_m(theta) x + e_m, where e_0 = 0, e_1 = (sigma_1/e) r and
e_{i+1} = (2 sigma_{i+1}/e)(A - cI) e_i - sigma_i sigma_{i+1} e_{i-1} + (2 sigma_{i+1}/e) p_i(theta) r.
The GPU runs the e recurrence in FP32; the error it adds is then relative to ||r||."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, chebyshev as Ch, lanczos as Lz


def residual_form(A, X, theta, m, lam, c, e, dtype=np.float64):
    s1 = e / (lam - c)
    R = (A @ X - X * theta)
    t = (theta - c) / e
    Rd = R.astype(dtype)
    Ad = A.astype(dtype)
    E_prev = np.zeros_like(Rd)
    E = (s1 / e * R).astype(dtype)
    p_prev, p, s = np.ones_like(theta), s1 * t, s1
    for _ in range(1, m):
        sn = 1.0 / (2.0 / s1 - s)
        src = (2.0 * sn / e * p).astype(dtype)
        E_next = (dtype(2.0 * sn / e) * (Ad @ E - dtype(c) * E) - dtype(s * sn) * E_prev
                  + Rd * src)
        E_prev, E = E, E_next
        p_prev, p = p, 2.0 * sn * t * p - s * sn * p_prev
        s = sn
    return X * p + E.astype(np.float64), R


@pytest.mark.parametrize("m", [1, 2, 20])
def test_residual_form_equals_filter(m):
    A = O.assemble(si.operator(si.CONFIGS[1], 2))
    w, V = np.linalg.eigh(A.toarray())
    rng = np.random.default_rng(m)
    X = V[:, :24] + 1e-3 * rng.standard_normal((A.shape[0], 24))     # near-Ritz vectors
    theta = np.einsum("ij,ij->j", X, A @ X) / np.einsum("ij,ij->j", X, X)
    beta = Lz.gershgorin_upper(A)
    lam, alpha = theta.min(), theta.max()
    c, e = (alpha + beta) / 2, (beta - alpha) / 2
    Y, _ = residual_form(A, X, theta, m, lam, c, e)
    ref = Ch.filter_block(A, X, m, lam, c, e)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_fp32_error_scales_with_residual():
    A = O.assemble(si.operator(si.CONFIGS[1], 3))
    w, V = np.linalg.eigh(A.toarray())
    beta = Lz.gershgorin_upper(A)
    errs = []
    for eps in (1e-2, 1e-5, 1e-8):
        rng = np.random.default_rng(0)
        X = V[:, :24] + eps * rng.standard_normal((A.shape[0], 24))
        theta = np.einsum("ij,ij->j", X, A @ X) / np.einsum("ij,ij->j", X, X)
        lam, alpha = theta.min(), theta.max()
        c, e = (alpha + beta) / 2, (beta - alpha) / 2
        ref = Ch.filter_block(A, X, 20, lam, c, e)
        Y32, R = residual_form(A, X, theta, 20, lam, c, e, dtype=np.float32)
        plain32 = Ch.filter_block(A.astype(np.float32), X.astype(np.float32), 20, np.float32(lam),
                                  np.float32(c), np.float32(e)).astype(np.float64)
        err = np.max(np.abs(Y32 - ref)) / np.max(np.abs(ref))
        err_plain = np.max(np.abs(plain32 - ref)) / np.max(np.abs(ref))
        rel_res = np.linalg.norm(R, axis=0).max() / np.abs(theta).max()
        errs.append(err)
        assert err < 1e-5 * max(rel_res, 1e-8), (eps, err, rel_res)
        if eps <= 1e-5:                          # plain FP32 filtering sits at its ~1e-6 floor
            assert err < 1e-2 * err_plain, (eps, err, err_plain)
    assert errs[2] < 1e-5 * errs[0]              # shrinks with the residual, no FP32 floor
