"""Pins of the grid transfer used for warm starts across sizes (no GPU)."""
import numpy as np

import scsf_inputs as si
from oracle import transfer as T, chfsi as C, operator as O, eig as E


def nodes(N):
    return (np.arange(N) + 1.0) / (N + 1)


def interp_1d(g, N0, N1):
    """1-D piecewise-linear interpolant with zero end values, by numpy.interp."""
    xp = np.concatenate([[0.0], nodes(N0), [1.0]])
    fp = np.concatenate([[0.0], g, [0.0]])
    return np.interp(nodes(N1), xp, fp)


def test_equal_sides_is_identity():
    rng = np.random.default_rng(0)
    F = rng.standard_normal((7, 7))
    np.testing.assert_array_equal(T.interpolate_field(F, 7), F)


def test_separable_fields_match_numpy_interp():
    # bilinear interpolation of g(x) h(y) is the product of the 1-D linear interpolants
    rng = np.random.default_rng(1)
    for N0, N1 in ((5, 9), (9, 5), (6, 13), (13, 6), (48, 53)):
        g, hh = rng.standard_normal(N0), rng.standard_normal(N0)
        F = np.outer(hh, g)                             # F[iy, ix] = h(iy) g(ix)
        ref = np.outer(interp_1d(hh, N0, N1), interp_1d(g, N0, N1))
        # both sides round the source position (relative error ~ N0 * eps in the fraction),
        # times a slope of at most 2 max|F| per cell, in each direction
        tol = 4 * N0 * np.finfo(float).eps * 2 * np.max(np.abs(F))
        np.testing.assert_allclose(T.interpolate_field(F, N1), ref, rtol=0, atol=tol)


def test_coarse_nodes_embedded_in_refined_grid():
    # N1 + 1 = 2 (N0 + 1): every other fine node is a coarse node, the rest are midpoints
    rng = np.random.default_rng(2)
    N0 = 6
    N1 = 2 * (N0 + 1) - 1
    F = rng.standard_normal((N0, N0))
    G = T.interpolate_field(F, N1)
    np.testing.assert_allclose(G[1::2, 1::2], F, rtol=0, atol=1e-15)
    P = np.pad(F, 1)
    mid_x = 0.5 * (P[1:-1, :-1] + P[1:-1, 1:])          # between columns, on coarse rows
    np.testing.assert_allclose(G[1::2, 0::2], mid_x, rtol=0, atol=1e-15)


def test_smooth_mode_error_is_second_order():
    # sin(pi x) sin(pi y) is zero on the boundary; interpolation error O(h0^2)
    errs = []
    for N0 in (16, 32, 64):
        x0 = nodes(N0)
        F = np.outer(np.sin(np.pi * x0), np.sin(np.pi * x0))
        N1 = 45
        x1 = nodes(N1)
        exact = np.outer(np.sin(np.pi * x1), np.sin(np.pi * x1))
        errs.append(np.max(np.abs(T.interpolate_field(F, N1) - exact)))
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1]


def test_block_is_columnwise():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((25, 3))
    Y = T.interpolate_block(X, 5, 8)
    for j in range(3):
        np.testing.assert_array_equal(Y[:, j], T.interpolate_field(X[:, j].reshape(5, 5), 8).ravel())


def test_sequence_across_sizes_gives_exact_eigenpairs():
    # warm start through the transfer still converges to the eigenpairs of each operator
    ops = [si.divk_operator(N, 4, 100 + N) for N in (14, 11, 16)]
    mats = [O.assemble(op) for op in ops]
    out = C.scsf_sequence(mats, 6, 10, 12, 1e-9, max_iter=300)
    for i, A in enumerate(mats):
        w, V = E.smallest_eigenpairs(A, 6, method="dense")
        assert out[i].converged
        np.testing.assert_allclose(out[i].evals, w, rtol=1e-8)
        assert np.max(E.subspace_sines(out[i].evecs, V)) < 1e-6
