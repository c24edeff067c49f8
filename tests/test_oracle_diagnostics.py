"""Pins of the sort diagnostics (no GPU): the one-sided subspace distance against closed forms
and an independent principal-angle routine, the high-frequency ratio against single Fourier
modes, mixtures of known energy and the Nyquist mode."""
import numpy as np
import pytest
import scipy.linalg

from oracle import diagnostics as D


def orthonormal(n, q, seed):
    return np.linalg.qr(np.random.default_rng(seed).standard_normal((n, q)))[0]


def test_distance_zero_for_the_same_subspace_in_another_basis():
    U = orthonormal(50, 6, 1)
    Q = orthonormal(6, 6, 2)
    assert D.one_sided_distance(U, U @ Q) < 1e-14


def test_distance_of_a_planar_rotation_is_its_sine():
    n = 9
    E = np.eye(n)
    for theta in (1e-6, 0.3, 1.0, np.pi / 2):
        U = E[:, :2]
        V = np.stack([E[:, 0], np.cos(theta) * E[:, 1] + np.sin(theta) * E[:, 2]], 1)
        assert D.one_sided_distance(U, V) == pytest.approx(np.sin(theta), rel=1e-12, abs=1e-15)


def test_distance_one_for_orthogonal_subspaces():
    E = np.eye(8)
    assert D.one_sided_distance(E[:, :3], E[:, 3:6]) == pytest.approx(1.0, abs=1e-15)


def test_distance_against_principal_angles_and_symmetry():
    for seed in range(5):
        U, V = orthonormal(40, 5, 10 + seed), orthonormal(40, 5, 20 + seed)
        V = np.linalg.qr(U + 0.3 * V)[0]        # a nearby subspace: angles well inside (0, pi/2)
        ang = scipy.linalg.subspace_angles(U, V)
        d = D.one_sided_distance(U, V)
        assert d == pytest.approx(np.sin(ang.max()), rel=1e-10)
        assert d == pytest.approx(D.one_sided_distance(V, U), rel=1e-10)
        assert 0.0 < d < 1.0


def test_order_neighbour_distances():
    ev = [orthonormal(30, 4, s) for s in range(5)]
    order = [3, 0, 4, 1, 2]
    d = D.order_neighbour_distances(ev, order, 3)
    assert d.shape == (4,)
    assert d[1] == pytest.approx(D.one_sided_distance(ev[0][:, :3], ev[4][:, :3]))


def mode(p, a, b, amp=1.0):
    x = np.arange(p)
    return amp * np.outer(np.cos(2 * np.pi * b * x / p), np.cos(2 * np.pi * a * x / p))


@pytest.mark.parametrize("a,b,high", [(0, 0, False), (3, 5, False), (19, 19, False),
                                      (20, 0, True), (0, 31, True), (25, 40, True)])
def test_highfreq_single_modes(a, b, high):
    p, p0 = 64, 20
    r = D.highfreq_ratio(mode(p, a, b), p0)
    assert r == pytest.approx(1.0 if high else 0.0, abs=1e-12)


def test_highfreq_mixture_and_nyquist():
    p, p0 = 64, 20
    # cos(3x) + 2 cos(25y): energies 1 : 4 over the same number of coefficients
    f = mode(p, 3, 0) + mode(p, 0, 25, 2.0)
    assert D.highfreq_ratio(f, p0) == pytest.approx(np.sqrt(4 / 5), rel=1e-12)
    # the Nyquist mode (a = p/2) has signed frequency p/2 >= p0
    assert D.highfreq_ratio(mode(p, p // 2, 0), p0) == pytest.approx(1.0, abs=1e-12)
    # channels add their energies; a constant field has no high part
    two = np.stack([mode(p, 1, 1, 3.0), mode(p, 30, 2)])
    e_low, e_high = 9.0 * 4, 1.0 * 4            # |F|^2 of a cos x cos mode: 4 (p^2 amp / 4)^2
    assert D.highfreq_ratio(two, p0) == pytest.approx(np.sqrt(e_high / (e_low + e_high)), rel=1e-12)
    assert D.highfreq_ratio(np.full((p, p), 2.5), p0) == pytest.approx(0.0, abs=1e-15)


def test_highfreq_odd_side_and_p0_one():
    p = 33
    x = np.random.default_rng(3).standard_normal((p, p))
    # p0 = 1 keeps only the mean: the ratio is the share of the fluctuation
    F2 = p * p * np.sum(x ** 2)
    dc2 = (x.sum()) ** 2
    assert D.highfreq_ratio(x, 1) == pytest.approx(np.sqrt(1 - dc2 / F2), rel=1e-12)
    # p0 above every signed frequency keeps everything
    assert D.highfreq_ratio(x, p // 2 + 1) == pytest.approx(0.0, abs=1e-7)
