"""Pins of the oracle's truncated-FFT greedy sort (Algorithm 2, App. F) -- no GPU."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import sort as S


def spatial_greedy(fields, start=0):
    """Naive greedy on the full spatial Frobenius distance (the ordering Section 3.1 starts
    from), written with plain loops."""
    n = len(fields)
    order, used, cur = [start], {start}, start
    for _ in range(n - 1):
        best, arg = np.inf, -1
        for j in range(n):
            if j in used:
                continue
            d = float(np.sum((fields[cur] - fields[j]) ** 2))
            if d < best:
                best, arg = d, j
        order.append(arg)
        used.add(arg)
        cur = arg
    return np.array(order)


def test_dc_term_is_mean_and_cosine_mode():
    p = 16
    rng = np.random.default_rng(0)
    f = rng.standard_normal((p, p)) + 3.0
    F = S.truncated_features(f, 4)
    assert F.shape == (1, 4, 4)
    assert F[0, 0, 0] == pytest.approx(f.mean(), rel=1e-13)
    y, x = np.meshgrid(np.arange(p), np.arange(p), indexing="ij")
    g = np.cos(2 * np.pi * 3 * x / p)
    G = S.truncated_features(g, 5)[0]
    expect = np.zeros((5, 5), complex)
    expect[0, 3] = 0.5
    np.testing.assert_allclose(G, expect, atol=1e-14)


def test_parseval_and_truncation_split():
    """App. F: full-spectrum distance equals the spatial one (normalised DFT), and equals the
    kept (SCSF metric) part plus the truncation tail."""
    ops = si.operators(si.CONFIGS[1], 6)
    p = ops[0].N
    Fi = S.truncated_features(ops[1].field, p)
    Fj = S.truncated_features(ops[4].field, p)
    full = np.sum(np.abs(Fi - Fj) ** 2) * p * p
    spatial = np.sum((ops[1].field - ops[4].field) ** 2)
    assert full == pytest.approx(spatial, rel=1e-12)
    p0 = 4
    kept = np.sum(np.abs(Fi[:, :p0, :p0] - Fj[:, :p0, :p0]) ** 2)
    mask = np.ones((p, p), bool)
    mask[:p0, :p0] = False
    tail = np.sum(np.abs((Fi - Fj)[:, mask]) ** 2)
    assert (kept + tail) * p * p == pytest.approx(spatial, rel=1e-12)


def test_full_spectrum_sort_equals_spatial_greedy():
    ops = si.operators(si.CONFIGS[1])
    fields = [o.field for o in ops]
    p = ops[0].N
    assert list(S.scsf_sort(fields, p)) == list(spatial_greedy(fields))


def test_greedy_bruteforce_and_ties():
    rng = np.random.default_rng(5)
    feats = rng.standard_normal((30, 1, 3, 3)) + 1j * rng.standard_normal((30, 1, 3, 3))
    feats[7] = feats[12]          # exact duplicates: the lower index must come first
    feats[21] = feats[12]
    order = S.greedy_order(feats, start=0)
    assert sorted(order) == list(range(30)) and order[0] == 0
    # brute force re-check of every step
    remaining = set(range(30)) - {0}
    for a, b in zip(order[:-1], order[1:]):
        d = {j: float(np.sum(np.abs(feats[a] - feats[j]) ** 2)) for j in remaining}
        best = min(d.values())
        assert b == min(j for j in remaining if d[j] == best)
        remaining.remove(b)
    pos = {v: i for i, v in enumerate(order)}
    assert pos[7] < pos[12] < pos[21] or pos[7] < pos[21]


def test_start_index_and_p0_too_large():
    ops = si.operators(si.CONFIGS[1], 8)
    order = S.scsf_sort([o.field for o in ops], 4, start=3)
    assert order[0] == 3 and sorted(order) == list(range(8))
    with pytest.raises(ValueError):
        S.truncated_features(ops[0].field, 33)
