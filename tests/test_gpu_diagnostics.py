"""Sort diagnostics on the GPU against the CPU oracle: the high-frequency ratio of the
coefficient fields, the one-sided subspace distance between solved eigenvector blocks, and the
full greedy order on the untruncated fields.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import diagnostics as D, sort as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, check_order_stepwise  # noqa: E402


@pytest.fixture(scope="module")
def h():
    return scsf.Handle()


def fields_of(cfg, count):
    return np.stack([si.operator(cfg, i).field for i in range(count)])


@pytest.mark.parametrize("cfgi,count,p0", [(2, 40, 20), (2, 12, 1), (2, 12, 40), (2, 8, 51),
                                           (1, 20, 4), (5, 10, 16)])
def test_highfreq_ratio_matches_oracle(h, cfgi, count, p0):
    say("highfreq", cfgi, count, p0)
    f = fields_of(si.CONFIGS[cfgi], count)
    if f.ndim == 3:
        f = f[:, None]
    got = host(scsf.scsf_highfreq_ratio(h, torch.tensor(f, device="cuda"), p0))
    ref = np.array([D.highfreq_ratio(x, p0) for x in f])
    say(float(ref.mean()))
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-7)


def test_highfreq_ratio_odd_side_and_modes(h):
    p = 33
    x = np.arange(p)
    m_low = np.outer(np.cos(2 * np.pi * 2 * x / p), np.cos(2 * np.pi * 3 * x / p))
    m_high = np.outer(np.cos(2 * np.pi * 16 * x / p), np.ones(p))
    f = np.stack([m_low, m_high, m_low + 2 * m_high, np.zeros((p, p))])[:, None]
    got = host(scsf.scsf_highfreq_ratio(h, torch.tensor(f, device="cuda"), 10))
    np.testing.assert_allclose(got, [0.0, 1.0, np.sqrt(4 * 1 / (4 * 1 + 0.5)), 0.0], atol=1e-7)
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_highfreq_ratio(h, torch.tensor(f, device="cuda"), 0)


def test_subspace_distance_on_solved_eigenvectors(h):
    """q = 10 lowest eigenvectors of the c1 operators (the paper's 10-dimensional subspaces)."""
    say("subspace distance")
    cfg = si.CONFIGS[1]
    ops = si.operators(cfg)
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1)
    order = S.scsf_sort([o.field for o in ops], cfg.p0)
    _, evecs, _ = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops], order, 2,
                                           prm)
    pairs = list(zip(order[:-1], order[1:])) + [(3, 3), (0, 7)]
    got = scsf.scsf_subspace_distance(h, evecs, 10, pairs)
    ev = [host(evecs[i]).T for i in range(len(ops))]
    ref = np.array([D.one_sided_distance(ev[a][:, :10], ev[b][:, :10]) for a, b in pairs])
    say(ref[:-2].mean())
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-13)
    assert got[-2] < 1e-13


@pytest.mark.parametrize("q", [1, 2, 17, 32])
def test_subspace_distance_closed_forms(h, q):
    n = 1000
    rng = np.random.default_rng(q)
    Q = np.linalg.qr(rng.standard_normal((n, q + 1)))[0]
    blocks = [Q[:, :q]]
    thetas = [1e-6, 0.4, np.pi / 2]
    for th in thetas:                               # rotate the last column towards Q[:, q]
        V = Q[:, :q].copy()
        V[:, -1] = np.cos(th) * Q[:, q - 1] + np.sin(th) * Q[:, q]
        blocks.append(V)
    B = torch.tensor(np.ascontiguousarray(np.stack([b.T for b in blocks])), device="cuda")
    got = scsf.scsf_subspace_distance(h, B, q, [(0, 1), (0, 2), (0, 3), (2, 2)])
    np.testing.assert_allclose(got[:3], np.sin(thetas), rtol=1e-9, atol=1e-12)
    assert got[3] < 1e-13
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_subspace_distance(h, B, q, [(0, 4)])
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_subspace_distance(h, B, 33, [(0, 1)])


def test_full_greedy_on_raw_fields(h):
    """Section 3.1's naive greedy: the spatial Frobenius distance on the untruncated fields."""
    f = fields_of(si.CONFIGS[2], 60).reshape(60, -1)
    flat = torch.tensor(f.astype(np.complex128), device="cuda")      # real fields, zero imaginary
    order = scsf.scsf_order_features(h, flat, start=0)
    check_order_stepwise(f, order)
