"""The spectral-window network on the GPU (FP32 training kernels, BF16 inference) against the
FP64 oracle, and what the trained network gains in the solver.  Needs an MI355X."""
import time

import numpy as np
import pytest

import scsf_inputs as si
from oracle import cnn, sort as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say  # noqa: E402


@pytest.fixture(scope="module")
def h():
    return scsf.Handle()


def rand_case(n=8, seed=0):
    rng = np.random.default_rng(seed)
    theta = cnn.init_params(seed) * 0.7
    theta[cnn.COUNT - 3:] = [3.0, 6.0, 0.5]            # output biases of a realistic size
    x = rng.standard_normal((n, 6, 16, 16)) * 0.5
    t = rng.standard_normal((n, 3)) + np.array([3.0, 6.0, 0.5])
    return theta, x, t


def dev32(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


def test_param_count():
    assert scsf.window_param_count() == cnn.COUNT


def test_forward_fp32_and_bf16(h):
    say("window forward")
    theta, x, t = rand_case()
    ref = cnn.forward(theta, x)
    y32 = scsf.scsf_window_forward(h, dev32(theta), dev32(x)).cpu().numpy()
    ybf = scsf.scsf_window_forward(h, dev32(theta), dev32(x), bf16=True).cpu().numpy()
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(y32 - ref)) <= 1e-5 * scale
    assert np.max(np.abs(ybf - ref)) <= 3e-2 * scale


def test_gradient_matches_oracle(h):
    say("window gradient")
    theta, x, t = rand_case(6, 1)
    loss_ref, g_ref = cnn.loss_and_grad(theta, x, t)
    loss, g = scsf.scsf_window_loss_grad(h, dev32(theta), dev32(x), dev32(t))
    g = g.cpu().numpy()
    assert loss == pytest.approx(loss_ref, rel=1e-5)
    o = 0
    for name, shp in cnn.SHAPES:
        size = int(np.prod(shp))
        a, b = g[o:o + size], g_ref[o:o + size]
        assert np.max(np.abs(a - b)) <= 1e-4 * max(np.max(np.abs(b)), 1e-12), name
        o += size


def test_input_labels_hints(h):
    say("window input / labels / hints")
    f = np.stack([o.field for o in si.operators(si.CONFIGS[5], 4)])
    feats = scsf.scsf_features(h, torch.tensor(f, device="cuda"), 16)
    x = scsf.scsf_window_input(h, feats).cpu().numpy()
    ref = cnn.window_features(np.stack([S.truncated_features(ff, 16) for ff in f]))
    assert np.max(np.abs(x - ref)) <= 1e-6 * np.max(np.abs(ref))
    rng = np.random.default_rng(3)
    ritz = np.sort(rng.uniform(10, 1000, size=(5, 12)), axis=1)
    beta = rng.uniform(5e3, 1e5, size=5)
    t = scsf.scsf_window_labels(h, torch.tensor(ritz, device="cuda"), 8,
                                torch.tensor(beta, device="cuda")).cpu().numpy()
    for i in range(5):
        assert t[i, 0] == pytest.approx(np.log(ritz[i, 0]), rel=1e-6)
        assert t[i, 1] == pytest.approx(np.log(ritz[i, 8]), rel=1e-6)
        assert t[i, 2] * 128 == pytest.approx(cnn.degree_label(ritz[i, 7], ritz[i, 8], beta[i]))
    out = torch.tensor([[3.0, 7.0, 0.5], [2.0, 5.0, 2.0]], device="cuda")
    hints = scsf.scsf_window_hints(h, out).cpu().numpy()
    np.testing.assert_allclose(hints[0], [np.exp(3.0), np.exp(7.0), 64.0], rtol=1e-12)
    assert hints[1, 2] == 128.0
    out2 = torch.tensor([[3.0, 7.0, 0.01]], device="cuda")
    assert scsf.scsf_window_hints(h, out2).cpu().numpy()[0, 2] == 8.0


def test_training_reduces_loss(h):
    say("window training")
    theta, x, t = rand_case(64, 4)
    p = scsf.scsf_window_init(h, 11)
    hist = scsf.scsf_window_train(h, p, dev32(x), dev32(t), 400, 2e-3)
    assert hist[-1] < 0.05 * hist[0], (hist[0], hist[-1])


def _solve(h, dops, order, prm, hints=None, ritz=None):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, vec, st = scsf.scsf_solve_sequence(h, dops, order, len(dops), prm, hints=hints, ritz=ritz)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, ev, st


def test_degree_hints_at_table_size_after_other_degrees(h):
    """Degree hints that all equal the largest degree (128) after a call with other degrees:
    the per-problem degrees on the device must be the requested ones, so the hinted solve
    repeats the plain degree-128 solve exactly (same iterations, same eigenvalues)."""
    say("degree hints at 128 after 20")
    cfg = si.CONFIGS[5]
    dops = [scsf.DeviceOperator(o) for o in si.operators(cfg, 8)]
    order = np.arange(len(dops))
    n = len(dops)
    prm20 = scsf.make_params(cfg.L, cfg.k, 20, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_DYNAMIC)
    prm64 = scsf.make_params(cfg.L, cfg.k, 128, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_DYNAMIC)
    _, ev20, st20 = _solve(h, dops, order, prm20, hints=np.tile([0.0, 0.0, 20.0], (n, 1)))
    _, ev_p, st_p = _solve(h, dops, order, prm64)
    _, ev_h, st_h = _solve(h, dops, order, prm20, hints=np.tile([0.0, 0.0, 128.0], (n, 1)))
    assert [s["degree"] for s in st_h] == [128] * n
    assert [s["iterations"] for s in st_h] == [s["iterations"] for s in st_p]
    assert sum(s["iterations"] for s in st_p) < sum(s["iterations"] for s in st20)
    np.testing.assert_allclose(ev_h.cpu().numpy(), ev_p.cpu().numpy(), rtol=1e-10)
    np.testing.assert_allclose(ev20.cpu().numpy(), ev_p.cpu().numpy(), rtol=1e-10)


def test_learned_window_gains_over_plain(h):
    """Train on solved config-5 operators, predict window and degree for held-out ones, and
    compare the held-out solves with and without the prediction."""
    say("learned window gain")
    cfg = si.CONFIGS[5]
    ops = si.operators(cfg, 48)
    dops = [scsf.DeviceOperator(o) for o in ops]
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    order = scsf.scsf_sort(h, fields, cfg.p0)
    train_idx, test_idx = order[:32], order[32:]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC)
    # training set: plain solves, labels from their Ritz values and bounds
    sub = [dops[i] for i in train_idx]
    ritz = torch.empty((len(sub), cfg.k), device="cuda", dtype=torch.float64)
    _, _, st = _solve(h, sub, np.arange(len(sub)), prm, ritz=ritz)
    beta = torch.tensor([s["beta"] for s in st], device="cuda", dtype=torch.float64)
    target = scsf.scsf_window_labels(h, ritz, cfg.L, beta)
    feats = scsf.scsf_features(h, fields, 16)
    x = scsf.scsf_window_input(h, feats)
    params = scsf.scsf_window_init(h, 5)
    hist = scsf.scsf_window_train(h, params, x[torch.tensor(train_idx, device="cuda")], target,
                                  600, 1e-3)
    say("loss", hist[0], hist[-1])
    out = scsf.scsf_window_forward(h, params, x[torch.tensor(test_idx, device="cuda")], bf16=True)
    hints = scsf.scsf_window_hints(h, out).cpu().numpy()
    tsub = [dops[i] for i in test_idx]
    t_plain, ev_p, st_p = _solve(h, tsub, np.arange(len(tsub)), prm)
    t_learn, ev_l, st_l = _solve(h, tsub, np.arange(len(tsub)), prm, hints=hints)
    it_p = sum(s["iterations"] for s in st_p)
    it_l = sum(s["iterations"] for s in st_l)
    used = sum(s["hint"] == 2 for s in st_l)
    say("plain", t_plain, it_p, "learned", t_learn, it_l, "hints used", used, "of", len(st_l))
    # both give the same eigenvalues (residual 1e-8 on both sides)
    np.testing.assert_allclose(ev_l.cpu().numpy(), ev_p.cpu().numpy(), rtol=1e-9)
    assert all(s["status"] == 0 for s in st_l)
    assert it_l < it_p and t_learn < t_plain
    # against the best fixed degree: on this family the labels put the degree at the table's
    # top for nearly every operator, so the plain method at the mean predicted degree is the
    # fair baseline.  The predicted window adds nothing beyond the degree (the learned solves
    # take about as many outer iterations); the check is that it costs nothing either.
    d_best = int(round(float(np.mean([s["degree"] for s in st_l]))))
    prm_best = scsf.make_params(cfg.L, cfg.k, d_best, cfg.tol, seed=1,
                                schedule=scsf.SCSF_SCHED_DYNAMIC)
    t_best, ev_b, st_b = _solve(h, tsub, np.arange(len(tsub)), prm_best)
    it_b = sum(s["iterations"] for s in st_b)
    say("best fixed degree", d_best, t_best, it_b)
    np.testing.assert_allclose(ev_l.cpu().numpy(), ev_b.cpu().numpy(), rtol=1e-9)
    assert it_l <= 1.15 * it_b
