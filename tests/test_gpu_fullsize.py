"""The benchmark workloads at their full sizes, in the launch configuration the benchmark times
(128 chains, 6 lanes, dynamic schedule, graphs, autotuned tiles and widths), against the CPU
oracle: every solve's status, the residuals of every pair (of a regular sample of the
operators for the two largest sets), orthonormality, the sort order, and sampled operators
against the oracle's shift-invert eigenpairs.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, eig as E, sort as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, check_pairs, check_order_stepwise  # noqa: E402
from test_gpu_batched import family_order  # noqa: E402

CHAINS, LANES = 128, 6


def bench_handle():
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, LANES)
    scsf.scsf_set_graphs(h, True)
    return h


def check_residuals(A, lam, X, tol, L):
    """Every pair: relative residual <= tol, ascending values, orthonormal vectors."""
    W = A @ X
    rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
    assert rel.max() <= tol * (1 + 1e-6), rel.max()
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(X.T @ X - np.eye(L))) < 1e-12


def test_poisson100_all_operators():
    """200 operators, n = 10^4, L = 100, k = 120, degree 20."""
    say("full size: poisson100")
    cfg = si.CONFIGS[2]
    ops = si.operators(cfg)
    h = bench_handle()
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    order = scsf.scsf_sort(h, fields, cfg.p0)
    check_order_stepwise(np.stack([S.truncated_features(o.field, cfg.p0) for o in ops]), order)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC)
    scsf.scsf_autotune(h, dops, [cfg.L] * len(ops), order, prm, probe=4)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, dops, order, CHAINS, prm)
    its = [s["iterations"] for s in stats]
    say("iterations mean", np.mean(its), "max", max(its))
    assert all(s["status"] == 0 for s in stats)
    for i, o in enumerate(ops):
        check_residuals(O.assemble(o), host(evals[i]), host(evecs[i]).T, cfg.tol, cfg.L)
    for i in (int(order[0]), int(np.argmax(its))):
        A = O.assemble(ops[i])
        w, V = E.smallest_eigenpairs(A, cfg.L + 10)
        check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)


def test_uneven_all_operators():
    """1000 operators, sides 48..128, L in {32, 64, 128}, both families, autotuned widths."""
    say("full size: uneven batch")
    cfg = si.CONFIGS[3]
    ops = si.operators(cfg)
    Ls = [si.mixed_L(cfg, i) for i in range(len(ops))]
    h = bench_handle()
    order = family_order(h, ops, cfg.p0)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(0, 0, cfg.degree, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_DYNAMIC)
    scsf.scsf_autotune(h, dops, Ls, order, prm, probe=4)
    evals, evecs, stats = scsf.scsf_solve_batched(h, dops, Ls, order, CHAINS, prm)
    its = [s["iterations"] for s in stats]
    say("iterations mean", np.mean(its), "max", max(its))
    assert all(s["status"] == 0 for s in stats)
    for i in range(0, len(ops), 5):
        check_residuals(O.assemble(ops[i]), host(evals[i]), host(evecs[i]).T, cfg.tol, Ls[i])
    largest = max(range(len(ops)), key=lambda j: (Ls[j], ops[j].N))
    for i in (int(order[0]), largest):
        A = O.assemble(ops[i])
        w, V = E.smallest_eigenpairs(A, Ls[i] + 10)
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], cfg.tol, w, V)


def test_mixed160_all_operators():
    """200 operators, n = 25600, L = 200, k = 240, FP32 filter: FP64 accuracy."""
    say("full size: mixed160")
    cfg = si.CONFIGS[4]
    ops = si.operators(cfg)
    h = bench_handle()
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    order = scsf.scsf_sort(h, fields, cfg.p0)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC, precision=scsf.SCSF_MIXED)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, dops, order, CHAINS, prm)
    its = [s["iterations"] for s in stats]
    say("iterations mean", np.mean(its), "max", max(its))
    assert all(s["status"] == 0 for s in stats)
    for i in range(0, len(ops), 10):
        check_residuals(O.assemble(ops[i]), host(evals[i]), host(evecs[i]).T, cfg.tol, cfg.L)
    i = int(order[0])
    A = O.assemble(ops[i])
    w, V = E.smallest_eigenpairs(A, cfg.L + 10)
    check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)


def test_aniso128_learned_window_all_operators():
    """2000 anisotropic operators: plain solves of the first 500 (sorted order) train the
    window network, whose BF16 predictions steer the other 1500 solves."""
    say("full size: learned window")
    cfg = si.CONFIGS[5]
    ops = si.operators(cfg)
    h = bench_handle()
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    order = scsf.scsf_sort(h, fields, cfg.p0)
    head, tail = [int(i) for i in order[:500]], [int(i) for i in order[500:]]
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC, precision=scsf.SCSF_MIXED)
    ritz = torch.empty((len(head), cfg.k), device="cuda", dtype=torch.float64)
    ev1, vec1, st1 = scsf.scsf_solve_sequence(h, [dops[i] for i in head], np.arange(len(head)),
                                              CHAINS, prm, ritz=ritz)
    beta = torch.tensor([s["beta"] for s in st1], device="cuda", dtype=torch.float64)
    target = scsf.scsf_window_labels(h, ritz, cfg.L, beta)
    x = scsf.scsf_window_input(h, scsf.scsf_features(h, fields, 16))
    params = scsf.scsf_window_init(h, 5)
    hist = scsf.scsf_window_train(h, params, x[torch.tensor(head, device="cuda")], target, 600,
                                  1e-3)
    assert hist[-1] < 0.05 * hist[0]
    out = scsf.scsf_window_forward(h, params, x[torch.tensor(tail, device="cuda")], bf16=True)
    hints = scsf.scsf_window_hints(h, out).cpu().numpy()
    ev2, vec2, st2 = scsf.scsf_solve_sequence(h, [dops[i] for i in tail], np.arange(len(tail)),
                                              CHAINS, prm, hints=hints)
    say("head iterations", np.mean([s["iterations"] for s in st1]),
        "tail iterations", np.mean([s["iterations"] for s in st2]),
        "hints used", sum(s["hint"] == 2 for s in st2))
    assert all(s["status"] == 0 for s in st1 + st2)
    for j in range(0, len(tail), 25):
        A = O.assemble(ops[tail[j]])
        check_residuals(A, host(ev2[j]), host(vec2[j]).T, cfg.tol, cfg.L)
    for j in (0, len(tail) // 2):
        A = O.assemble(ops[tail[j]])
        w, V = E.smallest_eigenpairs(A, cfg.L + 10)
        check_pairs(A, ev2[j], vec2[j].t(), cfg.L, cfg.tol, w, V)
