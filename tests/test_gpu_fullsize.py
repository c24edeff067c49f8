"""The benchmark workloads at their full sizes, in the launch configuration the benchmark times
(128 chains, 6 lanes, dynamic schedule, graphs, autotuned tiles and widths), against the CPU
oracle.

Every operator's L eigenvalues are compared with the oracle's, stored by
`tests/golden/make_fullsize_eigs.py` (ARPACK shift-invert of the assembled matrix to machine
tolerance, keyed by configuration and operator seed): within 1e-10 relative for the FP64 and
the mixed-precision solves at residual 1e-8 (the eigenvalue error of a pair with residual r
is at most r^2 / gap, Kato-Temple).  A returned pair that is not among the L smallest -- a
lambda_{L+1} pair in place of a skipped lambda_j -- fails that comparison.  Residuals,
orthonormality and ascending order are checked for every operator (for a regular sample of
the 2000 anisotropic operators, whose oracle assembly is slow), and the sort order step by
step.  Needs an MI355X."""
import os

import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, sort as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, check_order_stepwise  # noqa: E402
from test_gpu_batched import family_order  # noqa: E402

CHAINS, LANES = 128, 6
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def bench_handle():
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, LANES)
    scsf.scsf_set_graphs(h, True)
    return h


def golden(cfg):
    """(evals n_op x (max L + 1), L per operator) of the oracle, checked to belong to this
    generator (operator seeds)."""
    d = np.load(os.path.join(GOLDEN, f"fullsize_eigs_c{cfg.index}.npz"))
    seeds = d["seed"]
    assert len(seeds) == cfg.n_op
    assert all(int(seeds[i]) == si.op_seed(cfg.index, i) for i in range(cfg.n_op))
    return d["evals"], d["L"]


def check_evals(i, lam, ref, L, tol=1e-8, rel=1e-10):
    """L eigenvalues of operator i against the oracle's L + 1 smallest: within `rel`, or within
    the Kato-Temple bound 2 tol^2 lambda_j / gap_j where that is larger (tol = the relative
    residual of the solve; gap_j to the nearest other eigenvalue)."""
    assert lam.shape == (L,)
    w = ref[:L + 1]
    gap = np.minimum(np.diff(w)[:L], np.r_[np.inf, np.diff(w)[:L - 1]])
    bound = np.maximum(rel, 2.0 * tol * tol * w[:L] / gap)
    err = np.abs(lam - w[:L]) / np.abs(w[:L])
    assert np.all(err <= bound), (i, int(np.argmax(err / bound)), err.max())


def check_residuals(A, lam, X, tol, L):
    """Every pair: relative residual <= tol, ascending values, orthonormal vectors."""
    W = A @ X
    rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
    assert rel.max() <= tol * (1 + 1e-6), rel.max()
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(X.T @ X - np.eye(L))) < 1e-12


def test_poisson100_all_operators():
    """200 operators, n = 10^4, L = 100, k = 120, degree 30 (the benchmark's)."""
    say("full size: poisson100")
    cfg = si.CONFIGS[2]
    ref, _ = golden(cfg)
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
    ev = host(evals)
    for i, o in enumerate(ops):
        check_evals(i, ev[i], ref[i], cfg.L)
        check_residuals(O.assemble(o), ev[i], host(evecs[i]).T, cfg.tol, cfg.L)


def test_uneven_all_operators():
    """1000 operators, sides 48..128, L in {32, 64, 128}, both families, autotuned widths."""
    say("full size: uneven batch")
    cfg = si.CONFIGS[3]
    ref, Lref = golden(cfg)
    ops = si.operators(cfg)
    Ls = [si.mixed_L(cfg, i) for i in range(len(ops))]
    assert list(Lref) == Ls
    h = bench_handle()
    order = family_order(h, ops, cfg.p0)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(0, 0, cfg.degree, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_DYNAMIC)
    scsf.scsf_autotune(h, dops, Ls, order, prm, probe=4)
    evals, evecs, stats = scsf.scsf_solve_batched(h, dops, Ls, order, CHAINS, prm)
    its = [s["iterations"] for s in stats]
    say("iterations mean", np.mean(its), "max", max(its))
    assert all(s["status"] == 0 for s in stats)
    for i in range(len(ops)):
        lam = host(evals[i])
        check_evals(i, lam, ref[i], Ls[i])
        check_residuals(O.assemble(ops[i]), lam, host(evecs[i]).T, cfg.tol, Ls[i])


def test_uneven_mixed_precision_with_hints_all_operators():
    """The layered forms together on the 1000-operator uneven batch: FP32 filter, per-operator
    window hints (the stored oracle lambda_1 and lambda_{L+1}: the best a window predictor can
    give) and degree 20, in the benchmark's launch configuration; every operator against the
    FP64 oracle at 1e-10."""
    say("full size: uneven batch, mixed precision + hints")
    cfg = si.CONFIGS[3]
    ref, Lref = golden(cfg)
    ops = si.operators(cfg)
    Ls = [int(x) for x in Lref]
    hints = np.array([(ref[i, 0], ref[i, Ls[i]], cfg.degree) for i in range(len(ops))])
    h = bench_handle()
    order = family_order(h, ops, cfg.p0)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(0, 0, cfg.degree, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_DYNAMIC,
                           precision=scsf.SCSF_MIXED)
    scsf.scsf_autotune(h, dops, Ls, order, scsf.make_params(
        0, 0, cfg.degree, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_DYNAMIC), probe=4)
    evals, evecs, stats = scsf.scsf_solve_batched(h, dops, Ls, order, CHAINS, prm, hints=hints)
    its = [s["iterations"] for s in stats]
    say("iterations mean", np.mean(its), "max", max(its),
        "hints used", sum(s["hint"] == 2 for s in stats))
    assert all(s["status"] == 0 for s in stats)
    for i in range(len(ops)):
        lam = host(evals[i])
        check_evals(i, lam, ref[i], Ls[i])
    for i in range(0, len(ops), 10):
        check_residuals(O.assemble(ops[i]), host(evals[i]), host(evecs[i]).T, cfg.tol, Ls[i])


def test_mixed160_all_operators():
    """200 operators, n = 25600, L = 200, k = 240, FP32 filter: FP64 accuracy."""
    say("full size: mixed160")
    cfg = si.CONFIGS[4]
    ref, _ = golden(cfg)
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
    ev = host(evals)
    for i, o in enumerate(ops):
        check_evals(i, ev[i], ref[i], cfg.L)
        check_residuals(O.assemble(o), ev[i], host(evecs[i]).T, cfg.tol, cfg.L)


def learned_window_run(h, cfg, ops, dops, fields, precision):
    """The benchmark's learned-window step: plain solves of the first 500 operators of the
    sorted order train the window network, whose BF16 predictions (window and degree) steer
    the other 1500 solves.  Returns per-operator (evals, evecs) in operator order and the
    stats of both parts."""
    order = scsf.scsf_sort(h, fields, cfg.p0)
    head, tail = [int(i) for i in order[:500]], [int(i) for i in order[500:]]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC, precision=precision)
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
    res = {}
    for j, i in enumerate(head):
        res[i] = (ev1[j], vec1[j])
    for j, i in enumerate(tail):
        res[i] = (ev2[j], vec2[j])
    return res, st1 + st2


@pytest.mark.parametrize("precision", [scsf.SCSF_FP64, scsf.SCSF_MIXED], ids=["fp64", "mixed"])
def test_aniso128_learned_window_all_operators(precision):
    """2000 anisotropic operators (9-point, n = 16384, L = 64) in the benchmark's learned-window
    step, with the FP64 filter (the benchmark's value) and with the FP32 filter."""
    say("full size: learned window", precision)
    cfg = si.CONFIGS[5]
    ref, _ = golden(cfg)
    ops = si.operators(cfg)
    h = bench_handle()
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    dops = [scsf.DeviceOperator(o) for o in ops]
    res, stats = learned_window_run(h, cfg, ops, dops, fields, precision)
    assert all(s["status"] == 0 for s in stats)
    for i in range(len(ops)):
        check_evals(i, host(res[i][0]), ref[i], cfg.L)
    for i in range(0, len(ops), 40):
        check_residuals(O.assemble(ops[i]), host(res[i][0]), host(res[i][1]).T, cfg.tol, cfg.L)


def test_plate100_all_operators():
    """100 thin plates on a 100 x 100 grid (the paper's vibration size), L = 200, k = 240,
    degree 30, relative residual 1e-6 (the FP64 floor of these plates' lowest modes is about
    2e-8): generalized eigenvalues against the oracle's (the Kato-Temple bound of a 1e-6
    residual where it exceeds 1e-10), M-orthonormal eigenvectors, standard-form residuals."""
    say("full size: plate100")
    cfg = si.CONFIGS[6]
    ref, _ = golden(cfg)
    ops = si.operators(cfg)
    h = bench_handle()
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    order = scsf.scsf_sort(h, fields, cfg.p0)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC)
    scsf.scsf_autotune(h, dops, [cfg.L] * len(ops), order, prm, probe=4)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, dops, order, CHAINS, prm)
    its = [s["iterations"] for s in stats]
    say("iterations mean", np.mean(its), "max", max(its))
    assert all(s["status"] == 0 for s in stats)
    ev = host(evals)
    for i, o in enumerate(ops):
        check_evals(i, ev[i], ref[i], cfg.L, tol=cfg.tol)
        U = host(evecs[i]).T
        rho = o.rho.ravel()
        np.testing.assert_allclose(U.T @ (U * rho[:, None]), np.eye(cfg.L), atol=1e-10)
        check_residuals(O.assemble(o), ev[i], U * np.sqrt(rho)[:, None], cfg.tol, cfg.L)


def test_helmholtz80_all_operators():
    """100 Helmholtz operators -div(p grad u) - k^2 u on an 80 x 80 grid (n = 6400, the paper's
    Helmholtz size; indefinite, tens of negative eigenvalues down to about -10^3), the L = 200
    lowest eigenvalues, k = 240, degree 20, tol 1e-8, in the benchmark's launch configuration:
    every operator's eigenvalues against the oracle's, every pair's residual."""
    say("full size: helmholtz80")
    cfg = si.CONFIGS[7]
    ref, _ = golden(cfg)
    ops = si.operators(cfg)
    h = bench_handle()
    fields = torch.tensor(np.stack([o.field for o in ops]), device="cuda")
    order = scsf.scsf_sort(h, fields, cfg.p0)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_DYNAMIC)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, dops, order, CHAINS, prm)
    its = [s["iterations"] for s in stats]
    say("iterations mean", np.mean(its), "max", max(its))
    assert all(s["status"] == 0 for s in stats)
    ev = host(evals)
    for i, o in enumerate(ops):
        lam = ev[i]
        w = ref[i, :cfg.L]
        np.testing.assert_allclose(lam, w, rtol=1e-10, atol=1e-10 * np.abs(w).max())
        A = O.assemble(o)
        X = host(evecs[i]).T
        W = A @ X
        rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
        assert rel.max() <= cfg.tol * (1 + 1e-6)
        assert np.max(np.abs(X.T @ X - np.eye(cfg.L))) < 1e-12
