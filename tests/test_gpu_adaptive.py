"""Per-vector adaptive filter degrees on the GPU against the CPU oracle's adaptive ChFSI and the
exact eigenpairs: single solves, chained sequences (graphs against eager launches, bitwise),
uneven batches, the benchmark's launch shape at full size, and the rejected combinations.
Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, eig as E, chfsi as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, check_pairs  # noqa: E402
from test_gpu_batched import small_uneven, family_order  # noqa: E402
from test_gpu_graphs import assert_same  # noqa: E402


@pytest.fixture(scope="module")
def h():
    return scsf.Handle()


@pytest.mark.parametrize("i", [0, 1, 2])
def test_adaptive_solve_matches_oracle(h, i):
    """The same operator with one degree and with per-vector degrees: both reach the exact
    pairs; the adaptive solve agrees with the oracle's adaptive ChFSI, needs no more outer
    iterations than the uniform one, and its degrees stay in [m, 2m]."""
    say("adaptive solve c1 operator", i)
    cfg = si.CONFIGS[1]
    op = si.operator(cfg, i)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, cfg.L + 8)
    d = scsf.DeviceOperator(op)
    plain = scsf.scsf_solve(h, d, scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=3))
    ev, vec, _, _, st = scsf.scsf_solve(h, d, scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol,
                                                               seed=3, adaptive=1))
    ref = C.chfsi(A, cfg.L, cfg.k, cfg.degree, cfg.tol, seed=3, adaptive=True)
    say("plain", plain[4]["iterations"], plain[4]["filter_cols"], "adaptive", st["iterations"],
        st["filter_cols"], "degree", st["degree"], "oracle", ref.iterations, ref.filter_matvecs)
    assert st["status"] == 0 and st["nconv"] >= cfg.L
    check_pairs(A, ev, vec, cfg.L, cfg.tol, w, V)
    np.testing.assert_allclose(host(ev), ref.evals, rtol=1e-10)
    assert st["iterations"] <= plain[4]["iterations"]
    assert cfg.degree <= st["degree"] <= 2 * cfg.degree
    # the first iteration filters all k columns at m; later ones at most 2m + 2 each
    assert cfg.degree * cfg.k <= st["filter_cols"] <= (2 * cfg.degree + 2) * cfg.k * st["iterations"]


def test_adaptive_degree_cap_at_64(h):
    """degree 40: the per-vector degrees are capped at 64, not 80."""
    say("adaptive degree 40")
    cfg = si.CONFIGS[1]
    op = si.operator(cfg, 3)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, cfg.L + 8)
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op),
                                        scsf.make_params(cfg.L, cfg.k, 40, cfg.tol, seed=3,
                                                         adaptive=1))
    say(st)
    check_pairs(A, ev, vec, cfg.L, cfg.tol, w, V)
    assert 40 <= st["degree"] <= 64


@pytest.mark.parametrize("chains,lanes,sched", [(1, 1, 0), (3, 2, 0), (4, 2, 1)])
def test_adaptive_sequence_config1(chains, lanes, sched):
    say("adaptive sequence c1 chains", chains, "lanes", lanes, "schedule", sched)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, lanes)
    cfg = si.CONFIGS[1]
    ops = si.operators(cfg)
    dops = [scsf.DeviceOperator(o) for o in ops]
    order = np.arange(len(ops))
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1, schedule=sched, adaptive=1)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, dops, order, chains, prm)
    say([s["iterations"] for s in stats])
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, cfg.L + 8)
        assert stats[i]["status"] == 0
        assert cfg.degree <= stats[i]["degree"] <= 2 * cfg.degree
        check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)


def test_adaptive_graphs_match_eager():
    """The column degrees live on the device and change every iteration inside the captured
    post graph; replays must give the eager result bit for bit."""
    say("adaptive graphs vs eager")
    cfg = si.CONFIGS[1]
    dops = [scsf.DeviceOperator(o) for o in si.operators(cfg)]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_STATIC, adaptive=1)
    out = []
    for graphs in (False, True):
        h = scsf.Handle()
        scsf.scsf_set_lanes(h, 2)
        scsf.scsf_set_graphs(h, graphs)
        out.append(scsf.scsf_solve_sequence(h, dops, np.arange(len(dops)), 3, prm))
    assert_same(*out)


@pytest.mark.parametrize("tile", [1, 2, 4, 8])
def test_adaptive_batched_uneven(tile):
    """Uneven sizes and L in one batch, every staged-tile shape of the filter."""
    say("adaptive batched tile", tile)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    scsf.scsf_set_tile(h, tile)
    ops, Ls = small_uneven(10, 21)
    order = family_order(h, ops, 6)
    prm = scsf.make_params(0, 0, 16, 1e-8, seed=2, schedule=scsf.SCSF_SCHED_DYNAMIC, adaptive=1)
    evals, evecs, stats = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(o) for o in ops], Ls,
                                                  order, 4, prm)
    say([(s["iterations"], s["degree"]) for s in stats])
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, Ls[i] + 6, method="dense")
        assert stats[i]["status"] == 0
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], 1e-8, w, V)


def test_adaptive_config2_full_size_sampled():
    """The 10^4-node workload (L = 100, k = 120, degree 30) in the benchmark's launch shape
    (dynamic schedule, 6 lanes, graphs) on 24 operators: every pair's residual, sampled
    operators against shift-invert, and fewer outer iterations than one degree for all."""
    say("adaptive c2 sampled")
    cfg = si.CONFIGS[2]
    ops = si.operators(cfg, 24)
    dops = [scsf.DeviceOperator(o) for o in ops]
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 6)
    scsf.scsf_set_graphs(h, True)
    order = np.arange(len(ops))
    its = {}
    for ad in (0, 1):
        prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                               schedule=scsf.SCSF_SCHED_DYNAMIC, adaptive=ad)
        evals, evecs, stats = scsf.scsf_solve_sequence(h, dops, order, 8, prm)
        its[ad] = [s["iterations"] for s in stats]
        assert all(s["status"] == 0 for s in stats)
    say("plain", np.mean(its[0]), "adaptive", np.mean(its[1]))
    assert np.mean(its[1]) < np.mean(its[0])
    for i, o in enumerate(ops):
        A = O.assemble(o)
        X, lam = host(evecs[i]).T, host(evals[i])
        W = A @ X
        rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
        assert rel.max() <= cfg.tol * (1 + 1e-6)
    for i in (0, 13):
        A = O.assemble(ops[i])
        w, V = E.smallest_eigenpairs(A, cfg.L + 10)
        check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)


def test_adaptive_rejected_combinations(h):
    cfg = si.CONFIGS[1]
    ops = si.operators(cfg, 2)
    dops = [scsf.DeviceOperator(o) for o in ops]
    with pytest.raises(scsf.ScsfError) as e1:          # FP32 filter keeps one degree
        scsf.scsf_solve(h, dops[0], scsf.make_params(cfg.L, cfg.k, 20, cfg.tol, adaptive=1,
                                                     precision=scsf.SCSF_MIXED))
    assert e1.value.status == scsf.SCSF_EINVAL
    with pytest.raises(scsf.ScsfError) as e2:
        scsf.scsf_solve(h, dops[0], scsf.make_params(cfg.L, cfg.k, 20, cfg.tol, adaptive=2))
    assert e2.value.status == scsf.SCSF_EINVAL
    with pytest.raises(scsf.ScsfError) as e3:          # a degree hint fixes the degree
        scsf.scsf_solve_sequence(h, dops, [0, 1], 1,
                                 scsf.make_params(cfg.L, cfg.k, 20, cfg.tol, adaptive=1),
                                 hints=np.array([[0.0, 0.0, 30.0]] * 2))
    assert e3.value.status == scsf.SCSF_EINVAL
