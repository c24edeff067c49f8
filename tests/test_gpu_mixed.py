"""Mixed precision (FP32 filter in residual form, FP64 orthonormalisation / Rayleigh-Ritz /
residuals) against the FP64 CPU oracle.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, eig as E, sort as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import check_pairs, say  # noqa: E402


def test_mixed_solve_config1():
    say("mixed solve c1")
    cfg = si.CONFIGS[1]
    op = si.operator(cfg, 6)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, cfg.L + 8)
    h = scsf.Handle()
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=2, precision=scsf.SCSF_MIXED)
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op), prm)
    say(st)
    assert st["status"] == 0
    check_pairs(A, ev, vec, cfg.L, cfg.tol, w, V)


def test_mixed_tight_tolerance_below_fp32_floor():
    """The FP32 correction keeps converging: a 1e-11 residual (far below FP32 rounding of the
    filtered block) is reached."""
    say("mixed solve tol 1e-11")
    cfg = si.CONFIGS[1]
    op = si.operator(cfg, 9)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, cfg.L + 8)
    h = scsf.Handle()
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, 1e-11, seed=2, precision=scsf.SCSF_MIXED)
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op), prm)
    check_pairs(A, ev, vec, cfg.L, 1e-11, w, V)


@pytest.mark.parametrize("chains", [1, 4])
def test_mixed_sequence_config1(chains):
    say("mixed sequence c1", chains)
    cfg = si.CONFIGS[1]
    ops = si.operators(cfg, 10)
    order = S.scsf_sort([o.field for o in ops], cfg.p0)
    h = scsf.Handle()
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1, precision=scsf.SCSF_MIXED)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops], order,
                                                   chains, prm)
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, cfg.L + 8)
        check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)


def test_mixed_config4_sampled():
    """Config 4 shape (n = 25600, L = 200, k = 240) on a 3-operator prefix, 3 chains."""
    say("mixed c4 sampled")
    cfg = si.CONFIGS[4]
    ops = si.operators(cfg, 3)
    order = S.scsf_sort([o.field for o in ops], cfg.p0)
    h = scsf.Handle()
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1, precision=scsf.SCSF_MIXED,
                           schedule=scsf.SCSF_SCHED_DYNAMIC)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops], order,
                                                   3, prm)
    say([s["iterations"] for s in stats])
    i = int(order[0])
    A = O.assemble(ops[i])
    w, V = E.smallest_eigenpairs(A, cfg.L + 10)
    check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)
