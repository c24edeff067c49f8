"""Outer iterations replayed as HIP graphs against the same kernels launched one by one.

Each solve replays the captured graphs once per outer iteration, with the host's own uploads,
downloads and synchronisations between the replays; bitwise-equal eigenpairs and equal
iteration counts therefore check every replay against the eager run.  The static schedule is
used throughout: under the dynamic one the chain that claims an operator (and so its warm
start) depends on timing.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host  # noqa: E402
from test_gpu_batched import small_uneven  # noqa: E402


def both(run):
    out = []
    for graphs in (False, True):
        h = scsf.Handle()
        scsf.scsf_set_lanes(h, 2)
        scsf.scsf_set_graphs(h, graphs)
        out.append(run(h))
    return out


def assert_same(a, b):
    (ea, va, sa), (eb, vb, sb) = a, b
    assert [s["iterations"] for s in sa] == [s["iterations"] for s in sb]
    for x, y in zip(ea, eb):
        np.testing.assert_array_equal(host(x), host(y))
    for x, y in zip(va, vb):
        np.testing.assert_array_equal(host(x), host(y))


def test_graphs_sequence_fp64():
    say("graphs: fp64 sequence")
    cfg = si.CONFIGS[1]
    dops = [scsf.DeviceOperator(o) for o in si.operators(cfg)]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_STATIC)
    a, b = both(lambda h: scsf.scsf_solve_sequence(h, dops, np.arange(len(dops)), 3, prm))
    assert_same(a, b)


def test_graphs_batched_uneven():
    say("graphs: uneven batch")
    ops, Ls = small_uneven(10, 3)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(0, 0, 20, 1e-8, seed=2, schedule=scsf.SCSF_SCHED_STATIC)
    a, b = both(lambda h: scsf.scsf_solve_batched(h, dops, Ls, np.arange(len(ops)), 4, prm))
    assert_same(a, b)


def test_graphs_mixed_precision():
    say("graphs: mixed precision")
    ops = [si.divk_operator(40, 8, 50 + i) for i in range(6)]
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(20, 28, 20, 1e-8, seed=3, precision=scsf.SCSF_MIXED)
    a, b = both(lambda h: scsf.scsf_solve_sequence(h, dops, np.arange(6), 2, prm))
    assert_same(a, b)


def test_graphs_per_problem_degrees():
    """Degree hints 12..40: the iteration degree M changes as problems finish, so several
    graph sets are captured and replayed in turn."""
    say("graphs: per-problem degrees")
    cfg = si.CONFIGS[5]
    dops = [scsf.DeviceOperator(o) for o in si.operators(cfg, 8)]
    hints = np.array([[0.0, 0.0, d] for d in (12, 40, 20, 33, 16, 25, 12, 38)])
    prm = scsf.make_params(cfg.L, cfg.k, 20, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_STATIC)
    a, b = both(lambda h: scsf.scsf_solve_sequence(h, dops, np.arange(8), 4, prm, hints=hints))
    assert_same(a, b)
