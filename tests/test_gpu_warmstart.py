"""The warm start of Section 3.2 on operators that are truly close (App. E.7: the gain of the
method grows with the similarity of consecutive problems), through the C-ABI library: a chain
of generalized-Poisson operators whose GRF weights move by 1% per step.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, eig as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host  # noqa: E402

N, MODES, COUNT = 32, 8, 10


def chain():
    return si.perturbed_divk_chain(N, MODES, 42, COUNT, step=0.01)


def test_sort_restores_a_shuffled_chain():
    """Algorithm 2 started at the chain's first operator walks the shuffled chain in order."""
    say("warm start: sort restores the chain")
    ops = chain()
    perm = np.random.default_rng(3).permutation(COUNT)
    fields = torch.tensor(np.stack([ops[i].field for i in perm]), device="cuda")
    start = int(np.nonzero(perm == 0)[0][0])
    order = scsf.scsf_sort(scsf.Handle(), fields, 4, start=start)
    assert [int(perm[i]) for i in order] == list(range(COUNT))


@pytest.mark.parametrize("schedule", [scsf.SCSF_SCHED_STATIC, scsf.SCSF_SCHED_DYNAMIC])
def test_warm_start_carries_information(schedule):
    """One chain in order: every warm-started solve needs fewer outer iterations than the same
    solve from a random block, and both reach the dense eigenpairs."""
    say("warm start vs cold, schedule", schedule)
    ops = chain()
    dops = [scsf.DeviceOperator(o) for o in ops]
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 1)
    runs = {}
    for cold in (0, 1):
        prm = scsf.make_params(16, 24, 20, 1e-8, seed=1, schedule=schedule, cold_start=cold)
        ev, vec, st = scsf.scsf_solve_sequence(h, dops, np.arange(COUNT), 1, prm)
        assert all(s["status"] == 0 for s in st)
        runs[cold] = (host(ev), [s["iterations"] for s in st])
    warm_it, cold_it = runs[0][1], runs[1][1]
    say("warm", warm_it, "cold", cold_it)
    assert warm_it[0] == cold_it[0]                      # the chain head is cold either way
    assert all(w < c for w, c in zip(warm_it[1:], cold_it[1:]))
    assert sum(warm_it[1:]) <= 0.75 * sum(cold_it[1:])
    for i, o in enumerate(ops):
        w, _ = E.smallest_eigenpairs(O.assemble(o), 16, method="dense")
        for cold in (0, 1):
            np.testing.assert_allclose(runs[cold][0][i], w, rtol=1e-10)
