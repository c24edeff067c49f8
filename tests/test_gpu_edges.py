"""Edge cases of the solvers on the GPU against the dense oracle: a single wanted pair, a block
as wide as the matrix, the widest block (k = 256), general CSR operators, more chains than
operators, empty or out-of-range inputs, and a chain checkpointed to disk and resumed.
Needs an MI355X."""
import numpy as np
import pytest
import scipy.sparse as sp

import scsf_inputs as si
from oracle import operator as O, eig as E

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, check_pairs  # noqa: E402


@pytest.fixture(scope="module")
def h():
    return scsf.Handle()


def test_single_pair(h):
    say("edge: L = 1")
    N = 6
    op = si.divk_operator(N, 4, 3)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, 4, method="dense")
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op),
                                        scsf.make_params(1, 2, 20, 1e-10, seed=1))
    assert st["status"] == 0
    check_pairs(A, ev, vec, 1, 1e-10, w, V)


def test_block_as_wide_as_the_matrix(h):
    """k = n = 16 (fewer rows than Lanczos steps): the block spans the whole space."""
    say("edge: k = n")
    op = si.divk_operator(4, 4, 5)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, 16, method="dense")
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op),
                                        scsf.make_params(8, 16, 20, 1e-10, seed=1))
    assert st["status"] == 0
    check_pairs(A, ev, vec, 8, 1e-10, w, V)


def test_widest_block(h):
    """k = 256, the largest width (Jacobi in global scratch, Cholesky of width 256)."""
    say("edge: k = 256")
    op = si.divk_operator(20, 8, 9)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, 210, method="dense")
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op),
                                        scsf.make_params(200, 256, 20, 1e-8, seed=2))
    say(st)
    assert st["status"] == 0
    check_pairs(A, ev, vec, 200, 1e-8, w, V)


def test_csr_operators_solve_and_chain(h):
    """General CSR matrices through the single solve and a warm-started chain."""
    say("edge: CSR")
    ops = [si.divk_operator(18, 8, 40 + i) for i in range(3)]
    mats = [sp.csr_matrix(O.assemble(o)) for o in ops]
    dops = [scsf.DeviceOperator(csr=(A.indptr, A.indices, A.data)) for A in mats]
    prm = scsf.make_params(10, 16, 20, 1e-9, seed=3)
    ev, vec, _, _, st = scsf.scsf_solve(h, dops[0], prm)
    w, V = E.smallest_eigenpairs(mats[0], 16, method="dense")
    check_pairs(mats[0], ev, vec, 10, 1e-9, w, V)
    evs, vecs, sts = scsf.scsf_solve_sequence(h, dops, [2, 0, 1], 1, prm)
    for i, A in enumerate(mats):
        assert sts[i]["status"] == 0
        w, V = E.smallest_eigenpairs(A, 16, method="dense")
        check_pairs(A, evs[i], vecs[i].t(), 10, 1e-9, w, V)


def test_more_chains_than_operators():
    say("edge: chains > operators")
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 4)
    ops = [si.divk_operator(16, 8, 60 + i) for i in range(3)]
    prm = scsf.make_params(8, 12, 20, 1e-9, seed=4, schedule=scsf.SCSF_SCHED_DYNAMIC)
    ev, vec, st = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops], [0, 1, 2],
                                           10, prm)
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, 12, method="dense")
        assert st[i]["status"] == 0
        check_pairs(A, ev[i], vec[i].t(), 8, 1e-9, w, V)


def test_empty_and_out_of_range_inputs(h):
    lib = scsf.lib()
    prm = scsf.make_params(8, 12, 20, 1e-8)
    arr = (scsf.Operator * 1)()
    order = (scsf.c_int32 * 1)(0)
    d = torch.empty(16, device="cuda", dtype=torch.float64)
    st = lib.scsf_solve_sequence(h.ptr, arr, 0, order, 1, scsf.ctypes.byref(prm), scsf._ptr(d),
                                 scsf._ptr(d), None)
    assert st == scsf.SCSF_EINVAL                                   # no operators
    op = scsf.DeviceOperator(si.divk_operator(8, 4, 1))
    for bad in (scsf.make_params(8, 257, 20, 1e-8), scsf.make_params(8, 12, 129, 1e-8),
                scsf.make_params(8, 12, 0, 1e-8), scsf.make_params(8, 12, 20, 0.0),
                scsf.make_params(0, 12, 20, 1e-8), scsf.make_params(8, 65, 20, 1e-8),
                scsf.make_params(8, 12, 65, 1e-8, precision=scsf.SCSF_MIXED)):
        with pytest.raises(scsf.ScsfError) as e:                   # k > n = 64 in the last
            scsf.scsf_solve(h, op, bad)
        assert e.value.status == scsf.SCSF_EINVAL


def test_checkpoint_and_resume_of_a_chain(h, tmp_path):
    """The state of a warm-started chain is (position, X_next, theta_next).  A chain stopped
    after its third operator, its state written to disk and read back in a new handle, resumes
    with results identical to the uninterrupted chain."""
    say("edge: checkpoint / resume")
    cfg = si.CONFIGS[1]
    ops = [scsf.DeviceOperator(o) for o in si.operators(cfg, 6)]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=5)

    def run(h_, idx, X=None, th=None):
        out = []
        for i in idx:
            ev, _, X, th, st = scsf.scsf_solve(h_, ops[i], prm, X, th)
            out.append((host(ev), st["iterations"]))
        return out, X, th

    full, _, _ = run(h, range(6))
    head, X, th = run(h, range(3))
    np.savez(tmp_path / "chain.npz", pos=3, X=host(X).T, theta=host(th))
    ck = np.load(tmp_path / "chain.npz")
    h2 = scsf.Handle()
    Xr = torch.tensor(ck["X"], device="cuda").t()              # back to n x k column-major
    tail, _, _ = run(h2, range(int(ck["pos"]), 6), Xr, torch.tensor(ck["theta"], device="cuda"))
    for (a, ia), (b, ib) in zip(full, head + tail):
        np.testing.assert_array_equal(a, b)
        assert ia == ib
