"""The thin-plate vibration family on the GPU against the CPU oracle: the 13-point standard-form
step, its Gershgorin and Lanczos bounds, the batched filter, and solves (single, chained with
graphs, uneven sides) whose eigenvectors are returned M-orthonormal.  Needs an MI355X."""
import numpy as np
import pytest
import scipy.linalg

import scsf_inputs as si
from oracle import operator as O, eig as E, chebyshev as Ch, lanczos as Lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, to_dev, check_pairs  # noqa: E402


@pytest.fixture(scope="module")
def h():
    return scsf.Handle()


@pytest.mark.parametrize("N", [5, 17, 30, 64])
def test_plate_spmm_matches_assembled_matrix(h, N):
    say("plate spmm", N)
    op = si.plate_operator(N, 8, 40 + N)
    A = O.assemble(op)
    X = np.random.default_rng(N).standard_normal((op.n, 9))
    Y = host(scsf.scsf_spmm(h, scsf.DeviceOperator(op), to_dev(X)))
    ref = A @ X
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("tile", [1, 2, 4])
def test_plate_filter_batched_uneven(tile):
    say("plate filter batched tile", tile)
    h = scsf.Handle()
    scsf.scsf_set_tile(h, tile)
    ops = [si.plate_operator(N, 8, N) for N in (23, 14, 31)]
    ld = max(o.n for o in ops)
    X = np.random.default_rng(3).standard_normal((3, 11, ld))
    wins = []
    for o in ops:
        ub = Lz.gershgorin_upper(O.assemble(o))
        wins.append((0.0, 0.55 * ub, 0.45 * ub))
    Y = host(scsf.scsf_filter_batched(h, [scsf.DeviceOperator(o) for o in ops],
                                      torch.tensor(X, device="cuda"), 20, wins))
    for b, o in enumerate(ops):
        ref = Ch.filter_block(O.assemble(o), X[b, :, :o.n].T, 20, *wins[b])
        assert np.max(np.abs(Y[b, :, :o.n].T - ref)) <= 1e-11 * np.max(np.abs(ref)), b


def test_plate_bounds(h):
    op = si.plate_operator(24, 8, 9)
    A = O.assemble(op)
    bd = scsf.scsf_bounds(h, scsf.DeviceOperator(op))
    assert bd["gershgorin"] == pytest.approx(Lz.gershgorin_upper(A), rel=1e-12)
    lmax = np.linalg.eigvalsh(A.toarray())[-1]
    assert bd["lanczos"] >= lmax * (1 - 1e-12) and bd["beta"] >= lmax * (1 - 1e-12)


def check_generalized(op, evals, evecs, L, tol):
    """Eigenvalues against the dense generalized problem, K u = lambda M u, u^T M u = I."""
    K, M = O.assemble_plate_pair(op)
    w = scipy.linalg.eigh(K.toarray(), M.toarray(), eigvals_only=True)[:L]
    lam, U = host(evals), host(evecs)
    np.testing.assert_allclose(lam, w, rtol=1e-10)
    np.testing.assert_allclose(U.T @ (M @ U), np.eye(L), atol=1e-11)
    R = K @ U - (M @ U) * lam
    # the standard-form residual is <= tol; in the plain 2-norm it may grow by sqrt(cond M)
    rho = op.rho.ravel()
    bound = tol * np.sqrt(rho.max() / rho.min()) * (1 + 1e-6)
    assert np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(K @ U, axis=0)) <= bound


def test_plate_solve_single(h):
    say("plate solve")
    op = si.plate_operator(20, 8, 2)
    ev, vec, Xn, thn, st = scsf.scsf_solve(h, scsf.DeviceOperator(op),
                                           scsf.make_params(16, 24, 30, 1e-8, seed=1))
    say(st)
    assert st["status"] == 0
    check_generalized(op, ev, vec, 16, 1e-8)
    # the standard-form pairs against the oracle's (y = M^{1/2} u)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, 22)
    y = host(vec) * np.sqrt(op.rho.ravel())[:, None]
    check_pairs(A, ev, torch.tensor(y), 16, 1e-8, w, V)


@pytest.mark.parametrize("graphs", [False, True])
def test_plate_sequence(graphs):
    say("plate sequence graphs", graphs)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    scsf.scsf_set_graphs(h, graphs)
    ops = [si.plate_operator(18, 8, 100 + i) for i in range(6)]
    prm = scsf.make_params(12, 20, 30, 1e-8, seed=3, schedule=scsf.SCSF_SCHED_STATIC)
    ev, vec, st = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops],
                                           np.arange(6), 2, prm)
    say([s["iterations"] for s in st])
    for i, o in enumerate(ops):
        assert st[i]["status"] == 0
        check_generalized(o, ev[i], vec[i].t(), 12, 1e-8)


def test_plate_batched_uneven_sides():
    """Sides 16..26 in one batch: the grid transfer moves warm starts between sides."""
    say("plate batched")
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    ops = [si.plate_operator(N, 8, 200 + N) for N in (16, 21, 26, 18, 24, 16)]
    Ls = [8, 8, 12, 12, 8, 12]
    prm = scsf.make_params(0, 0, 30, 1e-8, seed=4)
    ev, vec, st = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(o) for o in ops], Ls,
                                          np.arange(6), 2, prm)
    for i, o in enumerate(ops):
        assert st[i]["status"] == 0
        check_generalized(o, ev[i], vec[i].t(), Ls[i], 1e-8)


def test_plate_rejects_mixed_precision(h):
    op = scsf.DeviceOperator(si.plate_operator(12, 4, 1))
    with pytest.raises(scsf.ScsfError) as e:
        scsf.scsf_solve(h, op, scsf.make_params(8, 12, 20, 1e-8, precision=scsf.SCSF_MIXED))
    assert e.value.status == scsf.SCSF_EINVAL
