"""Smallest-magnitude eigenpairs of indefinite operators (the Helmholtz family) on the GPU
against the dense eigensolver, the oracle's smallest-magnitude ChFSI and a closed form:
single solves, chained solves (graphs against eager launches), uneven batches and the
rejected combinations.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, magnitude as Mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host  # noqa: E402
from test_gpu_graphs import assert_same  # noqa: E402

MAG = scsf.SCSF_TARGET_MAGNITUDE


def check_magnitude_pairs(A, evals, evecs, L, tol):
    """Signed eigenvalues in |.| order against the dense spectrum; residuals; orthonormality;
    every vector in its eigenvalue's eigenspace where the |.|-neighbours are separated."""
    w, V = np.linalg.eigh(A.toarray())
    order = np.argsort(np.abs(w), kind="stable")
    ref = w[order[:L]]
    lam, X = host(evals), host(evecs)
    scale = np.abs(w).max()
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=1e-12 * scale)
    W = A @ X
    rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
    assert rel.max() <= tol * (1 + 1e-6)
    assert np.max(np.abs(X.T @ X - np.eye(L))) < 1e-12
    for j in range(L):
        others = np.delete(w, order[j])
        gap = np.min(np.abs(others - ref[j]))
        if gap > 1e-4 * scale:
            v = V[:, order[j]]
            dk = np.linalg.norm(W[:, j] - X[:, j] * lam[j]) / gap
            assert 1.0 - abs(v @ X[:, j]) <= max(1e-10, 2 * dk * dk + 1e-12), j


@pytest.mark.parametrize("N,L,k", [(20, 12, 20), (24, 12, 20)])
def test_helmholtz_single_solve(N, L, k):
    say("helmholtz solve", N, L, k)
    h = scsf.Handle()
    op = si.helmholtz_operator(N, 8, 30 + N)
    A = O.assemble(op)
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op),
                                        scsf.make_params(L, k, 20, 1e-9, seed=2, target=MAG))
    say(st)
    assert st["status"] == 0
    check_magnitude_pairs(A, ev, vec, L, 1e-9)
    ref = Mg.chfsi_magnitude(A, L, k, 20, 1e-9, seed=2, max_iter=5000)
    assert ref.converged
    np.testing.assert_allclose(host(ev), ref.evals, rtol=1e-10, atol=1e-12 * abs(ref.beta) ** 0.5)


def test_shifted_laplacian_closed_form():
    N = 24
    base = si.laplace_operator(N)
    h_ = 1.0 / (N + 1)
    s = np.sin(np.arange(1, N + 1) * np.pi * h_ / 2) ** 2
    mu = np.sort((4 / h_ ** 2 * (s[:, None] + s[None, :])).ravel())
    c = 0.5 * (mu[30] + mu[31]) + 7.1
    op = si.Stencil5(N=N, wx=base.wx, wy=base.wy, v=np.full((N, N), -c), field=base.field)
    h = scsf.Handle()
    ev, _, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op),
                                      scsf.make_params(14, 22, 20, 1e-10, seed=1, target=MAG))
    ref = (mu - c)[np.argsort(np.abs(mu - c), kind="stable")][:14]
    np.testing.assert_allclose(host(ev), ref, rtol=1e-10, atol=1e-9)
    # 31 eigenvalues lie below c: the lower end cannot be certified, the squared filter ran
    assert st["magnitude_route"] == 2


def test_short_negative_spectrum_takes_the_lower_end():
    """A Helmholtz operator with 9 negative eigenvalues and L = 30: the lowest converged pairs
    certify the 30 of smallest magnitude (route 1), in as few outer iterations as the plain
    method needs for the 30 algebraically smallest of the same operator."""
    say("helmholtz lower end")
    op = si.helmholtz_operator(20, 8, 7)
    A = O.assemble(op)
    h = scsf.Handle()
    d = scsf.DeviceOperator(op)
    ev, vec, _, _, st = scsf.scsf_solve(h, d, scsf.make_params(30, 40, 20, 1e-9, seed=2,
                                                               target=MAG))
    say(st)
    assert st["status"] == 0 and st["magnitude_route"] == 1
    check_magnitude_pairs(A, ev, vec, 30, 1e-9)
    _, _, _, _, st0 = scsf.scsf_solve(h, d, scsf.make_params(30, 40, 20, 1e-9, seed=2))
    assert st["iterations"] <= st0["iterations"] + 2


def test_magnitude_certificate_with_a_large_negative_outlier():
    """Eigenvalues -10, -1, 1, 2, ... (a diagonal CSR operator), L = 3: the three of smallest
    magnitude are -1, 1, 2, found at the lower end (the four lowest certify them)."""
    import scipy.sparse as sp
    lam = np.array([-10.0, -1.0] + list(np.arange(1.0, 59.0)))
    A = sp.diags(lam).tocsr()
    op = scsf.DeviceOperator(csr=(A.indptr, A.indices, A.data))
    ev, _, _, _, st = scsf.scsf_solve(scsf.Handle(), op,
                                      scsf.make_params(3, 8, 20, 1e-10, seed=6, target=MAG))
    assert st["magnitude_route"] == 1
    np.testing.assert_allclose(host(ev), [-1.0, 1.0, 2.0], rtol=1e-12)


def run_sequence(graphs, ops, prm):
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    scsf.scsf_set_graphs(h, graphs)
    return scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops], np.arange(len(ops)),
                                    2, prm)


def test_helmholtz_sequence_graphs_and_eager():
    say("helmholtz sequence")
    ops = [si.helmholtz_operator(22, 8, 500 + i) for i in range(6)]
    prm = scsf.make_params(12, 20, 20, 1e-9, seed=3, schedule=scsf.SCSF_SCHED_STATIC, target=MAG)
    a = run_sequence(False, ops, prm)
    b = run_sequence(True, ops, prm)
    assert_same(a, b)
    ev, vec, st = a
    say([s["iterations"] for s in st])
    for i, o in enumerate(ops):
        assert st[i]["status"] == 0
        check_magnitude_pairs(O.assemble(o), ev[i], vec[i].t(), 12, 1e-9)


def test_helmholtz_batched_uneven():
    say("helmholtz batched")
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    ops = [si.helmholtz_operator(N, 8, 600 + N) for N in (18, 25, 21, 27, 18)]
    Ls = [8, 12, 8, 12, 12]
    order = list(range(len(ops)))
    prm = scsf.make_params(0, 0, 20, 1e-9, seed=5, target=MAG)
    ev, vec, st = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(o) for o in ops], Ls, order, 2,
                                          prm)
    for i, o in enumerate(ops):
        assert st[i]["status"] == 0
        check_magnitude_pairs(O.assemble(o), ev[i], vec[i].t(), Ls[i], 1e-9)


def test_magnitude_rejected_combinations():
    h = scsf.Handle()
    d = scsf.DeviceOperator(si.helmholtz_operator(12, 4, 1))
    for bad in (dict(precision=scsf.SCSF_MIXED), dict(adaptive=1)):
        with pytest.raises(scsf.ScsfError) as e:
            scsf.scsf_solve(h, d, scsf.make_params(8, 12, 20, 1e-8, target=MAG, **bad))
        assert e.value.status == scsf.SCSF_EINVAL
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_solve(h, d, scsf.make_params(8, 12, 20, 1e-8, target=2))
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_solve_sequence(h, [d, d], [0, 1], 1, scsf.make_params(8, 12, 20, 1e-8, target=MAG),
                                 hints=np.array([[0.0, 0.0, 30.0]] * 2))
