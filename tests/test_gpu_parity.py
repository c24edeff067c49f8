"""Parity of the HIP path (through the C ABI) against the CPU oracle, step by step and end to
end.  Needs an MI355X."""
import numpy as np
import pytest
import scipy.sparse as sp

import scsf_inputs as si
from oracle import operator as O, eig as E, chebyshev as Ch, sort as S, lanczos as Lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def h():
    return scsf.Handle()


def to_dev(x):
    return scsf.as_colmajor(torch.tensor(np.asarray(x, np.float64), device="cuda"))


def host(x):
    return x.detach().cpu().numpy()


OPS5 = {
    "divk32": lambda: si.operator(si.CONFIGS[1], 0),
    "divk37_ragged": lambda: si.divk_operator(37, 8, 5),
    "potential40": lambda: si.potential_operator(40, 8, 3),
    "aniso24": lambda: si.aniso_operator(24, 8, 2),
}


# ------------------------------------------------------------------------------ operator
@pytest.mark.parametrize("name", list(OPS5))
def test_spmm_matches_assembled_matrix(h, name):
    op = OPS5[name]()
    say("spmm", name)
    A = O.assemble(op)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((A.shape[0], 13))
    Y = host(scsf.scsf_spmm(h, scsf.DeviceOperator(op), to_dev(X)))
    ref = A @ X
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_spmm_csr_matches(h):
    say("spmm csr")
    op = si.operator(si.CONFIGS[1], 3)
    A = sp.csr_matrix(O.assemble(op))
    rng = np.random.default_rng(2)
    X = rng.standard_normal((A.shape[0], 6))
    dA = scsf.DeviceOperator(csr=(A.indptr, A.indices, A.data))
    Y = host(scsf.scsf_spmm(h, dA, to_dev(X)))
    np.testing.assert_allclose(Y, A @ X, rtol=1e-13, atol=1e-13 * np.abs(A @ X).max())


# ------------------------------------------------------------------------------ filter
@pytest.mark.parametrize("m", [1, 2, 20, 31])
def test_filter_matches_oracle(h, m):
    say("filter m", m)
    op = si.operator(si.CONFIGS[1], 1)
    A = O.assemble(op)
    rng = np.random.default_rng(m)
    X = rng.standard_normal((A.shape[0], 24))
    ub = Lz.gershgorin_upper(A)
    lam, alpha = 150.0, 3000.0
    c, e = (alpha + ub) / 2, (ub - alpha) / 2
    Y = host(scsf.scsf_filter(h, scsf.DeviceOperator(op), to_dev(X), m, lam, c, e))
    ref = Ch.filter_block(A, X, m, lam, c, e)
    assert np.max(np.abs(Y - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_filter_on_sine_modes_closed_form(h):
    say("filter sine modes")
    N = 40
    hh = 1.0 / (N + 1)
    x = (np.arange(N) + 1.0) * hh
    modes = [(1, 1), (2, 1), (5, 7), (40, 40)]
    X = np.stack([np.outer(np.sin(j * np.pi * x), np.sin(i * np.pi * x)).ravel() for i, j in modes], 1)
    mu = np.array([4 / hh ** 2 * (np.sin(i * np.pi * hh / 2) ** 2 + np.sin(j * np.pi * hh / 2) ** 2)
                   for i, j in modes])
    lam, alpha, beta = mu[0], mu[1] * 1.5, 8 / hh ** 2
    c, e = (alpha + beta) / 2, (beta - alpha) / 2
    Y = host(scsf.scsf_filter(h, scsf.DeviceOperator(si.laplace_operator(N)), to_dev(X), 20, lam, c, e))
    np.testing.assert_allclose(Y, X * Ch.filter_gain(mu, 20, lam, c, e), rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------------------------ orthonormalisation
# k = 160 and 196 (the largest width whose packed factor fits in LDS) and 240 (global scratch)
@pytest.mark.parametrize("n,k,nl", [(1024, 24, 0), (1369, 40, 9), (10000, 120, 0), (4900, 70, 50),
                                    (16384, 160, 0), (9000, 176, 20), (12000, 200, 40)])
def test_orthonormalize(h, n, k, nl):
    say("orth", n, k, nl)
    rng = np.random.default_rng(n + k)
    V = np.linalg.qr(rng.standard_normal((n, nl)))[0] if nl else None
    X = rng.standard_normal((n, k)) @ np.diag(np.logspace(0, 3, k))   # uneven column norms
    Xd = to_dev(X)
    scsf.scsf_orthonormalize(h, Xd, None if V is None else to_dev(V))
    Q = host(Xd)
    assert np.max(np.abs(Q.T @ Q - np.eye(k))) < 1e-13
    P = X if V is None else X - V @ (V.T @ X)
    assert np.linalg.norm(P - Q @ (Q.T @ P)) <= 1e-11 * np.linalg.norm(P)
    if V is not None:
        assert np.max(np.abs(V.T @ Q)) < 1e-13


def test_orthonormalize_rank_deficient_uses_shift_or_reports(h):
    say("orth rank deficient")
    rng = np.random.default_rng(7)
    X = rng.standard_normal((2000, 30))
    X[:, 29] = X[:, 3] * (1 + 1e-13)                      # nearly duplicate column
    Xd = to_dev(X)
    try:
        scsf.scsf_orthonormalize(h, Xd)
    except scsf.ScsfError as err:
        assert err.status == scsf.SCSF_EBREAKDOWN
        return
    Q = host(Xd)
    assert np.max(np.abs(Q.T @ Q - np.eye(30))) < 1e-10


# ------------------------------------------------------------------------------ Rayleigh-Ritz
@pytest.fixture(params=[scsf.SCSF_EIG_TRIDIAG, scsf.SCSF_EIG_JACOBI], ids=["tridiag", "jacobi"])
def he(request):
    """A handle per Rayleigh-Ritz eigensolver."""
    hh = scsf.Handle()
    scsf.scsf_set_eigensolver(hh, request.param)
    return hh


OPS_RR = dict(OPS5, divk100=lambda: si.divk_operator(100, 8, 9),
              potential128=lambda: si.potential_operator(128, 8, 4))


@pytest.mark.parametrize("name,k", [("divk32", 24), ("divk37_ragged", 45), ("aniso24", 33),
                                    ("divk100", 160), ("potential128", 195),
                                    ("potential128", 240)])
def test_rayleigh_ritz_matches_oracle(he, name, k):
    h = he
    say("rr", name, k)
    op = OPS_RR[name]()
    A = O.assemble(op)
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.standard_normal((A.shape[0], k)))[0]
    Xd = to_dev(Q)
    th, res = scsf.scsf_rayleigh_ritz(h, scsf.DeviceOperator(op), Xd)
    G = Q.T @ (A @ Q)
    w, Z = np.linalg.eigh(0.5 * (G + G.T))
    np.testing.assert_allclose(host(th), w, rtol=1e-12, atol=1e-12 * np.abs(w).max())
    Xr = host(Xd)
    ref = Q @ Z
    for a, b in E.clusters(w, 1e-6):
        s = E.subspace_sines(ref[:, a:b], Xr[:, a:b])
        assert s.max() < 1e-9, (a, b, s.max())
    assert np.max(np.abs(Xr.T @ Xr - np.eye(k))) < 1e-13
    W = A @ Xr
    rr = np.linalg.norm(W - Xr * host(th), axis=0) / np.linalg.norm(W, axis=0)
    np.testing.assert_allclose(host(res), rr, rtol=1e-8, atol=1e-14)


def test_rayleigh_ritz_degenerate_clusters(he):
    """Exact eigenvectors of the Dirichlet Laplacian (doubly degenerate eigenvalues), mixed by a
    random rotation: the projected matrix has exactly repeated eigenvalues."""
    h = he
    say("rr degenerate")
    op = si.laplace_operator(12)
    A = O.assemble(op).toarray()
    w, V = np.linalg.eigh(A)
    k = 40
    R = np.linalg.qr(np.random.default_rng(5).standard_normal((k, k)))[0]
    Xd = to_dev(V[:, :k] @ R)
    th, res = scsf.scsf_rayleigh_ritz(h, scsf.DeviceOperator(op), Xd)
    np.testing.assert_allclose(host(th), w[:k], rtol=1e-12)
    Xr = host(Xd)
    assert np.max(np.abs(Xr.T @ Xr - np.eye(k))) < 1e-13
    assert host(res).max() < 1e-12
    for a, b in E.clusters(w[:k], 1e-6):
        assert E.subspace_sines(V[:, a:b], Xr[:, a:b]).max() < 1e-10


# ------------------------------------------------------------------------------ bounds
@pytest.mark.parametrize("name", ["divk32", "potential40", "aniso24"])
def test_bounds(h, name):
    say("bounds", name)
    op = OPS5[name]()
    A = O.assemble(op)
    b = scsf.scsf_bounds(h, scsf.DeviceOperator(op), 20, 5)
    w = np.linalg.eigvalsh(A.toarray())
    assert b["gershgorin"] == pytest.approx(Lz.gershgorin_upper(A), rel=1e-13)
    assert b["lanczos"] >= w[-1] * (1 - 1e-12)
    assert b["theta_min"] >= w[0] * (1 - 1e-10)
    assert b["beta"] == min(b["gershgorin"], b["lanczos"])
    assert b["beta"] >= w[-1] * (1 - 1e-12)


# ------------------------------------------------------------------------------ sort
def _fields(cfg, count):
    return [o.field for o in si.operators(cfg, count)]


@pytest.mark.parametrize("cfgi,count,p0", [(1, 20, 4), (1, 20, 32), (2, 60, 20)])
def test_features_match_oracle(h, cfgi, count, p0):
    say("features", cfgi, count, p0)
    f = _fields(si.CONFIGS[cfgi], count)
    got = host(scsf.scsf_features(h, torch.tensor(np.stack(f), device="cuda"), p0))
    ref = np.stack([S.truncated_features(x, p0) for x in f])
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def check_order_stepwise(feats, order, start=0):
    """Bit-exact order wherever the best two candidate distances differ by more than 1e-9
    (relative); at a near-tie the GPU's pick is accepted and the walk continues from it."""
    n = feats.shape[0]
    assert order[0] == start and sorted(order) == list(range(n))
    remaining = np.array(sorted(set(range(n)) - {start}))
    cur = start
    for pick in order[1:]:
        j, dbest, d = S.greedy_step(feats, cur, remaining)
        if pick != j:
            dp = d[np.searchsorted(remaining, pick)]
            assert abs(dp - dbest) <= 1e-9 * max(dp, dbest), (cur, pick, j)
        remaining = remaining[remaining != pick]
        cur = pick


@pytest.mark.parametrize("cfgi,count,p0", [(1, 20, 4), (2, 200, 20), (5, 300, 16)])
def test_sort_matches_oracle(h, cfgi, count, p0):
    say("sort", cfgi, count, p0)
    f = _fields(si.CONFIGS[cfgi], count)
    order = scsf.scsf_sort(h, torch.tensor(np.stack(f), device="cuda"), p0)
    feats = np.stack([S.truncated_features(x, p0) for x in f])
    check_order_stepwise(feats, order)


def test_sort_start_and_duplicates(h):
    say("sort duplicates")
    f = _fields(si.CONFIGS[1], 12)
    f[5] = f[2].copy()
    f[9] = f[2].copy()
    order = scsf.scsf_sort(h, torch.tensor(np.stack(f), device="cuda"), 4, start=7)
    ref = S.scsf_sort(f, 4, start=7)
    assert list(order) == list(ref)


def test_sort_nonfinite_fields_rejected(h):
    """A NaN field gives NaN distances: the walk still visits every operator exactly once
    (non-finite distances rank as +infinity) and the call reports SCSF_EINVAL."""
    say("sort: non-finite")
    f = torch.rand((5, 1, 8, 8), dtype=torch.float64, device="cuda")
    f[2, 0, 3, 3] = float("nan")
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_sort(h, f, 4)


def test_sort_invalid(h):
    f = torch.zeros((3, 1, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_sort(h, f, 9)


# ------------------------------------------------------------------------------ solve
def check_pairs(A, evals, evecs, L, tol, w_ref, V_ref, angle=1e-6):
    """Eigenvalues within 1e-10 relative of the reference, relative residuals <= tol,
    orthonormal vectors, and the subspace angle of every eigenvalue cluster (maximal runs of
    relative gap < 1e-2) against the reference.

    tol <= 1e-10: every cluster below L, a cluster straddling L cut at L, is held to `angle`
    without exception.  tol = 1e-8 cannot certify 1e-6 for clusters whose gap is below 1e-2 of
    the eigenvalue (Davis-Kahan: sin <= ||r|| / gap); there a cluster straddling L is skipped
    and the other clusters are held to max(angle, 2 x their Davis-Kahan bound)."""
    lam = host(evals)
    X = host(evecs)
    assert np.max(np.abs(lam - w_ref[:L]) / np.abs(w_ref[:L])) < 1e-10
    W = A @ X
    rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
    assert rel.max() <= tol * (1 + 1e-6)
    assert np.max(np.abs(X.T @ X - np.eye(L))) < 1e-12
    strict = tol <= 1e-10
    for a, b in E.clusters(w_ref):
        if a >= L:
            break
        if b > L and not strict:
            break
        b = min(b, L)
        s = E.subspace_sines(V_ref[:, a:b], X[:, a:b]).max()
        if strict:
            assert s <= angle, (a, b, s)
            continue
        gap = min(w_ref[a] - w_ref[a - 1] if a > 0 else np.inf, w_ref[b] - w_ref[b - 1])
        dk = np.max(np.linalg.norm(W - X * lam, axis=0)[a:b]) * np.sqrt(b - a) / gap
        assert s <= max(angle, 2 * dk), (a, b, s, dk)


def test_solve_cold_config1(h):
    say("solve cold c1")
    cfg = si.CONFIGS[1]
    op = si.operator(cfg, 0)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, cfg.L + 8)
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=3)
    ev, vec, Xn, thn, st = scsf.scsf_solve(h, scsf.DeviceOperator(op), prm)
    say(st)
    assert st["status"] == 0 and st["nconv"] >= cfg.L
    check_pairs(A, ev, vec, cfg.L, cfg.tol, w, V)


def test_solve_tight_tolerance_angles(h):
    say("solve tol 1e-12")
    cfg = si.CONFIGS[1]
    op = si.operator(cfg, 4)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, cfg.L + 8)
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, 1e-12, seed=3)
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op), prm)
    check_pairs(A, ev, vec, cfg.L, 1e-12, w, V, angle=1e-6)


def test_solve_laplacian_closed_form(h):
    say("solve laplacian")
    N = 32
    A = O.assemble(si.laplace_operator(N))
    hh = 1.0 / (N + 1)
    s = np.sin(np.arange(1, N + 1) * np.pi * hh / 2) ** 2
    lam = np.sort((4 / hh ** 2 * (s[:, None] + s[None, :])).ravel())
    prm = scsf.make_params(15, 24, 20, 1e-10, seed=1)      # lambda_16 = lambda_17: stop at 15
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(si.laplace_operator(N)), prm)
    np.testing.assert_allclose(host(ev), lam[:15], rtol=1e-10)


def test_solve_returns_the_L_smallest_when_pairs_enter_late(h):
    """The warm-start block holds the two smallest eigenvectors of a diagonal operator only as
    small admixtures of two guard columns, while exact eigenvectors of larger values (12
    missing) converge at once.  The solve must not stop when L pairs are locked while a smaller
    pair is still converging, and must return the L smallest locked pairs."""
    from test_oracle_numerics import planted_late_pairs
    say("solve: late pairs")
    A, X0, th0 = planted_late_pairs()
    A = A.tocsr()
    op = scsf.DeviceOperator(csr=(A.indptr, A.indices, A.data))
    prm = scsf.make_params(4, 6, 2, 1e-10, seed=3)
    Xp = torch.tensor(np.asfortranarray(X0).T.copy(), device="cuda").t()
    thp = torch.tensor(th0, device="cuda")
    ev, vec, _, _, st = scsf.scsf_solve(h, op, prm, Xp, thp)
    say(st)
    np.testing.assert_allclose(host(ev), [1.0, 2.0, 10.0, 11.0], rtol=1e-12)


def test_solve_warm_identical_operator_one_iteration(h):
    say("solve warm identical")
    cfg = si.CONFIGS[1]
    op = scsf.DeviceOperator(si.operator(cfg, 2))
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=3)
    ev, vec, Xn, thn, st = scsf.scsf_solve(h, op, prm)
    ev2, vec2, _, _, st2 = scsf.scsf_solve(h, op, prm, Xn, thn)
    assert st2["iterations"] == 1
    np.testing.assert_allclose(host(ev2), host(ev), rtol=1e-12)


def test_solve_nine_point(h):
    say("solve 9-point")
    op = si.aniso_operator(32, 8, 4)
    A = O.assemble(op)
    w, V = E.smallest_eigenpairs(A, 24)
    prm = scsf.make_params(16, 24, 20, 1e-8, seed=2)
    ev, vec, _, _, st = scsf.scsf_solve(h, scsf.DeviceOperator(op), prm)
    check_pairs(A, ev, vec, 16, 1e-8, w, V)


def test_solve_errors(h):
    say("solve errors")
    cfg = si.CONFIGS[1]
    op = scsf.DeviceOperator(si.operator(cfg, 5))
    with pytest.raises(scsf.ScsfError) as e1:
        scsf.scsf_solve(h, op, scsf.make_params(24, 24))
    assert e1.value.status == scsf.SCSF_EINVAL
    with pytest.raises(scsf.ScsfError) as e2:
        scsf.scsf_solve(h, op, scsf.make_params(16, 2000))
    assert e2.value.status == scsf.SCSF_EINVAL
    ev, vec, Xn, thn, st = scsf.scsf_solve(h, op, scsf.make_params(16, 24, max_iter=1),
                                           allow_notconv=True)
    assert st["status"] == scsf.SCSF_ENOTCONV and st["iterations"] == 1
    Xbad = Xn.clone()
    Xbad[5, 3] = float("nan")
    with pytest.raises(scsf.ScsfError) as e3:
        scsf.scsf_solve(h, op, scsf.make_params(16, 24), Xbad, thn)
    assert e3.value.status in (scsf.SCSF_ENUMERIC, scsf.SCSF_EBREAKDOWN)


# ------------------------------------------------------------------------------ sequences
@pytest.mark.parametrize("chains,lanes,sched", [(1, 1, 0), (3, 4, 0), (5, 2, 0), (4, 2, 1)])
def test_sequence_config1_matches_oracle(chains, lanes, sched):
    say("sequence c1 chains", chains, "lanes", lanes, "schedule", sched)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, lanes)
    cfg = si.CONFIGS[1]
    ops = si.operators(cfg)
    order = S.scsf_sort([o.field for o in ops], cfg.p0)
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1, schedule=sched)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops], order,
                                                   chains, prm)
    say([s["iterations"] for s in stats])
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, cfg.L + 8)
        check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)
        assert stats[i]["status"] == 0


def test_sequence_config2_sampled(h):
    """Config 2 (n = 10^4, L = 100, k = 120, degree 20) in the chunked launch shape of the
    benchmark, on a prefix of the sorted order; sampled operators against shift-invert."""
    say("sequence c2 sampled")
    cfg = si.CONFIGS[2]
    ops = si.operators(cfg, 16)
    order = S.scsf_sort([o.field for o in ops], cfg.p0)
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops], order,
                                                   8, prm)
    say([s["iterations"] for s in stats])
    for i in [int(order[0]), int(order[5]), int(order[-1])]:
        A = O.assemble(ops[i])
        w, V = E.smallest_eigenpairs(A, cfg.L + 10)
        check_pairs(A, evals[i], evecs[i].t(), cfg.L, cfg.tol, w, V)
