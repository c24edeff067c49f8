"""Uneven batches on the GPU: operators of different sizes and different L in one call, the
grid transfer for warm starts across sizes, and the feature order over mixed sizes, against
the CPU oracle.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, eig as E, sort as S, transfer as T, chebyshev as Ch, \
    lanczos as Lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, check_pairs, check_order_stepwise  # noqa: E402


@pytest.fixture(scope="module")
def h():
    return scsf.Handle()


# ------------------------------------------------------------------------------ transfer
@pytest.mark.parametrize("N0,N1,ncols", [(13, 21, 3), (21, 13, 2), (48, 53, 5), (128, 48, 2),
                                         (57, 57, 1), (1, 6, 1), (6, 1, 1)])
def test_interpolate_matches_oracle(h, N0, N1, ncols):
    say("interpolate", N0, N1, ncols)
    rng = np.random.default_rng(N0 * 1000 + N1)
    X = rng.standard_normal((N0 * N0, ncols))
    Y = host(scsf.scsf_interpolate(h, torch.tensor(X.T.copy(), device="cuda"), N0, N1)).T
    ref = T.interpolate_block(X, N0, N1)
    # rounding of the source position (~ N0 eps relative) times a slope <= 2 max|X| per cell
    tol = 4 * max(N0, 1) * np.finfo(float).eps * 2 * np.max(np.abs(X))
    assert np.max(np.abs(Y - ref)) <= tol
    if N0 == N1:
        np.testing.assert_array_equal(Y, X)


def test_interpolate_rejects_overlap_and_bad_sizes(h):
    X = torch.zeros((2, 100), dtype=torch.float64, device="cuda")
    lib = scsf.lib()
    # Y aliasing X
    st = lib.scsf_interpolate(h.ptr, 10, 10, 2, scsf._ptr(X), 100, scsf._ptr(X), 100)
    assert st == scsf.SCSF_EINVAL
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_interpolate(h, X, 0, 5)


# ------------------------------------------------------------------------------ order
def test_order_features_over_mixed_sizes(h):
    """Features of fields of different sides (1/p^2 scaling) ordered together."""
    say("order features mixed sizes")
    sides = [24, 31, 24, 40, 33, 31, 24, 40, 29, 35, 24, 33]
    f = [si.divk_operator(N, 8, 700 + i).field for i, N in enumerate(sides)]
    p0 = 6
    feats = torch.cat([scsf.scsf_features(h, torch.tensor(x[None], device="cuda"), p0) for x in f])
    order = scsf.scsf_order_features(h, feats, start=0)
    ref = np.stack([S.truncated_features(x, p0) for x in f])
    np.testing.assert_allclose(host(feats), ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))
    check_order_stepwise(ref, order)


# ------------------------------------------------------------------------------ solves
def small_uneven(count=14, seed=0):
    """Mixed families, sides 14..29, L in {4, 8, 12}: small enough for dense references."""
    rng = np.random.default_rng(seed)
    ops, Ls = [], []
    for i in range(count):
        N = int(rng.integers(14, 30))
        ops.append(si.divk_operator(N, 8, 300 + i) if i % 2 == 0
                   else si.potential_operator(N, 8, 300 + i))
        Ls.append(int(rng.choice([4, 8, 12])))
    return ops, Ls


def family_order(h, ops, p0):
    """Algorithm 2 within each family (div-K first, then -Laplace + V), concatenated."""
    order = []
    for fam in ("divk", "potential"):
        idx = [i for i, o in enumerate(ops) if o.family == fam]
        if not idx:
            continue
        feats = torch.cat([scsf.scsf_features(h, torch.tensor(ops[i].field[None], device="cuda"),
                                              p0) for i in idx])
        sub = scsf.scsf_order_features(h, feats, start=0)
        order += [idx[j] for j in sub]
    return order


FORMS = [scsf.SCSF_BATCH_GROUPED, scsf.SCSF_BATCH_ONE_SWEEP]
FORM_IDS = ["grouped", "one_sweep"]


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("chains,lanes,sched", [(1, 1, 0), (4, 2, 0), (6, 3, 1), (14, 4, 1)])
def test_batched_small_matches_oracle(chains, lanes, sched, form):
    """Widths 8 and 16 with L in {4, 8, 12}: in the one-sweep form the L = 4 problems sit in
    the last 8 columns of 16-wide blocks, beside problems with other L of the same width."""
    say("batched small chains", chains, "lanes", lanes, "schedule", sched, "form", form)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, lanes)
    scsf.scsf_set_batch_form(h, form)
    ops, Ls = small_uneven()
    order = family_order(h, ops, 6)
    prm = scsf.make_params(0, 0, 20, 1e-8, seed=2, schedule=sched)
    evals, evecs, stats = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(o) for o in ops], Ls,
                                                  order, chains, prm)
    say([s["iterations"] for s in stats])
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, Ls[i] + 6, method="dense")
        assert stats[i]["status"] == 0
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], 1e-8, w, V)


def test_batched_explicit_widths_and_single_operator(h):
    ops, Ls = small_uneven(3, 5)
    ks = [L + 6 for L in Ls]
    prm = scsf.make_params(0, 0, 16, 1e-8, seed=4)
    evals, evecs, stats = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(o) for o in ops], Ls,
                                                  [2, 0, 1], 2, prm, ks=ks)
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, Ls[i] + 6, method="dense")
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], 1e-8, w, V)
    e1, v1, s1 = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(ops[0])], [Ls[0]], [0], 1, prm)
    np.testing.assert_allclose(host(e1[0]), host(evals[0]), rtol=1e-10)


def test_block_width_rule():
    for L, k in [(1, 8), (4, 8), (8, 16), (32, 40), (64, 80), (100, 120), (128, 160), (200, 240)]:
        assert scsf.scsf_block_width(L) == k
        assert k >= L + int(np.ceil(0.2 * L))
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_block_width(0)


def test_batched_errors(h):
    ops, Ls = small_uneven(2, 7)
    d = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(0, 0, 20, 1e-8)
    with pytest.raises(scsf.ScsfError):                       # L >= k
        scsf.scsf_solve_batched(h, d, Ls, [0, 1], 1, prm, ks=[Ls[0], Ls[1] + 4])
    with pytest.raises(scsf.ScsfError):                       # not a permutation
        scsf.scsf_solve_batched(h, d, Ls, [0, 0], 1, prm)
    with pytest.raises(scsf.ScsfError):                       # hints fix the degree
        scsf.scsf_solve_batched(h, d, Ls, [0, 1], 1, scsf.make_params(0, 0, 20, 1e-8, adaptive=1),
                                hints=np.zeros((2, 3)))
    with pytest.raises(scsf.ScsfError):                       # L out of range
        scsf.scsf_solve_batched(h, d, [0, 4], [0, 1], 1, prm)


def test_batched_uneven_full_sizes_sampled(h):
    """The uneven workload at its real shapes (sides 48..128, L in {32, 64, 128}, both
    families) in the launch shape of the benchmark (dynamic schedule, 4 lanes), on a prefix of
    the operators: every pair's residual, and sampled operators against shift-invert."""
    say("batched uneven full sizes")
    cfg = si.CONFIGS[3]
    count = 24
    ops = si.operators(cfg, count)
    Ls = [si.mixed_L(cfg, i) for i in range(count)]
    order = family_order(h, ops, cfg.p0)
    prm = scsf.make_params(0, 0, cfg.degree, cfg.tol, seed=1, schedule=scsf.SCSF_SCHED_DYNAMIC)
    scsf.scsf_set_lanes(h, 4)
    evals, evecs, stats = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(o) for o in ops], Ls,
                                                  order, 8, prm)
    say([(o.N, L, s["iterations"]) for o, L, s in zip(ops, Ls, stats)])
    for i, o in enumerate(ops):
        assert stats[i]["status"] == 0
        A = O.assemble(o)
        X = host(evecs[i]).T
        lam = host(evals[i])
        W = A @ X
        rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
        assert rel.max() <= cfg.tol * (1 + 1e-6)
        assert np.all(np.diff(lam) >= 0)
    for i in sorted({order[0], order[count // 2], max(range(count), key=lambda j: ops[j].N)}):
        A = O.assemble(ops[i])
        w, V = E.smallest_eigenpairs(A, Ls[i] + 10)
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], cfg.tol, w, V)


@pytest.mark.parametrize("sched", [scsf.SCSF_SCHED_STATIC, scsf.SCSF_SCHED_DYNAMIC],
                         ids=["static", "dynamic"])
def test_batched_one_sweep_full_sizes_against_grouped(h, sched):
    """The uneven workload's shapes (sides 48..128, L in {32, 64, 128}, widths 48 / 96 / 160,
    both families) as one lockstep batch per lane: every pair's residual, the eigenvalues
    against the grouped form's, and sampled operators against shift-invert."""
    say("batched one sweep full sizes", sched)
    cfg = si.CONFIGS[3]
    count = 24
    ops = si.operators(cfg, count)
    Ls = [si.mixed_L(cfg, i) for i in range(count)]
    order = family_order(h, ops, cfg.p0)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(0, 0, cfg.degree, cfg.tol, seed=1, schedule=sched)
    g = scsf.Handle()
    scsf.scsf_set_lanes(g, 3)
    e_g, _, _ = scsf.scsf_solve_batched(g, dops, Ls, order, 8, prm)
    scsf.scsf_set_batch_form(g, scsf.SCSF_BATCH_ONE_SWEEP)
    evals, evecs, stats = scsf.scsf_solve_batched(g, dops, Ls, order, 8, prm)
    say([(o.N, L, s["iterations"]) for o, L, s in zip(ops, Ls, stats)])
    for i, o in enumerate(ops):
        assert stats[i]["status"] == 0 and stats[i]["nconv"] >= Ls[i]
        A = O.assemble(o)
        X = host(evecs[i]).T
        lam = host(evals[i])
        W = A @ X
        rel = np.linalg.norm(W - X * lam, axis=0) / np.linalg.norm(W, axis=0)
        assert rel.max() <= cfg.tol * (1 + 1e-6)
        assert np.all(np.diff(lam) >= 0)
        np.testing.assert_allclose(lam, host(e_g[i]), rtol=1e-10)
    for i in sorted({order[0], max(range(count), key=lambda j: Ls[j] * 1000 - ops[j].N)}):
        A = O.assemble(ops[i])
        w, V = E.smallest_eigenpairs(A, Ls[i] + 10)
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], cfg.tol, w, V)


def test_batch_form_errors(h):
    ops, Ls = small_uneven(2, 7)
    d = [scsf.DeviceOperator(o) for o in ops]
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_set_batch_form(h, 2)
    g = scsf.Handle()
    scsf.scsf_set_batch_form(g, scsf.SCSF_BATCH_ONE_SWEEP)
    with pytest.raises(scsf.ScsfError):                       # adaptive degrees
        scsf.scsf_solve_batched(g, d, Ls, [0, 1], 1, scsf.make_params(0, 0, 20, 1e-8, adaptive=1))
    with pytest.raises(scsf.ScsfError):                       # smallest magnitude
        scsf.scsf_solve_batched(g, d, Ls, [0, 1], 1, scsf.make_params(
            0, 0, 20, 1e-8, target=scsf.SCSF_TARGET_MAGNITUDE))


# ------------------------------------------------------------------------------ autotuner
def test_autotune_picks_valid_settings_and_solves():
    say("autotune")
    h = scsf.Handle()
    ops, Ls = small_uneven(12, 11)
    dops = [scsf.DeviceOperator(o) for o in ops]
    order = family_order(h, ops, 6)
    prm = scsf.make_params(0, 0, 20, 1e-8, seed=5)
    before = {L: scsf.scsf_tuned_width(h, L) for L in set(Ls)}
    assert all(before[L] == scsf.scsf_block_width(L) for L in before)
    scsf.scsf_autotune(h, dops, Ls, order, prm, probe=3)
    for L in set(Ls):
        k = scsf.scsf_tuned_width(h, L)
        assert k % 8 == 0 and k >= L + int(np.ceil(0.2 * L)) and k <= 256
        assert k <= min(o.n for o, LL in zip(ops, Ls) if LL == L)
        say("L", L, "width", k)
    for n in (900, 5000, 20000):
        for k in (16, 40, 80, 160, 240):
            assert scsf.scsf_tuned_tile(h, n, k) in (1, 2, 4)
    evals, evecs, stats = scsf.scsf_solve_batched(h, dops, Ls, order, 4, prm)
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, Ls[i] + 6, method="dense")
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], 1e-8, w, V)
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_autotune(h, dops, Ls, order, prm, probe=0)
    scsf.scsf_set_tile(h, 4)
    assert scsf.scsf_tuned_tile(h, 5000, 40) == 4 and scsf.scsf_tuned_tile(h, 20000, 240) == 4
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_set_tile(h, 3)
    evals, evecs, stats = scsf.scsf_solve_batched(h, dops, Ls, order, 4, prm)
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, Ls[i] + 6, method="dense")
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], 1e-8, w, V)


# ------------------------------------------------------------------------------ batched filter
@pytest.mark.parametrize("family,tile", [("five", 1), ("five", 2), ("five", 4), ("five", 8), ("nine", 2),
                                         ("nine", 8)])
def test_filter_batched_matches_oracle(family, tile):
    """B blocks of different grid sides (and, for the 5-point kind, operators with and without
    a potential) in one launch per step, against the oracle's filter of each block."""
    say("filter batched", family, "tile", tile)
    h = scsf.Handle()
    scsf.scsf_set_tile(h, tile)
    if family == "five":
        ops = [si.divk_operator(21, 8, 1), si.potential_operator(30, 8, 2),
               si.divk_operator(17, 8, 3), si.potential_operator(26, 8, 4)]
    else:
        ops = [si.aniso_operator(N, 8, 10 + N) for N in (19, 24, 13)]
    B, ncols, m = len(ops), 13, 20
    ld = max(o.n for o in ops)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((B, ncols, ld))
    wins = []
    for o in ops:
        A = O.assemble(o)
        ub = Lz.gershgorin_upper(A)
        lam, alpha = 0.05 * ub, 0.3 * ub
        wins.append((lam, (alpha + ub) / 2, (ub - alpha) / 2))
    Xd = torch.tensor(X, device="cuda")
    Y = host(scsf.scsf_filter_batched(h, [scsf.DeviceOperator(o) for o in ops], Xd, m, wins))
    np.testing.assert_array_equal(host(Xd), X)
    for b, o in enumerate(ops):
        A = O.assemble(o)
        ref = Ch.filter_block(A, X[b, :, :o.n].T, m, *wins[b])
        assert np.max(np.abs(Y[b, :, :o.n].T - ref)) <= 1e-11 * np.max(np.abs(ref)), b


@pytest.mark.parametrize("tile", [2, 4, 8])
def test_nine_point_sequence_every_tile(tile):
    """Chained 9-point solves with the staged filter pinned to each tile shape (8 columns x 1
    node per thread included): locking leaves partial column groups, against the dense
    eigenpairs."""
    say("nine-point sequence tile", tile)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    scsf.scsf_set_tile(h, tile)
    ops = [si.aniso_operator(20, 8, 60 + i) for i in range(4)]
    L = 8
    prm = scsf.make_params(L, 16, 24, 1e-8, seed=3)
    evals, evecs, stats = scsf.scsf_solve_sequence(h, [scsf.DeviceOperator(o) for o in ops],
                                                   np.arange(len(ops)), 2, prm)
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, L + 6, method="dense")
        assert stats[i]["status"] == 0
        check_pairs(A, evals[i], evecs[i].t(), L, 1e-8, w, V)


def test_filter_batched_errors():
    h = scsf.Handle()
    ops = [scsf.DeviceOperator(si.divk_operator(12, 8, 1)) for _ in range(2)]
    X = torch.zeros((2, 3, 144), dtype=torch.float64, device="cuda")
    with pytest.raises(scsf.ScsfError):                     # e <= 0
        scsf.scsf_filter_batched(h, ops, X, 5, [(1.0, 5.0, 0.0), (1.0, 5.0, 1.0)])
    with pytest.raises(scsf.ScsfError):                     # Y overlapping X
        scsf.scsf_filter_batched(h, ops, X, 5, [(1.0, 5.0, 1.0)] * 2, Y=X)
    mixed = [ops[0], scsf.DeviceOperator(si.aniso_operator(12, 8, 2))]
    with pytest.raises(scsf.ScsfError):                     # kinds differ
        scsf.scsf_filter_batched(h, mixed, X, 5, [(1.0, 5.0, 1.0)] * 2)


# ------------------------------------------------------------------------------ cold starts
def test_cold_start_sequence_equals_separate_solves():
    """cold_start = 1: every solve of a chain starts from the slot's seeded random block, so
    one chain over six operators gives the same pairs and iteration counts as six one-operator
    runs."""
    say("cold start sequence")
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 1)
    cfg = si.CONFIGS[1]
    ops = si.operators(cfg, 6)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=4, cold_start=1)
    ev, vec, st = scsf.scsf_solve_sequence(h, dops, np.arange(6), 1, prm)
    for i, o in enumerate(ops):
        e1, v1, s1 = scsf.scsf_solve_sequence(h, [dops[i]], [0], 1, prm)
        assert s1[0]["iterations"] == st[i]["iterations"]
        np.testing.assert_allclose(host(ev[i]), host(e1[0]), rtol=1e-12)
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, cfg.L + 8)
        check_pairs(A, ev[i], vec[i].t(), cfg.L, cfg.tol, w, V)
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_solve_sequence(h, dops, np.arange(6), 1,
                                 scsf.make_params(cfg.L, cfg.k, 20, cfg.tol, cold_start=2))


# ------------------------------------------------------------------------------ batched Gram
@pytest.mark.parametrize("n,k", [(1000, 24), (4099, 120), (777, 203)])
def test_gram_batched(n, k):
    say("gram batched", n, k)
    h = scsf.Handle()
    rng = np.random.default_rng(k)
    X = rng.standard_normal((5, k, n))
    G, ms = scsf.scsf_gram_batched(h, torch.tensor(X, device="cuda"), timed=True)
    assert ms > 0
    for b in range(5):
        ref = X[b] @ X[b].T
        np.testing.assert_allclose(host(G[b]), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    with pytest.raises(scsf.ScsfError):
        scsf.scsf_gram_batched(h, torch.zeros((2, 257, 300), dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("precision", [scsf.SCSF_FP64, scsf.SCSF_MIXED], ids=["fp64", "mixed"])
def test_batched_mixed_precision_and_hints_match_oracle(precision, form):
    """The layered forms on an uneven batch: FP32 filter (residual form), per-operator window
    and degree hints (here the oracle's lambda_1 and lambda_{L+1} and a degree per operator),
    sides and L differing within the batch, against the dense FP64 eigenpairs; in both batch
    forms (per-(L, k) batches, and one batch over every width)."""
    say("batched mixed + hints", precision, "form", form)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    scsf.scsf_set_batch_form(h, form)
    ops, Ls = small_uneven()
    order = family_order(h, ops, 6)
    ref = []
    hints = np.zeros((len(ops), 3))
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, Ls[i] + 6, method="dense")
        ref.append((A, w, V))
        hints[i] = (w[0], w[Ls[i]], 24 + 3 * (i % 3))
    prm = scsf.make_params(0, 0, 20, 1e-8, seed=2, schedule=scsf.SCSF_SCHED_DYNAMIC,
                           precision=precision)
    evals, evecs, stats = scsf.scsf_solve_batched(h, [scsf.DeviceOperator(o) for o in ops], Ls,
                                                  order, 4, prm, hints=hints)
    say([s["iterations"] for s in stats], [s["hint"] for s in stats])
    for i in range(len(ops)):
        A, w, V = ref[i]
        assert stats[i]["status"] == 0 and stats[i]["hint"] == 2
        check_pairs(A, evals[i], evecs[i].t(), Ls[i], 1e-8, w, V)
