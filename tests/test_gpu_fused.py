"""The fused filter (S Chebyshev steps of Algorithm 1 per launch, staged in LDS with their
halos) against the CPU oracle's filter and solves, through the C-ABI library: 5- and 9-point
operators of several sizes in one batch (ragged tiles, grid sides with halos wider than a
row), degrees below, at and above the group size, and chained solves with per-problem degrees
(hints) and with the plain degree.  Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si
from oracle import operator as O, eig as E, chebyshev as Ch, lanczos as Lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host, check_pairs  # noqa: E402

BATCHES = {
    "5pt": lambda: [si.divk_operator(37, 8, 5), si.divk_operator(30, 8, 6),
                    si.divk_operator(41, 8, 7)],
    "5pt_potential": lambda: [si.potential_operator(33, 8, 3), si.divk_operator(29, 8, 4)],
    "9pt": lambda: [si.aniso_operator(24, 8, 2), si.aniso_operator(19, 8, 3)],
    "9pt_128": lambda: [si.operator(si.CONFIGS[5], 0), si.operator(si.CONFIGS[5], 1)],
}


@pytest.mark.parametrize("S", [2, 3, 4])
@pytest.mark.parametrize("batch", sorted(BATCHES))
@pytest.mark.parametrize("m", [1, 3, 7, 20])
def test_fused_filter_matches_oracle(S, batch, m):
    say("fused filter S", S, batch, "m", m)
    ops = BATCHES[batch]()
    h = scsf.Handle()
    scsf.scsf_set_fused_steps(h, S)
    ncols = 13
    ld = max(o.N * o.N for o in ops)
    rng = np.random.default_rng(S * 100 + m)
    X = np.zeros((len(ops), ncols, ld))
    wins, refs = [], []
    for b, o in enumerate(ops):
        A = O.assemble(o)
        Xb = rng.standard_normal((A.shape[0], ncols))
        X[b, :, :A.shape[0]] = Xb.T
        ub = Lz.gershgorin_upper(A)
        lam, alpha = 0.0, 0.2 * ub
        c, e = (alpha + ub) / 2, (ub - alpha) / 2
        wins.append((lam, c, e))
        refs.append(Ch.filter_block(A, Xb, m, lam, c, e))
    Xd = torch.tensor(X, device="cuda")
    Y = host(scsf.scsf_filter_batched(h, [scsf.DeviceOperator(o) for o in ops], Xd, m, wins))
    for b, o in enumerate(ops):
        got = Y[b, :, :o.N * o.N].T
        assert np.max(np.abs(got - refs[b])) <= 1e-11 * np.max(np.abs(refs[b])), (b, m)


@pytest.mark.parametrize("S", [2, 3])
def test_fused_sequence_matches_oracle_and_unfused(S):
    """c1-sized chained solve (4 chains on 2 lanes, graphs): fused and unfused give the dense
    eigenpairs, in the same number of outer iterations.  The static schedule fixes every
    chain's operators (the dynamic one hands them out by timing, so warm starts would differ)."""
    say("fused sequence S", S)
    cfg = si.CONFIGS[1]
    ops = si.operators(cfg, 10)
    dops = [scsf.DeviceOperator(o) for o in ops]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_STATIC)
    runs = {}
    for fuse in (0, S):
        h = scsf.Handle()
        scsf.scsf_set_lanes(h, 2)
        scsf.scsf_set_fused_steps(h, fuse)
        runs[fuse] = scsf.scsf_solve_sequence(h, dops, np.arange(len(ops)), 4, prm)
    ev0, _, st0 = runs[0]
    ev1, vec1, st1 = runs[S]
    # the same recurrence node by node: equal iteration counts up to a rounding-level flip
    assert abs(sum(s["iterations"] for s in st1) - sum(s["iterations"] for s in st0)) <= 2
    np.testing.assert_allclose(host(ev1), host(ev0), rtol=1e-11)
    for i, o in enumerate(ops):
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, cfg.L + 8, method="dense")
        check_pairs(A, ev1[i], vec1[i].t(), cfg.L, cfg.tol, w, V)


def test_fused_hinted_degrees_on_nine_point_operators():
    """Per-problem degrees in one batch (hints 17..31) with the fused filter (S = 3): every
    degree is raised to the largest's residue mod 2 S, and the pairs match the oracle's."""
    say("fused hinted nine-point")
    cfg = si.CONFIGS[5]
    ops = [si.aniso_operator(30, 8, 40 + i) for i in range(8)]
    dops = [scsf.DeviceOperator(o) for o in ops]
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 2)
    scsf.scsf_set_fused_steps(h, 3)
    hints = np.array([[0.0, 0.0, 17.0 + 2 * i] for i in range(len(ops))])
    prm = scsf.make_params(24, 32, 20, 1e-9, seed=2, schedule=scsf.SCSF_SCHED_DYNAMIC)
    ev, vec, st = scsf.scsf_solve_sequence(h, dops, np.arange(len(ops)), 4, prm, hints=hints)
    say([s["degree"] for s in st], [s["iterations"] for s in st])
    for i, o in enumerate(ops):
        assert st[i]["status"] == 0
        A = O.assemble(o)
        w, V = E.smallest_eigenpairs(A, 32, method="dense")
        check_pairs(A, ev[i], vec[i].t(), 24, 1e-9, w, V)
