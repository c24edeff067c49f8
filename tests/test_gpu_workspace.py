"""The device-workspace contract of the C ABI and the per-phase solve times (Algorithm 3's
inputs and outputs in caller memory; the cost split of App. E.3), through the C-ABI library.
Needs an MI355X."""
import numpy as np
import pytest

import scsf_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402

from test_gpu_parity import say, host  # noqa: E402


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def workspace(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def test_single_solve_in_caller_workspace_matches_and_allocates_nothing():
    say("workspace: single solve")
    cfg = si.CONFIGS[2]
    op = scsf.DeviceOperator(si.operator(cfg, 3))
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=2)
    ref = scsf.scsf_solve(scsf.Handle(), op, prm)
    need = scsf.scsf_workspace_bytes(prm, op.n)
    say("workspace bytes", need)
    h = scsf.Handle()
    buf = workspace(need)
    scsf.scsf_set_workspace(h, buf)
    got = scsf.scsf_solve(h, op, prm)                    # first call: pinned staging, events
    before = free_bytes()
    got = scsf.scsf_solve(h, op, prm, out=got)           # outputs in the same caller tensors
    after = free_bytes()
    assert after == before, (before, after)
    assert scsf.scsf_workspace_peak(h) <= need
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    assert got[4]["iterations"] == ref[4]["iterations"]


def test_chained_solve_in_caller_workspace_allocates_nothing():
    """A chained solve (4 lanes, graphs) with the queried workspace: device free memory is the
    same before and after, and the results equal those of library-allocated buffers."""
    say("workspace: chained solve")
    cfg = si.CONFIGS[1]
    ops = [scsf.DeviceOperator(o) for o in si.operators(cfg)]
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1,
                           schedule=scsf.SCSF_SCHED_STATIC)
    order = np.arange(len(ops))
    chains = 8
    h0 = scsf.Handle()
    scsf.scsf_set_lanes(h0, 4)
    ev0, vec0, _ = scsf.scsf_solve_sequence(h0, ops, order, chains, prm)
    h = scsf.Handle()
    scsf.scsf_set_lanes(h, 4)
    need = scsf.scsf_workspace_bytes_sequence(h, prm, ops[0].n, len(ops), chains)
    say("workspace bytes", need)
    buf = workspace(need)
    scsf.scsf_set_workspace(h, buf)
    evals = torch.empty_like(ev0)
    evecs = torch.empty_like(vec0)
    scsf.scsf_solve_sequence(h, ops, order, chains, prm, evals, evecs)   # lanes, staging
    before = free_bytes()
    _, _, st = scsf.scsf_solve_sequence(h, ops, order, chains, prm, evals, evecs)
    after = free_bytes()
    assert after == before, (before, after)
    assert scsf.scsf_workspace_peak(h) <= need
    assert torch.equal(evals, ev0) and torch.equal(evecs, vec0)
    assert all(s["status"] == 0 for s in st)


def test_workspace_too_small_is_rejected_and_handle_recovers():
    say("workspace: too small")
    cfg = si.CONFIGS[1]
    op = scsf.DeviceOperator(si.operator(cfg, 0))
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1)
    need = scsf.scsf_workspace_bytes(prm, op.n)
    h = scsf.Handle()
    small = workspace(need // 2)
    scsf.scsf_set_workspace(h, small)
    with pytest.raises(scsf.ScsfError) as e:
        scsf.scsf_solve(h, op, prm)
    assert e.value.status == scsf.SCSF_ENOMEM
    scsf.scsf_set_workspace(h, None)                     # back to library-allocated buffers
    ev, _, _, _, st = scsf.scsf_solve(h, op, prm)
    assert st["status"] == 0


def test_phase_times_add_up_to_the_solve_time():
    """One operator of the mixed-precision workload's size (n = 25600, L = 200), FP64: the
    device times of the filter, orthonormalisation, Rayleigh-Ritz, residual and bound phases
    add up to the host wall time of the solve within 10%, and the handle's phase totals
    agree with the solve's."""
    say("phase times")
    cfg = si.CONFIGS[4]
    op = scsf.DeviceOperator(si.operator(cfg, 0))
    prm = scsf.make_params(cfg.L, cfg.k, cfg.degree, cfg.tol, seed=1)
    h = scsf.Handle()
    scsf.scsf_solve(h, op, prm)                          # warm: buffers, staging
    scsf.scsf_profile_read(h, reset=True)
    st = scsf.scsf_solve(h, op, prm)[4]
    prof = scsf.scsf_profile_read(h, reset=True)
    phases = [st[k] for k in ("ms_filter", "ms_orth", "ms_rr", "ms_resid", "ms_bound")]
    say(st["iterations"], "iterations; phases", phases, "wall", st["ms_wall"])
    assert all(p > 0 for p in phases)
    total = sum(phases)
    assert abs(total - st["ms_wall"]) <= 0.10 * st["ms_wall"], (total, st["ms_wall"])
    np.testing.assert_allclose([prof["phase_ms"][k] for k in scsf.PHASES], phases, rtol=1e-3)
