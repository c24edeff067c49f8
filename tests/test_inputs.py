"""The synthetic workload recipe (no GPU): seeds, shapes, value ranges and determinism of every
configuration and operator family."""
import numpy as np
import pytest

import scsf_inputs as si


def test_seed_rule():
    assert si.op_seed(2, 7) == 1_000_003 * 2 + 7
    # the operators of different configurations never share a seed (fewer than 10^6 each)
    assert si.op_seed(3, 999) < si.op_seed(4, 0)


@pytest.mark.parametrize("idx", sorted(si.CONFIGS))
def test_configurations_are_deterministic_and_well_formed(idx):
    cfg = si.CONFIGS[idx]
    a, b = si.operator(cfg, 3), si.operator(cfg, 3)
    for name in ("wx", "wy", "v", "cell", "D", "rho", "field"):
        x, y = getattr(a, name, None), getattr(b, name, None)
        if x is None:
            assert y is None
            continue
        np.testing.assert_array_equal(x, y)
        assert np.all(np.isfinite(x))
    assert 0 < cfg.L < cfg.k or cfg.family == "mixed"
    assert 1 <= cfg.degree <= 64 and cfg.p0 >= 1 and cfg.tol > 0
    if cfg.family != "mixed":
        assert a.N == cfg.sides[0]
    assert a.field.ndim == 3 and a.field.shape[1:] == (a.N, a.N)


def test_family_value_ranges():
    p = si.potential_operator(30, 8, 1)
    assert p.v.min() == pytest.approx(0.0) and p.v.max() == pytest.approx(100.0)
    d = si.divk_operator(30, 8, 1)
    assert np.all(d.wx > 0) and np.all(d.wy > 0) and d.v is None
    a = si.aniso_operator(20, 8, 1)
    k11, k12, k22 = a.cell[..., 0], a.cell[..., 1], a.cell[..., 2]
    assert np.all(k11 > 0) and np.all(k11 * k22 - k12 ** 2 > 0)        # SPD tensors
    h = si.helmholtz_operator(20, 8, 1)
    assert np.all(h.v < 0) and h.field.shape == (2, 20, 20)
    pl = si.plate_operator(20, 8, 1)
    assert np.all(pl.D > 0) and np.all(pl.rho > 0) and pl.field.shape == (2, 20, 20)


def test_uneven_configuration_draws():
    cfg = si.CONFIGS[3]
    sides = [si.operator(cfg, i).N for i in range(60)]
    Ls = [si.mixed_L(cfg, i) for i in range(60)]
    assert min(sides) >= 48 and max(sides) <= 128
    assert set(Ls) <= {32, 64, 128} and len(set(Ls)) == 3
    fams = [si.operator(cfg, i).family for i in range(6)]
    assert fams == ["divk", "potential"] * 3
