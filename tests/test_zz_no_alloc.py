"""scsf_bounds_noalloc (the bounds step with its scratch in the library's fixed device array,
for callers that cannot allocate) against scsf_bounds, through the C-ABI library: two calls in
a row, the second on a smaller operator, equal to the allocating entry point's outputs, with
device free memory unchanged.  Needs an MI355X."""
import pytest

import scsf_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2510_23215_amd import scsf  # noqa: E402


def test_noalloc_bounds_match_twice_then_smaller():
    h = scsf.Handle()
    big = scsf.DeviceOperator(si.operator(si.CONFIGS[5], 7))          # 9-point, n = 16384
    small = scsf.DeviceOperator(si.divk_operator(37, 8, 5))            # 5-point, n = 1369
    ref_big = scsf.scsf_bounds(h, big, 20, 11)
    ref_small = scsf.scsf_bounds(h, small, 20, 11)
    scsf.scsf_bounds_noalloc(h, big, 20, 11)                           # first use on the device
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info()[0]
    got_big = scsf.scsf_bounds_noalloc(h, big, 20, 11)
    got_small = scsf.scsf_bounds_noalloc(h, small, 20, 11)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == before
    assert got_big == ref_big
    assert got_small == ref_small


def test_noalloc_bounds_rejects_operators_beyond_its_scratch():
    h = scsf.Handle()
    op = scsf.DeviceOperator(si.divk_operator(520, 4, 1))              # n = 270400 > 2^18
    with pytest.raises(scsf.ScsfError) as e:
        scsf.scsf_bounds_noalloc(h, op, 20, 1)
    assert e.value.status == scsf.SCSF_EINVAL
