"""The allocation-free entry point kaldo_linewidths_noalloc against
kaldo_linewidths (same kernels on the library's device scratch array instead
of a caller workspace): bitwise the same linewidths, on two calls in a row
with the second on a smaller input (so the scratch array still holds the
first call's data), and a request larger than the array is refused."""
import numpy as np
import pytest

from oracle import phonons as oph
from synthetic import configs, models

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2602_23728_amd import kaldo as K  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def both(c, mesh, om, ev, ve, b, prec, subset=None):
    ref = K.linewidths(c, mesh, om, ev, ve, 300.0, b, prec, subset=subset)
    out = torch.full_like(ref, -7.0)
    K.linewidths_noalloc(c, mesh, om, ev, ve, 300.0, b, prec, subset=subset, out=out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("prec", [K.FP64, K.FP32])
def test_noalloc_matches_workspace_entry_point(prec):
    c = K.Crystal.from_model(models.diamond())
    b = configs.Broadening(adaptive=True)
    max_bytes = int(K.lib().kaldo_linewidths_noalloc_max_bytes())
    # first call: the 24^3 mesh (82,944 modes), the largest configuration
    big = (24, 24, 24)
    assert K.linewidths_workspace(c, big, prec) <= max_bytes
    om, ev, ve = K.phonons(c, big)
    ref, got = both(c, big, om, ev, ve, b, prec)
    assert np.array_equal(ref, got)
    # second call, smaller: a 5^3 mesh with oracle phonons, then a subset of it
    small = (5, 5, 5)
    o2, e2, v2 = (dev(x) for x in oph.phonons(models.diamond(), small))
    ref, got = both(c, small, o2, e2, v2, b, prec)
    assert np.array_equal(ref, got)
    sub = dev(np.arange(3, 750, 11, dtype=np.int32))
    ref, got = both(c, small, o2, e2, v2, b, prec, subset=sub)
    mask = np.zeros(750, bool)
    mask[np.arange(3, 750, 11)] = True
    assert np.array_equal(ref.reshape(-1)[mask], got.reshape(-1)[mask])
    assert np.all(got.reshape(-1)[~mask] == -7.0)
    c.device_status()
    c.close()


def test_noalloc_refuses_requests_beyond_the_scratch_array():
    c = K.Crystal.from_model(models.diamond())
    mesh = (40, 40, 40)  # FP64 workspace about 60 MB
    need = K.linewidths_workspace(c, mesh, K.FP64)
    assert need > int(K.lib().kaldo_linewidths_noalloc_max_bytes())
    om = torch.zeros(64000, 6, dtype=torch.float64, device="cuda")
    ev = torch.zeros(64000, 6, 6, 2, dtype=torch.float64, device="cuda")
    ve = torch.zeros(64000, 6, 3, dtype=torch.float64, device="cuda")
    out = torch.zeros(64000, 6, dtype=torch.float64, device="cuda")
    with pytest.raises(K.KaldoError) as e:
        K.linewidths_noalloc(c, mesh, om, ev, ve, 300.0, configs.Broadening(), K.FP64, out=out)
    assert e.value.status == -1 and "scratch" in str(e.value)
    c.close()
