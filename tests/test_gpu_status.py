"""Device-side validation of the C ABI: the kernels check the device-resident
inputs they read and record problems in the handle's status word, which
kaldo_device_status() returns and clears (KALDO_EINVAL for non-finite inputs
or subset indices out of range, KALDO_ENUMERIC for an imaginary mode above
nu_min or a phonon eigen-solver stopped at its sweep cap).  Every case is a
bad input made on the host; every kernel still runs to its normal end."""
import numpy as np
import pytest

from oracle import phonons as oph
from synthetic import configs, models

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2602_23728_amd import kaldo as K  # noqa: E402

B_ADAPT = configs.Broadening(adaptive=True)
B_FIXED = configs.Broadening(adaptive=False)
MESH = (3, 3, 3)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def setup():
    m = models.diamond()
    c = K.Crystal.from_model(m)
    om, ev, ve = oph.phonons(m, MESH)
    return m, c, om, ev, ve


def status(c):
    try:
        c.device_status()
        return 0, ""
    except K.KaldoError as e:
        return e.status, str(e)


@pytest.mark.parametrize("prec", [K.FP64, K.FP32, K.BF16X3])
def test_clean_inputs_report_ok(setup, prec):
    m, c, om, ev, ve = setup
    assert status(c)[0] == 0
    g = K.linewidths(c, MESH, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT, prec)
    K.kappa_rta(c, MESH, dev(om), dev(ve), g, 300.0, 0.1)
    assert status(c) == (0, "")


def test_gpu_phonons_converge_and_report_ok():
    for name, mesh in (("diamond", (5, 5, 5)), ("perovskite", (4, 4, 4))):
        c = K.Crystal.from_model(configs.build_model(name))
        K.phonons(c, mesh)
        assert status(c) == (0, ""), name
        c.close()


def test_sweep_cap_reports_non_convergence(monkeypatch):
    c = K.Crystal.from_model(models.diamond())
    monkeypatch.setenv("KALDO_JACOBI_SWEEPS", "1")
    om, _, _ = K.phonons(c, (3, 3, 3))
    rc, msg = status(c)
    assert rc == -4 and "did not converge" in msg
    assert torch.isfinite(om).all()  # the kernel still ran to its end
    assert status(c)[0] == 0          # the query cleared the word
    c.close()


@pytest.mark.parametrize("what", ["omega", "evec", "vel"])
@pytest.mark.parametrize("prec", [K.FP64, K.FP32])
def test_non_finite_inputs_give_einval(setup, what, prec):
    m, c, om, ev, ve = setup
    om2, ev2, ve2 = om.copy(), ev.copy(), ve.copy()
    if what == "omega":
        om2[4, 3] = np.nan
    elif what == "evec":
        ev2[7, 2, 5] = complex(np.inf, 0.0)
    else:
        ve2[11, 4, 1] = np.nan
    K.linewidths(c, MESH, dev(om2), dev(ev2), dev(ve2), 300.0, B_ADAPT, prec)
    rc, msg = status(c)
    assert rc == -1 and "non-finite" in msg
    assert status(c)[0] == 0


def test_imaginary_mode_above_floor_gives_enumeric(setup):
    m, c, om, ev, ve = setup
    om2 = om.copy()
    om2[5, 4] = -2 * np.pi * 1.0        # nu = -1 THz, |nu| above nu_min = 0.1 THz
    g = K.linewidths(c, MESH, dev(om2), dev(ev), dev(ve), 300.0, B_ADAPT, K.FP32)
    rc, msg = status(c)
    assert rc == -4 and "imaginary" in msg
    assert torch.isfinite(g).all()
    # below the floor a negative frequency is the masked zero branch: no error
    om3 = om.copy()
    om3[0, 0] = -2 * np.pi * 0.01
    K.linewidths(c, MESH, dev(om3), dev(ev), dev(ve), 300.0, B_ADAPT, K.FP32)
    assert status(c)[0] == 0


def test_subset_index_out_of_range_gives_einval(setup):
    m, c, om, ev, ve = setup
    n = om.size
    sub = np.array([3, n + 5, 17, -2], np.int32)
    out = torch.full((27, 6), -7.0, dtype=torch.float64, device="cuda")
    K.linewidths(c, MESH, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT, K.FP64, subset=dev(sub), out=out)
    rc, msg = status(c)
    assert rc == -1 and "subset" in msg
    g = out.cpu().numpy().reshape(-1)
    full = K.linewidths(c, MESH, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT, K.FP64).cpu().numpy().reshape(-1)
    assert np.allclose(g[[3, 17]], full[[3, 17]], rtol=1e-13, atol=0)
    mask = np.ones(n, bool)
    mask[[3, 17]] = False
    assert np.all(g[mask] == -7.0)


def test_kappa_non_finite_gamma_gives_einval(setup):
    m, c, om, ev, ve = setup
    g = K.linewidths(c, MESH, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT, K.FP32)
    g[2, 3] = float("nan")
    K.kappa_rta(c, MESH, dev(om), dev(ve), g, 300.0, 0.1)
    rc, msg = status(c)
    assert rc == -1 and "non-finite" in msg


@pytest.mark.parametrize("prec", [K.FP64, K.FP32, K.BF16X3])
def test_gamma_point_validation(setup, prec):
    m = models.supercell_gamma(models.diamond(), (2, 2, 2))
    c = K.Crystal.from_model(m)
    om, E = oph.phonons_gamma_real(m)
    K.linewidths_gamma(c, dev(om), dev(E), 300.0, B_FIXED, prec)
    assert status(c)[0] == 0
    E2 = E.copy()
    E2[3, 20] = np.nan
    K.linewidths_gamma(c, dev(om), dev(E2), 300.0, B_FIXED, prec)
    rc, msg = status(c)
    assert rc == -1 and "non-finite" in msg
    om2 = om.copy()
    om2[-1] = -om2[-1]
    K.linewidths_gamma(c, dev(om2), dev(E), 300.0, B_FIXED, prec)
    assert status(c)[0] == -4
    c.close()
