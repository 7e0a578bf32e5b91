"""The irreducible wedge on the GPU (restriction of the scattering calculation
to the irreducible Brillouin zone, results mapped back onto the full grid):
linewidths of the representatives' modes only, star-mapped, against the
full mesh, on the diamond 15^3 and perovskite 12^3 meshes.

* fixed width: equal to the full mesh after averaging degenerate clusters
  (the point group maps every term of Eq. gamma at q onto one at Rq);
* adaptive width (the configurations' own smearing): the widths of partners
  inside a degenerate multiplet follow the eigenvector gauge, which is not
  point-symmetric, so the wedge differs from the full mesh by that gauge
  freedom alone; checked on the conductivity against the oracle's stored
  full-mesh result.
"""
import os

import numpy as np
import pytest

from synthetic import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2602_23728_amd import kaldo as K  # noqa: E402
from paper_2602_23728_amd import learned as L  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
B_FIXED = configs.Broadening(adaptive=False)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def kappa_rel(k, ref):
    kb = np.trace(ref) / 3
    return max(abs(np.trace(k) / 3 - kb) / abs(kb), np.max(np.abs(k - ref)) / abs(kb))


# (config, precision, tolerance on cluster-averaged Gamma above 1e-3 max)
CASES = {"C2": (K.FP64, 1e-10), "C3": (K.FP32, 2e-5)}


@pytest.mark.parametrize("name", list(CASES))
def test_wedge_equals_full_mesh_fixed_width(name):
    prec, tol = CASES[name]
    cfg = configs.CONFIGS[name]
    m = configs.model_for(cfg)
    c = K.Crystal.from_model(m)
    mesh = cfg.mesh
    nq = int(np.prod(mesh))
    om, ev, ve = K.phonons(c, mesh)
    w = L.Wedge(m.lattice, m.frac, m.mass, mesh)
    full = K.linewidths(c, mesh, om, ev, ve, 300.0, B_FIXED, prec)
    wedge = L.plain_ibz_linewidths(c, w, om, ev, ve, 300.0, B_FIXED, prec)
    own = host(K.star_map(mesh, c.nb3, torch.arange(nq, dtype=torch.int32, device="cuda"), om,
                          full))
    got = host(wedge)
    c.device_status()
    big = own > 1e-3 * own.max()
    err = np.max(np.abs(got[big] - own[big]) / own[big])
    print(f"{name}: {w.n_ir} of {nq} q-points; wedge vs full (fixed width) max rel {err:.2e}")
    assert err <= tol
    assert np.max(np.abs(got - own)) <= tol * own.max()
    c.close()


@pytest.mark.parametrize("name", list(CASES))
def test_wedge_adaptive_against_stored_oracle(name):
    prec, _ = CASES[name]
    path = os.path.join(GOLDEN, f"{name.lower()}_oracle.npz")
    if not os.path.exists(path):
        pytest.skip(f"golden file missing: run tests/golden/make_golden.py {name}")
    g = np.load(path)
    cfg = configs.CONFIGS[name]
    m = configs.model_for(cfg)
    c = K.Crystal.from_model(m)
    mesh = cfg.mesh
    om, ev, ve = dev(g["omega"]), dev(g["evec"]), dev(g["vel"])
    w = L.Wedge(m.lattice, m.frac, m.mass, mesh)
    gam = L.plain_ibz_linewidths(c, w, om, ev, ve, 300.0, cfg.broadening, prec)
    kap = host(K.kappa_rta(c, mesh, om, ve, gam, 300.0, cfg.broadening.nu_min_thz))
    c.device_status()
    err = kappa_rel(kap, g["kappa"])
    print(f"{name}: wedge (adaptive width) kappa {np.trace(kap) / 3:.6g} vs full-mesh oracle "
          f"{np.trace(g['kappa']) / 3:.6g}: rel {err:.2e}")
    assert err <= 5e-3
    c.close()
