"""GPU full BTE (Eq. BTE, Eq. gamma1, Eq. sc_iter, Eq. inverse) against the
FP64 oracle on the same phonons: the scattering matrix element by element,
the direct inversion and the self-consistent iteration; the diamond 15^3
mesh against the oracle's stored rows and conductivity."""
import os

import numpy as np
import pytest

from oracle import bte as obte
from oracle import phonons as oph
from synthetic import configs, models

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2602_23728_amd import kaldo as K  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
B_ADAPT = configs.Broadening(adaptive=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_matrix(m, mesh, om, ev, ve, b):
    g0, g1 = obte.scattering_matrix(m, mesh, om, ev, ve, 300.0, b)
    A = g1 + np.diag(g0)
    act = obte.active_modes(om, g0, b.nu_min_thz)
    A[~act, :] = 0.0
    A[:, ~act] = 0.0
    A[np.flatnonzero(~act), np.flatnonzero(~act)] = 1.0
    return g0, g1, A, act


CASES = {
    "diamond": (lambda: models.diamond(), (4, 4, 4)),
    "random": (lambda: models.random_cell(11, 2), (3, 4, 5)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_scattering_matrix_matches_oracle(name):
    mk, mesh = CASES[name]
    m = mk()
    c = K.Crystal.from_model(m)
    om, ev, ve = oph.phonons(m, mesh)
    mat, g0 = K.scattering_matrix(c, mesh, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT)
    mat, g0 = host(mat), host(g0)
    c.device_status()
    og0, _, A, _ = oracle_matrix(m, mesh, om, ev, ve, B_ADAPT)
    np.testing.assert_allclose(g0, og0, rtol=1e-10, atol=1e-12 * og0.max())
    scale = np.abs(A).max()
    assert np.max(np.abs(mat - A)) <= 1e-10 * scale
    # bitwise reproducible
    mat2, _ = K.scattering_matrix(c, mesh, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT)
    assert np.array_equal(host(mat2), mat)
    c.close()


@pytest.mark.parametrize("name", list(CASES))
def test_direct_inversion_matches_oracle(name):
    mk, mesh = CASES[name]
    m = mk()
    nq = int(np.prod(mesh))
    c = K.Crystal.from_model(m)
    om, ev, ve = oph.phonons(m, mesh)
    mat, g0 = K.scattering_matrix(c, mesh, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT)
    lam, kap = K.bte_solve(c, mesh, dev(om), dev(ve), g0, 300.0, 0.1, mat)
    lam, kap = host(lam), host(kap)
    c.device_status()
    og0, og1, _, act = oracle_matrix(m, mesh, om, ev, ve, B_ADAPT)
    olam = obte.solve_inverse(og0, og1, ve, act)
    ok = obte.kappa_from_lambda(om, ve, olam, 300.0, m.volume, nq, act)
    kbar = np.trace(ok) / 3
    print(f"{name}: kappa_inv GPU {np.trace(kap) / 3:.10g} oracle {kbar:.10g}")
    assert np.max(np.abs(kap - ok)) <= 1e-8 * abs(kbar)
    assert np.max(np.abs(lam - olam)) <= 1e-8 * np.abs(olam).max()
    c.close()


@pytest.mark.parametrize("name", list(CASES))
def test_direct_inversion_with_a_raised_floor(name):
    """The solve leaves out every mode below its own nu_min: with the floor
    at the 40th percentile of the frequencies a scattered subset of modes
    drops out of the factorisation, whose solution must still be the
    oracle's on the remaining modes (and zero on the others)."""
    mk, mesh = CASES[name]
    m = mk()
    nq = int(np.prod(mesh))
    c = K.Crystal.from_model(m)
    om, ev, ve = oph.phonons(m, mesh)
    mat, g0 = K.scattering_matrix(c, mesh, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT)
    nu = om.ravel() / (2 * np.pi)
    floor = float(np.percentile(nu[nu > 0], 40))
    lam, kap = K.bte_solve(c, mesh, dev(om), dev(ve), g0, 300.0, floor, mat)
    lam, kap = host(lam), host(kap)
    c.device_status()
    og0, og1, _, _ = oracle_matrix(m, mesh, om, ev, ve, B_ADAPT)
    act = obte.active_modes(om, og0, floor)
    assert 0 < act.sum() < act.size
    olam = obte.solve_inverse(og0, og1, ve, act)
    ok = obte.kappa_from_lambda(om, ve, olam, 300.0, m.volume, nq, act)
    assert np.all(lam.reshape(-1, 3)[~act.ravel()] == 0.0)
    assert np.max(np.abs(lam - olam)) <= 1e-8 * np.abs(olam).max()
    assert np.max(np.abs(kap - ok)) <= 1e-8 * abs(np.trace(ok) / 3)
    c.close()


def test_direct_inversion_with_every_mode_decoupled():
    """A floor above every frequency leaves nothing to factorise: lambda and
    kappa are zero and the matrix is not touched."""
    mk, mesh = CASES["diamond"]
    m = mk()
    c = K.Crystal.from_model(m)
    om, ev, ve = oph.phonons(m, mesh)
    mat, g0 = K.scattering_matrix(c, mesh, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT)
    before = host(mat).copy()
    lam, kap = K.bte_solve(c, mesh, dev(om), dev(ve), g0, 300.0, 1e6, mat)
    lam, kap = host(lam), host(kap)
    c.device_status()
    assert np.all(lam == 0.0) and np.all(kap == 0.0)
    assert np.array_equal(host(mat), before)
    c.close()


def test_self_consistent_iteration_matches_oracle():
    mk, mesh = CASES["random"]
    m = mk()
    nq = int(np.prod(mesh))
    c = K.Crystal.from_model(m)
    om, ev, ve = oph.phonons(m, mesh)
    mat, g0 = K.scattering_matrix(c, mesh, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT)
    lam, kap, it, rc = K.bte_iterate(c, mesh, dev(om), dev(ve), g0, 300.0, 0.1, mat, 500, 1e-12)
    kap = host(kap)
    og0, og1, _, act = oracle_matrix(m, mesh, om, ev, ve, B_ADAPT)
    _, ok, oit = obte.solve_sc(og0, og1, ve, act, om, 300.0, m.volume, nq, 500, 1e-12)
    olam_i = obte.solve_inverse(og0, og1, ve, act)
    ok_i = obte.kappa_from_lambda(om, ve, olam_i, 300.0, m.volume, nq, act)
    print(f"SC: GPU {it} iterations, oracle {oit}; kappa {np.trace(kap) / 3:.10g} "
          f"oracle {np.trace(ok) / 3:.10g} inverse {np.trace(ok_i) / 3:.10g}")
    assert rc == 0 and abs(it - oit) <= 1
    assert np.max(np.abs(kap - ok)) <= 1e-9 * abs(np.trace(ok) / 3)
    assert np.max(np.abs(kap - ok_i)) <= 1e-9 * abs(np.trace(ok_i) / 3)
    c.close()


def test_iteration_reports_non_convergence():
    """On the diamond model the iteration does not contract (coalescence of
    two acoustic phonons into the flat optical band makes the off-diagonal
    part as large as twice the diagonal in some directions): status ENUMERIC,
    while the inversion still solves it."""
    m = models.diamond()
    mesh = (4, 4, 4)
    c = K.Crystal.from_model(m)
    om, ev, ve = oph.phonons(m, mesh)
    mat, g0 = K.scattering_matrix(c, mesh, dev(om), dev(ev), dev(ve), 300.0, B_ADAPT)
    _, _, it, rc = K.bte_iterate(c, mesh, dev(om), dev(ve), g0, 300.0, 0.1, mat, 150, 1e-12,
                                 check=False)
    assert rc == -4 and it == 150
    c.close()


def test_c2_scattering_matrix_and_inverse_golden():
    path = os.path.join(GOLDEN, "c2_bte_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("golden file missing: run tests/golden/make_bte_golden.py")
    gb = np.load(path)
    g = np.load(os.path.join(GOLDEN, "c2_oracle.npz"))
    cfg = configs.CONFIGS["C2"]
    m = configs.model_for(cfg)
    c = K.Crystal.from_model(m)
    mat, g0 = K.scattering_matrix(c, cfg.mesh, dev(g["omega"]), dev(g["evec"]), dev(g["vel"]),
                                  300.0, cfg.broadening)
    torch.cuda.synchronize()
    g0h = host(g0)
    np.testing.assert_allclose(g0h, gb["gamma0"], rtol=1e-10, atol=1e-12 * gb["gamma0"].max())
    nb3 = 6
    rows = np.concatenate([host(mat[q * nb3:(q + 1) * nb3]) for q in gb["rows_q"]])
    ref = gb["rows_val"] + 0.0
    act = obte.active_modes(g["omega"], gb["gamma0"], 0.1)
    ridx = np.concatenate([np.arange(q * nb3, (q + 1) * nb3) for q in gb["rows_q"]])
    for k, i in enumerate(ridx):
        ref[k, i] += gb["gamma0"][i]
    ref[:, ~act] = 0.0
    for k, i in enumerate(ridx):
        if not act[i]:
            ref[k, :] = 0.0
            ref[k, i] = 1.0
    assert np.max(np.abs(rows - ref)) <= 1e-10 * np.abs(ref).max()
    lam, kap = K.bte_solve(c, cfg.mesh, dev(g["omega"]), dev(g["vel"]), g0, 300.0, 0.1, mat)
    kap = host(kap)
    c.device_status()
    kbar = np.trace(gb["kappa_inv"]) / 3
    print(f"C2 kappa_inv GPU {np.trace(kap) / 3:.10g} oracle {kbar:.10g}")
    assert np.max(np.abs(kap - gb["kappa_inv"])) <= 1e-8 * abs(kbar)
    del mat
    c.close()
