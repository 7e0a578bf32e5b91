"""Pins of the oracle's full scattering matrix, self-consistent iteration and
direct inversion (Eq. BTE, Eq. gamma1, Eq. invBTE, Eq. sc_iter, Eq. inverse).

* the diagonal is the sum of the process rates, 2 Gamma of Eq. gamma;
* without the off-diagonal part the solution is the RTA (Eq. rta);
* the iteration of Eq. sc_iter converges to the inverse of Eq. inverse;
* detailed balance: D Gamma~ D^-1 (D = sqrt(n(n+1)) w) is symmetric when
  energy is conserved exactly, so its antisymmetric part shrinks in
  proportion to the energy mismatch over k_B T (the width of the smeared
  delta over the temperature), and its symmetric part is positive
  semi-definite; a wrong sign or a misplaced partner breaks both;
* a brute-force twin: explicit loops over every ordered triple of modes with
  the dense-supercell vertex and explicit -q lookups.
"""
import numpy as np
import pytest

from oracle import bruteforce, bte, kappa, linewidths, phonons
from oracle.constants import TWO_PI
from synthetic import configs, models

B_FIXED = configs.Broadening(adaptive=False)
B_ADAPT = configs.Broadening(adaptive=True)


def tr_consistent_phonons(model, mesh):
    """Oracle phonons with eta(-q) = eta(q)* and v(-q) = -v(q) (time-reversal
    partners share one solve)."""
    om, ev, ve = phonons.phonons(model, mesh)
    mq = bte.minus_index(mesh)
    for q in range(len(mq)):
        if mq[q] > q:
            om[mq[q]] = om[q]
            ev[mq[q]] = np.conj(ev[q])
            ve[mq[q]] = -ve[q]
    return om, ev, ve


@pytest.fixture(scope="module")
def random_case():
    m = models.random_cell(7, 2)
    mesh = (3, 3, 3)
    om, ev, ve = tr_consistent_phonons(m, mesh)
    return m, mesh, om, ev, ve


def test_diagonal_is_twice_the_linewidth(random_case):
    m, mesh, om, ev, ve = random_case
    g0, _ = bte.scattering_matrix(m, mesh, om, ev, ve, 300.0, B_ADAPT)
    G = linewidths.crystal_linewidths(m, mesh, om, ev, ve, 300.0, B_ADAPT)
    np.testing.assert_allclose(g0, 2.0 * G.reshape(-1), rtol=1e-12, atol=1e-15 * G.max())


def test_without_coupling_the_solution_is_the_rta(random_case):
    m, mesh, om, ev, ve = random_case
    nq = int(np.prod(mesh))
    g0, g1 = bte.scattering_matrix(m, mesh, om, ev, ve, 300.0, B_ADAPT)
    act = bte.active_modes(om, g0, 0.1)
    lam = bte.solve_inverse(g0, np.zeros_like(g1), ve, act)
    k = bte.kappa_from_lambda(om, ve, lam, 300.0, m.volume, nq, act)
    k_rta = kappa.kappa_rta(om, ve, g0.reshape(om.shape) / 2.0, 300.0, m.volume, nq, 0.1)
    np.testing.assert_allclose(k, k_rta, rtol=1e-12, atol=1e-14 * np.abs(k_rta).max())


def test_self_consistent_iteration_converges_to_the_inverse():
    """Eq. sc_iter from the RTA start reaches the solution of Eq. inverse (on a
    cell where the iteration contracts; the paper notes it converges when the
    off-diagonal part is smaller than the diagonal)."""
    m = models.random_cell(11, 2)
    mesh = (3, 4, 5)
    om, ev, ve = phonons.phonons(m, mesh)
    nq = int(np.prod(mesh))
    g0, g1 = bte.scattering_matrix(m, mesh, om, ev, ve, 300.0, B_ADAPT)
    act = bte.active_modes(om, g0, 0.1)
    lam_i = bte.solve_inverse(g0, g1, ve, act)
    lam_s, k_s, it = bte.solve_sc(g0, g1, ve, act, om, 300.0, m.volume, nq, 500, 1e-12)
    assert it < 500
    k_i = bte.kappa_from_lambda(om, ve, lam_i, 300.0, m.volume, nq, act)
    np.testing.assert_allclose(k_s, k_i, rtol=1e-10, atol=1e-12 * np.abs(k_i).max())
    # the solution is odd under time reversal (v is); the iteration's even
    # part is rounding that the even directions amplify, and kappa cannot see
    # it (c is even, v odd), so compare the odd parts of lambda
    tr = bte.time_reversal_partner(mesh, ev)
    odd = lambda x: 0.5 * (x - x[tr])  # noqa: E731
    np.testing.assert_allclose(odd(lam_i), lam_i, rtol=1e-8, atol=1e-10 * np.abs(lam_i).max())
    np.testing.assert_allclose(odd(lam_s), lam_i, rtol=1e-7, atol=1e-9 * np.abs(lam_i).max())
    # the coupling matters: the full solution differs from the RTA
    k_rta = kappa.kappa_rta(om, ve, g0.reshape(om.shape) / 2.0, 300.0, m.volume, nq, 0.1)
    assert abs(np.trace(k_i) - np.trace(k_rta)) > 1e-2 * abs(np.trace(k_rta))


def symmetric_form(g0, g1, om, act, T):
    w = om.reshape(-1)
    n = linewidths.bose(np.where(act, w, 1.0), T)
    D = np.sqrt(n * (n + 1.0)) * w
    idx = np.flatnonzero(act)
    A = g1[np.ix_(idx, idx)] + np.diag(g0[idx])
    return D[idx][:, None] * A / D[idx][None, :]


def test_detailed_balance_symmetry_and_definiteness():
    """Off the energy shell (|x| < 2 sigma) the population factors of the two
    ends of a process differ by a relative O(x/w) (and O(x/k_B T)): halving
    sigma halves the antisymmetric part of D Gamma~ D^-1, whose symmetric
    part stays positive semi-definite (up to that level)."""
    m = models.random_cell(7, 2)
    mesh = (4, 4, 4)
    om, ev, ve = tr_consistent_phonons(m, mesh)
    asym = []
    for sig in (0.4, 0.2, 0.1):
        b = configs.Broadening(adaptive=False, sigma_thz=sig)
        g0, g1 = bte.scattering_matrix(m, mesh, om, ev, ve, 300.0, b)
        act = bte.active_modes(om, g0, 0.1)
        S = symmetric_form(g0, g1, om, act, 300.0)
        H = 0.5 * (S + S.T)
        a = np.linalg.norm(S - S.T) / np.linalg.norm(S + S.T)
        e = np.linalg.eigvalsh(H)
        assert e.min() > -0.1 * a * e.max()
        asym.append(a)
    assert asym[0] < 0.01
    assert 1.4 < asym[0] / asym[1] < 2.6 and 1.4 < asym[1] / asym[2] < 2.6


def test_time_reversal_partner_map():
    """tr(q, s) sits at -q; applied twice it is the identity; for a solver's
    eigenvectors it pairs equal frequencies and opposite velocities."""
    m = models.diamond()
    mesh = (4, 4, 4)
    om, ev, ve = phonons.phonons(m, mesh)
    tr = bte.time_reversal_partner(mesh, ev)
    nb3 = om.shape[1]
    mq = bte.minus_index(mesh)
    assert np.array_equal(tr // nb3, np.repeat(mq, nb3))
    np.testing.assert_allclose(om.reshape(-1)[tr], om.reshape(-1), rtol=0, atol=1e-5)
    nu = om.reshape(-1) / TWO_PI
    iso = np.ones(om.size, bool)
    for q in range(om.shape[0]):
        for s in range(nb3):
            near = np.abs(nu[q * nb3:(q + 1) * nb3] - nu[q * nb3 + s]) < 1e-3
            iso[q * nb3 + s] = near.sum() == 1
    assert iso.sum() > 50
    assert np.array_equal(tr[tr[iso]], np.flatnonzero(iso))
    np.testing.assert_allclose(ve.reshape(-1, 3)[tr[iso]], -ve.reshape(-1, 3)[iso], atol=1e-8)


def test_scattering_matrix_matches_bruteforce_triples():
    m = models.random_cell(3, 2)
    mesh = (2, 2, 2)
    om, ev, ve = tr_consistent_phonons(m, mesh)
    T, b = 300.0, configs.Broadening(adaptive=False, sigma_thz=0.5)
    g0, g1 = bte.scattering_matrix(m, mesh, om, ev, ve, T, b)
    Vb = bruteforce.vertex_bruteforce(m, mesh, ev)  # [q, q1, s, s', s'']
    pts = phonons.mesh_points(mesh)
    N = np.asarray(mesh)

    def flat(c):
        c = np.mod(c, N)
        return (c[0] * N[1] + c[1]) * N[2] + c[2]

    nq, nb3 = om.shape
    nu = om / TWO_PI
    occ = np.where(nu >= 0.1, linewidths.bose(np.where(nu >= 0.1, om, 1.0), T), 0.0)
    sig = TWO_PI * 0.5
    pref = 2.0 * linewidths.PREFACTOR / nq
    G0 = np.zeros(nq * nb3)
    G1 = np.zeros((nq * nb3, nq * nb3))
    for q in range(nq):
        for q1 in range(nq):
            q2 = flat(-pts[q] - pts[q1])
            mq1, mq2 = flat(-pts[q1]), flat(-pts[q2])
            for s in range(nb3):
                for a in range(nb3):
                    for c in range(nb3):
                        if nu[q, s] < 0.1 or nu[q1, a] < 0.1 or nu[q2, c] < 0.1:
                            continue
                        w, w1, w2 = om[q, s], om[q1, a], om[q2, c]
                        base = pref * abs(Vb[q, q1, s, a, c]) ** 2 / (w * w1 * w2)
                        dp = base * (occ[q1, a] - occ[q2, c]) * float(
                            linewidths.smearing(w + w1 - w2, sig, 0))
                        dm = base * 0.5 * (occ[q1, a] + occ[q2, c] + 1) * float(
                            linewidths.smearing(w - w1 - w2, sig, 0))
                        row = q * nb3 + s
                        G0[row] += dp + dm
                        G1[row, q1 * nb3 + a] += dp * w1 / w
                        G1[row, mq1 * nb3 + a] -= dm * w1 / w
                        G1[row, mq2 * nb3 + c] -= (dp + dm) * w2 / w
    scale = np.abs(G1).max()
    assert scale > 0
    np.testing.assert_allclose(g0, G0, rtol=1e-10, atol=1e-13 * G0.max())
    np.testing.assert_allclose(g1, G1, rtol=1e-9, atol=1e-12 * scale)
