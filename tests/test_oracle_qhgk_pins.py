"""Pins of the oracle's QHGK conductivity (Eq. qhgk, Eq. qhgk_crystal):

* the diagonal of the generalised velocity matrix is the group velocity of
  Eq. groupvel (computed by the phonon code with its own derivative), and the
  matrix is Hermitian;
* the generalised heat capacity tends to c_mu of Eq. heatcap as the two
  frequencies meet (the reading of its prefactor), and the generalised
  lifetime's diagonal is 1/(2 Gamma);
* zone folding: a crystal's whole QHGK sum on an n^3 mesh (every pair of each
  q) equals Eq. qhgk for the Gamma point of its n^3 supercell, built from
  independent code (dense dynamical matrix, minimum-image separations, real
  eigenvectors); this fixes the velocity operator (with the basis offsets:
  without them the equality fails), its normalisation and 1/V;
* cubic isotropy of the whole sum on a cubic mesh, whose diagonal part is
  the RTA conductivity of Eq. rta.
"""
import numpy as np
import pytest

from oracle import kappa, phonons, qhgk
from oracle.constants import HBAR, KB, TWO_PI, U
from synthetic import models


@pytest.mark.parametrize("which", ["diamond", "random3"])
def test_velocity_matrix_diagonal_and_hermitian(which):
    m = models.diamond() if which == "diamond" else models.random_cell(7, 3)
    mesh = (3, 4, 3)
    om, ev, ve = phonons.phonons(m, mesh)
    pts = phonons.mesh_points(mesh)
    vmax = np.abs(ve).max()
    for q in [1, 7, 20, 33]:
        V = qhgk.velocity_matrix_crystal(m, pts[q] / np.array(mesh), om[q], ev[q])
        ok = om[q] / TWO_PI > 1e-3
        for a in range(3):
            np.testing.assert_allclose(V[a], V[a].conj().T, atol=1e-12 * vmax)
            d = np.diag(V[a])[ok]
            np.testing.assert_allclose(d.real, ve[q][ok, a], atol=1e-9 * vmax)
            assert np.abs(d.imag).max() <= 1e-12 * vmax


def test_heat_capacity_matrix_limit_and_lifetime_diagonal():
    T = 300.0
    w = np.array([5.0, 5.0 + 1e-3, 30.0, 60.0])              # rad/ps; the first two just apart
    c = qhgk.heat_capacity_matrix(w, T)
    cm = kappa.heat_capacity_kb(w, T)
    np.testing.assert_allclose(np.diag(c), cm, rtol=1e-14)
    # the limit: c(w, w + d) = c(w + d/2) + O(d^2)
    assert abs(c[0, 1] - kappa.heat_capacity_kb(np.array([5.0005]), T)[0]) < 1e-7 * cm[0]
    assert np.allclose(c, c.T, rtol=1e-14) and np.all(c > 0)
    # an explicit pair, from Eq. bose
    n = 1.0 / np.expm1(HBAR * w / (KB * T))
    want = HBAR / (KB * T) * w[2] * w[3] * (n[2] - n[3]) / (w[3] - w[2])
    assert abs(c[2, 3] - want) <= 1e-14 * want
    g = np.array([0.1, 0.2, 0.05, 0.3])
    tau = qhgk.lifetime_matrix(w, g)
    np.testing.assert_allclose(np.diag(tau), 1.0 / (2.0 * g), rtol=1e-15)
    assert np.allclose(tau, tau.T)


def _fold(model, mesh, gamma_const, T):
    om, ev, ve = phonons.phonons(model, mesh)
    G = np.full(om.shape, gamma_const)
    kc = qhgk.kappa_qhgk_crystal(model, mesh, om, ev, G, T, 0.1, interband_only=False)
    sc = models.supercell_gamma(model, mesh)
    oms, E = phonons.phonons_gamma_real(sc)
    ks, _ = qhgk.kappa_qhgk_gamma(sc, oms, E, np.full(oms.shape, gamma_const), T, 0.1)
    return kc, ks, (om, ev, ve)


@pytest.mark.parametrize("which", ["diamond", "perovskite"])
def test_zone_folding_crystal_vs_supercell(which):
    m = models.diamond() if which == "diamond" else models.perovskite(0)
    kc, ks, _ = _fold(m, (3, 3, 3), 0.3, 300.0)
    kbar = np.trace(kc) / 3
    assert kbar > 0
    assert np.max(np.abs(kc - ks)) <= 1e-9 * kbar


def test_zone_folding_needs_the_basis_offsets(monkeypatch):
    """With the derivative of the lattice-vector Bloch sum alone (no basis
    offsets) the interband matrix elements change and the crystal sum no
    longer equals the supercell's."""
    m = models.perovskite(0)
    mesh = (3, 3, 3)
    kc, ks, _ = _fold(m, mesh, 0.3, 300.0)
    kbar = np.trace(kc) / 3
    monkeypatch.setattr(qhgk, "separation_dq", lambda model, qf: phonons.dynamical_matrix_dq(model, qf))
    kw, _, _ = _fold(m, mesh, 0.3, 300.0)
    assert np.max(np.abs(kw - ks)) > 1e-4 * kbar
    assert np.max(np.abs(kc - ks)) <= 1e-9 * kbar


def test_cubic_isotropy_of_the_whole_sum():
    """With widths that depend on the frequency alone, the whole sum (intra-
    and interband) of a cubic crystal on a cubic mesh is isotropic.  (The
    interband part alone is not: inside a degenerate multiplet the split
    between the diagonal and the off-diagonal elements follows the eigenvector
    gauge, which is not point-symmetric; the sum over the multiplet is.)"""
    m = models.perovskite(0)
    mesh = (3, 3, 3)
    om, ev, ve = phonons.phonons(m, mesh)
    G = 0.02 + 0.01 * (om / om.max()) ** 2                   # a smooth mode-dependent width
    k = qhgk.kappa_qhgk_crystal(m, mesh, om, ev, G, 300.0, 0.1, interband_only=False)
    kbar = np.trace(k) / 3
    assert kbar > 0
    assert np.max(np.abs(k - kbar * np.eye(3))) <= 1e-9 * kbar
    # and the RTA part of that sum is the RTA conductivity of Eq. rta
    kr = kappa.kappa_rta(om, ve, G, 300.0, m.volume, 27, 0.1)
    ki = qhgk.kappa_qhgk_crystal(m, mesh, om, ev, G, 300.0, 0.1, interband_only=True)
    np.testing.assert_allclose(kr + ki, k, rtol=1e-10, atol=1e-12 * kbar)
