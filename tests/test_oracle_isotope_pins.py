"""Pins of the oracle's isotope scattering (Eq. isotope, Tamura):

* rotation invariance: rotating the Cartesian frame of every eigenvector
  (the crystal turned as a whole) leaves gamma_iso unchanged; the literal
  placement of the Cartesian sum outside |.|^2 does not, so this fixes the
  reading;
* completeness: summed over every partner (q', s') with the delta replaced by
  1, the overlaps give N_q sum_i g_i |eta_i(q,s)|^2 exactly;
* zone folding: a 3^3 mesh of the two-atom cell equals the Gamma point of its
  54-atom supercell (degenerate-cluster sums), which fixes the 1/N_q and the
  delta argument;
* brute force: explicit loops over q', s', i and a on a tiny mesh;
* limits: g = 0 gives 0, gamma_iso is linear in g, modes below nu_min get 0.
"""
import math

import numpy as np
import pytest

from oracle import isotope, phonons
from oracle.constants import TWO_PI
from synthetic import configs, models

B_FIXED = configs.Broadening(adaptive=False)
B_ADAPT = configs.Broadening(adaptive=True)
B_LORENTZ = configs.Broadening(shape=configs.LORENTZ, adaptive=False)


def clusters(nu, tol):
    order = np.argsort(nu, kind="stable")
    out, cur = [], [order[0]]
    for a, b in zip(order[:-1], order[1:]):
        if nu[b] - nu[a] < tol:
            cur.append(b)
        else:
            out.append(cur)
            cur = [b]
    out.append(cur)
    return out


@pytest.fixture(scope="module")
def random2():
    m = models.random_cell(11, 2)
    mesh = (3, 4, 5)
    return (m, mesh) + phonons.phonons(m, mesh)


def rotation(seed):
    rng = np.random.default_rng(seed)
    Q, R = np.linalg.qr(rng.normal(size=(3, 3)))
    return Q * np.sign(np.diag(R))


@pytest.mark.parametrize("b", [B_FIXED, B_ADAPT, B_LORENTZ], ids=["fixed", "adaptive", "lorentz"])
def test_rotation_invariance(random2, b):
    m, mesh, om, ev, ve = random2
    g = np.array([3.0e-4, 1.2e-4])
    ref = isotope.isotope_linewidths(m, mesh, om, ev, ve, g, b)
    R = rotation(1)
    nq, nb3, _ = ev.shape
    evr = np.einsum("ab,qibt->qiat", R, ev.reshape(nq, nb3 // 3, 3, nb3)).reshape(ev.shape)
    ver = ve @ R.T                                           # velocities turn with the frame
    rot = isotope.isotope_linewidths(m, mesh, om, evr, ver, g, b)
    assert ref.max() > 0
    np.testing.assert_allclose(rot, ref, rtol=1e-12, atol=1e-14 * ref.max())
    # the literal reading (Cartesian sum outside the modulus) is not invariant:
    # one partner's term changes under the same rotation
    q, s, q1, s1 = 1, 4, 7, 3
    e0, e1 = ev[q][:, s].reshape(2, 3), ev[q1][:, s1].reshape(2, 3)
    f0, f1 = evr[q][:, s].reshape(2, 3), evr[q1][:, s1].reshape(2, 3)
    lit = np.sum(g[:, None] * np.abs(np.conj(e0) * e1) ** 2)
    litr = np.sum(g[:, None] * np.abs(np.conj(f0) * f1) ** 2)
    tam = np.sum(g * np.abs(np.sum(np.conj(e0) * e1, axis=1)) ** 2)
    tamr = np.sum(g * np.abs(np.sum(np.conj(f0) * f1, axis=1)) ** 2)
    assert abs(tam - tamr) <= 1e-13 * abs(tam)
    assert abs(lit - litr) > 1e-3 * abs(lit)


def test_completeness_sum_rule(random2):
    m, mesh, om, ev, ve = random2
    nq, nb3, _ = ev.shape
    g = np.array([2.0e-4, 7.0e-5])
    for q, s in [(0, 3), (7, 0), (31, 5), (59, 2)]:
        O = isotope.overlaps(ev, q, s, g, 2)
        w = np.abs(ev[q][:, s].reshape(2, 3)) ** 2
        want = nq * np.sum(g * w.sum(axis=1))
        assert abs(O.sum() - want) <= 1e-12 * want


def test_zone_folding_crystal_vs_gamma_point():
    m = models.diamond()
    mesh = (3, 3, 3)
    om, ev, ve = phonons.phonons(m, mesh)
    g = np.array([2.0e-4, 5.0e-5])                          # the two sites differ
    gc = isotope.isotope_linewidths(m, mesh, om, ev, ve, g, B_FIXED)
    sc = models.supercell_gamma(m, mesh)
    oms, E = phonons.phonons_gamma_real(sc)
    g_sc = np.tile(g, 27)                                   # supercell atom = cell * N_b + basis
    gs = isotope.isotope_gamma_point(oms, E, g_sc, B_FIXED)
    nuc = om.reshape(-1) / TWO_PI
    order = np.argsort(nuc, kind="stable")
    nuc, gcf = nuc[order], gc.reshape(-1)[order]
    nus = oms / TWO_PI
    nuc = np.where(np.abs(nuc) < 0.05, 0.0, nuc)
    nus = np.where(np.abs(nus) < 0.05, 0.0, nus)
    assert np.allclose(nuc, nus, atol=1e-9)
    cl = clusters(nus, 1e-6)
    a = np.array([gcf[c].sum() for c in cl])
    b = np.array([gs[c].sum() for c in cl])
    assert a.max() > 0
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-12 * a.max())


def test_brute_force_loops():
    m = models.random_cell(3, 2)
    mesh = (2, 3, 2)
    om, ev, ve = phonons.phonons(m, mesh)
    g = np.array([1.5e-4, 4.0e-4])
    got = isotope.isotope_linewidths(m, mesh, om, ev, ve, g, B_FIXED)
    nq, nb3 = om.shape
    sig = TWO_PI * B_FIXED.sigma_thz
    for q in range(nq):
        for s in range(nb3):
            w = om[q, s]
            if w / TWO_PI < B_FIXED.nu_min_thz:
                assert got[q, s] == 0.0
                continue
            acc = 0.0
            for q1 in range(nq):
                for s1 in range(nb3):
                    w1 = om[q1, s1]
                    x = w - w1
                    if w1 / TWO_PI < B_FIXED.nu_min_thz or not abs(x) < 2 * sig:
                        continue
                    delta = math.exp(-(x * x) / (sig * sig)) / (math.sqrt(math.pi) * sig)
                    ov = 0.0
                    for i in range(2):
                        dot = 0j
                        for a in range(3):
                            dot += np.conj(ev[q, 3 * i + a, s]) * ev[q1, 3 * i + a, s1]
                        ov += g[i] * abs(dot) ** 2
                    acc += delta * ov
            want = math.pi / (2 * nq) * w * w * acc
            assert abs(got[q, s] - want) <= 1e-12 * max(abs(want), 1e-300)


def test_limits(random2):
    m, mesh, om, ev, ve = random2
    g1 = np.array([2.0e-4, 0.0])
    g2 = np.array([0.0, 3.0e-4])
    a = isotope.isotope_linewidths(m, mesh, om, ev, ve, g1, B_FIXED)
    b = isotope.isotope_linewidths(m, mesh, om, ev, ve, g2, B_FIXED)
    ab = isotope.isotope_linewidths(m, mesh, om, ev, ve, g1 + g2, B_FIXED)
    z = isotope.isotope_linewidths(m, mesh, om, ev, ve, np.zeros(2), B_FIXED)
    assert np.all(z == 0.0)
    np.testing.assert_allclose(ab, a + b, rtol=1e-13, atol=1e-16)
    low = om / TWO_PI < B_FIXED.nu_min_thz
    assert low.any() and np.all(ab[low] == 0.0) and np.all(ab[~low] >= 0.0)
