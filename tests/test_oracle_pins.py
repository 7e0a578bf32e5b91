"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test ties some part of the oracle to something other than itself: the
analytic nearest-neighbour diamond dispersion, finite differences, sum rules,
symmetries of the vertex and of the rates, zone folding between the crystal
and Gamma-point paths, and a brute-force dense-tensor vertex.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special

from oracle import bruteforce, kappa, linewidths, phonons
from oracle.constants import TWO_PI, U
from synthetic import configs, models

B_FIXED = configs.Broadening(adaptive=False)
B_ADAPT = configs.Broadening(adaptive=True)


@pytest.fixture(scope="module")
def diamond():
    return models.diamond()


def clusters(nu, tol=1e-4):
    out, start = [], 0
    for k in range(1, len(nu) + 1):
        if k == len(nu) or nu[k] - nu[k - 1] >= tol:
            out.append(slice(start, k))
            start = k
    return out


def cluster_sums(nu_row, g_row):
    return np.array([g_row[c].sum() for c in clusters(nu_row)])


# ---------------------------------------------------------------- inputs (T0, P3)

def test_fc3_matches_finite_difference_of_pair_energy():
    """Third derivative block of phi(r) vs an 8-point central difference."""
    k2, k3, r0 = 10.0, -60.0, 2.35
    rng = np.random.default_rng(3)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    d0 = r0 * n

    def E(d):
        r = np.linalg.norm(d)
        return 0.5 * k2 * (r - r0) ** 2 + k3 / 6.0 * (r - r0) ** 3

    h = 1e-3
    fd = np.zeros((3, 3, 3))
    eye = np.eye(3)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                s = 0.0
                for sa in (1, -1):
                    for sb in (1, -1):
                        for sc in (1, -1):
                            s += sa * sb * sc * E(d0 + h * (sa * eye[a] + sb * eye[b] + sc * eye[c]))
                fd[a, b, c] = s / (8 * h ** 3)
    an = models.pair_fc3_block(n, k2, k3, r0)
    assert np.max(np.abs(fd - an)) < 1e-4 * np.max(np.abs(an))


@pytest.mark.parametrize("builder", ["diamond", "perovskite", "glass"])
def test_acoustic_sum_rules(builder):
    m = configs.build_model(builder)
    nb = m.n_basis
    s2 = m.fc2.reshape(3 * nb, -1).reshape(3 * nb, m.n_rep * nb, 3).sum(axis=1)
    assert np.max(np.abs(s2)) < 1e-12 * np.max(np.abs(m.fc2))
    # sum over the third index of FC3 for every (first, second) pair
    acc = {}
    for i, j, k, v in zip(m.fc3_i, m.fc3_j, m.fc3_k, m.fc3_val):
        key = (i, j, k % 3)
        acc[key] = acc.get(key, 0.0) + v
    assert max(abs(v) for v in acc.values()) < 1e-12 * np.max(np.abs(m.fc3_val))


def test_fc3_counts_match_structure(diamond):
    # 13 atom triples per diamond basis atom, 185 for the perovskite, full blocks
    assert diamond.nnz == 27 * 26
    assert configs.build_model("perovskite").nnz == 27 * 185
    g = configs.build_model("glass")
    assert g.params["n_bonds"] == 1024 and g.nnz == 27 * (512 + 6 * 1024)


def test_three_zero_modes_at_gamma(diamond):
    om, _, _ = phonons.phonons_at(diamond, np.zeros(3))
    # diamond NN springs: 3 acoustic + 2 floppy zero modes (rank-4 D)
    assert np.sum(np.abs(om / TWO_PI) < 1e-5) >= 3


# ---------------------------------------------------------------- phonons (P1, P2)

def diamond_closed_form(qcart, a=models.DIAMOND_A, k2=10.0, m=models.SI_MASS):
    R = 0.5 * a * np.array([[0, 0, 0], [0, -1, -1], [-1, 0, -1], [-1, -1, 0]], float)
    S = np.abs(np.sum(np.exp(1j * (R @ qcart))))
    w2 = np.array([0, 0, k2 * (4 - S) / (3 * m), k2 * (4 + S) / (3 * m),
                   8 * k2 / (3 * m), 8 * k2 / (3 * m)]) * U
    return np.sort(np.sqrt(np.abs(w2)))


def test_diamond_dispersion_closed_form(diamond):
    B = phonons.reciprocal(diamond.lattice)
    rng = np.random.default_rng(0)
    for _ in range(30):
        f = rng.uniform(-0.5, 0.5, 3)
        om, _, _ = phonons.phonons_at(diamond, f)
        ref = diamond_closed_form(f @ B)
        assert np.allclose(np.sort(np.abs(om)), ref, rtol=1e-12, atol=1e-6 * ref.max())
    # optical frequency at Gamma, and the L and X points
    om, _, _ = phonons.phonons_at(diamond, np.zeros(3))
    assert abs(om.max() / TWO_PI - 15.2334) < 1e-4
    om, _, _ = phonons.phonons_at(diamond, np.array([0.5, 0.5, 0.5]))
    nu = np.sort(om / TWO_PI)
    assert np.allclose(nu[2:4], [7.6167, 13.1925], atol=1e-4)
    om, _, _ = phonons.phonons_at(diamond, np.array([0.0, 0.5, 0.5]))
    nu = np.sort(om / TWO_PI)
    assert np.allclose(nu[2:4], [10.7716, 10.7716], atol=1e-4)


def test_group_velocity_matches_finite_difference(diamond):
    B = phonons.reciprocal(diamond.lattice)
    Binv = np.linalg.inv(B)
    rng = np.random.default_rng(1)
    h = 1e-5
    for _ in range(10):
        f = rng.uniform(-0.45, 0.45, 3)
        om, _, v = phonons.phonons_at(diamond, f)
        qc = f @ B
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            op, _, _ = phonons.phonons_at(diamond, (qc + e) @ Binv)
            omn, _, _ = phonons.phonons_at(diamond, (qc - e) @ Binv)
            fd = (op - omn) / (2 * h)
            for s in (2, 3):  # the two dispersive branches (non-degenerate at random q)
                assert abs(fd[s] - v[s, c]) < 1e-6 * max(1.0, abs(v[s, c]))
        # flat optical and floppy branches carry no velocity
        assert np.max(np.abs(v[[0, 1, 4, 5]])) < 1e-8


def test_phonon_eigenvectors_orthonormal_and_phase_fixed(diamond):
    om, ev, _ = phonons.phonons(diamond, (3, 3, 3))
    for q in range(ev.shape[0]):
        assert np.allclose(ev[q].conj().T @ ev[q], np.eye(6), atol=1e-12)
        # some largest-modulus component (ties allowed) is real and positive
        mod = np.abs(ev[q])
        top = mod >= mod.max(axis=0)[None, :] - 1e-12
        ok = top & (np.abs(ev[q].imag) < 1e-14) & (ev[q].real > 0)
        assert np.all(ok.any(axis=0))


# ---------------------------------------------------------------- smearing (P11)

@pytest.mark.parametrize("shape,ref", [(linewidths.GAUSS, scipy.special.erf(2.0)),
                                       (linewidths.LORENTZ, 2.0 / math.pi * math.atan(4.0))])
def test_smearing_integral(shape, ref):
    for sigma in (0.3, 1.7):
        val, _ = scipy.integrate.quad(lambda x: float(linewidths.smearing(x, sigma, shape)),
                                      -2 * sigma, 2 * sigma, epsabs=1e-14, epsrel=1e-14)
        assert abs(val - ref) < 1e-12
        assert float(linewidths.smearing(2 * sigma, sigma, shape)) == 0.0


# ---------------------------------------------------------------- vertex (P4, P5, P10)

def test_vertex_matches_bruteforce_diamond(diamond):
    for mesh in [(2, 2, 2), (3, 3, 3)]:
        _, ev, _ = phonons.phonons(diamond, mesh)
        Vb = bruteforce.vertex_bruteforce(diamond, mesh, ev)
        nq = ev.shape[0]
        for q in range(nq):
            V, _ = linewidths.vertex_crystal(diamond, mesh, ev, q)
            scale = np.max(np.abs(Vb[q]))
            assert np.max(np.abs(V - Vb[q])) < 1e-12 * scale


def test_vertex_matches_bruteforce_random_cell():
    m = models.random_cell(seed=7, n_basis=2)
    mesh = (2, 3, 2)
    _, ev, _ = phonons.phonons(m, mesh)
    Vb = bruteforce.vertex_bruteforce(m, mesh, ev)
    for q in range(ev.shape[0]):
        V, _ = linewidths.vertex_crystal(m, mesh, ev, q)
        assert np.max(np.abs(V - Vb[q])) < 1e-12 * np.max(np.abs(Vb[q]))


def test_gamma_vertex_matches_bruteforce_random_glass():
    m = models.random_cluster_glass(seed=2, n_atoms=8)
    om, E = phonons.phonons_gamma_real(m)
    for mu in range(0, 24, 5):
        V = linewidths.vertex_gamma(m, E, mu)
        Vb = bruteforce.vertex_gamma_bruteforce(m, E, mu)
        assert np.max(np.abs(V - Vb)) < 1e-12 * np.max(np.abs(Vb))


def test_vertex_vanishes_for_uniform_translation(diamond):
    mesh = (3, 3, 3)
    _, ev, _ = phonons.phonons(diamond, mesh)
    ev = ev.copy()
    M = diamond.mass.sum()
    for a in range(3):
        t = np.zeros(6, complex)
        t[a::3] = np.sqrt(diamond.mass / M)
        ev[0][:, a] = t
    V, _ = linewidths.vertex_crystal(diamond, mesh, ev, 0)
    assert np.max(np.abs(V[:, 0:3])) <= 1e-12 * np.max(np.abs(V))
    # glass: the three uniform translations
    g = models.random_cluster_glass(seed=4, n_atoms=8)
    om, E = phonons.phonons_gamma_real(g)
    E = E.copy()
    Mt = g.mass.sum()
    for a in range(3):
        t = np.zeros(24)
        t[a::3] = np.sqrt(g.mass / Mt)
        E[:, a] = t
    Vg = linewidths.vertex_gamma(g, E, 0)
    Vref = linewidths.vertex_gamma(g, E, 10)
    assert np.max(np.abs(Vg)) <= 1e-12 * np.max(np.abs(Vref))


def test_vertex_permutation_symmetry(diamond):
    mesh = (4, 3, 3)
    _, ev, _ = phonons.phonons(diamond, mesh)
    nq = ev.shape[0]
    rng = np.random.default_rng(0)
    for q in rng.choice(nq, 4, replace=False):
        Vq, q2 = linewidths.vertex_crystal(diamond, mesh, ev, q)
        scale = np.max(np.abs(Vq))
        # swap second and third partner: V(q s; q2 s''; q1 s')
        for q1 in range(nq):
            assert np.max(np.abs(Vq[q1] - np.transpose(Vq[q2[q1]], (0, 2, 1)))) < 1e-12 * scale
        # swap first and second: V(q1 s'; q s; q2 s'')
        for q1 in rng.choice(nq, 3, replace=False):
            V1, q2b = linewidths.vertex_crystal(diamond, mesh, ev, q1)
            assert q2b[q] == q2[q1]
            assert np.max(np.abs(Vq[q1] - np.transpose(V1[q], (1, 0, 2)))) < 1e-12 * scale


def test_gamma_vertex_fully_symmetric():
    g = models.random_cluster_glass(seed=5, n_atoms=8)
    om, E = phonons.phonons_gamma_real(g)
    V = np.stack([linewidths.vertex_gamma(g, E, mu) for mu in range(24)])
    s = np.max(np.abs(V))
    assert np.max(np.abs(V - V.transpose(0, 2, 1))) < 1e-12 * s
    assert np.max(np.abs(V - V.transpose(1, 0, 2))) < 1e-12 * s


# ---------------------------------------------------------------- rates (P6-P9, P13)

@pytest.fixture(scope="module")
def c1_adaptive(diamond):
    mesh = (5, 5, 5)
    om, ev, ve = phonons.phonons(diamond, mesh)
    G = linewidths.crystal_linewidths(diamond, mesh, om, ev, ve, 300.0, B_ADAPT)
    return mesh, om, ev, ve, G


def test_time_reversal(c1_adaptive):
    mesh, om, _, _, G = c1_adaptive
    pts = phonons.mesh_points(mesh)
    N = np.asarray(mesh)
    nu = om / TWO_PI
    for q, n in enumerate(pts):
        m = np.mod(-n, N)
        qm = (m[0] * N[1] + m[1]) * N[2] + m[2]
        a, b = cluster_sums(nu[q], G[q]), cluster_sums(nu[qm], G[qm])
        assert np.allclose(a, b, rtol=1e-10, atol=1e-14)


def test_rates_nonnegative_and_masked(c1_adaptive):
    mesh, om, _, _, G = c1_adaptive
    nu = om / TWO_PI
    phys = nu >= 0.1
    assert np.all(G[~phys] == 0.0)
    assert np.all(G[nu > 2 * 0.1 * 4] >= 0.0)
    assert np.all(np.isfinite(G))


def test_quadratic_in_fc3(diamond):
    mesh = (3, 3, 3)
    om, ev, ve = phonons.phonons(diamond, mesh)
    G1 = linewidths.crystal_linewidths(diamond, mesh, om, ev, ve, 300.0, B_ADAPT)
    d2 = models.Model(**{**diamond.__dict__, "fc3_val": 2.0 * diamond.fc3_val})
    G2 = linewidths.crystal_linewidths(d2, mesh, om, ev, ve, 300.0, B_ADAPT)
    assert np.array_equal(G2, 4.0 * G1)


def test_zone_folding_crystal_vs_gamma_point(diamond):
    """3x3x3 mesh on the 2-atom cell == Gamma point of the 54-atom supercell."""
    mesh = (3, 3, 3)
    om, ev, ve = phonons.phonons(diamond, mesh)
    Gc = linewidths.crystal_linewidths(diamond, mesh, om, ev, ve, 300.0, B_FIXED)
    sc = models.supercell_gamma(diamond, mesh)
    oms, E = phonons.phonons_gamma_real(sc)
    Gs = linewidths.gamma_point_linewidths(sc, oms, E, 300.0, B_FIXED)
    nuc = om.reshape(-1) / TWO_PI
    order = np.argsort(nuc, kind="stable")
    nuc, gc = nuc[order], Gc.reshape(-1)[order]
    nus = oms / TWO_PI
    # the floppy zero modes are rounding noise in both; clamp them
    nuc = np.where(np.abs(nuc) < 0.05, 0.0, nuc)
    nus = np.where(np.abs(nus) < 0.05, 0.0, nus)
    assert np.allclose(nuc, nus, atol=1e-9)
    cl = clusters(nus, 1e-6)
    a = np.array([gc[c].sum() for c in cl])
    b = np.array([Gs[c].sum() for c in cl])
    assert np.allclose(a, b, rtol=1e-10, atol=1e-12 * a.max())
    assert a.max() > 0


def test_kappa_isotropic_cubic(c1_adaptive, diamond):
    mesh, om, _, ve, G = c1_adaptive
    k = kappa.kappa_rta(om, ve, G, 300.0, diamond.volume, 125, 0.1)
    kbar = np.trace(k) / 3
    assert kbar > 0
    assert np.max(np.abs(k - kbar * np.eye(3))) < 1e-10 * kbar


def test_linewidths_linear_in_temperature_in_classical_limit(diamond):
    """High-temperature limit of Eq. gamma with Eq. bose: n = k_B T/(hbar w) -
    1/2 + O(x), so (n1 - n2) and (n1 + n2 + 1) are both linear in T (their
    -1/2 parts cancel), and Gamma(2T)/Gamma(T) -> 2 with corrections of order
    x^2/12 (x = hbar w/k_B T < 4e-3 here).  A dropped or misplaced +1, a
    wrong population pairing or a wrong hbar/k_B factor breaks the ratio."""
    mesh = (3, 3, 3)
    om, ev, ve = phonons.phonons(diamond, mesh)
    g1 = linewidths.crystal_linewidths(diamond, mesh, om, ev, ve, 2.0e5, B_FIXED)
    g2 = linewidths.crystal_linewidths(diamond, mesh, om, ev, ve, 4.0e5, B_FIXED)
    big = g1 > 1e-3 * g1.max()
    assert big.sum() > 20
    assert np.max(np.abs(g2[big] / g1[big] - 2.0)) < 2e-5
    # at 300 K the same modes are far from the classical limit
    g0 = linewidths.crystal_linewidths(diamond, mesh, om, ev, ve, 300.0, B_FIXED)
    r = g1[big] / g0[big]
    assert np.max(np.abs(r - 2.0e5 / 300.0)) > 1.0
