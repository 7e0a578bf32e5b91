"""Pins of the oracle's populations, heat capacity, unit constants and
surrogate features against published constants, closed forms and
hand-computed values (nothing here re-evaluates the oracle's own formulas).

* Eq. bose: n(w) = 1/(e^x - 1), x = hbar w/(k_B T).  Pinned by n + 1 = e^x n,
  n(-w) = -1 - n(w), the classical limit n -> 1/x - 1/2, and n = 1 exactly at
  x = ln 2 with x built from the published ratio hbar/k_B.
* Eq. heatcap: c/k_B = x^2 e^x/(e^x - 1)^2.  Pinned by its value at x = 1,
  e/(e - 1)^2, the limit c -> k_B at high T, and c = hbar w dn/dT (the heat
  capacity of one oscillator of energy hbar w (n + 1/2)).
* U (1 eV/(A^2 amu) in ps^-2) equals the Faraday constant in C/mol times
  1e-1; KAPPA_UNIT (W/(m K) per k_B (A/ps)^2 ps/A^3) equals k_B 1e22.
"""
import math

import numpy as np

from oracle import kappa, linewidths, surrogate
from oracle.constants import HBAR, KAPPA_UNIT, KB, TWO_PI, U
from synthetic import configs, models

# CODATA 2018: hbar/k_B in K s (exact, from the exact hbar and k_B), the
# Faraday constant in C/mol and k_B in J/K.
HBAR_OVER_KB_KS = 7.6382325776e-12
FARADAY = 96485.33212
KB_SI = 1.380649e-23


def omega_at(x, T):
    """Angular frequency in rad/ps whose x = hbar w/(k_B T) is x."""
    return x * T / (HBAR_OVER_KB_KS * 1e12)


def test_hbar_over_kb_ratio():
    assert abs(HBAR / KB / 1e12 - HBAR_OVER_KB_KS) <= 1e-9 * HBAR_OVER_KB_KS


def test_bose_equals_one_at_ln2():
    for T in (10.0, 300.0, 1234.5):
        n = linewidths.bose(omega_at(math.log(2.0), T), T)
        assert abs(n - 1.0) < 1e-8


def test_bose_identities():
    T = 300.0
    x = np.array([1e-3, 0.1, 0.7, 1.0, 3.0, 12.0])
    w = omega_at(x, T)
    n = linewidths.bose(w, T)
    np.testing.assert_allclose(n + 1.0, np.exp(x) * n, rtol=1e-8)
    np.testing.assert_allclose(linewidths.bose(-w, T), -1.0 - n, rtol=1e-8)
    # classical limit: n = 1/x - 1/2 + x/12 + O(x^3)
    xs = np.array([1e-4, 1e-3, 1e-2])
    ns = linewidths.bose(omega_at(xs, T), T)
    np.testing.assert_allclose(ns, 1.0 / xs - 0.5 + xs / 12.0, rtol=1e-8)


def test_heat_capacity_closed_forms():
    T = 300.0
    c1 = kappa.heat_capacity_kb(omega_at(1.0, T), T)
    assert abs(c1 - math.e / (math.e - 1.0) ** 2) < 1e-8
    assert abs(math.e / (math.e - 1.0) ** 2 - 0.9206735942077923) < 1e-15
    # c -> k_B at high temperature: 1 - x^2/12 + O(x^4)
    for x in (1e-3, 1e-2):
        assert abs(kappa.heat_capacity_kb(omega_at(x, T), T) - (1.0 - x * x / 12.0)) < 1e-9
    # low temperature: x^2 e^-x
    x = 30.0
    assert abs(kappa.heat_capacity_kb(omega_at(x, T), T) / (x * x * math.exp(-x)) - 1.0) < 1e-8


def test_heat_capacity_is_temperature_derivative_of_mode_energy():
    """c = d/dT [hbar w (n + 1/2)] = hbar w dn/dT, by central differences of
    the (separately pinned) population."""
    w = np.array([1.0, 10.0, 60.0, 100.0])  # rad/ps
    T, h = 300.0, 1e-3
    dn = (linewidths.bose(w, T + h) - linewidths.bose(w, T - h)) / (2 * h)
    c_fd = HBAR * w * dn / KB
    np.testing.assert_allclose(kappa.heat_capacity_kb(w, T), c_fd, rtol=1e-7)


def test_unit_constant_U_is_faraday_over_ten():
    # 1 eV/(A^2 amu) = (e/m_u) V / A^2 = (F/1 g mol^-1) 1e20 s^-2 = F 1e-1 ps^-2
    assert abs(U - FARADAY * 0.1) <= 2e-9 * U
    assert abs(U - 9648.533212) < 1e-5


def test_kappa_unit_is_kb_times_1e22():
    # k_B [J/K] (A/ps)^2 ps / A^3 = k_B (1e2 m/s)^2 1e-12 s / 1e-30 m^3 = k_B 1e22 W/(m K)
    assert abs(KAPPA_UNIT - KB_SI * 1e22) <= 1e-15
    assert abs(KAPPA_UNIT - 0.1380649) <= 1e-15


def test_feature_values_hand_computed():
    """Feature row of two diamond modes on a 4x4x4 mesh, column by column.
    Lattice rows a_i = a/2 (0,1,1), (1,0,1), (1,1,0), so b1 = (2 pi/a)(-1,1,1).
    Mesh point (1,0,0) is q = b1/4: its own shortest image, every Cartesian
    component of magnitude (2 pi/a)/4.  Mesh point (3,0,0) is 3 b1/4, whose
    shortest image is q - b1 = -b1/4: the same magnitudes."""
    m = models.diamond()
    mesh = (4, 4, 4)
    nq, nb3 = 64, 6
    rng = np.random.default_rng(5)
    omega = rng.uniform(1.0, 90.0, (nq, nb3))
    vel = rng.normal(size=(nq, nb3, 3))
    dp = rng.uniform(0.0, 2.0, (nq, nb3))
    dm = rng.uniform(0.0, 2.0, (nq, nb3))
    q_a, q_b = 16, 48              # flat indices of (1,0,0) and (3,0,0)
    modes = [q_a * nb3 + 3, q_b * nb3 + 0]
    F = surrogate.features(m, mesh, omega, vel, dp, dm, modes)
    assert F.shape == (2, nb3 + 8)
    comp = 0.25 * 2.0 * math.pi / 5.43
    for row, (q, s) in enumerate(((q_a, 3), (q_b, 0))):
        f = F[row]
        assert abs(f[0] - omega[q, s] / TWO_PI) < 1e-14 * f[0]
        assert abs(f[1] - math.sqrt(float(np.sum(vel[q, s] ** 2)))) < 1e-14
        onehot = np.zeros(nb3)
        onehot[s] = 1.0
        np.testing.assert_array_equal(f[2:2 + nb3], onehot)
        np.testing.assert_allclose(f[2 + nb3:5 + nb3], [comp] * 3, rtol=1e-13)
        assert abs(f[5 + nb3] - comp * math.sqrt(3.0)) < 1e-13
        assert abs(f[6 + nb3] - math.log(1.0 + dp[q, s])) < 1e-14
        assert abs(f[7 + nb3] - math.log(1.0 + dm[q, s])) < 1e-14


def test_mode_weights_use_heat_capacity_and_star():
    """w = star c/k_B |v|^2 at x = 1: star e/(e-1)^2 |v|^2."""
    T = 300.0
    w = surrogate.mode_weights(np.array([omega_at(1.0, T)]), np.array([[1.0, 2.0, 2.0]]), T,
                               np.array([6.0]))
    assert abs(w[0] - 6.0 * 0.9206735942077923 * 9.0) < 1e-7


def test_natural_silicon_mass_variance():
    """g of natural silicon from its isotope masses and abundances: the
    literature value is 2.0e-4 (about 2.01e-4); a monoisotopic element gives 0."""
    assert abs(configs.mass_variance("Si") - 2.007e-4) < 1e-6
    assert configs.mass_variance("Cs") == 0.0
    assert len(configs.natural_g("perovskite")) == 5
