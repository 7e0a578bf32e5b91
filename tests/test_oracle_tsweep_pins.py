"""Pins of the oracle's temperature-sweep cache (multi-temperature
optimisation of "Performance and Scalability"; Eq. gamma, Eq. bose).

* decoupling: Gamma(T) rebuilt from the cached factors equals the direct
  Gamma(T) of Eq. gamma at several temperatures and both smearing forms;
* the T -> 0 limit: all populations vanish and only spontaneous decay
  (1/2 a-) remains, compared with the direct sum at 0.05 K;
* the classical limit: n -> k_B T/(hbar w), so Gamma/T tends to a
  population-free closed form of the cached factors;
* brute force: on a tiny mesh, explicit loops over every (q, s, q1, s', s'')
  with the dense-supercell vertex (no COO, no pattern tables) select the same
  partner pairs and give the same a+ and a-.
"""
import math

import numpy as np
import pytest

from oracle import bruteforce, linewidths, phonons, tsweep
from oracle.constants import HBAR, KB, TWO_PI
from synthetic import configs, models

B_FIXED = configs.Broadening(adaptive=False)
B_ADAPT = configs.Broadening(adaptive=True)
B_LORENTZ = configs.Broadening(shape=configs.LORENTZ, adaptive=False)

CASES = {
    "diamond-adaptive": (lambda: models.diamond(), (4, 4, 4), B_ADAPT),
    "random-fixed": (lambda: models.random_cell(11, 2), (3, 4, 5), B_FIXED),
    "random-lorentz": (lambda: models.random_cell(5, 2), (3, 3, 4), B_LORENTZ),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    mk, mesh, b = CASES[request.param]
    m = mk()
    om, ev, ve = phonons.phonons(m, mesh)
    cache = tsweep.linewidth_cache(m, mesh, om, ev, ve, b)
    return m, mesh, b, om, ev, ve, cache


@pytest.mark.parametrize("T", [40.0, 300.0, 1500.0])
def test_cache_reproduces_direct_gamma(case, T):
    m, mesh, b, om, ev, ve, cache = case
    direct = linewidths.crystal_linewidths(m, mesh, om, ev, ve, T, b)
    swept = tsweep.gamma_from_cache(cache, om, T, b.nu_min_thz)
    np.testing.assert_allclose(swept, direct, rtol=1e-12, atol=1e-14 * np.abs(direct).max())


def test_zero_temperature_limit_is_spontaneous_decay(case):
    m, mesh, b, om, ev, ve, cache = case
    direct = linewidths.crystal_linewidths(m, mesh, om, ev, ve, 0.05, b)
    decay = tsweep.spontaneous_decay(cache, om, b.nu_min_thz)
    assert decay.max() > 0
    np.testing.assert_allclose(direct, decay, rtol=1e-12, atol=1e-14 * decay.max())


def test_classical_limit(case):
    """n(w, T) = k_B T/(hbar w) - 1/2 + O(hbar w / k_B T), so Gamma(T)/T tends
    to (k_B/hbar) P/N_q sum [a+ (1/w1 - 1/w2) + 1/2 a- (1/w1 + 1/w2)]."""
    m, mesh, b, om, ev, ve, cache = case
    T = 2.0e6
    direct = linewidths.crystal_linewidths(m, mesh, om, ev, ve, T, b)
    flat = om.reshape(-1)
    inv = np.zeros_like(flat)
    ok = flat / TWO_PI >= b.nu_min_thz
    inv[ok] = 1.0 / flat[ok]
    i1, i2 = inv[cache["m1"]], inv[cache["m2"]]
    term = cache["a_plus"] * (i1 - i2) + 0.5 * cache["a_minus"] * (i1 + i2)
    rp = cache["row_ptr"]
    row = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    slope = np.bincount(row, weights=term, minlength=len(rp) - 1)
    slope = (KB / HBAR) * linewidths.PREFACTOR / cache["n_q"] * slope
    slope[~ok] = 0.0
    got = direct.reshape(-1) / T
    big = slope > 1e-6 * slope.max()
    np.testing.assert_allclose(got[big], slope[big], rtol=1e-5)


def test_cache_rows_against_brute_force():
    m = models.random_cell(3, 2)
    mesh = (2, 3, 2)
    b = B_FIXED
    om, ev, ve = phonons.phonons(m, mesh)
    cache = tsweep.linewidth_cache(m, mesh, om, ev, ve, b)
    Vb = bruteforce.vertex_bruteforce(m, mesh, ev)              # [q, q1, s, s', s'']
    pts = phonons.mesh_points(mesh)
    N = np.asarray(mesh)
    nq, nb3 = om.shape
    sig = TWO_PI * b.sigma_thz
    nu_min = b.nu_min_thz

    def g(x):
        return math.exp(-(x * x) / (sig * sig)) / (math.sqrt(math.pi) * sig)

    n_rows = 0
    for q in range(nq):
        for s in range(nb3):
            mu = q * nb3 + s
            lo, hi = cache["row_ptr"][mu], cache["row_ptr"][mu + 1]
            got = {(int(a), int(c)): (p, n) for a, c, p, n in
                   zip(cache["m1"][lo:hi], cache["m2"][lo:hi], cache["a_plus"][lo:hi],
                       cache["a_minus"][lo:hi])}
            want = {}
            w = om[q, s]
            if w / TWO_PI >= nu_min:
                for q1 in range(nq):
                    n2 = np.mod(-pts[q] - pts[q1], N)
                    q2 = (n2[0] * N[1] + n2[1]) * N[2] + n2[2]
                    for s1 in range(nb3):
                        for s2 in range(nb3):
                            w1, w2 = om[q1, s1], om[q2, s2]
                            if w1 / TWO_PI < nu_min or w2 / TWO_PI < nu_min:
                                continue
                            xp, xm = (w + w1) - w2, (w - w1) - w2
                            inp, inm = abs(xp) < 2 * sig, abs(xm) < 2 * sig
                            if not (inp or inm):
                                continue
                            v2 = abs(Vb[q, q1, s, s1, s2]) ** 2 / (w * w1 * w2)
                            want[(q1 * nb3 + s1, q2 * nb3 + s2)] = (
                                v2 * g(xp) if inp else 0.0, v2 * g(xm) if inm else 0.0)
            assert set(got) == set(want), (q, s)
            for k, (p, n) in want.items():
                scale = max(p, n, 1e-300)
                assert abs(got[k][0] - p) <= 1e-10 * scale and abs(got[k][1] - n) <= 1e-10 * scale
            n_rows += len(want) > 0
    assert n_rows > 0
