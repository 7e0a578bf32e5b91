"""Isotope (mass-disorder) scattering of the oracle, Eq. isotope.

Tamura's perturbation theory, as the paper states it ("Isotopic Scattering"):

    gamma_iso(q,s) = pi/(2 N_q) w(q,s)^2 sum_{q' s'} delta(w(q,s) - w(q',s'))
                     sum_i g_i |sum_a eta*_{ia}(q,s) eta_{ia}(q',s')|^2

with g_i = sum_iso f_iso (dM_iso/M_i)^2 the mass-variance parameter of basis
atom i.  Readings fixed here:
* the Cartesian sum sits inside the modulus (the overlap of the two modes'
  displacement patterns on atom i), which is Tamura's form and the one that
  does not change when the Cartesian axes are rotated; the printed formula
  puts the sum over i and a outside |.|^2, which would;
* delta is the smearing of Eq. broadening with the 2 sigma cut and the same
  nu_min masks as Eq. gamma (modes and partners below nu_min are excluded);
  the adaptive width is that of R9 applied to the elastic process: x = w - w'
  varies with the summed q' at the rate -v(q',s'), so
  sigma = max(floor, |v(q',s')| h / sqrt(12));
* gamma_iso is a linewidth in the convention of Eq. gamma (the paper adds the
  two: gamma = gamma_anh + gamma_iso, and tau = 1/(2 Gamma), Eq. lifetime).

Units: w rad/ps, sigma rad/ps, gamma_iso rad/ps.

This is test infrastructure: a plain, slow reference for the GPU library.
"""
from __future__ import annotations

import math

import numpy as np

from .constants import TWO_PI
from .linewidths import mesh_step2, smearing


def overlaps(evec, q, s, g, n_basis):
    """O[q', s'] = sum_i g_i |sum_a conj(eta_ia(q,s)) eta_ia(q',s')|^2."""
    nq, nb3, _ = evec.shape
    e0 = evec[q][:, s].reshape(n_basis, 3)
    E = evec.reshape(nq, n_basis, 3, nb3)
    dot = np.einsum("ia,qiat->qit", np.conj(e0), E)
    return np.einsum("i,qit->qt", np.asarray(g, float), np.abs(dot) ** 2)


def isotope_linewidths(model, mesh, omega, evec, vel, g, broadening, q_list=None):
    """gamma_iso [N_q, 3N_b] (rad/ps); rows not in q_list are left NaN."""
    nq, nb3 = omega.shape
    nb = nb3 // 3
    phys = omega / TWO_PI >= broadening.nu_min_thz
    if broadening.adaptive:
        h2 = mesh_step2(model.lattice, mesh)
        S = np.sum(vel * vel, axis=-1)                     # |v(q',s')|^2
        sig = np.maximum(np.sqrt(S * h2 / 12.0), TWO_PI * broadening.sigma_floor_thz)
    else:
        sig = np.full(omega.shape, TWO_PI * broadening.sigma_thz)
    out = np.full((nq, nb3), np.nan)
    for q in (range(nq) if q_list is None else q_list):
        for s in range(nb3):
            if not phys[q, s]:
                out[q, s] = 0.0
                continue
            w = omega[q, s]
            d = smearing(w - omega, sig, broadening.shape)      # (q', s')
            d = np.where(phys, d, 0.0)
            O = overlaps(evec, q, s, g, nb)
            out[q, s] = math.pi / (2.0 * nq) * w * w * np.sum(d * O)
    return out


def isotope_gamma_point(omega, E, g_atoms, broadening):
    """Eq. isotope for a Gamma-point solid (N_q = 1, real eigenvectors E
    [3N, 3N], g per atom of the cell), fixed width."""
    n3 = len(omega)
    n = n3 // 3
    phys = omega / TWO_PI >= broadening.nu_min_thz
    sig = TWO_PI * broadening.sigma_thz
    Er = E.reshape(n, 3, n3)
    out = np.zeros(n3)
    for mu in range(n3):
        if not phys[mu]:
            continue
        dot = np.einsum("ia,iat->it", Er[:, :, mu], Er)        # (atom, mu')
        O = np.einsum("i,it->t", np.asarray(g_atoms, float), dot ** 2)
        d = np.where(phys, smearing(omega[mu] - omega, np.full(n3, sig), broadening.shape), 0.0)
        out[mu] = math.pi / 2.0 * omega[mu] ** 2 * np.sum(d * O)
    return out
