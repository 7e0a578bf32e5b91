"""Quasi-harmonic Green-Kubo conductivity of the oracle (Eq. qhgk for a
Gamma-point solid, Eq. qhgk_crystal for the interband term of a crystal).

    kappa_ab = 1/V sum_{mu nu} c_{mu nu} v^a_{mu nu} tau_{mu nu} v^b_{nu mu}

Readings fixed here:
* Generalised heat capacity: c_{mu nu} = (hbar/T) w_mu w_nu (n_mu - n_nu) /
  (w_nu - w_mu), whose limit w_nu -> w_mu is the modal heat capacity c_mu of
  Eq. heatcap; the printed prefactor k_B/T misses that limit by hbar/k_B.
  Pairs closer than DEG_TOL_THZ use (c_mu + c_nu)/2 (the paper: c_mu for
  degenerate modes).
* Generalised velocities: the velocity operator of the cell, the q-derivative
  of the dynamical matrix written with the full separation of the two atoms
  (lattice vector plus basis offset, so that it does not depend on the phase
  convention of the eigenvectors), sandwiched between two modes and divided by
  2 sqrt(w_mu w_nu):
      v^a_{mu nu} = eta_mu^H [sum_l -i (R_l + tau_j - tau_i)_a e^{-i q.R_l}
                    Phi(0i, lj)/sqrt(m_i m_j)] eta_nu / (2 sqrt(w_mu w_nu)).
  Its diagonal is the group velocity of Eq. groupvel; the paper writes the
  matrix element without the normalisation.  For a Gamma-point solid the
  separations are the minimum-image vectors R_j - R_i.
* Generalised lifetimes (Lorentzian, as printed): tau_{mu nu} = g / (2 ((w_mu -
  w_nu)^2 + g^2)) with g = (Gamma_mu + Gamma_nu)/2, so that tau_{mu mu} =
  1/(2 Gamma_mu) is the lifetime of Eq. lifetime.
* Modes taken: nu >= nu_min and Gamma > GAMMA_FLOOR_REL max Gamma (as the RTA).
* V is the volume of the cell the sum runs over: N_q V_cell for a mesh.

This is test infrastructure: a plain, slow reference for the GPU library.
"""
from __future__ import annotations

import numpy as np

from .constants import HBAR, KAPPA_UNIT, KB, TWO_PI, U
from .kappa import GAMMA_FLOOR_REL, heat_capacity_kb
from .phonons import mesh_points

DEG_TOL_THZ = 1e-4
NU_FLOOR_THZ = 1e-3   # modes below it get no generalised velocity (as the group velocity)


def heat_capacity_matrix(omega, T):
    """c_{mu nu} / k_B for the modes of one block (all positive frequencies)."""
    w = np.asarray(omega, float)
    n = 1.0 / np.expm1(HBAR * w / (KB * T))
    dw = w[None, :] - w[:, None]                              # w_nu - w_mu
    deg = np.abs(dw) / TWO_PI < DEG_TOL_THZ
    with np.errstate(divide="ignore", invalid="ignore"):
        c = HBAR / (KB * T) * w[:, None] * w[None, :] * (n[:, None] - n[None, :]) / dw
    cm = heat_capacity_kb(w, T)
    return np.where(deg, 0.5 * (cm[:, None] + cm[None, :]), c)


def lifetime_matrix(omega, gamma):
    w = np.asarray(omega, float)
    g = 0.5 * (gamma[:, None] + gamma[None, :])
    dw = w[:, None] - w[None, :]
    return g / (2.0 * (dw * dw + g * g))


def separation_dq(model, qfrac):
    """(3, 3N_b, 3N_b): sum_l -i (R_l + tau_j - tau_i)_a e^{-i q.R_l} Phi/sqrt(mm)."""
    nb = model.n_basis
    phase = np.exp(-1j * TWO_PI * (model.rep @ np.asarray(qfrac, float)))
    R = model.rep @ model.lattice                             # (n_rep, 3)
    tau = model.frac @ model.lattice                          # (N_b, 3)
    m = np.repeat(model.mass, 3)
    inv = 1.0 / np.sqrt(np.outer(m, m))
    out = np.zeros((3, 3 * nb, 3 * nb), complex)
    for i in range(nb):
        for j in range(nb):
            sep = R + (tau[j] - tau[i])[None, :]             # (n_rep, 3)
            blk = model.fc2[3 * i:3 * i + 3, :, 3 * j:3 * j + 3]  # (3, n_rep, 3)
            for a in range(3):
                out[a, 3 * i:3 * i + 3, 3 * j:3 * j + 3] = np.einsum(
                    "xly,l->xy", blk, -1j * sep[:, a] * phase)
    return out * inv[None, :, :]


def velocity_matrix_crystal(model, qfrac, omega_q, eta_q):
    """v^a_{s s'} at one q (3, 3N_b, 3N_b), A/ps; 0 where a mode is below
    NU_FLOOR_THZ (zero modes, whose frequency is rounding noise)."""
    dD = separation_dq(model, qfrac) * U
    V = np.einsum("am,cab,bn->cmn", eta_q.conj(), dD, eta_q)
    pos = omega_q / TWO_PI >= NU_FLOOR_THZ
    norm = np.zeros((len(omega_q), len(omega_q)))
    wp = np.where(pos, omega_q, 1.0)
    norm[np.ix_(pos, pos)] = 1.0 / (2.0 * np.sqrt(np.outer(wp, wp)))[np.ix_(pos, pos)]
    return V * norm[None]


def _active(omega, gamma, nu_min_thz):
    g = np.asarray(gamma, float)
    gmax = np.max(g) if g.size else 0.0
    return (np.asarray(omega) / TWO_PI >= nu_min_thz) & (g > GAMMA_FLOOR_REL * gmax) & (g > 0)


def kappa_qhgk_crystal(model, mesh, omega, evec, gamma, T, nu_min_thz, interband_only=True):
    """3x3 kappa, W/(m K): the interband sum of Eq. qhgk_crystal (s != s'),
    or with interband_only=False every pair of each q (s == s' included: the
    RTA term with the generalised lifetime)."""
    pts = mesh_points(mesh)
    N = np.asarray(mesh, float)
    nq, nb3 = omega.shape
    act = _active(omega.reshape(-1), gamma.reshape(-1), nu_min_thz).reshape(nq, nb3)
    k = np.zeros((3, 3))
    for q in range(nq):
        a = act[q]
        if not a.any():
            continue
        V = velocity_matrix_crystal(model, pts[q] / N, omega[q], evec[q])[:, a][:, :, a]
        w = omega[q][a]
        W = heat_capacity_matrix(w, T) * lifetime_matrix(w, gamma[q][a])
        if interband_only:
            np.fill_diagonal(W, 0.0)
        k += np.real(np.einsum("mn,amn,bmn->ab", W, V, V.conj()))
    return KAPPA_UNIT * k / (nq * model.volume)


def minimum_image_separations(model):
    """(N, N, 3) R_j - R_i with the minimum-image convention of the cell."""
    d = model.frac[None, :, :] - model.frac[:, None, :]
    d -= np.round(d)
    return d @ model.lattice


def velocity_matrix_gamma(model, omega, E):
    """Gamma-point solid (one cell, real eigenvectors E [3N, 3N]): v^a
    (3, 3N, 3N) complex, A/ps (purely imaginary, antisymmetric).  Each bonded
    pair must have a single image within the force-constant range."""
    n = model.n_basis
    m = np.repeat(model.mass, 3)
    D = model.fc2.sum(axis=1) / np.sqrt(np.outer(m, m)) * U  # ps^-2
    sep = np.repeat(np.repeat(minimum_image_separations(model), 3, axis=0), 3, axis=1)
    pos = omega / TWO_PI >= NU_FLOOR_THZ
    wp = np.where(pos, omega, 1.0)
    norm = np.where(np.outer(pos, pos), 1.0 / (2.0 * np.sqrt(np.outer(wp, wp))), 0.0)
    out = np.empty((3, 3 * n, 3 * n), complex)
    for a in range(3):
        S = D * sep[:, :, a]
        out[a] = -1j * (E.T @ S @ E) * norm
    return out


def kappa_qhgk_gamma(model, omega, E, gamma, T, nu_min_thz):
    """(3x3 kappa W/(m K), mode diffusivity [3N] A^2/ps) of Eq. qhgk for a
    Gamma-point solid; the diffusivity is D_mu = 1/3 sum_a sum_nu
    |v^a_{mu nu}|^2 tau_{mu nu} over the taken modes."""
    act = _active(omega, gamma, nu_min_thz)
    V = velocity_matrix_gamma(model, omega, E)[:, act][:, :, act]
    w = omega[act]
    tau = lifetime_matrix(w, gamma[act])
    W = heat_capacity_matrix(w, T) * tau
    k = np.real(np.einsum("mn,amn,bmn->ab", W, V, V.conj()))
    diff = np.zeros(len(omega))
    diff[act] = np.einsum("mn,amn->m", tau, np.abs(V) ** 2) / 3.0
    return KAPPA_UNIT * k / model.volume, diff
