"""FP64 harmonic phonons of the oracle: frequencies, eigenvectors, velocities.

Follows the paper's "Interatomic Force Constants" section (mass-scaled
dynamical matrix, Eq. dynmat; its Bloch sum over replicas with the phase
e^{-i q.R_l}, Eq. dynmat_reciprocal; the Hermitian eigenproblem,
Eq. eigenvalue_crystal) and the Hellmann-Feynman group velocity, Eq. groupvel,
with the analytic q-derivative of the Bloch sum.

Readings where the paper is silent:
* q-mesh: Gamma-centred, q_n = sum_c (n_c / N_c) b_c, flattened in C order
  over (n1, n2, n3).
* Degenerate clusters (|dnu| < DEG_TOL_THZ after sorting) are rotated to
  diagonalise sum_c chat_c P^H (dD/dq_c) P with chat = (1,2,3)/sqrt(14);
  velocities are then the diagonal of eta^H dD/dq eta / (2 omega).
* Every eigenvector's phase is fixed: its largest-modulus component (first
  one on ties) is made real and positive.
* omega = sign(lambda) sqrt(|lambda| U); |nu| < NU_VEL_FLOOR_THZ gets v = 0.

This is test infrastructure: a plain, slow reference for the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .constants import TWO_PI, U

DEG_TOL_THZ = 1e-4
NU_VEL_FLOOR_THZ = 1e-3
C_HAT = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)


def mesh_points(mesh):
    """Integer mesh coordinates (N_q, 3), C order; q_frac = n / N."""
    n1, n2, n3 = mesh
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
    return g.reshape(-1, 3)


def reciprocal(lattice):
    """Rows b_c with a_i . b_c = 2 pi delta_ic (1/Angstrom)."""
    return TWO_PI * np.linalg.inv(lattice).T


def _dof_mass(model):
    return np.repeat(model.mass, 3)


def dynamical_matrix(model, qfrac):
    """D(q) = sum_l e^{-i q.R_l} Phi(0i, lj) / sqrt(m_i m_j), eV/(A^2 amu)."""
    phase = np.exp(-1j * TWO_PI * (model.rep @ np.asarray(qfrac, float)))
    K = np.einsum("alb,l->ab", model.fc2, phase)
    m = _dof_mass(model)
    return K / np.sqrt(np.outer(m, m))


def dynamical_matrix_dq(model, qfrac):
    """dD/dq_c, shape (3, 3N_b, 3N_b), eV A/(A^2 amu)."""
    phase = np.exp(-1j * TWO_PI * (model.rep @ np.asarray(qfrac, float)))
    R = model.rep @ model.lattice  # Cartesian replica vectors (n_rep, 3)
    m = _dof_mass(model)
    out = np.empty((3, 3 * model.n_basis, 3 * model.n_basis), complex)
    for c in range(3):
        out[c] = np.einsum("alb,l->ab", model.fc2, -1j * R[:, c] * phase) / np.sqrt(np.outer(m, m))
    return out


def _clusters(nu, tol):
    """Runs of consecutive sorted frequencies closer than tol."""
    out, start = [], 0
    for k in range(1, len(nu) + 1):
        if k == len(nu) or nu[k] - nu[k - 1] >= tol:
            out.append(list(range(start, k)))
            start = k
    return out


def fix_phase(evec):
    """Make each column's largest-modulus component real positive."""
    idx = np.argmax(np.abs(evec), axis=0)
    piv = evec[idx, np.arange(evec.shape[1])]
    return evec * (np.conj(piv) / np.abs(piv))[None, :]


def phonons_at(model, qfrac):
    """omega (rad/ps), eta (3N_b comp x 3N_b mode), v (3N_b x 3) in A/ps."""
    D = dynamical_matrix(model, qfrac)
    D = 0.5 * (D + D.conj().T)
    lam, eta = scipy.linalg.eigh(D)
    omega = np.sign(lam) * np.sqrt(np.abs(lam) * U)
    nu = omega / TWO_PI
    dD = dynamical_matrix_dq(model, qfrac)
    for cl in _clusters(nu, DEG_TOL_THZ):
        if len(cl) < 2:
            continue
        P = eta[:, cl]
        M = sum(C_HAT[c] * (P.conj().T @ dD[c] @ P) for c in range(3))
        M = 0.5 * (M + M.conj().T)
        _, W = scipy.linalg.eigh(M)
        eta[:, cl] = P @ W
    eta = fix_phase(eta)
    vel = np.zeros((len(omega), 3))
    ok = np.abs(nu) >= NU_VEL_FLOOR_THZ
    for c in range(3):
        d = np.real(np.einsum("am,ab,bm->m", eta.conj(), dD[c], eta))
        vel[ok, c] = d[ok] * U / (2.0 * omega[ok])
    return omega, eta, vel


def phonons(model, mesh):
    """All mesh points: omega [N_q][3N_b], eta [N_q][3N_b][3N_b], v [N_q][3N_b][3]."""
    pts = mesh_points(mesh)
    N = np.asarray(mesh, float)
    nq, nb3 = len(pts), 3 * model.n_basis
    om = np.empty((nq, nb3))
    ev = np.empty((nq, nb3, nb3), complex)
    ve = np.empty((nq, nb3, 3))
    for n, p in enumerate(pts):
        om[n], ev[n], ve[n] = phonons_at(model, p / N)
    return om, ev, ve


def phonons_gamma_real(model):
    """Gamma-point real symmetric problem: omega (3N,), E (3N comp x 3N mode) real."""
    K = model.fc2.sum(axis=1)
    m = _dof_mass(model)
    D = K / np.sqrt(np.outer(m, m))
    D = 0.5 * (D + D.T)
    lam, E = scipy.linalg.eigh(D)
    omega = np.sign(lam) * np.sqrt(np.abs(lam) * U)
    idx = np.argmax(np.abs(E), axis=0)
    E = E * np.sign(E[idx, np.arange(E.shape[1])])[None, :]
    return omega, E
