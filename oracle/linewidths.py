"""FP64 three-phonon linewidths of the oracle.

Definitions (paper, "Three-Phonon Scattering" subsection):
* Projected potential, Eq. phi3_proj, written for Bloch modes with the
  replica phases of Eq. dynmat_reciprocal and all-incoming momenta
  q + q1 + q2 = G (so q2 = -q - q1 on the mesh):
      V(qs; q1 s'; q2 s'') = sum_e Phi3_e / sqrt(m_i m_j m_k)
            eta_{i}(q,s) eta_{j}(q1,s') eta_{k}(q2,s'')
            e^{-i q1.R_{l'_e}} e^{-i q2.R_{l''_e}}
  evaluated as the paper's projection is organised ("Computational
  Implementation"): first contract the COO tensor with eta(q) on its
  home-cell index, then apply the q1-dependent phases and the two dense
  eigenvector products.  Phases are exact: q1.R = 2 pi sum_c n1_c l_c / N_c
  with the integer numerator reduced mod N_c.
* Rates, Eq. gamma with the population/delta factors of the Delta terms,
  in the reading fixed here:
      Gamma_mu = pi hbar U^3 / (8 N_q) sum_{q1,s',s''} m |V|^2/(w w1 w2)
                 [ (n1 - n2) g(x+, sig+) + 1/2 (n1 + n2 + 1) g(x-, sig-) ]
  with x+ = (w + w1) - w2 (coalescence), x- = (w - w1) - w2 (decay),
  m = [nu1 >= nu_min][nu2 >= nu_min], Gamma_mu = 0 for nu_mu < nu_min.
  (The printed Delta labels are paired with populations as above, the decay
  term carries 1/2 because the sum runs over ordered partner pairs, and 1/N_q
  normalises the Bloch sum; tau = 1/(2 Gamma), Eq. lifetime.)
* Smearing, Eq. broadening: Gaussian e^{-x^2/s^2}/(sqrt(pi) s) or Lorentzian
  (s/2)/(pi (x^2 + s^2/4)), both set to 0 unless |x| < 2 s.
* Adaptive width (the paper cites an adaptive scheme without its formula):
  s = max(s_floor, |dv| h / sqrt(12)), h^2 = (1/3) sum_c |b_c / N_c|^2 the
  mean-square mesh step, with dv+ = v(q1,s') + v(q2,s'') and
  dv- = -v(q1,s') + v(q2,s'').  (A per-axis sum sum_c (dv . b_c/N_c)^2 is not
  invariant under the point group when the b_c are not orthogonal; this is
  its rotation-invariant average and equals it on orthogonal meshes.)
* Populations, Eq. bose, quantum statistics.

Units: omega rad/ps, sigma rad/ps (input THz is cyclic: x 2 pi).

This is test infrastructure: a plain, slow reference for the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse

from .constants import HBAR, KB, TWO_PI, U
from .phonons import mesh_points, reciprocal

GAUSS = 0
LORENTZ = 1
PREFACTOR = math.pi * HBAR * U ** 3 / 8.0


def smearing(x, sigma, shape):
    """Normalised Gaussian or Lorentzian, cut to |x| < 2 sigma."""
    x = np.asarray(x, float)
    sigma = np.broadcast_to(np.asarray(sigma, float), x.shape)
    inside = np.abs(x) < 2.0 * sigma
    if shape == GAUSS:
        g = np.exp(-(x * x) / (sigma * sigma)) / (math.sqrt(math.pi) * sigma)
    elif shape == LORENTZ:
        g = (0.5 * sigma) / (math.pi * (x * x + 0.25 * sigma * sigma))
    else:
        raise ValueError(shape)
    return np.where(inside, g, 0.0)


def bose(omega, T):
    """n = 1/(exp(hbar w / kB T) - 1); omega in rad/ps."""
    return 1.0 / np.expm1(HBAR * np.asarray(omega, float) / (KB * T))


def mesh_step2(lattice, mesh):
    """h^2 = (1/3) sum_c |b_c / N_c|^2 (1/Angstrom^2)."""
    steps = reciprocal(lattice) / np.asarray(mesh, float)[:, None]
    return float(np.sum(steps * steps) / 3.0)


def adaptive_sigma(dv, h2, floor):
    """max(floor, sqrt(|dv|^2 h^2 / 12))."""
    S = np.sum(dv * dv, axis=-1)
    return np.maximum(np.sqrt(S * h2 / 12.0), floor)


class Patterns:
    """The FC3 COO grouped by its (second, third) index pair."""

    def __init__(self, model):
        nb = model.n_basis
        m = model.mass
        ib = model.fc3_i // 3
        jb = (model.fc3_j // 3) % nb
        kb = (model.fc3_k // 3) % nb
        self.coef = model.fc3_val / np.sqrt(m[ib] * m[jb] * m[kb])
        keys = model.fc3_j.astype(np.int64) * (3 * nb * model.n_rep) + model.fc3_k
        uniq, self.p_of_e = np.unique(keys, return_inverse=True)
        self.n_p = len(uniq)
        pj = uniq // (3 * nb * model.n_rep)
        pk = uniq % (3 * nb * model.n_rep)
        self.jrep = (pj // 3) // nb                   # replica of the 2nd index
        self.krep = (pk // 3) // nb                   # replica of the 3rd index
        self.jc = ((pj // 3) % nb) * 3 + pj % 3       # in-cell dof of 2nd index
        self.kc = ((pk // 3) % nb) * 3 + pk % 3
        self.i_e = model.fc3_i
        nb3 = 3 * nb
        self.nb3 = nb3
        # one-hot maps: entry -> pattern, pattern -> (jc, kc)
        self.E2P = scipy.sparse.csr_matrix(
            (np.ones(len(self.p_of_e)), (np.arange(len(self.p_of_e)), self.p_of_e)),
            shape=(len(self.p_of_e), self.n_p))
        self.P2JK = np.zeros((self.n_p, nb3 * nb3))
        self.P2JK[np.arange(self.n_p), self.jc * nb3 + self.kc] = 1.0


def vertex_crystal(model, mesh, evec, q, pat=None):
    """V[q1, s, s', s''] for the mode block at mesh point index q (all q1)."""
    pat = pat or Patterns(model)
    pts = mesh_points(mesh)
    N = np.asarray(mesh)
    nq, nb3 = len(pts), pat.nb3
    n = pts[q]
    q2_of_q1 = _q2_index(pts, n, N)
    # home-cell index contracted with eta(q): A[s, p]
    X = evec[q][pat.i_e, :] * pat.coef[:, None]          # (nnz, s)
    A = (pat.E2P.T @ X).T                                 # (s, p)
    # exact phases e^{-i (q1.R' + q2.R'')}: integer numerators reduced mod N
    n1 = pts                                              # (nq, 3)
    n2 = pts[q2_of_q1]
    f1 = np.sum(np.mod(n1[:, None, :] * model.rep[None, :, :], N) / N, axis=-1)  # (nq, rep)
    f2 = np.sum(np.mod(n2[:, None, :] * model.rep[None, :, :], N) / N, axis=-1)
    phase = np.exp(-1j * TWO_PI * (f1[:, pat.jrep] + f2[:, pat.krep]))  # (nq, p)
    # B[q1, s, jc, kc] = sum_p phase[q1, p] A[s, p] [p -> (jc, kc)]
    M = A.T[:, :, None] * pat.P2JK[:, None, :]            # (p, s, jc*kc)
    B = (phase @ M.reshape(pat.n_p, -1)).reshape(nq, nb3, nb3, nb3)
    T = np.matmul(B, evec[q2_of_q1][:, None, :, :])      # (q1, s, jc, s'')
    V = np.matmul(np.transpose(evec, (0, 2, 1))[:, None, :, :], T)  # (q1, s, s', s'')
    return V, q2_of_q1


def _q2_index(pts, n, N):
    n2 = np.mod(-n[None, :] - pts, N)
    return (n2[:, 0] * N[1] + n2[:, 1]) * N[2] + n2[:, 2]


def crystal_linewidths(model, mesh, omega, evec, vel, T, broadening, q_list=None,
                       stats=None):
    """Gamma [N_q, 3N_b] in rad/ps (rows not in q_list are left NaN).

    broadening: object with shape, adaptive, sigma_thz, sigma_floor_thz, nu_min_thz.
    stats: optional dict, filled with pass counts of the 2-sigma cut.
    """
    pat = Patterns(model)
    pts = mesh_points(mesh)
    N = np.asarray(mesh)
    nq, nb3 = len(pts), pat.nb3
    h2 = mesh_step2(model.lattice, mesh)
    nu = omega / TWO_PI
    phys = nu >= broadening.nu_min_thz
    occ = np.where(phys, bose(np.where(phys, omega, 1.0), T), 0.0)
    sig_fixed = TWO_PI * broadening.sigma_thz
    sig_floor = TWO_PI * broadening.sigma_floor_thz
    out = np.full((nq, nb3), np.nan)
    qs = range(nq) if q_list is None else q_list
    if stats is not None:
        # cand/passed: ordered (q1, s', s'') candidates and passes counted per
        # process over physical modes; blocks/blocks_pass: q1 blocks of a q with
        # any passing pair of any branch.  Per mode (all modes of the listed q,
        # masked ones included): mode_blocks/mode_blocks_pass count (mu, q1)
        # blocks and those with a pair passing in either process,
        # mode_cand/mode_pass the (mu, q1, s', s'') candidates and those
        # passing in either process; mode_phys the physical modes among them.
        stats.update(cand=0, passed=0, blocks=0, blocks_pass=0, mode_blocks=0,
                     mode_blocks_pass=0, mode_cand=0, mode_pass=0, mode_phys=0, n_q=0)
    for q in qs:
        V, q2 = vertex_crystal(model, mesh, evec, q, pat)
        w = omega[q][None, :, None, None]
        w1 = omega[:, None, :, None]
        w2 = omega[q2][:, None, None, :]
        m12 = (phys[:, None, :, None] & phys[q2][:, None, None, :])
        n1 = occ[:, None, :, None]
        n2 = occ[q2][:, None, None, :]
        if broadening.adaptive:
            v1 = vel[:, :, None, :]
            v2 = vel[q2][:, None, :, :]
            sp = adaptive_sigma(v1 + v2, h2, sig_floor)[:, None, :, :]
            sm = adaptive_sigma(-v1 + v2, h2, sig_floor)[:, None, :, :]
        else:
            sp = sm = np.full((1, 1, 1, 1), sig_fixed)
        xp = (w + w1) - w2
        xm = (w - w1) - w2
        gp = smearing(xp, np.broadcast_to(sp, xp.shape), broadening.shape)
        gm = smearing(xm, np.broadcast_to(sm, xm.shape), broadening.shape)
        safe = np.where(m12, w1 * w2, 1.0)
        pop = (n1 - n2) * gp + 0.5 * (n1 + n2 + 1.0) * gm
        with np.errstate(divide="ignore", invalid="ignore"):  # rows of masked modes
            term = np.where(m12, (np.abs(V) ** 2) * pop / (w * safe), 0.0)
            g = PREFACTOR / nq * term.sum(axis=(0, 2, 3))
        g[~phys[q]] = 0.0
        out[q] = g
        if stats is not None:
            passp = (np.abs(xp) < 2.0 * np.broadcast_to(sp, xp.shape)) & m12
            passm = (np.abs(xm) < 2.0 * np.broadcast_to(sm, xm.shape)) & m12
            anyp = (passp | passm) & phys[q][None, :, None, None]
            stats["cand"] += int(m12.sum() * phys[q].sum()) * 2
            stats["passed"] += int((passp & phys[q][None, :, None, None]).sum()
                                   + (passm & phys[q][None, :, None, None]).sum())
            stats["blocks"] += nq
            stats["blocks_pass"] += int(anyp.reshape(nq, -1).any(axis=1).sum())
            stats["mode_blocks"] += nq * nb3
            stats["mode_blocks_pass"] += int(anyp.any(axis=(2, 3)).sum())
            stats["mode_cand"] += nq * nb3 ** 3
            stats["mode_pass"] += int(anyp.sum())
            stats["mode_phys"] += int(phys[q].sum())
            stats["n_q"] += 1
    return out


# --------------------------------------------------------------------------
# Gamma-point (real eigenvectors, all atoms in one cell)
# --------------------------------------------------------------------------

def gamma_tensor_csr(model):
    """Phi3 / sqrt(m m m) as a CSR matrix with rows = first index a and
    columns = (b, c) flattened as b*3N + c."""
    n3 = 3 * model.n_basis
    m = np.repeat(model.mass, 3)
    coef = model.fc3_val / np.sqrt(m[model.fc3_i] * m[model.fc3_j] * m[model.fc3_k])
    return scipy.sparse.csr_matrix(
        (coef, (model.fc3_i, model.fc3_j.astype(np.int64) * n3 + model.fc3_k)),
        shape=(n3, n3 * n3))


def vertex_gamma(model, E, mu, T3=None):
    """V_mu[mu', mu''] = sum_abc Phi3_abc/sqrt(mmm) E_a,mu E_b,mu' E_c,mu''
    = E^T (A_mu E) with A_mu[b, c] = sum_a Phi3_abc E_a,mu / sqrt(mmm)."""
    n3 = E.shape[0]
    T3 = gamma_tensor_csr(model) if T3 is None else T3
    a_row = T3.T @ E[:, mu]                               # (b*n3 + c,)
    A = scipy.sparse.csr_matrix(a_row.reshape(n3, n3))
    W = A @ E
    return E.T @ W


def gamma_point_linewidths(model, omega, E, T, broadening, modes=None):
    """Gamma [3N] (rad/ps) for a Gamma-point solid (N_q = 1); modes not in
    `modes` are left NaN.  Fixed-width smearing (no velocities at one q)."""
    n3 = len(omega)
    T3 = gamma_tensor_csr(model)
    nu = omega / TWO_PI
    phys = nu >= broadening.nu_min_thz
    occ = np.where(phys, bose(np.where(phys, omega, 1.0), T), 0.0)
    sig = TWO_PI * broadening.sigma_thz
    m12 = phys[:, None] & phys[None, :]
    w1 = omega[:, None]
    w2 = omega[None, :]
    n1 = occ[:, None]
    n2 = occ[None, :]
    safe = np.where(m12, w1 * w2, 1.0)
    out = np.full(n3, np.nan)
    for mu in (range(n3) if modes is None else modes):
        if not phys[mu]:
            out[mu] = 0.0
            continue
        V = vertex_gamma(model, E, mu, T3)
        w = omega[mu]
        gp = smearing((w + w1) - w2, sig, broadening.shape)
        gm = smearing((w - w1) - w2, sig, broadening.shape)
        pop = (n1 - n2) * gp + 0.5 * (n1 + n2 + 1.0) * gm
        term = np.where(m12, V * V * pop / (w * safe), 0.0)
        out[mu] = PREFACTOR * term.sum()
    return out
