"""FP64 full scattering matrix of the linearised BTE, its self-consistent
iteration and its direct inversion (oracle).

TEST INFRASTRUCTURE ONLY: a plain reference for the GPU library.

Paper, "Boltzmann Transport Equation": the scattering matrix splits into a
diagonal part Gamma0 (Eq. BTE: the sum of the process rates) and an
off-diagonal coupling Gamma1 (Eq. gamma1); the mean free paths solve
v = (diag(Gamma0) + Gamma1) lambda (Eq. invBTE) and
kappa_ab = 1/(N_q V) sum c v_a lambda_b (Eq. kappa_general); lambda comes from
the self-consistent iteration (Eq. sc_iter) or from the inverse of the
matrix (Eq. inverse); with Gamma1 = 0 it is the RTA (Eq. rta).

Reading (the printed Eq. gamma1 lists four rates with one sign and no
frequency factors, which cannot reduce to the iteration the paper cites):
the rows follow the iterative scheme that Eq. sc_iter writes, in the form of
the adaptive-smearing reference the paper cites for its broadening.  For one
ordered candidate (q s; q1 s'; q2 s''), q + q1 + q2 = G, with
    d+ = 2 P |V|^2 (n1 - n2) g(x+) / (w w1 w2)          (coalescence)
    d- = 2 P |V|^2 1/2 (n1 + n2 + 1) g(x-) / (w w1 w2)   (decay)
(P = pi hbar U^3 / (8 N_q), the masks, cut and widths of the linewidths),
row mu = (q, s) receives
    Gamma0_mu        += d+ + d-            (so Gamma0 = 2 Gamma = 1/tau)
    Gamma1[mu, (q1, s')]  += d+ w1/w        (absorbed partner)
    Gamma1[mu, tr(q1, s')]  -= d- w1/w        (decay product)
    Gamma1[mu, tr(q2, s'')] -= (d+ + d-) w2/w (outgoing partner of both)
The physical partner phonons of the processes are at q1 (absorbed) and at
-q1, -q2 (emitted).  The vertex holds the eigenvector of q2; the emitted
phonon is the mode at -q2 whose eigenvector is its complex conjugate (time
reversal, D(-q) = D(q)*).  The column of an emitted partner (q', s') is
therefore its time-reversal partner tr(q', s') = (-q', t), t maximising
|sum_i eta_i(-q', t) eta_i(q', s')| (the overlap of eta(-q', t) with
eta(q', s')*): the same branch for a non-degenerate mode, the conjugate
vector's place inside a degenerate cluster (whose basis at -q' may list the
conjugate vectors in another order).  Modes that carry no conductivity in the RTA
(nu < nu_min, or Gamma not above 1e-8 max Gamma) are decoupled: their rows
and columns are dropped (lambda = 0).

The symmetric form: D Gamma~ D^-1 with D_mu = sqrt(n (n + 1)) w_mu (the
square root of the heat capacity, up to a constant) is symmetric when every
process conserves energy exactly (detailed balance); with a smeared delta
its antisymmetric part is of the order of the energy mismatch over k_B T.
"""
from __future__ import annotations

import numpy as np

from .constants import KAPPA_UNIT, TWO_PI
from .kappa import GAMMA_FLOOR_REL, heat_capacity_kb
from .linewidths import (PREFACTOR, Patterns, _q2_index, adaptive_sigma, bose, mesh_step2,
                         smearing, vertex_crystal)
from .phonons import mesh_points


def minus_index(mesh):
    """Flat index of -q for every mesh point q."""
    pts = mesh_points(mesh)
    N = np.asarray(mesh)
    m = np.mod(-pts, N)
    return (m[:, 0] * N[1] + m[:, 1]) * N[2] + m[:, 2]


def time_reversal_partner(mesh, evec):
    """tr[mode] = flat index of the mode at -q whose eigenvector is closest to
    the complex conjugate of this mode's (largest |overlap|, first on ties)."""
    nq, nb3, _ = evec.shape
    mq = minus_index(mesh)
    tr = np.empty(nq * nb3, dtype=np.int64)
    for q in range(nq):
        O = np.abs(evec[mq[q]].T @ evec[q])       # O[t, s] = |sum_i eta_i(-q, t) eta_i(q, s)|
        tr[q * nb3:(q + 1) * nb3] = mq[q] * nb3 + np.argmax(O, axis=0)
    return tr


class _Setup:
    """Per-call tables shared by the rows of one scattering matrix."""

    def __init__(self, model, mesh, omega, evec, T, broadening):
        self.pat = Patterns(model)
        self.nq, self.nb3 = omega.shape
        self.h2 = mesh_step2(model.lattice, mesh)
        nu = omega / TWO_PI
        self.phys = nu >= broadening.nu_min_thz
        self.occ = np.where(self.phys, bose(np.where(self.phys, omega, 1.0), T), 0.0)
        self.tr = time_reversal_partner(mesh, evec).reshape(self.nq, self.nb3)


def scattering_rows(model, mesh, omega, evec, vel, T, broadening, q, setup=None):
    """Rows (q, s) of the scattering matrix: (Gamma0 [3N_b], Gamma1 [3N_b, n])."""
    st = setup or _Setup(model, mesh, omega, evec, T, broadening)
    nq, nb3, phys, occ, tr = st.nq, st.nb3, st.phys, st.occ, st.tr
    n = nq * nb3
    g0 = np.zeros(nb3)
    g1 = np.zeros((nb3, n))
    if not phys[q].any():
        return g0, g1
    sig_fixed = TWO_PI * broadening.sigma_thz
    sig_floor = TWO_PI * broadening.sigma_floor_thz
    pref = 2.0 * PREFACTOR / nq
    b = np.arange(nb3)
    V, q2 = vertex_crystal(model, mesh, evec, q, st.pat)
    w = omega[q][None, :, None, None]
    w1 = omega[:, None, :, None]
    w2 = omega[q2][:, None, None, :]
    m12 = phys[:, None, :, None] & phys[q2][:, None, None, :] & phys[q][None, :, None, None]
    n1 = occ[:, None, :, None]
    n2 = occ[q2][:, None, None, :]
    if broadening.adaptive:
        v1 = vel[:, :, None, :]
        v2 = vel[q2][:, None, :, :]
        sp = adaptive_sigma(v1 + v2, st.h2, sig_floor)[:, None, :, :]
        sm = adaptive_sigma(-v1 + v2, st.h2, sig_floor)[:, None, :, :]
    else:
        sp = sm = np.full((1, 1, 1, 1), sig_fixed)
    gp = smearing((w + w1) - w2, np.broadcast_to(sp, V.shape), broadening.shape)
    gm = smearing((w - w1) - w2, np.broadcast_to(sm, V.shape), broadening.shape)
    safe_w = np.where(m12, w, 1.0)
    safe = np.where(m12, safe_w * (w1 * w2), 1.0)
    a2 = np.where(m12, np.abs(V) ** 2 / safe, 0.0)
    dp = pref * a2 * (n1 - n2) * gp                  # (q1, s, s', s'')
    dm = pref * a2 * 0.5 * (n1 + n2 + 1.0) * gm
    g0[:] = (dp + dm).sum(axis=(0, 2, 3))
    r1 = w1 / safe_w                                 # w1 / w
    r2 = w2 / safe_w                                 # w2 / w
    # columns: (q1, s'), tr(q1, s'), tr(q2, s'')
    col1 = (np.arange(nq)[:, None] * nb3 + b[None, :])            # (q1, s')
    colm1 = tr                                                    # tr(q1, s')
    colm2 = tr[q2]                                                # tr(q2, s'')
    absorbed = (dp * r1).sum(axis=3)                              # (q1, s, s')
    emitted1 = (dm * r1).sum(axis=3)                              # (q1, s, s')
    emitted2 = ((dp + dm) * r2).sum(axis=2)                       # (q1, s, s'')
    for s in range(nb3):
        np.add.at(g1[s], col1.reshape(-1), absorbed[:, s, :].reshape(-1))
        np.add.at(g1[s], colm1.reshape(-1), -emitted1[:, s, :].reshape(-1))
        np.add.at(g1[s], colm2.reshape(-1), -emitted2[:, s, :].reshape(-1))
    return g0, g1


def scattering_matrix(model, mesh, omega, evec, vel, T, broadening, q_list=None):
    """(Gamma0 [n], Gamma1 [n, n]) over all n = N_q 3N_b modes (rad/ps); with
    q_list only the rows of those q-points are filled."""
    st = _Setup(model, mesh, omega, evec, T, broadening)
    nq, nb3 = st.nq, st.nb3
    g0 = np.zeros(nq * nb3)
    g1 = np.zeros((nq * nb3, nq * nb3))
    for q in (range(nq) if q_list is None else q_list):
        r0, r1 = scattering_rows(model, mesh, omega, evec, vel, T, broadening, q, st)
        g0[q * nb3:(q + 1) * nb3] = r0
        g1[q * nb3:(q + 1) * nb3] = r1
    return g0, g1


def active_modes(omega, g0, nu_min_thz, gamma_floor_rel=GAMMA_FLOOR_REL):
    """Modes that carry conductivity: nu >= nu_min and Gamma0 above the floor
    (the same selection as the RTA conductivity, Gamma0 = 2 Gamma)."""
    om = np.asarray(omega, float).reshape(-1)
    gmax = np.max(g0) if g0.size else 0.0
    return (om / TWO_PI >= nu_min_thz) & (g0 > gamma_floor_rel * gmax) & (g0 > 0)


def kappa_from_lambda(omega, vel, lam, T, volume, nq, act):
    """Eq. kappa_general: 1/(N_q V) sum_mu c_mu v_mu,a lambda_mu,b (W/(m K))."""
    om = np.asarray(omega, float).reshape(-1)
    v = np.asarray(vel, float).reshape(-1, 3)
    c = np.zeros_like(om)
    c[act] = heat_capacity_kb(om[act], T)
    k = np.einsum("m,ma,mb->ab", c, v, lam)
    return KAPPA_UNIT * k / (nq * volume)


def solve_inverse(g0, g1, vel, act):
    """Eq. inverse: lambda = Gamma~^-1 v on the active modes (0 elsewhere)."""
    v = np.asarray(vel, float).reshape(-1, 3)
    idx = np.flatnonzero(act)
    A = g1[np.ix_(idx, idx)] + np.diag(g0[idx])
    lam = np.zeros_like(v)
    lam[idx] = np.linalg.solve(A, v[idx])
    return lam


def solve_sc(g0, g1, vel, act, omega, T, volume, nq, n_iterations=200, tolerance=1e-12):
    """Eq. sc_iter from the RTA start lambda0 = v / Gamma0, stopped when the
    relative change of Tr(kappa)/3 falls below `tolerance` or after
    `n_iterations` updates.  Returns (lambda, kappa, iterations)."""
    v = np.asarray(vel, float).reshape(-1, 3)
    idx = np.flatnonzero(act)
    G1 = g1[np.ix_(idx, idx)]
    d = g0[idx][:, None]
    lam_a = v[idx] / d
    lam = np.zeros_like(v)
    lam[idx] = lam_a
    kap = kappa_from_lambda(omega, vel, lam, T, volume, nq, act)
    it = 0
    for it in range(1, n_iterations + 1):
        lam_a = v[idx] / d - (G1 @ lam_a) / d
        lam[idx] = lam_a
        k_new = kappa_from_lambda(omega, vel, lam, T, volume, nq, act)
        k0, k1 = np.trace(kap) / 3, np.trace(k_new) / 3
        kap = k_new
        if abs(k1 - k0) <= tolerance * abs(k0):
            break
    return lam, kap, it
