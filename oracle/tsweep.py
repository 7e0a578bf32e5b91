"""Temperature sweeps from a cached projection (oracle).

The paper separates the temperature-invariant part of the linewidth
calculation from the populations ("Performance and Scalability",
multi-temperature optimisation): the projection of the third-order IFCs on
three phonon modes (Eq. phi3_proj) is computed once and reused for every
temperature.  In Eq. gamma (read as in `oracle.linewidths`) every factor but
the Bose populations of the partners is independent of T: |V|^2, the energy
cut |x| < 2 sigma, the smearing g(x; sigma) (the adaptive widths come from
group velocities) and 1/(w w1 w2).  So per mode mu and ordered partner pair
(m1, m2) = ((q1, s'), (q2, s'')) with both partners physical and at least one
process inside its cut:

    a+ = |V|^2 g(x+; sigma+) / (w w1 w2),   a- = |V|^2 g(x-; sigma-) / (w w1 w2)

and then, for any T,

    Gamma_mu(T) = pi hbar U^3 / (8 N_q) sum [ a+ (n1 - n2) + 1/2 a- (n1 + n2 + 1) ]

with n = n_BE(w, T) (Eq. bose).  Pairs outside both cuts contribute zero at
every T and are not stored.  The cache is a list of rows, one per mode, in
the order (q1, s', s'') of the direct sum.

This is test infrastructure: a plain, slow reference for the GPU library.
"""
from __future__ import annotations

import numpy as np

from .constants import TWO_PI
from .linewidths import (PREFACTOR, Patterns, adaptive_sigma, bose, mesh_step2, smearing,
                         vertex_crystal)
from .phonons import mesh_points


def linewidth_cache(model, mesh, omega, evec, vel, broadening, q_list=None):
    """Temperature-independent factors of Eq. gamma for the modes of the
    listed q (all q by default).

    Returns a dict: row_ptr int64 [n_modes + 1] (rows of modes not listed, or
    below nu_min, are empty), m1, m2 int64 flat partner-mode indices,
    a_plus, a_minus FP64 (the coalescence and decay factors above, each zero
    when its own process fails its cut), and n_q."""
    pat = Patterns(model)
    pts = mesh_points(mesh)
    nq, nb3 = len(pts), pat.nb3
    h2 = mesh_step2(model.lattice, mesh)
    phys = omega / TWO_PI >= broadening.nu_min_thz
    sig_fixed = TWO_PI * broadening.sigma_thz
    sig_floor = TWO_PI * broadening.sigma_floor_thz
    rows = [None] * (nq * nb3)
    qs = range(nq) if q_list is None else q_list
    for q in qs:
        V, q2 = vertex_crystal(model, mesh, evec, q, pat)          # (q1, s, s', s'')
        w = omega[q][None, :, None, None]
        w1 = omega[:, None, :, None]
        w2 = omega[q2][:, None, None, :]
        m12 = phys[:, None, :, None] & phys[q2][:, None, None, :]
        if broadening.adaptive:
            v1 = vel[:, :, None, :]
            v2 = vel[q2][:, None, :, :]
            sp = adaptive_sigma(v1 + v2, h2, sig_floor)[:, None, :, :]
            sm = adaptive_sigma(-v1 + v2, h2, sig_floor)[:, None, :, :]
        else:
            sp = sm = np.full((1, 1, 1, 1), sig_fixed)
        xp = (w + w1) - w2
        xm = (w - w1) - w2
        spb = np.broadcast_to(sp, xp.shape)
        smb = np.broadcast_to(sm, xm.shape)
        keep = m12 & ((np.abs(xp) < 2.0 * spb) | (np.abs(xm) < 2.0 * smb))
        gp = smearing(xp, spb, broadening.shape)
        gm = smearing(xm, smb, broadening.shape)
        safe = np.where(m12, w1 * w2, 1.0)
        with np.errstate(divide="ignore", invalid="ignore"):      # rows of masked modes
            base = np.where(m12, np.abs(V) ** 2 / (w * safe), 0.0)
        ap = base * gp
        am = base * gm
        q1_idx = np.arange(nq)
        for s in range(nb3):
            mu = q * nb3 + s
            if not phys[q, s]:
                rows[mu] = (np.zeros(0, np.int64),) * 2 + (np.zeros(0),) * 2
                continue
            k1, s1, s2 = np.nonzero(keep[:, s, :, :])               # C order: q1, s', s''
            rows[mu] = (q1_idx[k1] * nb3 + s1, q2[k1] * nb3 + s2, ap[k1, s, s1, s2],
                        am[k1, s, s1, s2])
    empty = (np.zeros(0, np.int64),) * 2 + (np.zeros(0),) * 2
    rows = [r if r is not None else empty for r in rows]
    counts = np.array([len(r[0]) for r in rows], np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(counts)])
    cat = [np.concatenate([r[k] for r in rows]) for k in range(4)]
    return dict(row_ptr=row_ptr, m1=cat[0].astype(np.int64), m2=cat[1].astype(np.int64),
                a_plus=cat[2], a_minus=cat[3], n_q=nq)


def gamma_from_cache(cache, omega, T, nu_min_thz):
    """Gamma [N_q, 3N_b] (rad/ps) at temperature T from the cached factors:
    the populations of Eq. bose applied to each stored pair."""
    flat = omega.reshape(-1)
    phys = flat / TWO_PI >= nu_min_thz
    occ = np.where(phys, bose(np.where(phys, flat, 1.0), T), 0.0)
    n1 = occ[cache["m1"]]
    n2 = occ[cache["m2"]]
    term = cache["a_plus"] * (n1 - n2) + 0.5 * cache["a_minus"] * (n1 + n2 + 1.0)
    rp = cache["row_ptr"]
    row = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    g = np.bincount(row, weights=term, minlength=len(rp) - 1)
    g = PREFACTOR / cache["n_q"] * g
    g[~phys] = 0.0
    return g.reshape(omega.shape)


def spontaneous_decay(cache, omega, nu_min_thz):
    """The T -> 0 limit of Eq. gamma: with every population zero only the decay
    term 1/2 a- survives."""
    rp = cache["row_ptr"]
    row = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    g = PREFACTOR / cache["n_q"] * np.bincount(row, weights=0.5 * cache["a_minus"],
                                               minlength=len(rp) - 1)
    g[omega.reshape(-1) / TWO_PI < nu_min_thz] = 0.0
    return g.reshape(omega.shape)
