"""FP64 two-phonon joint density of states of the oracle.

The scattering phase space the paper lists among its computed properties
(the phase-space quantity of the "Phonon Properties and Scattering" and
plotting sections; it gives no formula).  Read here as the energy-conserving
partner count of each process with the same smearing, cut, masks and widths
as the linewidths, without the vertex and populations:

    D+(q,s) = (1/N_q) sum_{q1,s',s''} m g((w + w1) - w2; sig+)
    D-(q,s) = (1/N_q) sum_{q1,s',s''} m g((w - w1) - w2; sig-)

with q2 = -q - q1 and m = [nu1 >= nu_min][nu2 >= nu_min]; D = 0 for modes
below nu_min.  Units: ps/rad.

This is test infrastructure.
"""
from __future__ import annotations

import numpy as np

from .constants import TWO_PI
from .linewidths import _q2_index, adaptive_sigma, mesh_step2, smearing
from .phonons import mesh_points


def jdos(model, mesh, omega, vel, broadening, q_list=None):
    """(D+, D-) arrays [N_q, 3N_b]; rows not in q_list are NaN."""
    pts = mesh_points(mesh)
    N = np.asarray(mesh)
    nq, nb3 = omega.shape
    h2 = mesh_step2(model.lattice, mesh)
    nu = omega / TWO_PI
    phys = nu >= broadening.nu_min_thz
    sig_fixed = TWO_PI * broadening.sigma_thz
    sig_floor = TWO_PI * broadening.sigma_floor_thz
    dp = np.full((nq, nb3), np.nan)
    dm = np.full((nq, nb3), np.nan)
    for q in (range(nq) if q_list is None else q_list):
        q2 = _q2_index(pts, pts[q], N)
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
        gp = smearing(xp, np.broadcast_to(sp, xp.shape), broadening.shape)
        gm = smearing(xm, np.broadcast_to(sm, xm.shape), broadening.shape)
        dp[q] = np.where(m12, gp, 0.0).sum(axis=(0, 2, 3)) / nq
        dm[q] = np.where(m12, gm, 0.0).sum(axis=(0, 2, 3)) / nq
        dp[q][~phys[q]] = 0.0
        dm[q][~phys[q]] = 0.0
    return dp, dm
