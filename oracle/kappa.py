"""FP64 heat capacity and RTA conductivity of the oracle.

Heat capacity, Eq. heatcap: c = k_B x^2 e^x / (e^x - 1)^2, x = hbar w / k_B T.
RTA conductivity, Eq. rta, with the lifetime of Eq. lifetime, tau = 1/(2 Gamma):
    kappa_ab = 1/(N_q V) sum_mu c_mu v_mu,a v_mu,b tau_mu
over modes with nu >= nu_min and Gamma > GAMMA_FLOOR_REL * max(Gamma): a mode
whose linewidth vanishes (no energy-conserving partner, or a vertex that is
zero by symmetry and only rounding noise remains) would otherwise carry an
unbounded lifetime.  Output W/(m K).

This is test infrastructure: a plain reference for the GPU library.
"""
from __future__ import annotations

import numpy as np

from .constants import HBAR, KAPPA_UNIT, KB, TWO_PI

GAMMA_FLOOR_REL = 1e-8


def heat_capacity_kb(omega, T):
    """c / k_B (dimensionless)."""
    x = HBAR * np.asarray(omega, float) / (KB * T)
    return x * x * np.exp(x) / np.expm1(x) ** 2


def kappa_rta(omega, vel, gamma, T, volume, nq, nu_min_thz, gamma_floor_rel=GAMMA_FLOOR_REL):
    """3x3 kappa in W/(m K). omega/gamma (N_q, 3N_b) rad/ps, vel (..., 3) A/ps."""
    om = np.asarray(omega, float).reshape(-1)
    g = np.asarray(gamma, float).reshape(-1)
    v = np.asarray(vel, float).reshape(-1, 3)
    gmax = np.max(g) if g.size else 0.0
    use = (om / TWO_PI >= nu_min_thz) & (g > gamma_floor_rel * gmax) & (g > 0)
    c = np.zeros_like(om)
    c[use] = heat_capacity_kb(om[use], T)
    tau = np.zeros_like(om)
    tau[use] = 1.0 / (2.0 * g[use])
    k = np.einsum("m,ma,mb->ab", c * tau, v, v)
    return KAPPA_UNIT * k / (nq * volume)
