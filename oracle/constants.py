"""Physical constants and unit conversions of the FP64 oracle (CODATA 2018).

Inputs are eV, Angstrom, amu, K; angular frequencies are rad/ps, velocities
Angstrom/ps, linewidths rad/ps, conductivity W/(m K).
"""
import math

EV_J = 1.602176634e-19          # J per eV (exact)
AMU_KG = 1.66053906660e-27      # kg per amu
HBAR_JS = 1.054571817e-34       # J s
KB_JK = 1.380649e-23            # J/K (exact)

HBAR = HBAR_JS / EV_J * 1e12    # eV ps
KB = KB_JK / EV_J               # eV / K
# 1 eV/(A^2 amu) expressed in ps^-2: turns FC2/mass into omega^2
U = EV_J / (1e-20 * AMU_KG) * 1e-24
TWO_PI = 2.0 * math.pi
# W/(m K) per [k_B * (A/ps)^2 * ps / A^3]
KAPPA_UNIT = KB_JK * (1e2) ** 2 * 1e-12 / 1e-30
