"""The five synthetic workloads and the readings they fix.

Each config names a lattice builder from `synthetic.models`, a Gamma-centred
q-mesh, the temperature and the energy-conservation smearing.  Values the
paper leaves open are fixed here as named constants:

* NU_MIN_THZ = 0.1: modes (and scattering partners) below this cyclic
  frequency get no linewidth and no conductivity share (the paper's
  `min_frequency` selective calculation).
* SIGMA_THZ = 0.1: fixed Gaussian width, cyclic, in THz.
* SIGMA_FLOOR_THZ = 0.01: lower bound of the adaptive width.
* T_KELVIN = 300.
"""
from __future__ import annotations

import dataclasses
from functools import lru_cache

from . import models

NU_MIN_THZ = 0.1
SIGMA_THZ = 0.1
SIGMA_FLOOR_THZ = 0.01
T_KELVIN = 300.0

GAUSS = 0
LORENTZ = 1

# Natural isotope compositions (mass in u, abundance), for the isotope
# scattering inputs: g = sum_iso f (1 - m_iso / m_avg)^2 of each element
# (the mass-variance parameter of the paper's "Isotopic Scattering"; the
# library takes g as an input).
ISOTOPES = {
    "Si": ((27.97692653465, 0.92223), (28.9764946649, 0.04685), (29.973770136, 0.03092)),
    "Pb": ((203.9730440, 0.014), (205.9744657, 0.241), (206.9758973, 0.221),
           (207.9766525, 0.524)),
    "Cs": ((132.905451961, 1.0),),
    "I": ((126.904472, 1.0),),
}


def mass_variance(element: str) -> float:
    iso = ISOTOPES[element]
    m_avg = sum(m * f for m, f in iso) / sum(f for _, f in iso)
    return sum(f * (1.0 - m / m_avg) ** 2 for m, f in iso) / sum(f for _, f in iso)


def natural_g(builder: str):
    """g per basis atom of a model builder's cell with natural compositions:
    the diamond cell is silicon; the perovskite sites A, B, X x 3 are taken as
    Cs, Pb and I (masses 133, 207, 127)."""
    if builder == "diamond":
        return [mass_variance("Si")] * 2
    if builder == "perovskite":
        return [mass_variance("Cs"), mass_variance("Pb")] + [mass_variance("I")] * 3
    raise ValueError(builder)


@dataclasses.dataclass(frozen=True)
class Broadening:
    shape: int = GAUSS
    adaptive: bool = False
    sigma_thz: float = SIGMA_THZ
    sigma_floor_thz: float = SIGMA_FLOOR_THZ
    nu_min_thz: float = NU_MIN_THZ


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    builder: str
    mesh: tuple
    temperature: float
    broadening: Broadening
    description: str


CONFIGS = {
    "C1": Config("C1", "diamond", (5, 5, 5), T_KELVIN, Broadening(adaptive=False),
                 "diamond 2-atom cell, NN springs k2=10 k3=-60, 5x5x5 mesh, "
                 "Gaussian sigma=0.1 THz"),
    "C2": Config("C2", "diamond", (15, 15, 15), T_KELVIN, Broadening(adaptive=True),
                 "diamond 2-atom cell, 15x15x15 mesh (20,250 modes), adaptive Gaussian"),
    "C3": Config("C3", "perovskite", (12, 12, 12), T_KELVIN, Broadening(adaptive=True),
                 "cubic ABX3 5-atom cell, seeded springs, 12x12x12 mesh (25,920 modes), "
                 "adaptive Gaussian"),
    "C4": Config("C4", "glass", (1, 1, 1), T_KELVIN, Broadening(adaptive=False),
                 "512-atom displaced-diamond glass, Gamma point (1,536 modes), "
                 "Gaussian sigma=0.1 THz"),
    "C5": Config("C5", "diamond", (24, 24, 24), T_KELVIN, Broadening(adaptive=True),
                 "diamond 2-atom cell, 24x24x24 mesh (82,944 modes), adaptive Gaussian"),
}


@lru_cache(maxsize=None)
def build_model(builder: str) -> models.Model:
    if builder == "diamond":
        return models.diamond()
    if builder == "perovskite":
        return models.perovskite(0)
    if builder == "glass":
        return models.glass(0)
    if builder == "glass46":
        return models.glass(0, cutoff=4.6)
    raise KeyError(builder)


def model_for(cfg: str | Config) -> models.Model:
    c = CONFIGS[cfg] if isinstance(cfg, str) else cfg
    return build_model(c.builder)
