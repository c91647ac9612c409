"""Parameters of the per-photon physics beyond the core path (setup inputs only).

Defaults: aerosol tau0 = 0.02, Gamma = -1.28 and the micro-roughness halo (f, n, r0) =
(0.135, 3.5, 0.1 deg) are the paper's values (sections 2.3.3 and 2.4.2).  The rest are synthetic
site and hardware values: 30 deg zenith angle, a 2.7 km site (520 mmHg, 8 mmHg water, 12 C),
dome seeing of 0.1 arcsec per axis, a halo truncated at 1 deg, a 50 nm field-free layer, a
four-vane spider holding the secondary of the three-mirror telescope, and the second kick of the
hybrid atmosphere for the synthetic screens (r0 = 0.15 m, L0 = 30 m, the paper's split
kappa_crit = 2 pi / (1.5 r0)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Tuple

from .atmosphere import J_FRACTIONS

# Flag bits of the extra physics (the same bits as the library's PHX_F_* flags).
PHYS_AEROSOL = 1 << 4
PHYS_DISPERSION = 1 << 5
PHYS_DOME = 1 << 6
PHYS_HALO = 1 << 7
PHYS_SPIDER = 1 << 11
PHYS_DEAD_LAYER = 1 << 12
PHYS_SECOND_KICK = 1 << 13
PHYS_FIELD_DIFFUSION = 1 << 14
PHYS_GHOSTS = 1 << 15
PHYS_EXTRA = (PHYS_AEROSOL | PHYS_DISPERSION | PHYS_DOME | PHYS_HALO | PHYS_SPIDER |
              PHYS_DEAD_LAYER)
MAX_LAYERS = 8

ARCSEC = math.radians(1.0 / 3600.0)


@dataclass
class Extras:
    zenith: float = math.radians(30.0)
    zenith_pa: float = math.radians(60.0)
    tau0: float = 0.02
    gamma: float = -1.28
    pressure: float = 520.0          # mmHg
    water: float = 8.0               # mmHg
    temperature: float = 12.0        # deg C
    lam0: float = 600e-9             # refraction of this wavelength is taken out (m)
    dome_sigma: float = 0.1 * ARCSEC
    halo_f: float = 0.135
    halo_n: float = 3.5
    halo_r0: float = math.radians(0.1)
    halo_max: float = math.radians(1.0)
    dead: float = 50e-9              # m
    vanes: int = 4
    vane_angle: float = math.radians(45.0)
    vane_width: float = 0.03
    vane_r_in: float = 1.6
    vane_r_out: float = 4.4
    vane_z_lo: float = 6.45
    vane_z_hi: float = 6.95
    # hybrid atmosphere (second kick): the screens' r0 and L0, the split wavenumber
    # 2 pi / (1.5 r0) of the paper, the finest screen's Nyquist wavenumber (1 cm pixels) and
    # each layer's share of the turbulence integral
    kick_r0: float = 0.15
    kick_L0: float = 30.0
    kick_kappa_crit: float = 2.0 * math.pi / (1.5 * 0.15)
    kick_kappa_max: float = math.pi / 0.01
    kick_fraction: Tuple[float, ...] = field(
        default_factory=lambda: tuple(J_FRACTIONS) + (0.0,) * (MAX_LAYERS - len(J_FRACTIONS)))

    # field model of the diffusion (100 um device at 173 K): 40 V overdepletion, 5e11 cm^-3 bulk
    # doping, 5e13 cm^-3 surface layers 0.5 um deep (the field stays above 2.4e5 V/m), collection
    # 2 um above the front surface
    si_voltage: float = 40.0
    si_n_bulk: float = 5e17
    si_n_back: float = 5e19
    si_s_back: float = 0.5e-6
    si_n_front: float = 5e19
    si_s_front: float = 0.5e-6
    si_z_collect: float = 2e-6

    def replace(self, **kw) -> "Extras":
        return replace(self, **kw)


def tma_extras() -> Extras:
    """Extras for the three-mirror telescope (spider between the secondary and the start plane)."""
    return Extras()


def paraboloid_extras(focal: float = 10.0) -> Extras:
    """Extras for the 1 m paraboloid: a four-vane spider 0.5 m below the start plane."""
    return Extras(vane_width=0.01, vane_r_in=0.0, vane_r_out=0.6,
                  vane_z_lo=focal + 0.5, vane_z_hi=focal + 0.6, vane_angle=0.0)
