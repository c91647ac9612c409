"""Source catalogs and spectral energy distributions (setup inputs; section 2.2).

A source is given by the tangent-plane coordinates (xi, eta) of its nominal direction, which are the
paper's n_x, n_y of section 2.2 (n_z = -sqrt(1 - n_x^2 - n_y^2)).  Extended sources are
ellipsoidal Sersic profiles (section 2.2.1) with index n, normalisation b_n, semi-axis scales a, b
(radians, major and minor) and position angle.  With b_n chosen so that P(2n, b_n) = 1/2
(regularised lower incomplete gamma) the scale radius r0 is the half-light radius, and a is the
half-light radius along the major axis.

SEDs: ``sed = -1`` means a top-hat that is flat in photon number per unit wavelength on
[lam_lo, lam_hi] (monochromatic when lam_lo == lam_hi).  ``sed = k >= 0`` selects row k of an
``SEDTable``: f_lambda (energy flux per unit wavelength) per wavelength bin on a shared grid.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

H_PLANCK = 6.62607015e-34
C_LIGHT = 299792458.0
K_BOLTZ = 1.380649e-23


@dataclass
class SEDTable:
    lam_edges: np.ndarray   # [K+1] metres, increasing
    flux: np.ndarray        # [n_sed, K] f_lambda per bin (any units)

    @property
    def n_sed(self) -> int:
        return int(self.flux.shape[0])


@dataclass
class Sources:
    xi: np.ndarray
    eta: np.ndarray
    kind: np.ndarray            # 0 point, 1 Sersic
    sed: np.ndarray             # -1 top-hat, else SEDTable row
    lam_lo: np.ndarray
    lam_hi: np.ndarray
    redshift: np.ndarray
    sersic_n: np.ndarray
    sersic_bn: np.ndarray
    sersic_a: np.ndarray
    sersic_b: np.ndarray
    sersic_pa: np.ndarray
    n_photons: np.ndarray       # uint64

    def __len__(self) -> int:
        return int(self.xi.shape[0])

    @property
    def total_photons(self) -> int:
        return int(self.n_photons.sum())

    def subset(self, idx) -> "Sources":
        return Sources(**{k: getattr(self, k)[idx] for k in self.__dataclass_fields__})


def point_sources(xi, eta, n_photons, lam_lo=320e-9, lam_hi=1080e-9) -> Sources:
    xi = np.atleast_1d(np.asarray(xi, float))
    eta = np.atleast_1d(np.asarray(eta, float))
    m = xi.shape[0]
    z = np.zeros(m)
    return Sources(xi, eta, np.zeros(m, np.int32), -np.ones(m, np.int32),
                   np.full(m, lam_lo), np.full(m, lam_hi), z.copy(), z.copy(), z.copy(),
                   z.copy(), z.copy(), z.copy(),
                   np.broadcast_to(np.asarray(n_photons, np.uint64), (m,)).copy())


def sersic_bn(n):
    """b_n with P(2n, b_n) = 1/2, so that r0 is the half-light radius."""
    from scipy.special import gammaincinv
    return gammaincinv(2.0 * np.asarray(n, float), 0.5)


def blackbody_flambda(lam_mid, T):
    """Planck f_lambda (arbitrary normalisation), lam in metres."""
    x = H_PLANCK * C_LIGHT / (lam_mid * K_BOLTZ * T)
    return lam_mid ** -5 / np.expm1(x)


def blackbody_table(temperatures, lam_lo=320e-9, lam_hi=1080e-9, step=1e-9) -> SEDTable:
    k = int(round((lam_hi - lam_lo) / step))
    edges = lam_lo + step * np.arange(k + 1)
    mid = 0.5 * (edges[:-1] + edges[1:])
    T = np.asarray(temperatures, float)[:, None]
    f = blackbody_flambda(mid[None, :], T)
    f = f / f.max(axis=1, keepdims=True)
    return SEDTable(edges, f)


def power_law_counts(rng: np.random.Generator, m: int, slope: float = -1.5, lo: float = 10.0,
                     hi: float = 1e7) -> np.ndarray:
    """Integer photon counts with dN/dn proportional to n^slope on [lo, hi] (inverse CDF)."""
    a = slope + 1.0
    u = rng.uniform(size=m)
    if abs(a) < 1e-12:
        x = lo * (hi / lo) ** u
    else:
        x = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
    return np.floor(x).astype(np.uint64)
