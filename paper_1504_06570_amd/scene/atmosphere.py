"""Frozen-flow turbulence screens (setup inputs; section 2.3.1).

OPD screens W (metres of optical path) are synthesised by FFT from the von Karman spectrum
(section 2.3.1, spectrum (k^2 + L0^-2)^-11/6) at several nested pixel scales that tile
periodically (section 2.3.1: screens on several scales, the smaller repeated on the larger).

Readings of the paper used here:
* Phase power spectral density Phi(kappa) = 0.4898 r0^(-5/3) (kappa^2 + kappa0^2)^(-11/6), kappa in
  rad/m, kappa0 = 2 pi / L0.  For L0 -> infinity its structure function is 6.88 (r/r0)^(5/3).
  OPD = phase * lambda_ref / (2 pi) with lambda_ref = 500 nm, so r0 refers to 500 nm.
* Each layer i carries a fraction f_i of the turbulence integral J; since r0^(-5/3) is proportional to
  J, r0_i = f_i^(-3/5) r0.
* Spectral split over scales: scale s with pixel p_s holds the modes kappa_lo(s) <= |kappa| <
  kappa_hi(s); kappa_hi of a coarse scale is half its Nyquist frequency (0.5 pi / p_s), which is
  kappa_lo of the next finer scale; the finest scale goes up to its Nyquist frequency.  The sum over
  scales is the full spectrum on the finest grid (no refractive/diffractive split: the whole
  spectrum is applied refractively).
* Layer heights 0, 0.5, 1, 2, 4, 8, 16 km (section 2.3.1, seven-layer model).  The site's
  measured J percentiles and wind statistics are not available; fractions and winds are
  synthetic (speeds 5 -> 30 m/s linear in layer index, directions uniform from the scene seed).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

LAYER_HEIGHTS = (0.0, 500.0, 1000.0, 2000.0, 4000.0, 8000.0, 16000.0)
J_FRACTIONS = (0.50, 0.10, 0.08, 0.08, 0.08, 0.08, 0.08)
VK_CONST = 0.4898  # = 0.023 (2 pi)^(5/3): phase PSD constant for kappa in rad/m


@dataclass
class Atmosphere:
    heights: np.ndarray           # [L] metres above the M1 vertex
    wind: np.ndarray              # [L, 2] m/s
    pixels: np.ndarray            # [S] metres per screen pixel
    n: int                        # screen side (pixels)
    opd: np.ndarray               # float32 [L, S, n, n], metres
    r0: float = 0.15
    L0: float = 30.0
    lambda_ref: float = 500e-9
    meta: dict = field(default_factory=dict)

    @property
    def n_layers(self) -> int:
        return int(self.opd.shape[0])

    @property
    def n_scales(self) -> int:
        return int(self.opd.shape[1])


def scale_bands(pixels: Sequence[float], n: int):
    """(kappa_lo, kappa_hi) per scale; pixels ordered coarse -> fine."""
    bands = []
    for k, p in enumerate(pixels):
        lo = 0.0 if k == 0 else 0.5 * np.pi / pixels[k - 1]
        hi = np.pi / p if k == len(pixels) - 1 else 0.5 * np.pi / p
        bands.append((lo, hi))
    return bands


def vk_phase_psd(kappa, r0, L0):
    k0 = 0.0 if not np.isfinite(L0) else 2.0 * np.pi / L0
    return VK_CONST * r0 ** (-5.0 / 3.0) * (kappa * kappa + k0 * k0) ** (-11.0 / 6.0)


def opd_screen(rng: np.random.Generator, n: int, pixel: float, r0: float, L0: float,
               band, lambda_ref: float = 500e-9) -> np.ndarray:
    """One periodic OPD screen (float64, metres) holding the modes of ``band``."""
    dk = 2.0 * np.pi / (n * pixel)
    k1 = np.fft.fftfreq(n, d=1.0 / n) * dk
    kx, ky = np.meshgrid(k1, k1, indexing="xy")
    kappa = np.hypot(kx, ky)
    mask = (kappa >= band[0]) & (kappa < band[1]) & (kappa > 0)
    psd = np.zeros_like(kappa)
    psd[mask] = vk_phase_psd(kappa[mask], r0, L0)
    amp = np.sqrt(psd) * dk
    noise = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    # E|c|^2 = 2 Phi dk^2, so the real part alone has the target covariance
    phase = np.fft.ifft2(noise * amp).real * (n * n)
    return phase * (lambda_ref / (2.0 * np.pi))


def make_atmosphere(seed: int, n: int = 2048, pixels=(1.0, 0.1, 0.01), r0: float = 0.15,
                    L0: float = 30.0, heights=LAYER_HEIGHTS, fractions=J_FRACTIONS,
                    speeds=None, lambda_ref: float = 500e-9, kappa_cut=None) -> Atmosphere:
    """kappa_cut: keep only the modes below this wavenumber (rad/m) -- the low-frequency screens
    of the hybrid two-kick atmosphere (section 2.3.2), whose higher modes act through the second
    kick instead.  The random draws are the same as without the cut."""
    rng = np.random.default_rng(seed)
    L = len(heights)
    if speeds is None:
        speeds = np.linspace(5.0, 30.0, L)
    direction = rng.uniform(0.0, 2.0 * np.pi, L)
    wind = np.stack([speeds * np.cos(direction), speeds * np.sin(direction)], axis=1)
    bands = scale_bands(pixels, n)
    if kappa_cut is not None:
        bands = [(lo, min(hi, kappa_cut)) for lo, hi in bands]
    opd = np.empty((L, len(pixels), n, n), dtype=np.float32)
    for i in range(L):
        r0_i = fractions[i] ** (-3.0 / 5.0) * r0
        for s, p in enumerate(pixels):
            opd[i, s] = opd_screen(rng, n, p, r0_i, L0, bands[s], lambda_ref).astype(np.float32)
    return Atmosphere(np.asarray(heights, float), wind, np.asarray(pixels, float), n, opd,
                      r0=r0, L0=L0, lambda_ref=lambda_ref,
                      meta=dict(seed=seed, fractions=list(fractions), bands=bands))


def uniform_gradient_atmosphere(gx: float, gy: float, n: int = 64, pixels=(1.0,),
                                heights=(0.0,), wind=((0.0, 0.0),)) -> Atmosphere:
    """A periodic ramp screen whose centred-difference gradient is (gx, gy) everywhere except
    across its seam, which is placed half a period away from the origin (screen index n/2).
    Photons that stay within |x|, |y| < (n/2 - 2) * pixel never see the seam."""
    L, S = len(heights), len(pixels)
    opd = np.zeros((L, S, n, n), dtype=np.float32)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ii = (i + n // 2) % n
    jj = (j + n // 2) % n
    for s, p in enumerate(pixels):
        opd[:, s] = (gx * p * ii + gy * p * jj).astype(np.float32)
    return Atmosphere(np.asarray(heights, float), np.asarray(wind, float), np.asarray(pixels, float),
                      n, opd, r0=np.inf, L0=np.inf)
