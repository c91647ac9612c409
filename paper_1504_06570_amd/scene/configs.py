"""Synthetic scenes for the five workloads (seeded; setup inputs only).

* ``tiny``:       paraboloid D = 1 m, f = 10 m, one on-axis 500 nm source, 1e5 photons, 64^2 chip,
                  no coatings, no silicon (the landing point is binned).
* ``telescope``:  generated three-mirror anastigmat + camera, 21 x 21 point sources over the square
                  inscribed in the 3.5 deg field, 1e7 photons, flat photon SED 320-1080 nm,
                  coatings, 100 um silicon, diffusion; the 4096^2 chip sits at the field centre.
* ``full``:       ``telescope`` optics + 7 frozen-flow von Karman layers, 1e9 photons from one star
                  at a random field position; the chip is centred on the star's paraxial image.
* ``batched``:    ``full`` stack, 1e4 sources over one chip's sky footprint (80 % stars, 20 %
                  Sersic), power-law photon counts, blackbody SEDs.
* ``gradients``:  ``full`` stack, 25 sources on a 5 x 5 grid, 1e7 photons each, 22 perturbation
                  parameters.

``scale`` shrinks photon counts (and ``screen_n`` the screens) for CPU-sized test cases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import coatings as _coat
from .atmosphere import Atmosphere, make_atmosphere
from .optics import Prescription, paraboloid, paraxial_image, tma_camera
from .physics import Extras
from .sources import (SEDTable, Sources, blackbody_table, point_sources, power_law_counts,
                      sersic_bn)

PHYS_ATMOSPHERE = 1
PHYS_COATINGS = 2
PHYS_SILICON = 4
PHYS_DIFFUSION = 8
PHYS_ALL = PHYS_ATMOSPHERE | PHYS_COATINGS | PHYS_SILICON | PHYS_DIFFUSION

# Perturbation vector layout (22 parameters): M2 (dx, dy, tx, ty, dz), camera (dx, dy, tx, ty, dz),
# M1 Zernike Z4..Z15 (Noll) amplitudes in metres.
N_PERTURB = 22
PERTURB_NAMES = ([f"m2_{k}" for k in ("dx", "dy", "tx", "ty", "dz")] +
                 [f"cam_{k}" for k in ("dx", "dy", "tx", "ty", "dz")] +
                 [f"m1_z{j}" for j in range(4, 16)])
PERTURB_RANGE = np.array([0.5e-3, 0.5e-3, 1e-4, 1e-4, 25e-6] * 2 + [0.5e-6] * 12)

FIELD_HALF_DEG = 1.75
SQUARE_HALF_DEG = FIELD_HALF_DEG / math.sqrt(2.0)


@dataclass
class Scene:
    name: str
    prescription: Prescription
    sources: Sources
    coatings: Optional[np.ndarray] = None         # float32 [n][N_S][N_LAM]
    atmosphere: Optional[Atmosphere] = None
    sed: Optional[SEDTable] = None
    physics: int = 0
    seed: int = 1
    exposure: float = 15.0
    pupil_margin: float = 0.0
    perturbation: np.ndarray = field(default_factory=lambda: np.zeros(N_PERTURB))
    meta: dict = field(default_factory=dict)
    extras: Optional[Extras] = None               # parameters of the PHYS_EXTRA bits
    reflectance: Optional[np.ndarray] = None      # float32 like coatings: ghost reflection


def _coated_tma(chip_center=(0.0, 0.0)):
    return tma_camera(chip_center=chip_center,
                      coatings=dict(mirror=_coat.MIRROR, ar=_coat.AR, filter=_coat.FILTER,
                                    detector=_coat.DETECTOR_AR))


def tiny(scale: float = 1.0) -> Scene:
    src = point_sources([0.0], [0.0], int(round(1e5 * scale)), 500e-9, 500e-9)
    return Scene("tiny", paraboloid(), src, physics=0, seed=1)


def _grid_counts(total: int, m: int) -> np.ndarray:
    base, extra = divmod(total, m)
    return np.array([base + 1] * extra + [base] * (m - extra), np.uint64)


def telescope(scale: float = 1.0) -> Scene:
    t = np.tan(np.radians(np.linspace(-SQUARE_HALF_DEG, SQUARE_HALF_DEG, 21)))
    X, Y = np.meshgrid(t, t, indexing="xy")
    counts = _grid_counts(int(round(1e7 * scale)), 441)
    src = point_sources(X.ravel(), Y.ravel(), counts, 320e-9, 1080e-9)
    return Scene("telescope", _coated_tma(), src, _coat.standard_tables(),
                 physics=PHYS_COATINGS | PHYS_SILICON | PHYS_DIFFUSION, seed=2)


def hybrid(scale: float = 1.0, screen_n: int = 2048, scene_seed: int = 3) -> Scene:
    """``full`` with the hybrid two-kick atmosphere (section 2.3.2): the same screens limited to
    wavenumbers below kappa_crit = 2 pi / (1.5 r0), the modes above it applied as the per-layer
    second kick."""
    from .physics import PHYS_SECOND_KICK, Extras
    s = full(scale, screen_n, scene_seed)
    x = Extras()
    s.atmosphere = make_atmosphere(scene_seed, n=screen_n, kappa_cut=x.kick_kappa_crit)
    s.physics = PHYS_ALL | PHYS_SECOND_KICK
    s.extras = x
    s.name = "hybrid"
    return s


def full(scale: float = 1.0, screen_n: int = 2048, scene_seed: int = 3) -> Scene:
    rng = np.random.default_rng(scene_seed)
    # uniform in the 1.75 deg disc
    r = np.radians(FIELD_HALF_DEG) * math.sqrt(rng.uniform())
    phi = rng.uniform(0.0, 2.0 * np.pi)
    xi, eta = math.tan(r) * math.cos(phi), math.tan(r) * math.sin(phi)
    pres = _coated_tma()
    cx, cy = paraxial_image(pres, xi, eta)
    pres = _coated_tma(chip_center=(cx, cy))
    atm = make_atmosphere(scene_seed, n=screen_n)
    src = point_sources([xi], [eta], int(round(1e9 * scale)), 320e-9, 1080e-9)
    return Scene("full", pres, src, _coat.standard_tables(), atm, physics=PHYS_ALL, seed=3,
                 pupil_margin=0.3, meta=dict(star=(xi, eta)))


def batched(scale: float = 1.0, screen_n: int = 2048, scene_seed: int = 4, n_src: int = 10000,
            slope: float = -1.5) -> Scene:
    rng = np.random.default_rng(scene_seed)
    pres = _coated_tma()
    half = 0.5 * 4096 * 10e-6 / pres.focal_length          # chip half-width on the sky (rad)
    xi = np.tan(rng.uniform(-half, half, n_src))
    eta = np.tan(rng.uniform(-half, half, n_src))
    counts = power_law_counts(rng, n_src, slope=slope)
    if scale != 1.0:
        counts = np.maximum(np.floor(counts * scale), 1).astype(np.uint64)
    temps = np.exp(rng.uniform(np.log(3000.0), np.log(30000.0), n_src))
    sed = blackbody_table(temps)
    src = point_sources(xi, eta, counts)
    src.sed = np.arange(n_src, dtype=np.int32)
    gal = rng.uniform(size=n_src) < 0.2
    n = rng.uniform(0.5, 4.0, n_src)
    arcsec = np.radians(1.0 / 3600.0)
    re = rng.uniform(0.2, 3.0, n_src) * arcsec
    q = rng.uniform(0.3, 1.0, n_src)
    src.kind = gal.astype(np.int32)
    src.sersic_n = np.where(gal, n, 0.0)
    src.sersic_bn = np.where(gal, sersic_bn(np.where(gal, n, 1.0)), 0.0)
    src.sersic_a = np.where(gal, re, 0.0)
    src.sersic_b = np.where(gal, re * q, 0.0)
    src.sersic_pa = np.where(gal, rng.uniform(0.0, np.pi, n_src), 0.0)
    atm = make_atmosphere(scene_seed, n=screen_n)
    return Scene("batched", pres, src, _coat.standard_tables(), atm, sed, physics=PHYS_ALL,
                 seed=4, pupil_margin=0.3)


def gradients(scale: float = 1.0, screen_n: int = 2048, scene_seed: int = 5) -> Scene:
    t = np.tan(np.radians(np.linspace(-SQUARE_HALF_DEG, SQUARE_HALF_DEG, 5)))
    X, Y = np.meshgrid(t, t, indexing="xy")
    src = point_sources(X.ravel(), Y.ravel(), int(round(1e7 * scale)), 320e-9, 1080e-9)
    atm = make_atmosphere(scene_seed, n=screen_n)
    return Scene("gradients", _coated_tma(), src, _coat.standard_tables(), atm,
                 physics=PHYS_ALL, seed=5, pupil_margin=0.3)


CONFIGS = dict(tiny=tiny, telescope=telescope, full=full, batched=batched, gradients=gradients,
               hybrid=hybrid)
