"""Optical prescriptions for the synthetic scenes (setup, not the per-photon trace).

Global frame: z points to the sky, the primary-mirror (M1) vertex sits at the origin,
photons arrive travelling towards -z.  A surface is the set of points

    z = z_vertex + S(r),  S(r) = c r^2 / (1 + sqrt(1 - (1 + kappa) c^2 r^2)) + sum_{i=3..10} alpha_i r^i

which is the conic + polynomial asphere of the paper (section 2.4.1, surface equation) with
c = 1/R.  c > 0 means the surface rises away from the axis (concave as seen from above).

Two prescriptions are provided:

* ``paraboloid(...)``: one paraboloidal mirror (kappa = -1) and a flat detector at its focus.
* ``tma_camera(...)``: a three-mirror anastigmat with the first-order parameters of the paper's
  survey telescope (8.36 m primary, 3.4 m secondary, 5.0 m tertiary, f/1.234, 3.5 deg field),
  three fused-silica lenses and a filter.  The paper deliberately does not publish the
  telescope's design (section 4), so the layout is *generated* here: a paraxial (first-order)
  solve of curvatures and spacings, Seidel third-order conditions for the three mirror conics,
  a field-flattening lens for the Petzval sum, and an exact re-expression of each mirror conic as a
  different base conic plus alpha_4, alpha_6, alpha_8 terms (so the even-asphere code path is
  exercised without degrading the design).  This module uses textbook paraxial/Seidel optics
  only; it does not trace real rays.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

MIRROR = 0
REFRACT = 1
DETECTOR = 2

VACUUM = 0
GLASS = 1
SILICON = 2

# Fused silica, Malitson (1965) Sellmeier coefficients (lambda in micrometres).  The paper gives the
# Sellmeier form (section 2.4.1) but no glass data.
SILICA_B = (0.6961663, 0.4079426, 0.8974794)
SILICA_C_UM2 = (0.0684043 ** 2, 0.1162414 ** 2, 9.896161 ** 2)


def silica_index(lam_m: float) -> float:
    """Design-time index (first-order layout only; the trace evaluates its own)."""
    l2 = (lam_m * 1e6) ** 2
    s = 1.0
    for b, c in zip(SILICA_B, SILICA_C_UM2):
        s += b * l2 / (l2 - c)
    return math.sqrt(s)


@dataclass
class Surface:
    name: str
    kind: int
    z: float
    curvature: float = 0.0
    conic: float = 0.0
    alpha: Tuple[float, ...] = (0.0,) * 8      # alpha_3 .. alpha_10
    r_in: float = 0.0
    r_out: float = 1.0
    medium: int = VACUUM                        # medium after the surface (in travel order)
    coating: int = -1                           # coating table index, -1 = none
    group: int = 0                              # rigid-body perturbation group (0 = none)


@dataclass
class Chip:
    """A rectangular device on the detector surface (section 2.4.1; paper Table 1)."""
    center_x: float
    center_y: float
    pixel: float = 10e-6
    nx: int = 4096
    ny: int = 4096

    @property
    def x0(self) -> float:
        return self.center_x - 0.5 * self.nx * self.pixel

    @property
    def y0(self) -> float:
        return self.center_y - 0.5 * self.ny * self.pixel


@dataclass
class Silicon:
    thickness: float = 100e-6      # t_Si (m)
    temperature: float = 173.0     # device temperature (K)
    sigma_max: float = 4e-6        # diffusion sigma for a conversion at the entrance surface (m)


@dataclass
class Prescription:
    name: str
    surfaces: List[Surface]
    chip: Chip
    silicon: Silicon = field(default_factory=Silicon)
    pupil_r_in: float = 0.0          # sampling annulus on M1 (section 2.2)
    pupil_r_out: float = 0.5
    z_start: float = 11.0            # plane above every optic where the optics trace starts
    obscuration_z: float = 0.0       # plane of the central obscuration disk (M2 shadow)
    obscuration_r: float = 0.0       # 0 = no obscuration
    glass_b: Tuple[float, float, float] = SILICA_B
    glass_c_um2: Tuple[float, float, float] = SILICA_C_UM2
    group_pivot: Tuple[Tuple[float, float, float], ...] = ((0.0, 0.0, 0.0),) * 3
    focal_length: float = 0.0        # paraxial effective focal length (m), informational
    notes: dict = field(default_factory=dict)

    def replace(self, **kw) -> "Prescription":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------------------------
# Config "plain method, tiny": one paraboloid, detector at its focus.
# ----------------------------------------------------------------------------------------------
def paraboloid(diameter: float = 1.0, focal: float = 10.0, npix: int = 64,
               pixel: float = 10e-6) -> Prescription:
    """Paraboloid mirror (R = 2f, kappa = -1) with a flat detector at z = f.

    The optical axis goes through the centre of pixel (npix/2, npix/2), so that the perfect focus
    is not on a pixel corner: x0 = y0 = -(npix/2 + 1/2) * pixel.
    """
    m1 = Surface("M1", MIRROR, z=0.0, curvature=1.0 / (2.0 * focal), conic=-1.0,
                 r_in=0.0, r_out=0.5 * diameter, medium=VACUUM)
    det = Surface("DET", DETECTOR, z=focal, curvature=0.0, r_in=0.0, r_out=0.05,
                  medium=SILICON)
    half = npix // 2
    chip = Chip(center_x=-(half + 0.5) * pixel + 0.5 * npix * pixel,
                center_y=-(half + 0.5) * pixel + 0.5 * npix * pixel,
                pixel=pixel, nx=npix, ny=npix)
    return Prescription("paraboloid", [m1, det], chip,
                        pupil_r_in=0.0, pupil_r_out=0.5 * diameter,
                        z_start=focal + 1.0, obscuration_z=focal, obscuration_r=0.0,
                        focal_length=focal)


# ----------------------------------------------------------------------------------------------
# Paraxial y-nu trace and Seidel sums in the sequential ("unfolded") convention: axis along the
# initial travel direction (downwards, z_W = -z), curvature positive when the centre of curvature
# lies downstream, refractive index negative after an odd number of reflections, refraction
# n'u' = n u - h c (n' - n), transfer h_next = h + d u'.
# ----------------------------------------------------------------------------------------------
def _paraxial(seq, h0, u0):
    """seq: list of (c_W, n, n_next, d_to_next).  Returns per-surface (h, u_in, u_out)."""
    h, u = h0, u0
    out = []
    for c, n, n2, d in seq:
        u2 = (n * u - h * c * (n2 - n)) / n2
        out.append((h, u, u2))
        h = h + d * u2
        u = u2
    return out, h, u


def _seidel(seq, conics, marg, chief):
    """Third-order sums S_I, S_II, S_III, S_IV (Welford's forms, aspheric conic terms added)."""
    (hm0, um0), (hc0, uc0) = marg, chief
    pm, _, _ = _paraxial(seq, hm0, um0)
    pc, _, _ = _paraxial(seq, hc0, uc0)
    lag = None
    S = np.zeros(4)
    for k, ((c, n, n2, d), (h, u, u2), (hb, ub, ub2)) in enumerate(zip(seq, pm, pc)):
        if lag is None:
            lag = n * (ub * h - u * hb)
        A = n * (u + h * c)
        Ab = n * (ub + hb * c)
        du = u2 / n2 - u / n
        kap = conics[k]
        asp = kap * c ** 3 * (n2 - n) * h ** 4
        S[0] += -A * A * h * du + asp
        S[1] += -A * Ab * h * du + (asp * hb / h if h != 0 else 0.0)
        S[2] += -Ab * Ab * h * du + (asp * (hb / h) ** 2 if h != 0 else 0.0)
        S[3] += -lag * lag * c * (1.0 / n2 - 1.0 / n)
    return S


def tma_camera(chip_center: Tuple[float, float] = (0.0, 0.0),
               coatings: Optional[dict] = None) -> Prescription:
    """The generated three-mirror anastigmat + camera, loaded from ``tma_camera.json`` (written by
    ``tma_design.py``).

    coatings: mapping surface role -> coating table index, roles 'mirror', 'ar', 'filter',
    'detector'.
    """
    with open(os.path.join(os.path.dirname(__file__), "tma_camera.json")) as f:
        d = json.load(f)
    cm = coatings or {}
    surfaces = []
    for s in d["surfaces"]:
        role = s["role"]
        surfaces.append(Surface(s["name"], s["kind"], s["z"], s["curvature"], s["conic"],
                                tuple(s["alpha"]), s["r_in"], s["r_out"], s["medium"],
                                cm.get(role, -1), s["group"]))
    chip = Chip(center_x=chip_center[0], center_y=chip_center[1])
    return Prescription("tma_camera", surfaces, chip, pupil_r_in=d["pupil_r_in"],
                        pupil_r_out=d["pupil_r_out"], z_start=d["z_start"],
                        obscuration_z=d["obscuration_z"], obscuration_r=d["obscuration_r"],
                        group_pivot=tuple(tuple(p) for p in d["group_pivot"]),
                        focal_length=d["focal_length"], notes=d.get("notes", {}))


def paraxial_sequence(p: Prescription, lam: float = 600e-9):
    """Unfolded paraxial sequence of every surface before the detector, plus the detector's
    distance from the last surface (used for chip placement only)."""
    seq = []
    n = 1.0
    surfs = p.surfaces
    for k, s in enumerate(surfs[:-1]):
        if s.kind == MIRROR:
            n2 = -n
        else:
            mag = silica_index(lam) if s.medium == GLASS else 1.0
            n2 = mag if n > 0 else -mag
        znext = surfs[k + 1].z
        seq.append((-s.curvature, n, n2, -(znext - s.z)))
        n = n2
    return seq


def paraxial_image(p: Prescription, xi: float, eta: float, lam: float = 600e-9):
    """Paraxial chief-ray image of a source at tangent coordinates (xi, eta) on the detector
    (stop at the first surface).  Setup-only: used to centre a chip on a star."""
    seq = paraxial_sequence(p, lam)
    nz = np.sqrt(1.0 - xi * xi - eta * eta)
    _, hx, _ = _paraxial(seq, 0.0, xi / nz)
    _, hy, _ = _paraxial(seq, 0.0, eta / nz)
    return float(hx), float(hy)
