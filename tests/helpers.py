"""Small synthetic scenes shared by the oracle pins and the GPU parity tests."""
from __future__ import annotations

import numpy as np

from paper_1504_06570_amd.scene import configs as C
from paper_1504_06570_amd.scene import optics as Op
from paper_1504_06570_amd.scene.atmosphere import uniform_gradient_atmosphere
from paper_1504_06570_amd.scene.sources import point_sources


def flat_detector_scene(n_photons=20000, r_in=0.0, r_out=0.5, lam=500e-9, xi=0.0, eta=0.0,
                        physics=0, coatings=None, det_coating=-1, npix=1000, pixel=1e-3):
    """A single flat detector at z = 0 facing the sky: the landing point is the pupil sample."""
    det = Op.Surface("DET", Op.DETECTOR, 0.0, 0.0, 0.0, (0.0,) * 8, 0.0, 10.0, Op.SILICON,
                     det_coating, 0)
    chip = Op.Chip(0.0, 0.0, pixel=pixel, nx=npix, ny=npix)
    p = Op.Prescription("flat", [det], chip, pupil_r_in=r_in, pupil_r_out=r_out, z_start=1.0,
                        obscuration_z=0.5, obscuration_r=0.0)
    src = point_sources([xi], [eta], n_photons, lam, lam)
    return C.Scene("flat", p, src, coatings, physics=physics, seed=11)


def mirror_chain_scene(n_photons=2000):
    """Paraboloid M1 + two conics whose foci are chained (M2 images the M1 focus onto F2, M3
    images F2 onto F3): a perfect on-axis focus at every pupil radius.  Geometry of the generated
    telescope's first three mirrors."""
    ref = C.telescope(scale=1e-4).prescription
    c1, c2, c3 = (s.curvature for s in ref.surfaces[:3])
    z2, z3 = ref.surfaces[1].z, ref.surfaces[2].z
    # paraxial axis crossings
    y = 1e-3
    m1 = -2 * c1 * y
    F1 = y / (-m1)
    y2 = y + m1 * z2
    m2 = m1 + 2 * c2 * y2
    F2 = z2 + y2 / m2
    y3 = y2 + m2 * (z2 - z3)
    m3 = m2 - 2 * c3 * y3
    F3 = z3 - y3 / m3

    def kappa(p, q):
        e = (p - q) / (p + q)
        return -e * e

    k2 = kappa(-(F1 - z2), z2 - F2)
    k3 = kappa(F2 - z3, F3 - z3)
    surfs = [Op.Surface("M1", Op.MIRROR, 0.0, c1, -1.0, (0.0,) * 8, 2.5, 4.18),
             Op.Surface("M2", Op.MIRROR, z2, c2, k2, (0.0,) * 8, 0.0, 1.7),
             Op.Surface("M3", Op.MIRROR, z3, c3, k3, (0.0,) * 8, 0.0, 2.5),
             Op.Surface("DET", Op.DETECTOR, F3, 0.0, 0.0, (0.0,) * 8, 0.0, 0.5, Op.SILICON)]
    chip = Op.Chip(-0.5e-5, -0.5e-5, pixel=10e-6, nx=64, ny=64)
    p = Op.Prescription("chain", surfs, chip, pupil_r_in=2.5, pupil_r_out=4.18, z_start=z2 + 1.0,
                        obscuration_z=z2, obscuration_r=0.0)
    src = point_sources([0.0], [0.0], n_photons, 600e-9, 600e-9)
    return C.Scene("chain", p, src, physics=0, seed=12), F3


def paraboloid_gradient_scene(gx, gy, lam, n_photons=4000, height=0.0):
    s = C.tiny()
    s.atmosphere = uniform_gradient_atmosphere(gx, gy, n=64, pixels=(1.0,), heights=(height,))
    s.physics = C.PHYS_ATMOSPHERE
    s.sources = point_sources([0.0], [0.0], n_photons, lam, lam)
    s.prescription = s.prescription.replace(chip=Op.Chip(0.0, 0.0, 10e-6, 4096, 4096))
    return s


def plate_scene(thickness, tilt, lam=600e-9, n_photons=200):
    """Plane-parallel fused-silica plate (camera group, tilted by `tilt` about x at its front
    vertex) above a flat detector; vertical light from a tiny pupil."""
    surfs = [Op.Surface("Pa", Op.REFRACT, 1.0, 0.0, 0.0, (0.0,) * 8, 0.0, 0.5, Op.GLASS, -1, 2),
             Op.Surface("Pb", Op.REFRACT, 1.0 - thickness, 0.0, 0.0, (0.0,) * 8, 0.0, 0.5,
                        Op.VACUUM, -1, 2),
             Op.Surface("DET", Op.DETECTOR, 0.0, 0.0, 0.0, (0.0,) * 8, 0.0, 1.0, Op.SILICON)]
    chip = Op.Chip(0.0, 0.0, 1e-5, 1000, 1000)
    p = Op.Prescription("plate", surfs, chip, pupil_r_in=0.0, pupil_r_out=1e-4, z_start=2.0,
                        group_pivot=((0, 0, 0), (0, 0, 0), (0.0, 0.0, 1.0)))
    src = point_sources([0.0], [0.0], n_photons, lam, lam)
    s = C.Scene("plate", p, src, physics=0, seed=13)
    th = np.zeros(C.N_PERTURB)
    th[7] = tilt  # camera tx
    s.perturbation = th
    return s


def fold_scene(D=2.0, delta=0.3, r0=0.5, n_photons=300, physics=0, lam=600e-9):
    """Flat mirror at z = 0 (perturbation group 1, the surface that also carries the Zernike
    terms) reflecting vertical light up to a flat detector at z = D (group 2, pivot a height
    `delta` above its vertex).  At zero perturbation the landing point is the pupil sample, and
    the first derivatives of the landing point have closed forms."""
    m = Op.Surface("FLAT", Op.MIRROR, 0.0, 0.0, 0.0, (0.0,) * 8, 0.0, r0, Op.VACUUM, -1, 1)
    det = Op.Surface("DET", Op.DETECTOR, D, 0.0, 0.0, (0.0,) * 8, 0.0, 2.0, Op.SILICON, -1, 2)
    chip = Op.Chip(0.0, 0.0, pixel=1e-3, nx=1000, ny=1000)
    p = Op.Prescription("fold", [m, det], chip, pupil_r_in=0.0, pupil_r_out=0.9 * r0,
                        z_start=D + 1.0, obscuration_z=0.0, obscuration_r=0.0,
                        group_pivot=((0.0, 0.0, 0.0), (0.0, 0.0, 0.1), (0.0, 0.0, D + delta)))
    src = point_sources([0.0], [0.0], n_photons, lam, lam)
    return C.Scene("fold", p, src, physics=physics, seed=14)


def noll_zernike(j, u, v):
    """Noll-indexed Zernike polynomial from its radial/azimuthal definition (Noll 1976)."""
    from math import factorial
    nm = {4: (2, 0), 5: (2, -2), 6: (2, 2), 7: (3, -1), 8: (3, 1), 9: (3, -3), 10: (3, 3),
          11: (4, 0), 12: (4, 2), 13: (4, -2), 14: (4, 4), 15: (4, -4)}
    n, m = nm[j]
    rho = np.hypot(u, v)
    phi = np.arctan2(v, u)
    ma = abs(m)
    R = sum((-1) ** k * factorial(n - k) / (factorial(k) * factorial((n + ma) // 2 - k) *
                                             factorial((n - ma) // 2 - k)) * rho ** (n - 2 * k)
            for k in range((n - ma) // 2 + 1))
    if m == 0:
        return np.sqrt(n + 1) * R
    ang = np.cos(ma * phi) if m > 0 else np.sin(ma * phi)
    return np.sqrt(2 * (n + 1)) * R * ang


def newton_cycle_scene(n_photons=2000):
    """A surface on which Newton's iteration never converges, for the NONCONV outcome.  Newton on
    G(t) = t^3 - 2t + 2 has the superattracting two-cycle t = 0 <-> 1.  A paraboloid (kappa = -1,
    curvature c) with an r^3 term a3, met by a ray in its x-z plane of slope dz/dx = -1 through
    (x0, 0, z0) of its frame, has f = z - S = z0 - x0 + u - (c/2) u^2 - a3 |u|^3 along the ray
    (u = x, here u < 0); choosing f = K G((u - a)/b) with a = 2^(1/3) b puts the conic root where
    the iteration starts (t = 0).  A flat vacuum window at z = 0 holds a tiny pupil on the axis;
    the surface is decentred by -x0 (group 1) so the light crosses its frame at x0."""
    import math
    b, m, x0 = -0.1, -1.0, -1.0
    a = 2 ** (1 / 3) * b
    K = m * b / (3 * 2 ** (2 / 3) - 2)
    c = 6 * K * a / b ** 3
    a3 = K / b ** 3
    z0 = 2 * K - K * a ** 3 / b ** 3 + 2 * K * a / b + x0 * m
    V = -z0
    win = Op.Surface("WIN", Op.REFRACT, 0.0, 0.0, 0.0, (0.0,) * 8, 0.0, 10.0, Op.VACUUM)
    mir = Op.Surface("NC", Op.MIRROR, V, c, -1.0, (a3,) + (0.0,) * 7, 0.0, 10.0, Op.VACUUM, -1, 1)
    det = Op.Surface("DET", Op.DETECTOR, 5.0, 0.0, 0.0, (0.0,) * 8, 0.0, 100.0, Op.SILICON)
    chip = Op.Chip(0.0, 0.0, 1e-3, 100, 100)
    p = Op.Prescription("newton_cycle", [win, mir, det], chip, pupil_r_in=0.0, pupil_r_out=1e-9,
                        z_start=1.0, obscuration_z=0.0, obscuration_r=0.0,
                        group_pivot=((0, 0, 0), (0.0, 0.0, V), (0, 0, 0)))
    src = point_sources([math.sqrt(0.5)], [0.0], n_photons, 500e-9, 500e-9)
    s = C.Scene("newton_cycle", p, src, physics=0, seed=21)
    th = np.zeros(C.N_PERTURB)
    th[0] = -x0
    s.perturbation = th
    s.meta = dict(a=a, b=b, x0=x0, z0=z0)
    return s
