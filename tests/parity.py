"""GPU-vs-oracle comparison helpers (used by the gpu-marked tests and the smoke check)."""
from __future__ import annotations

import numpy as np

import oracle as O

# A photon whose decision margin (oracle) is below this is a boundary photon: a rounding-level
# difference between the two implementations may flip one of its decisions.
BOUNDARY_MARGIN = 1e-7
POS_TOL = 1e-9          # metres: landing and electron positions


def match(gpu_ev: np.ndarray, orc_ev: np.ndarray):
    """Align both event arrays on (source, photon)."""
    kg = gpu_ev["source"].astype(np.int64) * (1 << 40) + gpu_ev["photon"].astype(np.int64)
    ko = orc_ev["source"].astype(np.int64) * (1 << 40) + orc_ev["photon"].astype(np.int64)
    ig, io = np.argsort(kg), np.argsort(ko)
    g, o = gpu_ev[ig], orc_ev[io]
    assert np.array_equal(kg[ig], ko[io]), "photon sets differ"
    return g, o


def chip_of(scene):
    """(x0, y0, pixel) of a scene's chip, for the pixel-edge rule of compare / images_agree."""
    c = scene.prescription.chip
    return (c.x0, c.y0, c.pixel)


def near_pixel_edge(ev, chip, pos_tol=POS_TOL):
    """Photons whose electron position lies within pos_tol of a pixel edge: positions agree only to
    pos_tol, so their pixel index is not unique."""
    if chip is None:
        return np.zeros(len(ev), bool)
    x0, y0, p = chip
    fx = (ev["xe"] - x0) / p
    fy = (ev["ye"] - y0) / p
    dx = np.abs(fx - np.round(fx)) * p
    dy = np.abs(fy - np.round(fy)) * p
    return (dx < pos_tol) | (dy < pos_tol)


def compare(gpu_ev, orc_ev, pos_tol=POS_TOL, chip=None):
    """Returns a report dict; raises AssertionError on a parity failure.  With the chip geometry,
    detected photons within pos_tol of a pixel edge (oracle position) are compared by position
    only."""
    g, o = match(gpu_ev, orc_ev)
    boundary = o["margin"] < BOUNDARY_MARGIN
    same = g["status"] == o["status"]
    same &= g["surface"] == o["surface"]
    bad = ~same & ~boundary
    assert not bad.any(), (
        f"{bad.sum()} non-boundary status mismatches; first: gpu {g[bad][:3]} oracle {o[bad][:3]}")
    ok = same & ~boundary
    dx = np.abs(g["x"] - o["x"])[ok]
    dy = np.abs(g["y"] - o["y"])[ok]
    conv = ok & (o["status"] <= O.OFF_CHIP)
    dxe = np.abs(g["xe"] - o["xe"])[conv]
    dye = np.abs(g["ye"] - o["ye"])[conv]
    worst = max([0.0] + [float(a.max()) for a in (dx, dy, dxe, dye) if a.size])
    assert worst <= pos_tol, f"position mismatch {worst:.3e} m > {pos_tol:.1e} m"
    det = conv & (o["status"] == O.DETECTED) & ~near_pixel_edge(o, chip, pos_tol)
    assert np.array_equal(g["pix_i"][det], o["pix_i"][det])
    assert np.array_equal(g["pix_j"][det], o["pix_j"][det])
    lam = np.abs(g["lam"] - o["lam"]).max() if len(g) else 0.0
    return dict(n=len(g), boundary=int(boundary.sum()), boundary_frac=float(boundary.mean()) if len(g) else 0.0,
                status_mismatch_boundary=int((~same).sum()), worst_pos=worst, worst_lam=float(lam),
                detected=int((o["status"] == O.DETECTED).sum()))


def image_without_boundary(img: np.ndarray, ev: np.ndarray) -> np.ndarray:
    """Subtract boundary photons' own contributions (detected ones) from an image."""
    out = img.astype(np.int64).copy()
    b = ev[(ev["margin"] < BOUNDARY_MARGIN) & (ev["status"] == O.DETECTED)]
    np.subtract.at(out, (b["pix_j"], b["pix_i"]), 1)
    return out


def images_agree(gpu_img, orc_img, gpu_ev, orc_ev, chip=None):
    """Per-pixel counts equal after removing the boundary photons' contributions from each side
    (each side's own decision for those photons)."""
    g, o = match(gpu_ev, orc_ev)
    boundary = (o["margin"] < BOUNDARY_MARGIN) | near_pixel_edge(o, chip)
    gi = gpu_img.astype(np.int64).copy()
    oi = orc_img.astype(np.int64).copy()
    gb = g[boundary & (g["status"] == O.DETECTED)]
    ob = o[boundary & (o["status"] == O.DETECTED)]
    np.subtract.at(gi, (gb["pix_j"], gb["pix_i"]), 1)
    np.subtract.at(oi, (ob["pix_j"], ob["pix_i"]), 1)
    return np.array_equal(gi, oi)
