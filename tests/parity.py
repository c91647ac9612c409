"""GPU-vs-oracle comparison helpers (used by the gpu-marked tests and the smoke check).

The rule (per-photon parity of a Monte Carlo sample path driven by the same random numbers):
  * a *boundary photon* is one whose smallest decision margin in the oracle -- distance of its
    electron position to a pixel edge in pixels, |u - T| of a roulette, the relative distance to
    an aperture edge, to the silicon thickness or to total internal reflection, a rejection
    sampler's acceptance test, the distance of an SED draw's uniform to its bin's edges -- is
    below BOUNDARY_MARGIN; a rounding-level difference between the two implementations may flip
    one of its decisions.  The SED bin choice compares the same uniform with CDF sums that the
    two sides form in the same order, equal to K eps (1.7e-13 for 761 bins), so the oracle
    records its distance scaled by 1e5: the band is 1e-12 there (taken unscaled, 1e-7 of the
    uniform would mark 2e-7 K = 1.5e-4 of the photons of a blackbody source);
  * every other photon has the same status and deciding surface on both sides, its last position
    (and, when converted, its electron position) within the position bar (POS_TOL, wider for a
    photon that the spider's edge diffraction makes sensitive to rounding: position_bar), and
    when detected the same pixel;
  * boundary photons are fewer than 1e-5 of the photons (asserted by the tests);
  * images agree after each side's boundary photons are taken out of its own image.
BOUNDARY_MARGIN = 1e-7 is 1e-12 m at the 10 um pixels of the telescope's chip; the measured
worst position deviation of a converted photon is below 1e-13 m, so no detected photon away from
the boundary band can change pixel.
"""
from __future__ import annotations

import numpy as np

import oracle as O

BOUNDARY_MARGIN = 1e-7
POS_TOL = 1e-9          # metres: landing and electron positions
# A photon whose spider edge diffraction turns it by delta / d per metre of edge distance d
# (oracle event field `cond`) carries a position difference at the vanes, at rounding level, into
# its final position amplified by cond x the path after the spider.  Its position bar is
# UPSTREAM_EPS x SPIDER_PATH x cond when that exceeds POS_TOL: UPSTREAM_EPS is five times the
# largest position difference measured before M1 (1.9e-13 m, photons vignetted at M1 in the
# headline's parity sample; the vanes lie on the same straight path), SPIDER_PATH bounds the lever
# of a turn at
# the spider: the path from the vanes to the detector along the telescope is 25 m (vane tops 6.95 m
# above M1, M1 to M2 and M2 to M3 6.3 m each, M3 to the detector 4.3 m; tested against the
# prescription), and the focal length that carries a turn to the focal plane is 10.3 m.  Its
# status, surface and pixel must still be equal.
UPSTREAM_EPS = 1e-12    # metres
SPIDER_PATH = 30.0      # metres


def position_bar(orc_ev, pos_tol=POS_TOL):
    """Per-photon position bar: pos_tol, or wider for a photon conditioned by the spider."""
    return np.maximum(pos_tol, UPSTREAM_EPS * SPIDER_PATH * orc_ev["cond"])


def match(gpu_ev: np.ndarray, orc_ev: np.ndarray):
    """Align both event arrays on (source, photon)."""
    kg = gpu_ev["source"].astype(np.int64) * (1 << 40) + gpu_ev["photon"].astype(np.int64)
    ko = orc_ev["source"].astype(np.int64) * (1 << 40) + orc_ev["photon"].astype(np.int64)
    ig, io = np.argsort(kg), np.argsort(ko)
    g, o = gpu_ev[ig], orc_ev[io]
    assert np.array_equal(kg[ig], ko[io]), "photon sets differ"
    return g, o


def chip_of(scene):
    """(x0, y0, pixel) of a scene's chip (kept for callers that report pixel geometry)."""
    c = scene.prescription.chip
    return (c.x0, c.y0, c.pixel)


def deviations(g, o):
    """Per photon the largest coordinate difference of the last position and, for converted
    photons, of the electron position (metres); NaN where statuses or surfaces differ."""
    d = np.maximum.reduce([np.abs(g[f] - o[f]) for f in ("x", "y", "z")])
    conv = o["status"] <= O.OFF_CHIP
    de = np.maximum(np.abs(g["xe"] - o["xe"]), np.abs(g["ye"] - o["ye"]))
    d = np.where(conv, np.maximum(d, de), d)
    same = (g["status"] == o["status"]) & (g["surface"] == o["surface"])
    return np.where(same, d, np.nan)


def group_worst(g, o, d, mask):
    """Worst deviation per (status, deciding surface) over the photons in mask, with the photon
    that carries it: {"STATUS@surface": (worst, n, source, photon)}."""
    out = {}
    st, sf = o["status"][mask], o["surface"][mask]
    dm, src, ph = d[mask], o["source"][mask], o["photon"][mask]
    for key in sorted(set(zip(st.tolist(), sf.tolist()))):
        m = (st == key[0]) & (sf == key[1])
        i = int(np.argmax(dm[m]))
        out[f"{O.STATUS[key[0]]}@{key[1]}"] = (float(dm[m][i]), int(m.sum()), int(src[m][i]),
                                               int(ph[m][i]))
    return out


def compare(gpu_ev, orc_ev, pos_tol=POS_TOL, chip=None):
    """Returns a report dict; raises AssertionError on a parity failure (see the module
    docstring).  `chip` is accepted for older callers and not used: pixel edges are part of the
    oracle's decision margin."""
    g, o = match(gpu_ev, orc_ev)
    boundary = o["margin"] < BOUNDARY_MARGIN
    same = (g["status"] == o["status"]) & (g["surface"] == o["surface"])
    bad = ~same & ~boundary
    assert not bad.any(), (
        f"{bad.sum()} non-boundary status mismatches; first: gpu {g[bad][:3]} oracle {o[bad][:3]}")
    ok = same & ~boundary
    d = deviations(g, o)
    groups = group_worst(g, o, d, ok)
    worst = max([0.0] + [v[0] for v in groups.values()])
    conv = ok & (o["status"] <= O.OFF_CHIP)
    worst_conv = float(d[conv].max()) if conv.any() else 0.0
    bar = position_bar(o, pos_tol)
    over = ok & (d > bar)
    if over.any():
        i = int(np.argmax(np.where(over, d / bar, 0.0)))
        raise AssertionError(f"position mismatch {d[i]:.3e} m > {bar[i]:.1e} m at "
                             f"{O.STATUS[o['status'][i]]}@{o['surface'][i]} (source "
                             f"{o['source'][i]}, photon {o['photon'][i]})")
    det = ok & (o["status"] == O.DETECTED)
    flips = det & ((g["pix_i"] != o["pix_i"]) | (g["pix_j"] != o["pix_j"]))
    assert not flips.any(), (f"{flips.sum()} non-boundary detected photons in different pixels; "
                             f"first: gpu {g[flips][:2]} oracle {o[flips][:2]}")
    lam = np.abs(g["lam"] - o["lam"]).max() if len(g) else 0.0
    return dict(n=len(g), boundary=int(boundary.sum()),
                boundary_frac=float(boundary.mean()) if len(g) else 0.0,
                status_mismatch_boundary=int((~same).sum()), worst_pos=worst,
                worst_converted=worst_conv, worst_lam=float(lam),
                widened=int((ok & (bar > pos_tol)).sum()),
                detected=int((o["status"] == O.DETECTED).sum()),
                groups={k: v[0] for k, v in groups.items()},
                worst_photon=(max(groups, key=lambda kk: groups[kk][0]),) + groups[
                    max(groups, key=lambda kk: groups[kk][0])][2:] if groups else None)


def image_without_boundary(img: np.ndarray, ev: np.ndarray) -> np.ndarray:
    """Subtract boundary photons' own contributions (detected ones) from an image."""
    out = img.astype(np.int64).copy()
    b = ev[(ev["margin"] < BOUNDARY_MARGIN) & (ev["status"] == O.DETECTED)]
    np.subtract.at(out, (b["pix_j"], b["pix_i"]), 1)
    return out


def images_agree(gpu_img, orc_img, gpu_ev, orc_ev, chip=None):
    """Per-pixel counts equal after removing the boundary photons' contributions from each side
    (each side's own decision for those photons).  `chip` is not used (see compare)."""
    g, o = match(gpu_ev, orc_ev)
    boundary = o["margin"] < BOUNDARY_MARGIN
    gi = gpu_img.astype(np.int64).copy()
    oi = orc_img.astype(np.int64).copy()
    gb = g[boundary & (g["status"] == O.DETECTED)]
    ob = o[boundary & (o["status"] == O.DETECTED)]
    np.subtract.at(gi, (gb["pix_j"], gb["pix_i"]), 1)
    np.subtract.at(oi, (ob["pix_j"], ob["pix_i"]), 1)
    return np.array_equal(gi, oi)
