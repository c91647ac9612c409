"""Synthetic coating tables (setup inputs).

The paper feeds each coated surface a table of transmission probability against incidence angle
and wavelength (section 2.4.2, coating paragraph; Table 1 "coating" row) but publishes none.  The
tables here are smooth synthetic stand-ins with the paper's *shape*: mirrors that keep ~90 % of
the photons, anti-reflection coatings at ~99 %, a band-pass filter whose edges shift blue with
angle, and a detector AR coating.

Table layout (shared with the trace): float32 ``T[coating][k_s][k_lambda]`` on a uniform grid in
s = sin^2(theta_incidence) (``S_MAX``/``N_S``) and wavelength (``LAM0``/``DLAM``/``N_LAM``).  The
grid is uniform in sin^2(theta) because an interference filter's edge shift is linear in it.
"""
from __future__ import annotations

import numpy as np

N_S = 61
S_MAX = 0.3
N_LAM = 801
LAM0 = 300e-9
DLAM = 1e-9

MIRROR, AR, FILTER, DETECTOR_AR = 0, 1, 2, 3


def grid():
    s = np.linspace(0.0, S_MAX, N_S)
    lam = LAM0 + DLAM * np.arange(N_LAM)
    return s, lam


def _mirror(s, lam):
    x = (lam - 700e-9) / 400e-9
    return 0.92 - 0.04 * x * x - 0.03 * s


def _ar(s, lam):
    x = (lam - 700e-9) / 400e-9
    return 0.99 - 0.01 * x * x - 0.02 * s


def _filter(s, lam, lam_c0=625e-9, half=75e-9, edge=4e-9, n_eff=2.0, peak=0.95, leak=1e-4):
    shift = np.sqrt(1.0 - s / (n_eff * n_eff))
    lo = (lam_c0 - half) * shift
    hi = (lam_c0 + half) * shift
    t = peak / ((1.0 + np.exp(-(lam - lo) / edge)) * (1.0 + np.exp((lam - hi) / edge)))
    return t + leak


def _detector_ar(s, lam):
    x = (lam - 700e-9) / 400e-9
    return 0.97 - 0.01 * x * x - 0.03 * s


def standard_tables() -> np.ndarray:
    """Four coatings [MIRROR, AR, FILTER, DETECTOR_AR] as float32 [4][N_S][N_LAM]."""
    s, lam = grid()
    S, L = np.meshgrid(s, lam, indexing="ij")
    out = np.stack([_mirror(S, L), _ar(S, L), _filter(S, L), _detector_ar(S, L)])
    return np.clip(out, 0.0, 1.0).astype(np.float32)


ROLES = {"mirror": MIRROR, "ar": AR, "filter": FILTER, "detector": DETECTOR_AR}

# Share of the photons not transmitted that a coating reflects (ghosts); the rest is absorbed.
# Mirrors: their table is already the reflection probability (no ghost branch).
REFLECT_SHARE = {MIRROR: 0.0, AR: 0.9, FILTER: 0.95, DETECTOR_AR: 0.85}


def standard_reflectance(tables=None) -> np.ndarray:
    """Reflection probabilities R[coating][k_s][k_lambda] for the ghost branch (section 2.4.2: the
    coating description carries reflection and transmission): a fixed share of 1 - T (interference
    filters reflect what they do not pass; anti-reflection coatings reflect most of their small
    loss), float32 on the transmission grid, R <= 1 - T."""
    t = standard_tables() if tables is None else np.asarray(tables, np.float32)
    share = np.array([REFLECT_SHARE[c] for c in range(t.shape[0])], np.float32)
    r = share[:, None, None] * (1.0 - t.astype(np.float64))
    return np.clip(r, 0.0, 1.0 - t).astype(np.float32)
