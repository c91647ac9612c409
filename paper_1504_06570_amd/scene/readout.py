"""Parameters of the sensor readout chain (setup inputs; section 2.5 electronic readout).

Synthetic values for a 16-amplifier 4k x 4k device (8 x 2 segments of 512 x 2048 pixels): full well
1e5 electrons, 15 s exposure with 0.02 e-/s/pixel dark current, 1e-4 hot and 1e-4 dead pixels,
1e-6 hot-column ends, charge transfer efficiencies 0.999995 (parallel) and 0.999998 (serial),
gains 1.5-1.9 e-/ADU, biases near 1000 ADU and read noise 4.5-6.5 e- varying between amplifiers,
non-linearity 0.02, small bit-error widths on the low bits, 10 overscan rows and columns.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np

MAX_AMPS = 32


def _per_amp(seed, lo, hi):
    rng = np.random.default_rng(seed)
    return tuple(float(v) for v in rng.uniform(lo, hi, MAX_AMPS))


@dataclass
class Readout:
    seed: int = 21
    amp_nx: int = 8
    amp_ny: int = 2
    over_x: int = 10
    over_y: int = 10
    full_well: float = 1e5
    exposure: float = 15.0
    dark_rate: float = 0.02
    hot_fraction: float = 1e-4
    dead_fraction: float = 1e-4
    hot_column_fraction: float = 1e-6
    cte_parallel: float = 0.999995
    cte_serial: float = 0.999998
    nonlinearity: float = 0.02
    gain: Tuple[float, ...] = field(default_factory=lambda: _per_amp(1, 1.5, 1.9))
    bias: Tuple[float, ...] = field(default_factory=lambda: _per_amp(2, 990.0, 1010.0))
    read_noise: Tuple[float, ...] = field(default_factory=lambda: _per_amp(3, 4.5, 6.5))
    bit_sigma: Tuple[float, ...] = (0.02, 0.01, 0.005) + (0.0,) * 13

    def replace(self, **kw) -> "Readout":
        return replace(self, **kw)
