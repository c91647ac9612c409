"""Reference arithmetic of the per-source moments for the tests: the exact integer sums of
quantised electron positions, and the centroids and central second moments as the plain
definition (1/n) sum (x - mean)^2 etc., evaluated exactly in rational arithmetic and rounded once
(the library forms them on the device, phx_moments); the adjoint's cotangent coefficients of a
loss of the moments (d mean/d x_i = 1/n, d Ixx/d x_i = 2 (x_i - mean)/n, d Ixy/d x_i =
(y_i - mean y)/n)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

Q_LOG2 = 44          # positions quantised to x 2^44 (the library's PHX_MOMENT_Q_LOG2)
WORDS = 12


def quantised_sums(xe, ye):
    """(n, SX, SY, SXX, SYY, SXY) of positions given on the host."""
    q = float(1 << Q_LOG2)
    X = [int(v) for v in np.rint(np.asarray(xe, np.float64) * q)]
    Y = [int(v) for v in np.rint(np.asarray(ye, np.float64) * q)]
    return (len(X), sum(X), sum(Y), sum(a * a for a in X), sum(b * b for b in Y),
            sum(a * b for a, b in zip(X, Y)))


def moments_from_sums(sums) -> np.ndarray:
    """Per source (n, mean x, mean y, Ixx, Iyy, Ixy); n = 0 gives a zero row."""
    q = 1 << Q_LOG2
    out = np.zeros((len(sums), 6))
    for i, (n, sx, sy, sxx, syy, sxy) in enumerate(sums):
        if n == 0:
            continue
        out[i] = (n, float(Fraction(sx, n * q)), float(Fraction(sy, n * q)),
                  float(Fraction(n * sxx - sx * sx, n * n * q * q)),
                  float(Fraction(n * syy - sy * sy, n * n * q * q)),
                  float(Fraction(n * sxy - sx * sy, n * n * q * q)))
    return out


def words_of(sums) -> np.ndarray:
    """Moment words [n][12] (int64 storage) holding the given sums (128-bit two's complement)."""
    w = np.zeros((len(sums), WORDS), np.uint64)
    for i, (n, *vals) in enumerate(sums):
        w[i, 0] = n
        for k, v in enumerate(vals):
            v &= (1 << 128) - 1
            w[i, 2 + 2 * k] = v & ((1 << 64) - 1)
            w[i, 3 + 2 * k] = v >> 64
    return w.view(np.int64)


def adjoint_seeds(mom, gout) -> np.ndarray:
    """Cotangent coefficients [n][8] from moments [n][6] and dL/d(mean x, mean y, Ixx, Iyy, Ixy)
    [n][5]: (g0, g1, 2 g2, 2 g3, g4) / n, mean x, mean y, 0; zero rows for n = 0."""
    mom = np.asarray(mom, np.float64)
    g = np.asarray(gout, np.float64)
    out = np.zeros((len(mom), 8))
    n = mom[:, 0]
    ok = n > 0
    inv = np.where(ok, 1.0 / np.where(ok, n, 1.0), 0.0)
    out[:, 0] = g[:, 0] * inv
    out[:, 1] = g[:, 1] * inv
    out[:, 2] = 2.0 * g[:, 2] * inv
    out[:, 3] = 2.0 * g[:, 3] * inv
    out[:, 4] = g[:, 4] * inv
    out[:, 5] = np.where(ok, mom[:, 1], 0.0)
    out[:, 6] = np.where(ok, mom[:, 2], 0.0)
    return out
