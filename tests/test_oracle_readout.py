"""Pins of the oracle's sensor readout chain (section 2.4.3 saturation and bleeding, section 2.5
electronic readout) against conservation laws, exact laws of the random draws and closed forms
(no GPU)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_1504_06570_amd.scene.readout import Readout


@pytest.fixture(scope="module", autouse=True)
def _build_oracle():
    O.build()


def _quiet(**kw):
    """A readout with every random effect off: no dark current, defects, transfer losses, read
    noise, non-linearity or bit errors; gain 1, bias 0."""
    base = dict(amp_nx=2, amp_ny=2, over_x=4, over_y=4, dark_rate=0.0, hot_fraction=0.0,
                dead_fraction=0.0, hot_column_fraction=0.0, cte_parallel=1.0, cte_serial=1.0,
                nonlinearity=0.0, gain=(1.0,) * 32, bias=(0.0,) * 32, read_noise=(0.0,) * 32,
                bit_sigma=(0.0,) * 16, full_well=1000.0)
    base.update(kw)
    return Readout(**base)


def test_bleeding_conserves_charge_up_to_full_half_rows():
    """Every half-row keeps min(its charge, n w), no pixel exceeds w, and nothing crosses the
    implant at the middle of the row."""
    rp = _quiet()
    rng = np.random.default_rng(0)
    img = rng.integers(0, 900, (16, 64)).astype(np.uint32)
    img[3, 10] = 20000
    img[5, 31] = 80000          # next to the implant, saturating its whole half-row
    img[7, 40:44] = 5000
    out = O.bleed(rp, img)
    w, h = 1000, 32
    assert out.max() <= w
    for j in range(16):
        for a, b in ((0, h), (h, 64)):
            want = min(int(img[j, a:b].astype(np.int64).sum()), (b - a) * w)
            assert int(out[j, a:b].astype(np.int64).sum()) == want
    assert np.all(out[5, :32] == w) and np.array_equal(out[5, 32:], img[5, 32:])


def test_bleeding_of_one_pixel_spreads_symmetrically():
    """One pixel with excess 4 w in an empty row fills the closest pixels on both sides in turn
    (ties toward the row's end): the pixels p-2 .. p+2 end full, the rest empty."""
    rp = _quiet()
    img = np.zeros((1, 64), np.uint32)
    img[0, 12] = 5000
    out = O.bleed(rp, img)
    assert np.array_equal(np.nonzero(out[0])[0], np.arange(10, 15))
    assert np.all(out[0, 10:15] == 1000)
    img[0, 12] = 4000      # excess 3 w: the tie at distance 2 goes toward the row's end (left)
    out = O.bleed(rp, img)
    assert np.array_equal(np.nonzero(out[0])[0], np.arange(10, 14))


def test_dark_current_has_mean_and_variance_rate_times_exposure():
    """Dark electrons per pixel: normal with mean and variance mu = rate x exposure, rounded
    (mean mu, variance mu + 1/12 within 5 sigma)."""
    rp = _quiet(dark_rate=2.0, exposure=15.0)
    img = np.zeros((128, 128), np.uint32)
    _, _, work, _, _ = O.readout(rp, img)
    d = work.astype(np.float64).ravel()
    n, mu = d.size, 30.0
    assert abs(d.mean() - mu) < 5 * math.sqrt(mu / n)
    assert abs(d.var() - (mu + 1 / 12)) < 5 * mu * math.sqrt(2.0 / n)


def test_hot_dead_pixels_and_hot_columns():
    """Hot pixels (set to w) and dead pixels (emptied) in their fractions (binomial, 5 sigma);
    every pixel behind a hot-column end in its segment column is at w, and the chance that a
    segment column holds no end is (1 - f)^sh."""
    rp = _quiet(hot_fraction=0.01, dead_fraction=0.02)
    img = np.full((128, 128), 10, np.uint32)
    _, _, work, _, _ = O.readout(rp, img)
    n = img.size
    for val, f in ((1000, 0.01), (0, 0.02)):
        k = (work == val).sum()
        assert abs(k - n * f) < 5 * math.sqrt(n * f * (1 - f))
    f = 0.005
    rp = _quiet(hot_column_fraction=f)
    _, _, work, _, _ = O.readout(rp, img)
    sh = 64
    clean = 0
    for half, rows in ((0, np.arange(0, 64)), (1, np.arange(127, 63, -1))):
        seg = work[rows]                         # rows ordered away from the register
        hot = seg == 1000
        # once hot, stays hot along the readout chain
        assert np.all(np.diff(hot.astype(int), axis=0) >= 0)
        clean += (~hot.any(axis=0)).sum()
    p = (1 - f) ** sh
    m = 2 * 128
    assert abs(clean - m * p) < 5 * math.sqrt(m * p * (1 - p))


def test_parallel_transfer_trail_is_negative_binomial():
    """A single pixel of n electrons at parallel index r, transfer inefficiency eps: the counts in
    slots r + f follow the negative binomial law of failures before r + 1 successes (chi-square
    over f = 0, 1, 2, >= 3), and no electron is lost with enough overscan."""
    eps, r, n = 2e-3, 40, 200000
    rp = _quiet(cte_parallel=1.0 - eps, full_well=1e9, over_y=20, amp_nx=1, amp_ny=1)
    img = np.zeros((64, 8), np.uint32)
    img[r, 3] = n
    _, _, work, par, ser = O.readout(rp, img)
    col = par[0, :, 3].astype(np.int64)
    assert col.sum() == n and col[:r].sum() == 0
    pmf = stats.nbinom.pmf(np.arange(3), r + 1, 1 - eps)
    exp_ = n * np.append(pmf, 1 - pmf.sum())
    obs = np.append(col[r:r + 3], col[r + 3:].sum())
    assert ((obs - exp_) ** 2 / exp_).sum() < stats.chi2.ppf(1 - 1e-4, 3)
    assert np.array_equal(ser[0, :, :8], par[0])       # serial transfers perfect


def test_serial_transfer_trail_and_conservation():
    """Serial inefficiency moves charge along the register only, by the same law with c + 1
    transfers; total charge is conserved when the overscan holds the trail."""
    eps, c, n = 3e-3, 30, 100000
    rp = _quiet(cte_serial=1.0 - eps, full_well=1e9, over_x=20, amp_nx=1, amp_ny=1)
    img = np.zeros((8, 40), np.uint32)
    img[2, c] = n
    _, _, _, par, ser = O.readout(rp, img)
    row = ser[0, 2].astype(np.int64)
    assert row.sum() == n and row[:c].sum() == 0
    pmf = stats.nbinom.pmf(np.arange(3), c + 1, 1 - eps)
    exp_ = n * np.append(pmf, 1 - pmf.sum())
    obs = np.append(row[c:c + 3], row[c + 3:].sum())
    assert ((obs - exp_) ** 2 / exp_).sum() < stats.chi2.ppf(1 - 1e-4, 3)


def test_segment_geometry_and_ideal_digitiser():
    """Without noise or bit errors the digitiser is floor(e / G + B); each segment is read from its
    register edge (rows from the device edge) and its amplifier end, into [sh + over_y, sw +
    over_x] with empty overscan."""
    G, B = 2.0, 1000.3
    rp = _quiet(gain=(G,) * 32, bias=(B,) * 32)
    rng = np.random.default_rng(4)
    img = rng.integers(0, 999, (32, 32)).astype(np.uint32)
    out, _, _, par, ser = O.readout(rp, img)
    assert out.shape == (4, 20, 20)
    want = np.floor(ser / G + B).astype(np.uint16)
    assert np.array_equal(out, want)
    # amplifier 0: rows from the bottom edge; amplifier 2 (top half): rows from the top edge
    assert np.array_equal(ser[0, :16, :16], img[:16, :16])
    assert np.array_equal(ser[2, :16, :16], img[31:15:-1, :16])
    assert np.array_equal(ser[1, :16, :16], img[:16, 16:])
    assert ser[:, 16:, :].sum() == 0 and ser[:, :, 16:].sum() == 0


def test_nonlinearity_read_noise_and_bit_errors():
    """ADU = e / (G (1 + N e / W)) + B; read noise adds a normal of sigma electrons (output
    variance sigma^2 / G^2 + 1/12 for the floor); a bit error of width sigma_i on bit i leaves the
    other bits as the ideal digitiser sets them and makes bit i a fair coin when sigma_i >> 1."""
    W, N = 1000.0, 0.05
    rp = _quiet(nonlinearity=N, gain=(1.5,) * 32, bias=(100.25,) * 32)
    img = np.full((16, 16), 800, np.uint32)
    out, _, _, _, ser = O.readout(rp, img)
    e = ser.astype(np.float64)
    assert np.array_equal(out, np.floor(e / (1.5 * (1 + N * e / W)) + 100.25).astype(np.uint16))
    rp = _quiet(read_noise=(5.0,) * 32, bias=(1000.0,) * 32, over_x=0, over_y=0)
    img = np.zeros((128, 128), np.uint32)
    out, _, _, _, _ = O.readout(rp, img)
    v = out.astype(np.float64).ravel()
    assert abs(v.var() - (25 + 1 / 12)) < 5 * 25 * math.sqrt(2.0 / v.size)
    assert abs(v.mean() - 999.5) < 5 * 5 / math.sqrt(v.size)
    rp = _quiet(bit_sigma=(0.0, 0.0, 20.0) + (0.0,) * 13, bias=(1000.37,) * 32, over_x=0, over_y=0)
    img = np.random.default_rng(5).integers(0, 999, (128, 128)).astype(np.uint32)
    out, _, _, _, ser = O.readout(rp, img)
    ideal = np.floor(ser + 1000.37).astype(np.int64)
    o = out.astype(np.int64)
    assert np.array_equal(o & ~4, ideal & ~4)
    b2 = (o >> 2) & 1
    assert abs(b2.mean() - 0.5) < 5 * 0.5 / math.sqrt(b2.size)
