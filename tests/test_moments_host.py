"""Host-side moment arithmetic: the exact integer sums and their conversion to centroids and
central second moments (no GPU)."""
import numpy as np

from paper_1504_06570_amd import phx as P


def _words(sums):
    w = np.zeros((len(sums), P.MOMENT_WORDS), np.uint64)
    for i, (n, *vals) in enumerate(sums):
        w[i, 0] = n
        for k, v in enumerate(vals):
            v &= (1 << 128) - 1
            w[i, 2 + 2 * k] = v & ((1 << 64) - 1)
            w[i, 3 + 2 * k] = v >> 64
    return w.view(np.int64)


def test_words_round_trip_signed_128_bit():
    sums = [(3, -5, 7, 2 ** 100 + 3, 1, -(2 ** 90) - 1), (0, 0, 0, 0, 0, 0)]
    assert P.moment_sums(_words(sums)) == sums


def test_moments_of_a_point_cloud():
    """A far-off-axis 10 um cloud: the rational evaluation keeps full relative precision of the
    tiny central moments where naive sums in floating point would cancel."""
    rng = np.random.default_rng(0)
    x = 0.031 + 10e-6 * rng.standard_normal(5000)
    y = -0.022 + 7e-6 * rng.standard_normal(5000) + 0.3 * (x - 0.031)
    m = P.moments_from_sums([P.quantised_sums(x, y)])[0]
    q = 2.0 ** -P.MOMENT_Q_LOG2
    xq, yq = np.rint(x / q) * q, np.rint(y / q) * q
    # reference: two-pass central moments in extended precision on the quantised positions
    xl, yl = xq.astype(np.longdouble), yq.astype(np.longdouble)
    mx, my = xl.mean(), yl.mean()
    want = [len(x), mx, my, ((xl - mx) ** 2).mean(), ((yl - my) ** 2).mean(),
            ((xl - mx) * (yl - my)).mean()]
    np.testing.assert_allclose(m, np.array(want, np.float64), rtol=1e-13, atol=0)


def test_empty_source_is_zero():
    assert np.all(P.moments_from_sums([(0, 0, 0, 0, 0, 0)]) == 0)
