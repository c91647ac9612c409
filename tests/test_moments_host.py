"""The tests' reference moment arithmetic (no GPU): word encoding, and the exact rational
centroids and central second moments against an independent extended-precision two-pass
evaluation."""
import numpy as np

from paper_1504_06570_amd import phx as P
from tests import moments_ref as R


def test_words_round_trip_signed_128_bit():
    sums = [(3, -5, 7, 2 ** 100 + 3, 1, -(2 ** 90) - 1), (0, 0, 0, 0, 0, 0)]
    assert P.moment_sums(R.words_of(sums)) == sums
    assert R.Q_LOG2 == P.MOMENT_Q_LOG2 and R.WORDS == P.MOMENT_WORDS


def test_moments_of_a_point_cloud():
    """A far-off-axis 10 um cloud: the rational evaluation keeps full relative precision of the
    tiny central moments where naive sums in floating point would cancel."""
    rng = np.random.default_rng(0)
    x = 0.031 + 10e-6 * rng.standard_normal(5000)
    y = -0.022 + 7e-6 * rng.standard_normal(5000) + 0.3 * (x - 0.031)
    m = R.moments_from_sums([R.quantised_sums(x, y)])[0]
    q = 2.0 ** -R.Q_LOG2
    xq, yq = np.rint(x / q) * q, np.rint(y / q) * q
    # reference: two-pass central moments in extended precision on the quantised positions
    xl, yl = xq.astype(np.longdouble), yq.astype(np.longdouble)
    mx, my = xl.mean(), yl.mean()
    want = [len(x), mx, my, ((xl - mx) ** 2).mean(), ((yl - my) ** 2).mean(),
            ((xl - mx) * (yl - my)).mean()]
    np.testing.assert_allclose(m, np.array(want, np.float64), rtol=1e-13, atol=0)


def test_empty_source_is_zero():
    assert np.all(R.moments_from_sums([(0, 0, 0, 0, 0, 0)]) == 0)
    assert np.all(R.adjoint_seeds(np.zeros((1, 6)), np.ones((1, 5))) == 0)
