"""The C ABI's result calls: phx_moments (per-source centroids and central second moments from
the exact moment words, rounded once) against the exact rational definition, on adversarial
words and on a traced catalogue; phx_read_image against the device image."""
import numpy as np
import pytest

from paper_1504_06570_amd.scene import configs as C
from tests import moments_ref as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def phx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_06570_amd import phx as P
    return P


def _adversarial_sums(rng, k):
    out = [(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0), (1, -1, 1, 1, 1, -1),
           # ties at the 53-bit rounding point: (2^53 + 1) 2^-44 and (2^54 + 2) / 2^45
           (1, 2 ** 53 + 1, -(2 ** 53 + 1), 0, 0, 0), (2, 2 ** 54 + 2, 2 ** 54 + 6, 0, 0, 0),
           # a far-off-axis tight cloud: n SXX - SX^2 cancels in 150 of 156 bits
           (2 ** 33 + 7, (2 ** 33 + 7) * (2 ** 43 + 12345), -(2 ** 33 + 7) * (2 ** 42 + 9),
            (2 ** 33 + 7) * (2 ** 43 + 12345) ** 2 + 3 * 2 ** 40,
            (2 ** 33 + 7) * (2 ** 42 + 9) ** 2 + 5, -(2 ** 33 + 7) * (2 ** 43 + 12345) * (2 ** 42 + 9) - 1)]
    for _ in range(k):
        n = int(rng.integers(1, 2 ** 62))
        vals = [int(rng.integers(-2 ** 62, 2 ** 62)) * int(rng.integers(1, 2 ** 60)) for _ in range(5)]
        out.append((n, *vals))
    return out


def test_moments_call_equals_the_exact_definition(phx):
    import torch
    s = C.tiny(scale=0.01)
    tr = phx.Tracer(s)
    sums = _adversarial_sums(np.random.default_rng(3), 400)
    w = torch.from_numpy(R.words_of(sums)).cuda()
    got = tr.moments(w).cpu().numpy()
    want = R.moments_from_sums(sums)
    assert np.array_equal(got, want), np.nonzero(got != want)
    tr.close()


def test_moments_of_a_traced_catalogue_and_the_image_copy(phx):
    import torch
    s = C.telescope(scale=0.01)
    tr = phx.Tracer(s)
    m = tr.new_moments()
    img, _, _, _ = tr.trace(moments=m)
    got = tr.moments(m).cpu().numpy()
    host = tr.read_image(img)
    torch.cuda.synchronize()
    want = R.moments_from_sums(phx.moment_sums(m))
    assert np.array_equal(got, want)
    assert (got[:, 0] > 0).all()
    assert np.array_equal(host, img.cpu().numpy().view(np.uint32)) and host.sum() > 0
    with pytest.raises(phx.PhxError):
        tr._check(tr.L.phx_read_image(tr.ctx, img.data_ptr(), host.ctypes.data, host.size - 1,
                                      None))
    with pytest.raises(phx.PhxError):
        tr._check(tr.L.phx_moments(tr.ctx, None, 3, None, None))
    tr.close()
