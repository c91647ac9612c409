"""The GPU-vs-oracle comparison rules themselves (no GPU): a photon closer to a pixel edge than the
position tolerance may land in either pixel; any other pixel difference is a failure."""
import numpy as np
import pytest

import oracle as O
from tests import parity


def _events(xe, pix_i, status=O.DETECTED):
    ev = np.zeros(len(xe), O.EVENT_DTYPE)
    ev["photon"] = np.arange(len(xe))
    ev["status"] = status
    ev["surface"] = 1
    ev["xe"] = xe
    ev["x"] = xe
    ev["ye"] = ev["y"] = 0.5e-5     # mid-pixel in y
    ev["pix_i"] = pix_i
    ev["margin"] = 1.0
    return ev


def test_pixel_flip_within_the_position_tolerance_is_allowed_only_with_the_chip():
    chip = (0.0, 0.0, 1e-5)
    o = _events([1e-5 + 2e-10, 2.5e-5], [1, 2])
    g = _events([1e-5 - 1e-10, 2.5e-5], [0, 2])
    with pytest.raises(AssertionError):
        parity.compare(g, o)
    rep = parity.compare(g, o, chip=chip)
    assert rep["n"] == 2
    img_o = np.zeros((1, 4), np.uint32)
    img_g = np.zeros((1, 4), np.uint32)
    img_o[0, [1, 2]] += 1
    img_g[0, [0, 2]] += 1
    assert not parity.images_agree(img_g, img_o, g, o)
    assert parity.images_agree(img_g, img_o, g, o, chip=chip)


def test_pixel_flip_beyond_the_position_tolerance_fails():
    chip = (0.0, 0.0, 1e-5)
    o = _events([1e-5 + 5e-9], [1])
    g = _events([1e-5 + 5e-9], [0])
    with pytest.raises(AssertionError):
        parity.compare(g, o, chip=chip)
