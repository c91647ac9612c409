"""The benchmark's own workloads against the oracle: the full configuration (one star, seven
frozen-flow layers of 2048^2 screens at 1 m / 10 cm / 1 cm, the telescope with coatings, silicon,
diffusion, the 4096^2 chip), the default launch shape the benchmark settles on (chunks of 2^26
photons, the two-stream pipeline, 16 / 48 / 2 workgroups per compute unit, the shape the autotuner
settles on), the pre-roll on, three chunks of photons; then the same star with the extra
per-photon physics, through the hybrid two-kick atmosphere, and with ghost reflections, as the
benchmark runs them.  Every 50th photon of the launch (4e6 photons) is recorded and traced by the
oracle alone, by its index; they must agree photon by photon and pixel by pixel.  Boundary photons
(an oracle decision margin below the parity module's bar) are counted against the whole sample,
the culled photons included: the pre-roll's decisions are exact integer comparisons, and a culled
photon is one the oracle does not convert, so both sides leave it out of the image.  The oracle's
own rate of such photons on these workloads is 2e-6 (core), 5e-6 (extra physics), 9e-6 (hybrid
atmosphere, whose second-kick sampler adds decisions) and 3.5e-6 (ghosts) over 2e6 photons, so a
sample of 4e6 resolves the 1e-5 bar."""
import numpy as np
import pytest

import oracle as O
from paper_1504_06570_amd.scene import configs as C
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def phx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_06570_amd import phx as P
    return P


N_SAMPLED = 3 << 26   # three chunks of the default size
STRIDE = 50


def sampled_parity(phx, s, kind):
    """Traces N_SAMPLED photons of scene s in the default launch shape with the pre-roll on,
    records every STRIDE-th and checks it against the oracle; returns the report."""
    import torch
    tr = phx.Tracer(s)
    flags = int(s.physics) | phx.F_CULL
    stats = tr.new_stats()
    img, _, _, evb = tr.trace(flags=flags, stats=stats, photon_count=N_SAMPLED,
                              event_stride=STRIDE)
    torch.cuda.synchronize()
    g = phx.events_to_numpy(evb).copy()
    gimg = img.cpu().numpy().view(np.uint32)
    st = stats.cpu().numpy()
    tr.close()
    assert len(g) == (N_SAMPLED + STRIDE - 1) // STRIDE
    assert np.array_equal(g["photon"], np.arange(0, N_SAMPLED, STRIDE, dtype=np.uint64))
    tab = phx.stats_table(st)
    assert int(gimg.sum()) == int(tab[phx.DETECTED].sum()) > 0
    o = O.Oracle(s).trace_list(0, g["photon"], threads=16)
    # culled photons are ones the oracle does not convert
    culled = g["status"] == phx.CULLED
    assert culled.any()
    assert not np.isin(o["status"][culled], [O.DETECTED, O.OFF_CHIP]).any()
    rep = parity.compare(g[~culled], o[~culled])
    frac = rep["boundary"] / len(g)
    print(f"{kind} sample: {len(g)} photons, {int(culled.sum())} culled, boundary fraction of "
          f"the sample {frac:.2e};", {k: v for k, v in rep.items() if k != "groups"})
    print("worst deviation per status@surface:", rep["groups"])
    assert frac < 1e-5
    assert rep["detected"] > 10000
    # every sampled detected photon is counted in its pixel of the launch's image
    det = (g["status"] == phx.DETECTED) & ~culled
    assert np.all(gimg[g["pix_j"][det], g["pix_i"][det]] > 0)
    return rep, g, o, culled


def test_headline_configuration_sampled_against_the_oracle(phx):
    s = C.full()
    tr = phx.Tracer(s)
    cfg = tr.launch_config()
    tr.close()
    assert cfg["chunk_log2"] == 26 and cfg["pipeline"] == 1
    assert (cfg["generate_blocks_per_cu"], cfg["front_blocks_per_cu"],
            cfg["back_blocks_per_cu"]) == (16, 48, 2)
    rep, g, o, culled = sampled_parity(phx, s, "headline")
    assert 0.5 < culled.mean() < 0.99


def _full_size_next(kind):
    from paper_1504_06570_amd.scene import coatings as cm
    from paper_1504_06570_amd.scene import physics as X
    if kind == "hybrid":
        return C.hybrid()
    s = C.full()
    if kind == "extras":
        s.physics = C.PHYS_ALL | X.PHYS_EXTRA
        s.extras = X.tma_extras()
    else:
        s.physics = C.PHYS_ALL | X.PHYS_GHOSTS
        s.reflectance = cm.standard_reflectance()
    return s


@pytest.mark.parametrize("kind", ["extras", "hybrid", "ghosts"])
def test_next_rows_at_full_size_sampled_against_the_oracle(phx, kind):
    """The extra per-photon physics (aerosol, dispersion, dome seeing, halo, spider, dead layer),
    the hybrid two-kick atmosphere and the ghost reflections on the headline star at full size,
    as the benchmark runs them."""
    rep, g, o, culled = sampled_parity(phx, _full_size_next(kind), kind)
    if kind == "extras":
        for status in (phx.EXTINCT, phx.DEAD, phx.OBSCURED):
            assert (o["status"][~culled] == status).any()
