"""The benchmark's own workloads against the oracle: the full configuration (one star, seven
frozen-flow layers of 2048^2 screens at 1 m / 10 cm / 1 cm, the telescope with coatings, silicon,
diffusion, the 4096^2 chip), the default launch shape the benchmark settles on (chunks of 2^26
photons, the two-stream pipeline, 16 / 48 / 2 workgroups per compute unit, the shape the autotuner
settles on), the pre-roll on, three chunks of photons; then the same star with the extra
per-photon physics, through the hybrid two-kick atmosphere, and with ghost reflections, as the
benchmark runs them; and the many-source workload (1e4 sources, 9.5e7 photons), every photon of
it.  Every 50th photon of the launch (4e6 photons) is recorded and traced by the
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


def test_batched_catalogue_every_photon_against_the_oracle(phx):
    """The benchmark's many-source workload at full size -- 1e4 stars and Sersic galaxies with
    blackbody SEDs and power-law photon counts (9.5e7 photons), seven layers of 2048^2 screens, the
    telescope, coatings, silicon and diffusion -- as one graph-replayed batched launch in the
    default launch shape with the pre-roll on.  Every photon's record equals the oracle's (the
    oracle traced source block by source block), boundary photons are fewer than 1e-5 of all, and
    the image equals the oracle's after each side's boundary photons are taken out of its own."""
    import torch
    s = C.batched()
    tr = phx.Tracer(s)
    flags = int(s.physics) | phx.F_CULL
    stats = tr.new_stats()
    img, _, _, evb = tr.trace(flags=flags, stats=stats, event_stride=1, batched=True)
    torch.cuda.synchronize()
    g_all = phx.events_to_numpy(evb).copy()
    gimg = img.cpu().numpy().view(np.uint32).astype(np.int64)
    tab = phx.stats_table(stats.cpu().numpy())
    del evb, img
    tr.close()
    torch.cuda.empty_cache()
    counts = s.sources.n_photons.astype(np.int64)
    total = int(counts.sum())
    assert len(g_all) == total
    assert int(gimg.sum()) == int(tab[phx.DETECTED].sum()) > 0
    starts = np.concatenate([[0], np.cumsum(counts)])
    orc = O.Oracle(s)
    oimg = np.zeros(orc.image_shape, np.uint32)
    adj_g = np.zeros(gimg.shape, np.int64)
    adj_o = np.zeros(gimg.shape, np.int64)
    boundary = detected = n_culled = 0
    worst = worst_conv = 0.0
    for blk in np.array_split(np.arange(len(counts)), 20):
        cb = np.zeros(len(counts), np.uint64)
        cb[blk] = counts[blk]
        o = orc.trace_sources(counts=cb, image=oimg, threads=16)
        g = g_all[starts[blk[0]]:starts[blk[-1] + 1]]
        assert len(g) == len(o)
        culled = g["status"] == phx.CULLED
        assert not np.isin(o["status"][culled], [O.DETECTED, O.OFF_CHIP]).any()
        rep = parity.compare(g[~culled], o[~culled])
        boundary += rep["boundary"]
        detected += rep["detected"]
        n_culled += int(culled.sum())
        worst = max(worst, rep["worst_pos"])
        worst_conv = max(worst_conv, rep["worst_converted"])
        gm, om = parity.match(g[~culled], o[~culled])
        b = om["margin"] < parity.BOUNDARY_MARGIN
        gb = gm[b & (gm["status"] == O.DETECTED)]
        ob = om[b & (om["status"] == O.DETECTED)]
        np.add.at(adj_g, (gb["pix_j"], gb["pix_i"]), 1)
        np.add.at(adj_o, (ob["pix_j"], ob["pix_i"]), 1)
        del o, g, gm, om
    print(f"batched catalogue: {total} photons, {n_culled} culled, {detected} detected, "
          f"{boundary} boundary ({boundary / total:.2e}), worst deviation {worst:.2e} m "
          f"(converted {worst_conv:.2e} m)")
    assert boundary / total < 1e-5
    assert np.array_equal(gimg - adj_g, oimg.astype(np.int64) - adj_o)


def test_gradient_configuration_forward_sampled_against_the_oracle(phx):
    """The forward trace of the benchmark's gradient workload at full size: 25 stars on a 5 x 5
    grid over the field, 1e7 photons each, seven layers of 2048^2 screens, the telescope with its
    22 perturbation parameters set as the benchmark sets them (decenters, tilts and pistons of M2
    and the camera, Zernike terms of M1), coatings, silicon and diffusion, pre-roll on.  Every 50th
    photon of the launch equals the oracle's (traced with the same perturbation), boundary photons
    counted against the sample."""
    import torch
    s = C.gradients()
    theta = np.random.default_rng(5).uniform(-1, 1, C.N_PERTURB) * C.PERTURB_RANGE
    tr = phx.Tracer(s)
    tr.set_perturbation(theta)
    flags = int(s.physics) | phx.F_CULL
    stats = tr.new_stats()
    img, _, _, evb = tr.trace(flags=flags, stats=stats, event_stride=STRIDE)
    torch.cuda.synchronize()
    g = phx.events_to_numpy(evb).copy()
    gimg = img.cpu().numpy().view(np.uint32)
    tab = phx.stats_table(stats.cpu().numpy())
    tr.close()
    counts = s.sources.n_photons.astype(np.int64)
    total = int(counts.sum())
    assert len(g) == (total + STRIDE - 1) // STRIDE
    assert int(gimg.sum()) == int(tab[phx.DETECTED].sum()) > 0
    orc = O.Oracle(s, theta=theta)
    o = np.zeros(len(g), O.EVENT_DTYPE)
    for src in np.unique(g["source"]):
        m = g["source"] == src
        o[m] = orc.trace_list(int(src), g["photon"][m], threads=16)
    culled = g["status"] == phx.CULLED
    assert culled.any()
    assert not np.isin(o["status"][culled], [O.DETECTED, O.OFF_CHIP]).any()
    rep = parity.compare(g[~culled], o[~culled])
    frac = rep["boundary"] / len(g)
    print(f"gradient workload sample: {len(g)} photons, {int(culled.sum())} culled, boundary "
          f"fraction of the sample {frac:.2e};", {k: v for k, v in rep.items() if k != "groups"})
    assert frac < 1e-5
    assert rep["detected"] > 10000
    det = (g["status"] == phx.DETECTED) & ~culled
    assert np.all(gimg[g["pix_j"][det], g["pix_i"][det]] > 0)
