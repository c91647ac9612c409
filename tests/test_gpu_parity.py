"""GPU trace (through the C ABI) against the CPU oracle, photon by photon and pixel by pixel."""
import numpy as np
import pytest

import oracle as O
from paper_1504_06570_amd.scene import configs as C
from paper_1504_06570_amd.scene import optics as Op
from paper_1504_06570_amd.scene.sources import blackbody_table, sersic_bn
from tests import helpers as H
from tests import moments_ref as R
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def phx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_06570_amd import phx as P
    return P


def run_both(P, scene, stride=1, threads=8, flags=None, photon_count=0, photon_begin=0):
    import torch
    tr = P.Tracer(scene)
    stats = tr.new_stats()
    img, stats, _, evb = tr.trace(stats=stats, event_stride=stride, flags=flags,
                                  photon_count=photon_count, photon_begin=photon_begin)
    torch.cuda.synchronize()
    gev = P.events_to_numpy(evb)
    gimg = img.cpu().numpy().view(np.uint32)
    orc = O.Oracle(scene)
    oimg = np.zeros(orc.image_shape, np.uint32)
    counts = None if not photon_count else np.full(len(scene.sources), photon_count)
    oev = orc.trace_sources(counts=counts, begin=photon_begin, image=oimg, threads=threads)
    tr.close()
    return gev, gimg, oev, oimg, stats.cpu().numpy()


def test_tiny_paraboloid_focus(phx):
    """Paraboloid point focus: every GPU photon lands within 1e-12 m of the axis in pixel
    (32, 32), binned counts equal the transmitted photons, photon by photon equal to the oracle."""
    s = C.tiny()
    gev, gimg, oev, oimg, st = run_both(phx, s)
    rep = parity.compare(gev, oev, chip=parity.chip_of(s))
    assert rep["boundary"] == 0
    assert np.max(np.hypot(gev["x"], gev["y"])) < 1e-12
    assert gimg[32, 32] == len(gev) == gimg.sum() == 100000
    assert np.array_equal(gimg, oimg)
    tab = phx.stats_table(st)
    assert tab[phx.DETECTED].sum() == 100000


def test_telescope_parity(phx):
    """Generated three-mirror telescope + camera, coatings, silicon, diffusion, 441 sources."""
    s = C.telescope(scale=0.02)
    gev, gimg, oev, oimg, st = run_both(phx, s)
    rep = parity.compare(gev, oev, chip=parity.chip_of(s))
    assert rep["boundary_frac"] < 1e-5
    assert parity.images_agree(gimg, oimg, gev, oev, chip=parity.chip_of(s))
    assert gimg.sum() == (gev["status"] == phx.DETECTED).sum()


def test_telescope_cull_keeps_image(phx):
    """Pre-roll culling (section 3.2) removes only photons that cannot be detected."""
    import torch
    s = C.telescope(scale=0.02)
    s.prescription = s.prescription.replace(chip=Op.Chip(0.0, 0.0, 10e-6, 4096, 4096))
    tr = phx.Tracer(s)
    a, st_a, _, _ = tr.trace(stats=tr.new_stats())
    b, st_b, _, _ = tr.trace(stats=tr.new_stats(), flags=int(s.physics) | phx.F_CULL)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ta, tb = phx.stats_table(st_a), phx.stats_table(st_b)
    assert ta[phx.DETECTED].sum() == tb[phx.DETECTED].sum()
    assert tb[phx.CULLED].sum() > 0.5 * s.sources.total_photons


def test_full_atmosphere_parity_small_screens(phx):
    """Seven frozen-flow layers (256^2 screens at three scales) + the telescope."""
    s = C.full(scale=2e-4, screen_n=256)
    gev, gimg, oev, oimg, st = run_both(phx, s)
    rep = parity.compare(gev, oev, chip=parity.chip_of(s))
    assert rep["boundary_frac"] < 1e-5
    assert rep["detected"] > 1000
    assert parity.images_agree(gimg, oimg, gev, oev, chip=parity.chip_of(s))


def test_sersic_and_blackbody_parity(phx):
    """Extended Sersic sources and tabulated blackbody SEDs through the full stack."""
    s = C.batched(scale=2e-3, screen_n=128, n_src=200)
    gev, gimg, oev, oimg, st = run_both(phx, s)
    rep = parity.compare(gev, oev, chip=parity.chip_of(s))
    assert rep["boundary_frac"] < 1e-5
    assert parity.images_agree(gimg, oimg, gev, oev, chip=parity.chip_of(s))


def test_perturbed_optics_parity(phx):
    """Decentred/tilted secondary and camera, Zernike-deformed primary."""
    s = C.gradients(scale=2e-3, screen_n=128)
    rng = np.random.default_rng(3)
    s.perturbation = rng.uniform(-1, 1, C.N_PERTURB) * C.PERTURB_RANGE
    gev, gimg, oev, oimg, st = run_both(phx, s)
    rep = parity.compare(gev, oev, chip=parity.chip_of(s))
    assert rep["boundary_frac"] < 1e-5


def test_split_launch_and_repeat_are_bit_identical(phx):
    """Photons are keyed by index: [0, k) + [k, n) equals [0, n); a repeat is identical."""
    import torch
    s = C.full(scale=1e-4, screen_n=128)
    s.prescription = s.prescription.replace(chip=Op.Chip(s.prescription.chip.center_x,
                                                         s.prescription.chip.center_y, 10e-6, 512, 512))
    tr = phx.Tracer(s)
    n = int(s.sources.n_photons[0])
    a, _, _, _ = tr.trace(photon_count=n)
    b = tr.new_image()
    tr.trace(b, photon_count=n // 3)
    tr.trace(b, photon_begin=n // 3, photon_count=n - n // 3)
    c, _, _, _ = tr.trace(photon_count=n)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
    assert int(a.sum()) > 0


def test_error_paths(phx):
    """Host-side validation returns errors instead of launching."""
    s = C.tiny()
    tr = phx.Tracer(s)
    with pytest.raises(phx.PhxError):
        tr.trace(src_begin=0, src_end=5)
    with pytest.raises(phx.PhxError):
        tr.trace(flags=phx.F_ATMOSPHERE)
    bad = C.tiny()
    bad.prescription.surfaces[0].r_out = float("nan")
    with pytest.raises(phx.PhxError):
        phx.Tracer(bad)


def test_preroll_events_consistent(phx):
    """With the pre-roll on, every photon it removes is one that the full trace does not detect,
    and every other photon has exactly the record it has without the pre-roll."""
    import torch
    s = C.full(scale=2e-4, screen_n=128)
    tr = phx.Tracer(s)
    _, _, _, ea = tr.trace(event_stride=1)
    _, _, _, eb = tr.trace(event_stride=1, flags=int(s.physics) | phx.F_CULL)
    torch.cuda.synchronize()
    a, b = phx.events_to_numpy(ea), phx.events_to_numpy(eb)
    assert np.array_equal(a["photon"], b["photon"])
    culled = b["status"] == phx.CULLED
    assert culled.mean() > 0.5
    assert not np.isin(a["status"][culled], [phx.DETECTED, phx.OFF_CHIP]).any()
    keep = ~culled
    for f in ("status", "surface", "pix_i", "pix_j"):
        assert np.array_equal(a[f][keep], b[f][keep]), f
    for f in ("x", "y", "xe", "ye", "lam"):
        assert np.array_equal(a[f][keep], b[f][keep]), f


def test_moments_equal_sums_over_events(phx):
    """The exact moment words equal the quantised sums over the same launch's event records,
    source by source (the 128-bit wavefront reduction and atomics lose nothing)."""
    import torch
    s = C.telescope(scale=0.01)
    tr = phx.Tracer(s)
    m = tr.new_moments()
    _, _, _, ev = tr.trace(moments=m, event_stride=1)
    torch.cuda.synchronize()
    e = phx.events_to_numpy(ev)
    got = phx.moment_sums(m)
    conv = e["status"] <= phx.OFF_CHIP
    assert conv.sum() > 1000
    for si in range(len(s.sources)):
        sel = conv & (e["source"] == si)
        assert got[si] == R.quantised_sums(e["xe"][sel], e["ye"][sel]), si
    tr.close()


def test_geometric_preroll_culls_only_primary_vignetting(phx):
    """With the atmosphere the pupil annulus is sampled wider than the primary; the pre-roll drops
    samples farther out than the bounded atmospheric displacement.  With coatings that never cull,
    every photon it drops is vignetted at the primary in the full trace (or, for the red photons
    the escape test removes, crosses the silicon), and every other photon keeps its record."""
    import torch
    s = C.full(scale=2e-4, screen_n=128)
    s.coatings = np.ones_like(s.coatings)
    tr = phx.Tracer(s)
    _, _, _, ea = tr.trace(event_stride=1)
    _, _, _, eb = tr.trace(event_stride=1, flags=int(s.physics) | phx.F_CULL)
    torch.cuda.synchronize()
    a, b = phx.events_to_numpy(ea), phx.events_to_numpy(eb)
    culled = b["status"] == phx.CULLED
    prim = (a["status"] == phx.VIGNETTED) & (a["surface"] == 0)
    assert (culled & prim).mean() > 0.03
    assert np.all((prim | (a["status"] == phx.ESCAPED))[culled])
    keep = ~culled
    for f in ("status", "surface", "pix_i", "pix_j", "x", "y", "xe", "ye"):
        assert np.array_equal(a[f][keep], b[f][keep]), f
    tr.close()


def test_escape_preroll_culls_only_certain_escapes(phx):
    """Red photons with coatings that never cull: the pre-roll's escape test removes photons whose
    conversion distance times the smallest refracted cosine exceeds the silicon thickness; none of
    them converts in the full trace (those that reach the silicon escape it), and every other
    photon keeps its record."""
    import torch
    s = C.telescope(scale=0.002)
    s.coatings = np.ones_like(s.coatings)
    s.sources.lam_lo[:] = 950e-9
    s.sources.lam_hi[:] = 1080e-9
    tr = phx.Tracer(s)
    _, _, _, ea = tr.trace(event_stride=1)
    img_b, _, _, eb = tr.trace(event_stride=1, flags=int(s.physics) | phx.F_CULL)
    img_a, _, _, _ = tr.trace()
    torch.cuda.synchronize()
    assert torch.equal(img_a, img_b)
    a, b = phx.events_to_numpy(ea), phx.events_to_numpy(eb)
    culled = b["status"] == phx.CULLED
    escaped = a["status"] == phx.ESCAPED
    assert culled.sum() > 0.2 * escaped.sum() > 0
    assert not np.isin(a["status"][culled], [phx.DETECTED, phx.OFF_CHIP]).any()
    assert escaped[culled].mean() > 0.5, np.bincount(a["status"][culled])
    keep = ~culled
    for f in ("status", "surface", "pix_i", "pix_j", "x", "y", "xe", "ye"):
        assert np.array_equal(a[f][keep], b[f][keep]), f
    tr.close()


def test_photon_index_crossing_32_bits(phx):
    """Photon indices around 2^32 (the Philox counter's high word turns over): GPU and oracle
    agree photon by photon, with the pre-roll and the atmosphere on."""
    s = C.full(scale=2e-4, screen_n=128)
    begin = (1 << 32) - 3000
    flags = int(s.physics) | phx.F_CULL
    gev, gimg, oev, oimg, _ = run_both(phx, s, flags=flags, photon_count=6000, photon_begin=begin)
    assert gev["photon"].min() == begin and gev["photon"].max() == begin + 5999
    g, o = parity.match(gev, oev)
    culled = g["status"] == phx.CULLED
    assert 0 < culled.sum() < len(g)
    rep = parity.compare(g[~culled], o[~culled])
    assert rep["boundary_frac"] < 1e-5
    assert not np.isin(o["status"][culled], [phx.DETECTED, phx.OFF_CHIP]).any()


def _parity_with_cull(phx, gev, oev):
    g, o = parity.match(gev, oev)
    culled = g["status"] == phx.CULLED
    assert not np.isin(o["status"][culled], [phx.DETECTED, phx.OFF_CHIP]).any()
    rep = parity.compare(g[~culled], o[~culled])
    assert rep["boundary_frac"] < 1e-5
    return g, o, culled


def test_ragged_counts_and_a_single_photon(phx):
    """Photon counts that fill no bitmap word, wavefront or workgroup evenly, at an odd first
    index: 100003 photons from index 17, and one photon alone, with the pre-roll and the
    atmosphere on; GPU and oracle agree photon by photon and the image counts the detected."""
    s = C.full(scale=2e-4, screen_n=128)
    flags = int(s.physics) | phx.F_CULL
    for count, begin in ((100003, 17), (1, 12345)):
        gev, gimg, oev, oimg, _ = run_both(phx, s, flags=flags, photon_count=count,
                                           photon_begin=begin)
        assert len(gev) == count and gev["photon"].min() == begin
        assert gev["photon"].max() == begin + count - 1
        g, o, culled = _parity_with_cull(phx, gev, oev)
        assert int(gimg.sum()) == int((g["status"] == phx.DETECTED).sum())


def test_last_chunk_of_one_photon(phx):
    """Chunks of 2^16 photons and a launch of 2^16 + 1: the second chunk holds one photon and
    runs through the two-stream pipeline like the first; GPU and oracle agree photon by photon."""
    import torch
    s = C.full(scale=2e-4, screen_n=128)
    flags = int(s.physics) | phx.F_CULL
    n = (1 << 16) + 1
    tr = phx.Tracer(s)
    tr.set_launch_config(chunk_log2=16, pipeline=1)
    stats = tr.new_stats()
    img, stats, _, evb = tr.trace(stats=stats, event_stride=1, flags=flags, photon_count=n)
    torch.cuda.synchronize()
    gev = phx.events_to_numpy(evb)
    gimg = img.cpu().numpy().view(np.uint32)
    tr.close()
    oev = O.Oracle(s).trace_sources(counts=np.full(len(s.sources), n), threads=8)
    assert len(gev) == n
    g, o, culled = _parity_with_cull(phx, gev, oev)
    assert int(gimg.sum()) == int((g["status"] == phx.DETECTED).sum())


def test_largest_chunk_and_the_top_of_the_index_range(phx):
    """The largest launch shape's chunk (2^27 photons, two buffers of it pipelined) with a ragged
    second chunk, every 9973rd photon recorded and traced by the oracle alone; and photon indices
    just below 2^64 (the end of the 64-bit counter).  GPU and oracle agree photon by photon."""
    import torch
    s = C.full(scale=2e-4, screen_n=256)
    flags = int(s.physics) | phx.F_CULL
    tr = phx.Tracer(s)
    tr.set_launch_config(chunk_log2=27, pipeline=1)
    n, stride = (1 << 27) + 4097, 9973
    img, _, _, evb = tr.trace(flags=flags, photon_count=n, event_stride=stride)
    torch.cuda.synchronize()
    g = phx.events_to_numpy(evb).copy()
    tr.close()
    assert len(g) == (n + stride - 1) // stride
    assert np.array_equal(g["photon"], np.arange(0, n, stride, dtype=np.uint64))
    o = O.Oracle(s).trace_list(0, g["photon"], threads=8)
    _parity_with_cull(phx, g, o)
    assert int(img.sum()) > 0
    # the last 4000 photons below 2^64
    begin = (1 << 64) - 4001
    gev, gimg, oev, oimg, _ = run_both(phx, s, flags=flags, photon_count=4000, photon_begin=begin)
    assert int(gev["photon"].max()) == (1 << 64) - 2
    _parity_with_cull(phx, gev, oev)


def test_newton_cycle_is_nonconv(phx):
    """A surface on which Newton's iteration cycles (tests/helpers.newton_cycle_scene): every
    photon is counted as NONCONV at that surface, photon by photon equal to the oracle, with
    nothing binned."""
    s = H.newton_cycle_scene(20000)
    gev, gimg, oev, oimg, st = run_both(phx, s)
    assert np.all(gev["status"] == phx.NONCONV) and np.all(gev["surface"] == 1)
    rep = parity.compare(gev, oev)
    assert rep["boundary"] == 0
    tab = phx.stats_table(st)
    assert tab[phx.NONCONV, 2] == 20000 and tab.sum() == 20000
    assert gimg.sum() == 0


def test_non_finite_screens_are_refused(phx):
    """A screen holding a NaN or an infinity is refused at load (PHX_ERR_INVALID), after which the
    atmosphere cannot be traced (PHX_ERR_STATE) until good screens are loaded."""
    import copy
    s = C.full(scale=1e-6, screen_n=64)
    tr = phx.Tracer(s)
    for bad in (np.nan, np.inf, -np.inf):
        atm = copy.deepcopy(s.atmosphere)
        atm.opd = np.array(atm.opd, np.float32)
        atm.opd[3, 2, 10, 20] = bad
        with pytest.raises(phx.PhxError, match="NaN or infinite"):
            tr.load_screens(atm)
        with pytest.raises(phx.PhxError, match="without loaded screens"):
            tr.trace()
    tr.load_screens(s.atmosphere)
    img, _, _, _ = tr.trace()
    tr.close()
