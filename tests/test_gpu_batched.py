"""Batched (graph-replayed, tunable launch shape) trace against the plain per-source launches.

Photons are keyed by (seed, source, index), so a single launch over many sources of uneven
photon counts, any launch shape, and any replay of a captured graph must bin exactly the photons
that one launch per source bins."""
import numpy as np
import pytest

from paper_1504_06570_amd.scene import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def phx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_06570_amd import phx as P
    return P


@pytest.fixture(scope="module")
def scene():
    # 10^3 sources, power-law counts 10..1e5 after scaling, stars + Sersic galaxies, blackbodies
    return C.batched(scale=1e-2, screen_n=256, n_src=1000)


def per_source(phx, tr, scene):
    import torch
    img = tr.new_image()
    stats = tr.new_stats()
    for s in range(len(scene.sources)):
        tr.trace(img, stats=stats, src_begin=s, src_end=s + 1)
    torch.cuda.synchronize()
    return img, stats


def test_batched_equals_per_source(phx, scene):
    import torch
    tr = phx.Tracer(scene)
    ref_img, ref_stats = per_source(phx, tr, scene)
    img, stats, _, _ = tr.trace(stats=tr.new_stats(), batched=True)
    one, one_stats, _, _ = tr.trace(stats=tr.new_stats())
    torch.cuda.synchronize()
    assert int(ref_img.sum()) > 0
    assert torch.equal(img, ref_img) and torch.equal(one, ref_img)
    assert torch.equal(stats, ref_stats) and torch.equal(one_stats, ref_stats)
    tr.close()


def test_graph_replays_match_eager(phx, scene):
    """Each replay of the captured graph, with eager work and synchronisation in between,
    adds exactly one eager trace's counts."""
    import torch
    tr = phx.Tracer(scene)
    eager, _, _, _ = tr.trace()
    img = tr.new_image()
    for k in range(1, 4):
        tr.trace(img, batched=True)
        torch.cuda.synchronize()
        assert torch.equal(img, eager * k), k
        tr.trace(tr.new_image(), src_begin=0, src_end=7)   # unrelated eager work
        torch.cuda.synchronize()
    tr.close()


@pytest.mark.parametrize("cfg", [
    dict(dynamic_tiles=1),
    dict(chunk_log2=16, dynamic_tiles=1),
    dict(chunk_log2=17, generate_blocks_per_cu=1, front_blocks_per_cu=3, back_blocks_per_cu=1),
    dict(generate_blocks_per_cu=64, front_blocks_per_cu=64, back_blocks_per_cu=16),
    dict(pipeline=0),
    dict(pipeline=0, chunk_log2=16, dynamic_tiles=1),
])
def test_launch_shapes_bin_the_same_photons(phx, scene, cfg):
    import torch
    tr = phx.Tracer(scene)
    flags = int(scene.physics) | phx.F_CULL
    ref, ref_st, _, _ = tr.trace(stats=tr.new_stats(), flags=flags)
    tr.set_launch_config(**cfg)
    assert {k: tr.launch_config()[k] for k in cfg} == cfg
    for batched in (False, True):
        img, st, _, _ = tr.trace(stats=tr.new_stats(), flags=flags, batched=batched)
        torch.cuda.synchronize()
        assert torch.equal(img, ref), (cfg, batched)
        assert torch.equal(st, ref_st), (cfg, batched)
    tr.close()


def test_launch_config_validation(phx, scene):
    tr = phx.Tracer(C.tiny())
    for bad in (dict(chunk_log2=15), dict(chunk_log2=28), dict(back_blocks_per_cu=0),
                dict(front_blocks_per_cu=65), dict(dynamic_tiles=2), dict(pipeline=2)):
        with pytest.raises(phx.PhxError):
            tr.set_launch_config(**bad)
    tr.close()


def test_autotune_picks_a_valid_shape_and_keeps_results(phx, scene):
    import torch
    tr = phx.Tracer(scene)
    flags = int(scene.physics) | phx.F_CULL
    ref, _, _, _ = tr.trace(flags=flags)
    best = tr.autotune(flags=flags)
    assert best == tr.launch_config()
    assert 16 <= best["chunk_log2"] <= 27 and best["dynamic_tiles"] in (0, 1)
    img, _, _, _ = tr.trace(flags=flags, batched=True)
    torch.cuda.synchronize()
    assert torch.equal(img, ref)
    # graph replays tuned with the pipeline on: the captured graph holds both streams
    tr.set_launch_config(pipeline=1)
    best = tr.autotune(flags=flags, batched=True)
    assert best == tr.launch_config() and best["pipeline"] == 1
    for _ in range(3):   # replays with eager work between them, each equal to the eager trace
        img, _, _, _ = tr.trace(flags=flags, batched=True)
        eager, _, _, _ = tr.trace(flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(img, ref) and torch.equal(eager, ref)
    tr.close()


def test_batched_moments_match_per_source(phx, scene):
    """Per-source moment words are exact integer sums: a batched launch reproduces the
    per-source launches bit for bit."""
    import torch
    tr = phx.Tracer(scene)
    m_ref = tr.new_moments()
    rows = list(range(0, len(scene.sources), 97))
    for s in rows:
        tr.trace(moments=m_ref, src_begin=s, src_end=s + 1)
    m = tr.new_moments()
    tr.trace(moments=m, batched=True)
    torch.cuda.synchronize()
    assert torch.equal(m[rows], m_ref[rows])
    assert int(m[:, 0].sum()) > 0
    tr.close()


def test_source_aligned_chunks_match(phx):
    """Launches of a few big sources are cut at source boundaries and their survivors sorted by
    time; images, statistics and moment words equal those of the evenly cut launch."""
    import torch
    s = C.gradients(scale=2e-4, screen_n=128)
    tr = phx.Tracer(s)
    kw = dict(src_begin=10, src_end=15, photon_count=20000, flags=int(s.physics) | phx.F_CULL)
    ref, ref_st, ref_m, _ = tr.trace(stats=tr.new_stats(), moments=tr.new_moments(), **kw)
    tr.set_launch_config(chunk_log2=16)      # chunk 65536: each source (20000) is >= chunk / 8
    img, st, m, _ = tr.trace(stats=tr.new_stats(), moments=tr.new_moments(), **kw)
    torch.cuda.synchronize()
    assert int(ref.sum()) > 0 and int(ref_m[10:15, 0].min()) > 0
    assert torch.equal(img, ref) and torch.equal(st, ref_st) and torch.equal(m, ref_m)
    tr.close()


def test_zero_count_sources_and_events(phx):
    """Sources without photons between others (the decode's guide must skip them), one launch
    against per-source launches, with event records checked photon by photon."""
    import torch
    s = C.batched(scale=1e-2, screen_n=256, n_src=64)
    counts = s.sources.n_photons.copy()
    counts[1::3] = 0
    counts[-1] = 0
    s.sources.n_photons[:] = counts
    tr = phx.Tracer(s)
    ref = tr.new_image()
    for k in range(len(s.sources)):
        if counts[k]:
            tr.trace(ref, src_begin=k, src_end=k + 1)
    img, _, _, ev = tr.trace(event_stride=1)
    torch.cuda.synchronize()
    assert int(ref.sum()) > 0 and torch.equal(img, ref)
    e = phx.events_to_numpy(ev)
    assert len(e) == int(counts.sum())
    expect = np.repeat(np.arange(len(counts)), counts.astype(np.int64))
    assert np.array_equal(e["source"], expect)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    assert np.array_equal(e["photon"].astype(np.int64), np.arange(len(e)) - first[expect])
    tr.close()
