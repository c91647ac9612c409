"""Adjoint trace (phx_adjoint) against closed forms, the oracle's gradient and finite differences.

The derivative is pathwise: each photon keeps its random numbers (keyed by photon index) and its
discrete decisions.  Per-photon Jacobians come from the adjoint's diagnostic output."""
import numpy as np
import pytest

import oracle as O
from paper_1504_06570_amd.scene import configs as C
from tests import moments_ref as R
from tests import helpers as H

pytestmark = pytest.mark.gpu

RANGE = C.PERTURB_RANGE


@pytest.fixture(scope="module")
def phx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_06570_amd import phx as P
    return P


def gpu_jacobians(P, scene, photon_count, src_begin=0, src_end=None):
    """Per-photon Jacobians [n_src, photon_count, 2, 22], converted mask, and event records."""
    import torch
    tr = P.Tracer(scene)
    src_end = len(scene.sources) if src_end is None else src_end
    ns = src_end - src_begin
    seeds = torch.zeros((ns, 8), dtype=torch.float64)
    g, jac = tr.adjoint(seeds, src_begin=src_begin, src_end=src_end, photon_count=photon_count,
                        jac_stride=1)
    _, _, _, ev = tr.trace(src_begin=src_begin, src_end=src_end, photon_count=photon_count,
                           event_stride=1)
    torch.cuda.synchronize()
    e = P.events_to_numpy(ev).reshape(ns, photon_count)
    j = jac.cpu().numpy().reshape(ns, photon_count, 2, C.N_PERTURB)
    tr.close()
    assert np.all(g.cpu().numpy() == 0)
    return j, e["status"] <= P.OFF_CHIP, e


def test_fold_mirror_closed_forms(phx):
    """The same closed forms that pin the oracle's gradient: mirror tilt turns the ray by twice
    the angle, detector shift and pivoted tilt, Zernike slopes from the Noll definition."""
    s = H.fold_scene(n_photons=2000)
    j, conv, e = gpu_jacobians(phx, s, 2000)
    j, conv, e = j[0], conv[0], e[0]
    assert conv.all()
    D, delta, R = 2.0, 0.3, 0.5
    x, y = e["xe"], e["ye"]
    want = np.zeros_like(j)
    want[:, 1, 2] = -2 * D
    want[:, 0, 3] = 2 * D
    want[:, 0, 5] = -1.0
    want[:, 1, 6] = -1.0
    want[:, 1, 7] = -delta
    want[:, 0, 8] = delta
    h = 1e-6
    for i, zj in enumerate(range(4, 16)):
        u, v = x / R, y / R
        want[:, 0, 10 + i] = -2 * D * (H.noll_zernike(zj, u + h, v) - H.noll_zernike(zj, u - h, v)) / (2 * h) / R
        want[:, 1, 10 + i] = -2 * D * (H.noll_zernike(zj, u, v + h) - H.noll_zernike(zj, u, v - h)) / (2 * h) / R
    np.testing.assert_allclose(j, want, rtol=1e-7, atol=1e-8)


def compare_with_oracle(P, scene, count, sources, threads=8, tol=5e-6):
    j, conv, e = gpu_jacobians(P, scene, count)
    orc = O.Oracle(scene)
    h = 1e-3 * RANGE
    n_cmp = 0
    for si in sources:
        oj, frozen = orc.jacobian(si, 0, count, h, threads=threads)
        both = frozen & conv[si]
        n_cmp += both.sum()
        scale = np.abs(oj[both]).max(axis=(0, 1), keepdims=True) + 1e-30
        err = np.abs(j[si][both] - oj[both]) / scale
        assert err.max() <= tol, (si, err.max(axis=(0, 1)))
        # photons the oracle keeps frozen are converted on the GPU too (up to boundary photons)
        assert (frozen & ~conv[si]).sum() <= max(1, 1e-3 * frozen.sum())
    return n_cmp


def test_perturbed_telescope_matches_oracle(phx):
    """Moved and tilted groups, Zernike-deformed primary, three lenses, filter, coatings,
    silicon and diffusion: per-photon Jacobians agree with the oracle's extrapolated central
    differences to its accuracy (a few parts in 1e6 of each parameter's largest effect)."""
    s = C.telescope(scale=1e-4)
    rng = np.random.default_rng(21)
    s.perturbation = rng.uniform(-1, 1, C.N_PERTURB) * RANGE
    n = compare_with_oracle(phx, s, 3000, sources=[0, 110, 220, 330, 440])
    assert n > 300


def test_full_stack_matches_oracle(phx):
    """The same with seven atmosphere layers in front (deflected rays enter the optics)."""
    s = C.gradients(scale=1e-4, screen_n=128)
    rng = np.random.default_rng(22)
    s.perturbation = rng.uniform(-1, 1, C.N_PERTURB) * RANGE
    n = compare_with_oracle(phx, s, 3000, sources=[0, 12, 24])
    assert n > 100


def test_benchmark_gradient_scene_matches_oracle(phx):
    """The benchmark's gradient workload itself (seven layers of 2048^2 screens, the perturbation
    the benchmark sets): the first 3000 photons of three of its 25 stars."""
    s = C.gradients()
    s.perturbation = np.random.default_rng(5).uniform(-1, 1, C.N_PERTURB) * RANGE
    n = compare_with_oracle(phx, s, 3000, sources=[0, 12, 24])
    assert n > 100


def test_full_stack_with_extra_physics_matches_oracle(phx):
    """Dispersion, dome seeing, the halo, the spider, aerosol extinction and the dead layer on top
    of the full stack: none depends on the perturbation, so the photons' Jacobians still agree
    with the oracle's central differences (and the same photons are removed on both sides)."""
    from paper_1504_06570_amd.scene import physics as X
    s = C.gradients(scale=1e-4, screen_n=128)
    s.physics = int(s.physics) | X.PHYS_EXTRA
    s.extras = X.tma_extras()
    rng = np.random.default_rng(23)
    s.perturbation = rng.uniform(-1, 1, C.N_PERTURB) * RANGE
    n = compare_with_oracle(phx, s, 3000, sources=[0, 12, 24])
    assert n > 100


def test_hybrid_atmosphere_matches_oracle(phx):
    """The hybrid two-kick atmosphere in front of the perturbed optics: the second kick does not
    depend on the perturbation, so the Jacobians agree with the oracle's central differences."""
    from paper_1504_06570_amd.scene import physics as X
    from paper_1504_06570_amd.scene.atmosphere import make_atmosphere
    s = C.gradients(scale=1e-4, screen_n=128)
    s.extras = X.tma_extras()
    s.atmosphere = make_atmosphere(5, n=128, kappa_cut=s.extras.kick_kappa_crit)
    s.physics = int(s.physics) | X.PHYS_SECOND_KICK
    rng = np.random.default_rng(24)
    s.perturbation = rng.uniform(-1, 1, C.N_PERTURB) * RANGE
    n = compare_with_oracle(phx, s, 3000, sources=[0, 12, 24])
    assert n > 100


def test_field_diffusion_matches_oracle(phx):
    """With the field model of the diffusion the electron offset depends on the depth through the
    sigma table; the Jacobians (which carry d sigma / d depth through the refracted direction)
    agree with the oracle's central differences."""
    from paper_1504_06570_amd.scene import physics as X
    s = C.telescope(scale=1e-4)
    s.physics = int(s.physics) | X.PHYS_FIELD_DIFFUSION
    s.extras = X.tma_extras()
    rng = np.random.default_rng(25)
    s.perturbation = rng.uniform(-1, 1, C.N_PERTURB) * RANGE
    # the oracle integrates each photon's collection time in every finite-difference trace
    n = compare_with_oracle(phx, s, 800, sources=[0, 220, 440])
    assert n > 50


def test_vjp_equals_sum_of_jacobians(phx):
    """The reduced gradient equals sum_i xbar_i J_x,i + ybar_i J_y,i assembled on the host from
    the per-photon Jacobians (seeds, decode and fixed-order reductions)."""
    import torch
    s = C.gradients(scale=2e-4, screen_n=128)
    s.perturbation = np.random.default_rng(23).uniform(-1, 1, C.N_PERTURB) * RANGE
    tr = phx.Tracer(s)
    n = 2000
    ns = len(s.sources)
    m = tr.new_moments()
    _, _, _, ev = tr.trace(moments=m, photon_count=n, event_stride=1)
    mom = tr.moments(m).cpu().numpy()
    gout = np.random.default_rng(24).standard_normal((ns, 5))
    seeds = R.adjoint_seeds(mom, gout)
    g, jac = tr.adjoint(torch.from_numpy(seeds), photon_count=n, jac_stride=1)
    g2 = tr.adjoint(torch.from_numpy(seeds), photon_count=n)
    # the library's own cotangent coefficients from the words and dL/d(moments)
    g3 = tr.adjoint_moments(m, torch.from_numpy(gout), photon_count=n)
    torch.cuda.synchronize()
    assert torch.equal(g3, g2)
    e = phx.events_to_numpy(ev)
    j = jac.cpu().numpy()
    conv = e["status"] <= phx.OFF_CHIP
    sd = seeds[e["source"]]
    dx, dy = e["xe"] - sd[:, 5], e["ye"] - sd[:, 6]
    xb = np.where(conv, sd[:, 0] + sd[:, 2] * dx + sd[:, 4] * dy, 0.0)
    yb = np.where(conv, sd[:, 1] + sd[:, 3] * dy + sd[:, 4] * dx, 0.0)
    want = (xb[:, None] * j[:, 0] + yb[:, None] * j[:, 1]).sum(axis=0)
    got, got2 = g.cpu().numpy(), g2.cpu().numpy()
    scale = np.abs(want * RANGE).max()
    assert np.abs((got - want) * RANGE).max() <= 1e-10 * scale
    assert np.abs((got2 - want) * RANGE).max() <= 1e-10 * scale
    tr.close()


def test_adjoint_is_deterministic(phx):
    """Repeats give the same bits, with the chunk pipeline on two streams or on one."""
    import torch
    s = C.gradients(scale=2e-4, screen_n=128)
    tr = phx.Tracer(s)
    seeds = torch.ones((len(s.sources), 8), dtype=torch.float64)
    a = tr.adjoint(seeds, photon_count=3000).clone()
    b = tr.adjoint(seeds, photon_count=3000).clone()
    tr.set_launch_config(pipeline=0)
    c = tr.adjoint(seeds, photon_count=3000).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
    tr.close()


def moments_on(P, e, sel, ns):
    """Exact moments of the selected events, per source."""
    sums = []
    for si in range(ns):
        k = sel & (e["source"] == si)
        sums.append(R.quantised_sums(e["xe"][k], e["ye"][k]))
    return R.moments_from_sums(sums)


def test_central_differences_on_frozen_set(phx):
    """Per-source centroid and second-moment gradients agree with central differences of the GPU
    forward at h = 1e-3 of each parameter's range, both taken over the photons whose decisions
    do not change between the nominal and the +-h traces: relative error <= 1e-4."""
    import torch
    s = C.gradients(scale=2e-4, screen_n=128)
    theta0 = np.random.default_rng(25).uniform(-1, 1, C.N_PERTURB) * RANGE
    ns, n = len(s.sources), 4000
    tr = phx.Tracer(s)

    def events(theta):
        tr.set_perturbation(theta)
        _, _, _, ev = tr.trace(photon_count=n, event_stride=1)
        torch.cuda.synchronize()
        return phx.events_to_numpy(ev)

    e0 = events(theta0)
    conv0 = e0["status"] <= phx.OFF_CHIP
    fd = np.zeros((ns, 5, C.N_PERTURB))
    keep = conv0.copy()
    runs = []
    for k in range(C.N_PERTURB):
        h = 1e-3 * RANGE[k]
        tp, tm = theta0.copy(), theta0.copy()
        tp[k] += h
        tm[k] -= h
        ep, em = events(tp), events(tm)
        same = ((ep["status"] <= phx.OFF_CHIP) & (em["status"] <= phx.OFF_CHIP) &
                (ep["surface"] == e0["surface"]) & (em["surface"] == e0["surface"]))
        keep &= same
        runs.append((ep, em, h))
    assert keep.sum() > 0.99 * conv0.sum()
    for k, (ep, em, h) in enumerate(runs):
        mp, mm = moments_on(phx, ep, keep, ns), moments_on(phx, em, keep, ns)
        fd[:, :, k] = (mp[:, 1:] - mm[:, 1:]) / (2 * h)
    # adjoint on the same set: per-photon Jacobians restricted to it, one output at a time
    tr.set_perturbation(theta0)
    _, jac = tr.adjoint(torch.zeros((ns, 8), dtype=torch.float64), photon_count=n, jac_stride=1)
    torch.cuda.synchronize()
    j = jac.cpu().numpy()
    m0 = moments_on(phx, e0, keep, ns)
    adj = np.zeros_like(fd)
    for si in range(ns):
        k = keep & (e0["source"] == si)
        N = k.sum()
        dx, dy = e0["xe"][k] - m0[si, 1], e0["ye"][k] - m0[si, 2]
        Jx, Jy = j[k, 0], j[k, 1]
        adj[si, 0] = Jx.sum(0) / N
        adj[si, 1] = Jy.sum(0) / N
        adj[si, 2] = 2 * (dx[:, None] * Jx).sum(0) / N
        adj[si, 3] = 2 * (dy[:, None] * Jy).sum(0) / N
        adj[si, 4] = ((dy[:, None] * Jx) + (dx[:, None] * Jy)).sum(0) / N
    a, b = adj * RANGE, fd * RANGE
    # each entry to 1e-4 of itself, above a floor of 1e-6 of its row's largest entry (the central
    # differences' truncation error, O(h^2) relative, and the rounding of the GPU positions over
    # 2h are far below it; entries that vanish by symmetry meet the floor)
    row = np.abs(b).max(axis=2, keepdims=True)
    err = np.abs(a - b)
    bound = 1e-4 * np.abs(b) + 1e-6 * row
    worst = (err / bound).max()
    print(f"adjoint vs central differences: worst error / bound {worst:.3f}, "
          f"worst relative error of entries above 1e-3 of their row "
          f"{(err / np.abs(b))[np.abs(b) > 1e-3 * row].max():.2e}")
    assert np.all(err <= bound), worst
    tr.close()


def test_autograd_function_backward(phx):
    """psf_moments(theta).backward() equals the adjoint called with the same cotangents, and
    its value equals the host moments of the forward words."""
    import torch
    from paper_1504_06570_amd.autograd import psf_moments
    s = C.gradients(scale=2e-4, screen_n=128)
    tr = phx.Tracer(s)
    theta = torch.tensor(np.random.default_rng(26).uniform(-1, 1, C.N_PERTURB) * RANGE,
                         dtype=torch.float64, requires_grad=True)
    out = psf_moments(theta, tr, photon_count=3000)
    w = torch.tensor(np.random.default_rng(27).standard_normal(out.shape), dtype=torch.float64)
    (out * w.to(out.device)).sum().backward()
    tr.set_perturbation(theta.detach().numpy())
    m = tr.new_moments()
    tr.trace(moments=m, photon_count=3000)
    torch.cuda.synchronize()
    mom = R.moments_from_sums(phx.moment_sums(m))
    assert np.array_equal(out.detach().cpu().numpy(), mom[:, 1:])
    g = tr.adjoint(torch.from_numpy(R.adjoint_seeds(mom, w.numpy())), photon_count=3000)
    torch.cuda.synchronize()
    assert torch.equal(theta.grad, g.cpu())
    tr.close()


def test_adjoint_error_paths(phx):
    import torch
    s = C.tiny()
    tr = phx.Tracer(s)
    with pytest.raises(phx.PhxError):
        tr.adjoint(torch.zeros((2, 8), dtype=torch.float64))      # wrong seed rows
    with pytest.raises(phx.PhxError):
        tr.adjoint(torch.zeros((3, 8), dtype=torch.float64), src_begin=0, src_end=3)
    tr.close()
