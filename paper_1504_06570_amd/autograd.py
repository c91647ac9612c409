"""Differentiable PSF moments: torch.autograd.Function over the trace and its adjoint.

``psf_moments(theta, tracer)`` traces the tracer's sources with the optics perturbed by
``theta`` (22 parameters: two rigid-body groups x (shift x, shift y, tilt x, tilt y, piston), then
the primary's Zernike Z4..Z15 amplitudes) and returns per source the mean electron position and
the central second moments (Ixx, Iyy, Ixy) of its converted photons.  The backward pass calls the
library's adjoint trace: the pathwise derivative with every photon's random numbers and discrete
decisions held fixed (a fixed-seed estimator).  Both passes run in the library's HIP kernels.
"""
from __future__ import annotations


def _function():
    import torch

    class _PsfMoments(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, tracer, kw):
            th = theta.detach().to("cpu", torch.float64).numpy()
            tracer.set_perturbation(th)
            src_begin = kw.get("src_begin", 0)
            src_end = kw.get("src_end", None)
            src_end = tracer.n_sources if src_end is None else src_end
            words = tracer.new_moments()
            image = tracer.new_image()
            tracer.trace(image, moments=words, **kw)
            mom = tracer.moments(words)[src_begin:src_end, 1:]
            ctx.tracer, ctx.kw, ctx.words, ctx.theta = tracer, dict(kw), words, th
            ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
            return mom.to(theta.device)

        @staticmethod
        def backward(ctx, gout):
            tr = ctx.tracer
            tr.set_perturbation(ctx.theta)
            kw = {k: v for k, v in ctx.kw.items() if k not in ("stats", "event_stride", "events")}
            grad = tr.adjoint_moments(ctx.words, gout.detach(), **kw)
            return grad.to(ctx.theta_device, ctx.theta_dtype), None, None

    return _PsfMoments


_FN = None


def psf_moments(theta, tracer, **trace_kw):
    """theta: float64 tensor [22] -> tensor [n_sources, 5] of (mean x, mean y, Ixx, Iyy, Ixy) in
    metres / square metres (detector frame).  trace_kw: flags, seed, src_begin, src_end,
    photon_begin, photon_count, stream (as Tracer.trace)."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(theta, tracer, trace_kw)


def moment_names():
    return ["mean_x", "mean_y", "Ixx", "Iyy", "Ixy"]

