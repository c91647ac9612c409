"""Benchmark: photons/s of the full atmosphere + optics + sensor photon trace on one MI355X.

Workload (one step): one star at a random field position, 1e9 photons, seven frozen-flow von
Karman layers (2048^2 screens at 1 m / 10 cm / 1 cm), the generated three-mirror telescope +
camera with coatings, 100 um silicon with diffusion, a 4096^2 chip centred on the star.  Inputs
are synthetic and resident on the GPU before timing; the image accumulates across steps.

Prints one JSON line.  `--gpus N` with N > 1 exits: the trace runs on one GPU (photons shard by
key across GPUs with one image sum, which is not implemented).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photons/s (atm+optics+sensor) on 1 MI355X vs oracle; adjoint/forward cost ratio"
PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1504_06570_amd", "csrc", "phx_trace.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "trace_kernel_full_1e9_pmc.json")

PEAK_INT32_TOPS = 78.6    # 32-bit integer VALU lane operations: 256 CU x 4 SIMD x 32 lanes x 2.4 GHz
OP_COUNTS = os.path.join(ROOT, "profiles", "oracle_op_counts_full.json")
FP64_FIELDS = ("add", "mul", "div", "sqrt", "trans")
# Implementation traffic of the sky stage (not the method's): the 7-double start-plane state each
# traced photon hands to the optics stage.
STATE_BYTES = 7 * 8
# Integer operations of one Philox4x32-10 block: ten rounds of two 32x32 -> 64-bit products, two
# three-way XORs (four XORs) and two key additions.
PHILOX_INT_OPS = 10 * 8
# The pre-roll's algorithmic work per generated photon, a lower bound: the block holding its
# wavelength and pupil radius and the block holding the first (most selective) roulette word.
PREROLL_BLOCKS = 2


def op_counts():
    """The oracle counting build's mean operations per photon by outcome (committed table)."""
    try:
        return json.load(open(OP_COUNTS))
    except (OSError, ValueError):
        return None


def front_bytes_per_photon(n_layers, n_scales, counts=None):
    """Algorithmic bytes per traced photon of the sky stage: the screen footprints the method
    gathers (from the counting build when its table is there: 7 layers x 3 scales x 32 B)."""
    if counts is not None:
        return counts["by_outcome"]["all"]["sky"]["gather_bytes"]
    return n_layers * n_scales * 4 * 8


def back_ops_by_class(stats, counts):
    """FP64 operations of the optics + sensor stage for this launch's traced photons, per class
    (add/sub, mul, div, sqrt, transcendental): each outcome group's count in the launch statistics
    times its mean count in the oracle's counting build (a group absent from the counted sample
    takes the mean of its status)."""
    from paper_1504_06570_amd import phx
    tab = phx.stats_table(stats)
    by = counts["by_outcome"]

    def ops(rec, f):
        return rec["optics"][f] + rec["sensor"][f]
    total = {f: 0.0 for f in FP64_FIELDS}
    for st in range(phx.N_STATUS):
        if st == phx.CULLED:
            continue
        for col in range(tab.shape[1]):
            n = float(tab[st, col])
            if n == 0:
                continue
            key = f"{phx.STATUS[st]}@{col - 1}"
            same = [v for k, v in by.items() if k.split("@")[0] == phx.STATUS[st]]
            for f in FP64_FIELDS:
                if key in by:
                    total[f] += n * ops(by[key], f)
                else:
                    total[f] += n * (np.mean([ops(v, f) for v in same]) if same
                                     else ops(by["all"], f))
    return total


def back_flops(stats, counts):
    """FP64 operations of the optics + sensor stage (every class counted as one operation)."""
    return sum(back_ops_by_class(stats, counts).values())


# FP64 operation classes of the op-rate probe (probe_fp64's kind codes)
OP_KINDS = {"fma": (0, 4000), "div": (1, 1000), "sqrt": (2, 1000), "exp": (3, 400),
            "log": (4, 200), "sin": (5, 200), "div_refined": (6, 2000),
            "sqrt_refined": (7, 2000)}


def fp64_op_rates(threads=1 << 22, reps=3):
    """Operations per second of each FP64 class as compiled for this GPU (probe_fp64 of
    libphx_probe.so: 8 independent chains per thread, so the issue rate is measured, not the
    latency); None when the probe library is not built."""
    import ctypes as C
    import torch
    from paper_1504_06570_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        return None
    lib = C.CDLL(B.PROBE_LIB)
    lib.probe_fp64.argtypes = [C.c_int, C.c_void_p, C.c_uint64, C.c_int, C.c_void_p]
    lib.probe_fp64.restype = C.c_int
    out = torch.empty(threads, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    rates = {}
    for name, (kind, iters) in OP_KINDS.items():
        def run():
            rc = lib.probe_fp64(kind, out.data_ptr(), threads, iters, C.c_void_p(stream.cuda_stream))
            if rc != 0:
                raise SystemExit(f"bench.py: probe_fp64 returned {rc}")
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rates[name] = threads * iters * 8 / (ms * 1e-3)
    return rates


def philox_rate(threads=1 << 22, iters=64, reps=3):
    """Philox4x32-10 blocks per second as the trace kernels compute them (probe_philox of
    libphx_probe.so); None when the probe library is not built."""
    import ctypes as C
    import torch
    from paper_1504_06570_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        return None
    lib = C.CDLL(B.PROBE_LIB)
    lib.probe_philox.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.c_void_p]
    lib.probe_philox.restype = C.c_int
    out = torch.empty(threads, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run():
        rc = lib.probe_philox(out.data_ptr(), threads, iters, C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise SystemExit(f"bench.py: probe_philox returned {rc}")
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    return threads * iters * 8 / (e0.elapsed_time(e1) / reps * 1e-3)


def per_class_seconds(ops, rates):
    """Time of FP64 operations by class at the measured rates: additions and multiplications
    paired into fused multiply-adds, divisions and square roots at the rates of the refined
    hardware estimates (the faster forms, so the bound is the stricter one), transcendentals at
    the harmonic mean of exp, log and sin."""
    trans = 3.0 / (1.0 / rates["exp"] + 1.0 / rates["log"] + 1.0 / rates["sin"])
    div = max(rates["div"], rates["div_refined"])
    sqrt = max(rates["sqrt"], rates["sqrt_refined"])
    return ((ops["add"] + ops["mul"]) / (2.0 * rates["fma"]) + ops["div"] / div +
            ops["sqrt"] / sqrt + ops["trans"] / trans)


def kernel_hash():
    h = hashlib.sha256()
    for p in (KERNEL_SRC, os.path.join(ROOT, "paper_1504_06570_amd", "csrc", "phx_internal.h")):
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(n_launch_photons, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None if it is missing or was taken on a different kernel source."""
    try:
        d = json.load(open(PMC_SUMMARY))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash() or d.get("photons") != n_launch_photons:
        return None
    # keys carry the template arguments of the instantiation (`front_kernel<false, false>`); the
    # headline command launches one instantiation of each kernel
    hbm = d.get("hbm_bytes_per_launch", {})
    keys = [k for k in hbm if k == kernel or k.startswith(kernel + "<")]
    return hbm[keys[0]] if len(keys) == 1 else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, n_photons, threads):
    """The oracle on the host: photons [0, n_photons) of the headline star, full physics, no
    pre-roll (the oracle traces every photon to its fate), split over `threads` threads."""
    import oracle as O
    orc = O.Oracle(scene)
    img = np.zeros(orc.image_shape, np.uint32)
    counts = np.array([n_photons], np.uint64)
    t0 = time.perf_counter()
    orc.trace_sources(counts=counts, image=img, events=False, threads=threads)
    dt = time.perf_counter() - t0
    return n_photons / dt, dt


def batched_leg(steps, per_source_steps=1, variant_slope=-1.1):
    """Many uneven sources: one graph-replayed launch over all of them (launch shape picked by
    the autotuner) against one plain launch per source, on the same GPU and the same photons."""
    import numpy as np
    import torch
    from paper_1504_06570_amd import phx
    from paper_1504_06570_amd.scene import configs as C
    t0 = time.perf_counter()
    scene = C.batched()
    tr = phx.Tracer(scene)
    print(f"# batched setup {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    flags = int(scene.physics) | phx.F_CULL
    counts = scene.sources.n_photons.astype(np.int64)
    total = int(counts.sum())
    t0 = time.perf_counter()
    best = tr.autotune(flags=flags, batched=True)   # graph replays, two streams captured
    t_tune = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # untimed first passes of both forms into fresh images: they must be identical
    one_b = tr.new_image()
    tr.trace(one_b, flags=flags, batched=True)
    one_p = tr.new_image()
    for s in range(len(counts)):
        tr.trace(one_p, flags=flags, src_begin=s, src_end=s + 1, photon_count=int(counts[s]))
    torch.cuda.synchronize()
    same = bool(torch.equal(one_b, one_p))
    del one_p
    img = tr.new_image()
    e0.record(stream)
    for _ in range(steps):
        tr.trace(img, flags=flags, batched=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(per_source_steps):
        for s in range(len(counts)):
            tr.trace(img, flags=flags, src_begin=s, src_end=s + 1, photon_count=int(counts[s]))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1) / per_source_steps
    same = same and bool(torch.equal(img, one_b * (steps + per_source_steps)))
    tr.close()
    print(f"# batched {ms_b:.2f} ms, per-source {ms_p:.2f} ms, tune {t_tune:.1f}s {best}",
          file=sys.stderr, flush=True)
    # the same catalogue with counts drawn from a shallower power law (slope -1.1), the photon
    # total the configuration quotes (~3e9); batched launch only
    variant = None
    if variant_slope is not None:
        sv = C.batched(slope=variant_slope)
        tv = phx.Tracer(sv)
        tot_v = int(sv.sources.n_photons.astype(np.int64).sum())
        tv.set_launch_config(**{k: v for k, v in best.items()})
        img_v = tv.new_image()
        tv.trace(img_v, flags=flags, batched=True)
        torch.cuda.synchronize()
        e0.record(stream)
        tv.trace(img_v, flags=flags, batched=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_v = e0.elapsed_time(e1)
        tv.close()
        variant = {"slope": variant_slope, "photons_per_step": tot_v, "ms_per_step": ms_v,
                   "value": tot_v / (ms_v * 1e-3)}
        print(f"# batched slope {variant_slope}: {tot_v:.3e} photons, {ms_v:.1f} ms",
              file=sys.stderr, flush=True)
    return {
        "workload": f"{len(counts)} sources (80% stars, 20% Sersic), power-law counts slope -1.5 "
                    f"on [10, 1e7], blackbody SEDs, full atmosphere + optics + sensor",
        "photons_per_step": total,
        "value": total / (ms_b * 1e-3),
        "ms_per_step": ms_b,
        "per_source_value": total / (ms_p * 1e-3),
        "per_source_ms_per_step": ms_p,
        "speedup_vs_per_source": ms_p / ms_b,
        "images_identical": same,
        "launch_config": best,
        "autotune_s": t_tune,
        "variant": variant,
    }


def gradient_leg(steps):
    """Fixed-seed gradients of per-source centroids and second moments with respect to the 22
    optics parameters: 25 stars on a 5 x 5 grid, 1e7 photons each, full atmosphere + optics +
    sensor.  Times the forward trace with moments and the adjoint trace of the same photons."""
    import numpy as np
    import torch
    from paper_1504_06570_amd import phx
    from paper_1504_06570_amd.scene import configs as C
    t0 = time.perf_counter()
    scene = C.gradients()
    tr = phx.Tracer(scene)
    theta = np.random.default_rng(5).uniform(-1, 1, C.N_PERTURB) * C.PERTURB_RANGE
    tr.set_perturbation(theta)
    print(f"# gradient setup {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    flags = int(scene.physics) | phx.F_CULL
    total = int(scene.sources.n_photons.sum())
    stream = torch.cuda.current_stream()
    img = tr.new_image()
    m = tr.new_moments()
    tr.trace(img, flags=flags, moments=m)
    torch.cuda.synchronize()
    dmom = torch.from_numpy(np.random.default_rng(6).standard_normal((len(scene.sources), 5)))
    grad = tr.adjoint_moments(m, dmom, flags=flags)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        m.zero_()
        tr.trace(img, flags=flags, moments=m)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1) / steps
    tr.set_timing(True)
    e0.record(stream)
    for _ in range(steps):
        tr.adjoint_moments(m, dmom, flags=flags, grad=grad)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_a = e0.elapsed_time(e1) / steps
    kt = tr.get_timing()
    tr.set_timing(False)
    tr.close()
    print(f"# forward {ms_f:.2f} ms, adjoint {ms_a:.2f} ms, kernels {kt}", file=sys.stderr,
          flush=True)
    return {
        "workload": "25 stars on a 5x5 field grid, 1e7 photons each, full atmosphere + optics + "
                    "sensor, perturbed optics; gradients of per-source centroid and second "
                    "moments with respect to 22 parameters",
        "photons_per_step": total,
        "forward_ms": ms_f,
        "adjoint_ms": ms_a,
        "adjoint_forward_ratio": ms_a / ms_f,
        "forward_photons_per_s": total / (ms_f * 1e-3),
        "adjoint_photons_per_s": total / (ms_a * 1e-3),
        "adjoint_stage_ms": {k: kt[k] / steps for k in ("generate", "compact", "front", "back")},
    }


def extras_leg(tr, scene, flags, steps, n_ph, core_ms, tune=True):
    """The headline step with aerosol extinction, dispersion, dome seeing, the micro-roughness
    halo, the spider and the dead layer switched on (their kernels' EXTRA instantiations): time
    per step, its cost against the core step, and each kernel's duration on a single stream."""
    import torch
    from paper_1504_06570_amd import phx
    from paper_1504_06570_amd.scene import physics as X
    tr.load_physics(X.tma_extras())
    fx = flags | X.PHYS_EXTRA
    base_cfg = tr.launch_config()
    t0 = time.perf_counter()
    # the leg's own launch shape (unless the command fixes it); the tracer's is restored after
    tuned = tr.autotune(flags=fx) if tune else base_cfg
    t_tune = time.perf_counter() - t0
    img = tr.new_image()
    stats = tr.new_stats()
    tr.trace(img, flags=fx)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    tr.set_timing(True)
    e0.record(stream)
    for _ in range(steps):
        tr.trace(img, flags=fx, stats=stats)
    e1.record(stream)
    torch.cuda.synchronize()
    kt = tr.get_timing()
    tr.set_timing(False)
    ms = e0.elapsed_time(e1) / steps
    st = stats.cpu().numpy()
    tab = phx.stats_table(st) / steps
    traced = float(st[phx.STAT_TRACED]) / steps
    # each kernel alone (single stream)
    tr.set_launch_config(pipeline=0)
    tr.set_timing(True)
    tr.trace(tr.new_image(), flags=fx)
    torch.cuda.synchronize()
    kti = tr.get_timing()
    tr.set_timing(False)
    tr.set_launch_config(**base_cfg)
    ci = max(kti["chunks"], 1.0)
    atm = scene.atmosphere
    f_ms = kti["front"] / ci
    f_bytes = traced * front_bytes_per_photon(atm.n_layers, atm.n_scales) / ci
    f_gbs = f_bytes / (f_ms * 1e-3) * 1e-9
    print(f"# extra physics {ms:.2f} ms/step ({ms / core_ms:.2f}x core), tuned {tuned} in "
          f"{t_tune:.1f}s, kernels {kt}", file=sys.stderr, flush=True)
    return {
        "workload": "the headline star with aerosol extinction, dispersion, dome seeing, the "
                    "micro-roughness halo, a four-vane spider and a 50 nm dead layer on "
                    "(pre-roll on; its geometric cull is off with entrance kicks)",
        "photons_per_step": n_ph,
        "ms_per_step": ms,
        "value": n_ph / (ms * 1e-3),
        "cost_vs_core": ms / core_ms,
        "traced_per_step": traced,
        "detected_per_step": float(tab[phx.DETECTED].sum()),
        "extinct_per_step": float(tab[phx.EXTINCT].sum()),
        "dead_per_step": float(tab[phx.DEAD].sum()),
        "obscured_per_step": float(tab[phx.OBSCURED].sum()),
        "stage_ms_per_step": {k: kt[k] / steps for k in ("generate", "compact", "front", "back")},
        "stage_ms_single_stream": {k: kti[k] for k in ("generate", "compact", "front", "back")},
        "front_kernel_single_stream": {"bound": "hbm", "achieved": f_gbs, "peak": PEAK_HBM_GBS,
                                       "unit": "GB/s", "frac": f_gbs / PEAK_HBM_GBS,
                                       "launch_ms": f_ms},
        "back_kernel_single_stream_ms": kti["back"] / ci,
        "launch_config": tuned,
        "autotune_s": t_tune,
    }


def ghost_leg(tr, flags, steps, n_ph, core_ms, tune=True):
    """The headline step with ghost reflections: filter, lens and detector coatings reflect what
    they do not transmit (a fixed share), and reflected photons are traced non-sequentially."""
    import numpy as np
    import torch
    from paper_1504_06570_amd import phx
    from paper_1504_06570_amd.scene import coatings as cm
    rt = np.ascontiguousarray(cm.standard_reflectance(), np.float32)
    tr._check(tr.L.phx_load_reflectance(tr.ctx, rt.ctypes.data, *rt.shape))
    fx = flags | phx.F_GHOSTS
    # the ghost trace's own launch shape, tuned on a quarter of the step (four chunks) unless the
    # command fixes it; the tracer's shape is restored afterwards
    base_cfg = tr.launch_config()
    t0 = time.perf_counter()
    tuned = tr.autotune(flags=fx, photon_count=1 << 28) if tune else base_cfg
    t_tune = time.perf_counter() - t0
    img = tr.new_image()
    stats = tr.new_stats()
    tr.trace(img, flags=fx)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        tr.trace(img, flags=fx, stats=stats)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = stats.cpu().numpy()
    tab = phx.stats_table(st) / steps
    tr.set_launch_config(**base_cfg)
    rel = f" ({ms / core_ms:.2f}x core)" if core_ms else ""
    print(f"# ghosts {ms:.2f} ms/step{rel}, tuned {tuned} in {t_tune:.1f}s", file=sys.stderr,
          flush=True)
    return {
        "workload": "the headline star with ghost reflections (filter, lens and detector "
                    "coatings reflect 0.95 / 0.9 / 0.85 of what they do not transmit; pre-roll "
                    "on without its coating tests)",
        "photons_per_step": n_ph,
        "ms_per_step": ms,
        "value": n_ph / (ms * 1e-3),
        "cost_vs_core": ms / core_ms if core_ms else None,
        "traced_per_step": float(st[phx.STAT_TRACED]) / steps,
        "detected_per_step": float(tab[phx.DETECTED].sum()),
        "off_chip_per_step": float(tab[phx.OFF_CHIP].sum()),
        "launch_config": tuned,
        "autotune_s": t_tune,
    }


def launch_shape(text):
    """--launch G,F,B[,C]: pre-roll, sky and optics workgroups per compute unit, and optionally
    the chunk size's log2."""
    v = [int(x) for x in text.split(",")]
    if len(v) not in (3, 4):
        raise SystemExit("bench.py: --launch takes G,F,B or G,F,B,C")
    shape = dict(generate_blocks_per_cu=v[0], front_blocks_per_cu=v[1], back_blocks_per_cu=v[2])
    if len(v) == 4:
        shape["chunk_log2"] = v[3]
    return shape


def ghosts_only(args):
    """The ghost leg alone on the headline star (for profiling it): the launch shape from
    --launch, else the leg's own tuning."""
    from paper_1504_06570_amd import phx
    from paper_1504_06570_amd.scene import configs as C
    n_ph = int(args.photons)
    scene = C.full()
    scene.sources.n_photons[:] = n_ph
    tr = phx.Tracer(scene)
    if args.launch:
        tr.set_launch_config(**launch_shape(args.launch))
    out = ghost_leg(tr, int(scene.physics) | phx.F_CULL, max(args.steps, 1), n_ph, None,
                    tune=not (args.launch or args.no_autotune))
    tr.close()
    return out


def hybrid_leg(steps, n_ph, core_ms, launch=None):
    """The headline star through the hybrid two-kick atmosphere: the same seven layers with their
    screens limited to wavenumbers below kappa_crit = 2 pi / (1.5 r0) and the higher modes applied
    as the per-layer second kick (pre-roll on; its geometric cull is off with the kick)."""
    import torch
    from paper_1504_06570_amd import phx
    from paper_1504_06570_amd.scene import configs as C
    t0 = time.perf_counter()
    scene = C.hybrid()
    scene.sources.n_photons[:] = n_ph
    tr = phx.Tracer(scene)
    setup = time.perf_counter() - t0
    flags = int(scene.physics) | phx.F_CULL
    t0 = time.perf_counter()
    if launch is None:
        tuned = tr.autotune(flags=flags)   # the leg's own launch shape
    else:
        tr.set_launch_config(**launch)     # the shape the command fixes
        tuned = tr.launch_config()
    t_tune = time.perf_counter() - t0
    img = tr.new_image()
    stats = tr.new_stats()
    tr.trace(img, flags=flags)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    tr.set_timing(True)
    e0.record(stream)
    for _ in range(steps):
        tr.trace(img, flags=flags, stats=stats)
    e1.record(stream)
    torch.cuda.synchronize()
    kt = tr.get_timing()
    tr.set_timing(False)
    ms = e0.elapsed_time(e1) / steps
    st = stats.cpu().numpy()
    tab = phx.stats_table(st) / steps
    tr.set_launch_config(pipeline=0)
    tr.set_timing(True)
    tr.trace(tr.new_image(), flags=flags)
    torch.cuda.synchronize()
    kti = tr.get_timing()
    tr.set_timing(False)
    ci = max(kti["chunks"], 1.0)
    traced = float(st[phx.STAT_TRACED]) / steps
    atm = scene.atmosphere
    f_ms = kti["front"] / ci
    f_gbs = traced * front_bytes_per_photon(atm.n_layers, atm.n_scales) / ci / (f_ms * 1e-3) * 1e-9
    tr.close()
    print(f"# hybrid atmosphere {ms:.2f} ms/step ({ms / core_ms:.2f}x core), setup {setup:.1f}s, "
          f"tuned {tuned} in {t_tune:.1f}s", file=sys.stderr, flush=True)
    return {
        "workload": "the headline star through the hybrid two-kick atmosphere (screens below "
                    "kappa_crit = 2 pi / (1.5 r0), second kick per layer; phase variance above "
                    "kappa_crit 0.167 summed over layers)",
        "photons_per_step": n_ph,
        "ms_per_step": ms,
        "value": n_ph / (ms * 1e-3),
        "cost_vs_core": ms / core_ms,
        "traced_per_step": traced,
        "detected_per_step": float(tab[phx.DETECTED].sum()),
        "stage_ms_per_step": {k: kt[k] / steps for k in ("generate", "compact", "front", "back")},
        "stage_ms_single_stream": {k: kti[k] for k in ("generate", "compact", "front", "back")},
        "front_kernel_single_stream": {"bound": "hbm", "achieved": f_gbs, "peak": PEAK_HBM_GBS,
                                       "unit": "GB/s", "frac": f_gbs / PEAK_HBM_GBS,
                                       "launch_ms": f_ms},
        "back_kernel_single_stream_ms": kti["back"] / ci,
        "launch_config": tuned,
        "autotune_s": t_tune,
    }


READOUT_BYTES_PER_PIXEL = 46   # zero both slot buffers (8), bleed copy (8), defects (8),
                               # parallel read + add (8), serial read + add (8), digitise (6)


def readout_leg(tr, img, steps):
    """The readout chain (bleeding, dark current, defects, per-electron parallel and serial
    transfers, digitisation) of one step's 4096^2 image of the headline star on 16 amplifiers."""
    import torch
    from paper_1504_06570_amd.scene.readout import Readout
    rp = Readout()
    out = tr.readout(img, rp)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        out = tr.readout(img, rp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ny, nx = img.shape
    electrons = float(img.double().sum().item())
    # electrons each transfer stage draws a delay for (after bleeding, dark current and defects:
    # hot pixels and hot columns at full well dominate)
    _, work, par, _ = tr.readout(img, rp, stages=True)
    torch.cuda.synchronize()
    moved = float(work.view(torch.int32).double().sum().item() +
                  par.view(torch.int32).double().sum().item())
    del work, par
    gbs = READOUT_BYTES_PER_PIXEL * nx * ny / (ms * 1e-3) * 1e-9
    print(f"# readout {ms:.3f} ms ({electrons:.3e} electrons in, {moved:.3e} transferred)",
          file=sys.stderr, flush=True)
    return {
        "workload": "readout chain of one step's 4096^2 image of the headline star (16 amplifiers "
                    "8 x 2, 10 overscan rows and columns, full well 1e5, CTE 0.999995 / 0.999998)",
        "pixels": nx * ny,
        "electrons": electrons,
        "ms_per_readout": ms,
        "pixels_per_s": nx * ny / (ms * 1e-3),
        "electrons_per_s": electrons / (ms * 1e-3),
        "transfer_electron_draws": moved,
        "transfer_draws_per_s": moved / (ms * 1e-3),
        "hbm_algorithmic": {"bytes_per_pixel": READOUT_BYTES_PER_PIXEL, "achieved": gbs,
                            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS},
        "adu_shape": list(out.shape),
    }


def copy_probe():
    """A plain 1 GiB device copy, for calibrating the HBM byte counters."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": a.numel() * 4}))


def gather_probe(footprints_mib=(4, 64, 256, 940, 2816), threads=1 << 24, reps=10):
    """Random gathers of 32-byte records (one screen-cell record of the sky stage) over tables of
    several sizes, by the probe kernel of libphx_probe.so: each thread makes 7 dependent rounds
    of 1 or 3 independent gathers (the sky stage's 7 layers, one or all 3 screen scales in
    flight).  940 MiB is the footprint of the seven finest screens, 2816 MiB that of all 21
    screens of the headline workload.  Prints one JSON line: records per second and the rate in
    128-byte lines (the L2 line each missing record brings in)."""
    import ctypes as C
    import torch
    from paper_1504_06570_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        raise SystemExit(f"bench.py: {B.PROBE_LIB} is not built (python -c 'import "
                         "__graft_entry__ as g; g.build()')")
    lib = C.CDLL(B.PROBE_LIB)
    lib.probe_gather.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_int,
                                 C.c_int, C.c_uint32, C.c_void_p]
    lib.probe_gather.restype = C.c_int
    stream = torch.cuda.current_stream()
    out = torch.empty(threads, dtype=torch.int32, device="cuda")
    rows = []
    for mib in footprints_mib:
        n_rec = mib * (1 << 20) // 32
        table = torch.zeros(n_rec * 8, dtype=torch.int32, device="cuda")
        for width in (1, 3):
            def run(seed):
                rc = lib.probe_gather(table.data_ptr(), n_rec, out.data_ptr(), threads, 7, width,
                                      seed, C.c_void_p(stream.cuda_stream))
                if rc != 0:
                    raise SystemExit(f"bench.py: probe_gather returned {rc}")
            run(1)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for r in range(reps):
                run(2 + r)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            recs = threads * 7 * width
            rows.append({"footprint_mib": mib, "in_flight_per_thread": width, "records": recs,
                         "ms": ms, "records_per_s": recs / (ms * 1e-3),
                         "record_GBps": recs * 32 / (ms * 1e-3) * 1e-9,
                         "line_GBps": recs * 128 / (ms * 1e-3) * 1e-9})
            print(f"# gather {mib} MiB x{width}: {rows[-1]['records_per_s']:.3e} records/s",
                  file=sys.stderr, flush=True)
        del table
    print(json.dumps({"gather_probe": rows}), flush=True)


_KERNEL_NAME = None


def kernel_short_name(name):
    """`back_kernel<false, false, false>` from a demangled rocprofv3 kernel name."""
    import re
    global _KERNEL_NAME
    if _KERNEL_NAME is None:
        _KERNEL_NAME = re.compile(r"([A-Za-z_]\w*(?:<[^()]*>)?)\(")
    m = _KERNEL_NAME.search(name)
    return m.group(1) if m else name[:48]


def summarize_stats(csv_path):
    """Table of a rocprofv3 `--stats` kernel summary (its *_kernel_stats.csv): calls, average and
    total duration per kernel, in milliseconds."""
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    agg = {}
    for r in rows:
        k = kernel_short_name(r["Name"])
        a = agg.setdefault(k, [0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"]) * 1e-6
    tot = sum(a[1] for a in agg.values()) or 1.0
    lines = [f"{'kernel':40s} {'calls':>7s} {'avg_ms':>9s} {'total_ms':>10s} {'pct':>6s}"]
    for k, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{k[:40]:40s} {n:7d} {t / n:9.4f} {t:10.2f} {100 * t / tot:6.2f}")
    return "\n".join(lines)


def _counter_rows(d):
    """{(kernel, counter): [values per dispatch]} of a rocprofv3 `--pmc` run's directory."""
    import csv
    import glob
    out = {}
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        for r in csv.DictReader(open(f)):
            k = kernel_short_name(r.get("Kernel_Name") or r.get("Kernel-Name") or "")
            out.setdefault((k, r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    return out


def summarize_pmc(dirs, copy_dirs, photons, json_out):
    """Per-dispatch means of the counters of several rocprofv3 `--pmc` runs of the headline command,
    and the HBM bytes per launch from FETCH_SIZE and WRITE_SIZE scaled by what the same counters
    read for a plain device copy of known size (the two `--copy-probe` runs).  Writes the JSON that
    the benchmark's `traffic` field reads (keyed to the kernel source's hash) and returns a
    table."""
    rows = {}
    for d in dirs:
        for key, v in _counter_rows(d).items():
            rows.setdefault(key, []).extend(v)
    copy = {}
    for d in copy_dirs:
        for key, v in _counter_rows(d).items():
            copy.setdefault(key, []).extend(v)
    copy_bytes = float(1 << 30)
    # the copy is the dispatch that fetches the most; its write counter is read on the same kernel
    fk = max((k for k in copy if k[1] == "FETCH_SIZE"), key=lambda k: max(copy[k]))
    fetch_kib = max(copy[fk])
    write_kib = max(copy.get((fk[0], "WRITE_SIZE"), [0.0]))
    fetch_factor = copy_bytes / 1024 / fetch_kib
    write_factor = copy_bytes / 1024 / write_kib if write_kib else None
    kernels = sorted({k for k, _ in rows})
    mean = {k: {c: float(np.mean(v)) for (kk, c), v in rows.items() if kk == k} for k in kernels}
    calls = {k: max(len(v) for (kk, _), v in rows.items() if kk == k) for k in kernels}
    hbm = {}
    for k, m in mean.items():
        if "FETCH_SIZE" in m and "WRITE_SIZE" in m and write_factor:
            hbm[k] = (m["FETCH_SIZE"] * fetch_factor + m["WRITE_SIZE"] * write_factor) * 1024
    rec = {
        "kernel_hash": kernel_hash(),
        "photons": int(photons),
        "calibration": {"copy_bytes_each_way": copy_bytes, "copy_kernel": fk[0],
                        "copy_fetch_kib": fetch_kib, "copy_write_kib": write_kib,
                        "fetch_factor": fetch_factor, "write_factor": write_factor},
        "hbm_bytes_per_launch": hbm,
        "counters_per_dispatch": mean,
        "dispatches": calls,
    }
    with open(json_out, "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# copy calibration: {fk[0]} reads {fetch_kib:.0f} KiB FETCH_SIZE and writes "
             f"{write_kib:.0f} KiB WRITE_SIZE for 1 GiB each way -> fetch factor "
             f"{fetch_factor:.3f}, write factor {write_factor:.3f}", ""]
    for k in sorted(kernels, key=lambda k: -hbm.get(k, 0.0)):
        if not any(t in k for t in ("_kernel", "bucket_", "compact_")):
            continue
        lines.append(f"{k}   dispatches {calls[k]}" +
                     (f"   HBM bytes per launch {hbm[k]:.4e}" if k in hbm else ""))
        for c in sorted(mean[k]):
            lines.append(f"    {c:28s} {mean[k][c]:.4e}")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--photons", type=float, default=1e9)
    ap.add_argument("--no-cull", action="store_true", help="time without the pre-roll only")
    ap.add_argument("--cpu-sample", type=float, default=8e7)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--op-probe", action="store_true",
                    help="issue rates of the FP64 operation classes (fma, div, sqrt, exp, log, "
                         "sin) and of Philox blocks")
    ap.add_argument("--gather-probe", action="store_true",
                    help="random 32-byte record gathers over tables of 4 MiB - 2.75 GiB (the "
                         "memory system's rate for the sky stage's access pattern)")
    ap.add_argument("--no-compare", action="store_true", help="skip the run without the pre-roll")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-source batched leg")
    ap.add_argument("--no-gradient", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the legs with the per-photon physics beyond the core path and the "
                         "hybrid atmosphere")
    ap.add_argument("--only", choices=("batched", "gradient", "ghosts"), default=None,
                    help="run one secondary leg alone and print its record (for profiling)")
    ap.add_argument("--launch", default=None, metavar="G,F,B[,C]",
                    help="fixed launch shape (pre-roll, sky and optics workgroups per compute "
                         "unit, optionally the chunk size's log2) in place of the autotuner, so "
                         "that a profile holds only the timed launches")
    ap.add_argument("--no-single-stream", action="store_true",
                    help="skip the step with both stages on one stream")
    ap.add_argument("--summarize-stats", default=None, metavar="CSV",
                    help="print the table of a rocprofv3 --stats kernel summary and exit")
    ap.add_argument("--summarize-pmc", nargs="+", default=None, metavar="DIR",
                    help="rocprofv3 --pmc output directories of the headline command: print "
                         "per-dispatch counter means, write the HBM traffic summary and exit")
    ap.add_argument("--copy-dirs", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="with --summarize-pmc: the two --copy-probe counter runs")
    ap.add_argument("--pmc-json", default=PMC_SUMMARY)
    args = ap.parse_args()
    if args.summarize_stats:
        print(summarize_stats(args.summarize_stats))
        return
    if args.summarize_pmc:
        if not args.copy_dirs:
            raise SystemExit("bench.py: --summarize-pmc needs --copy-dirs")
        print(summarize_pmc(args.summarize_pmc, args.copy_dirs, args.photons, args.pmc_json))
        return
    if args.gpus != 1:
        print(f"bench.py: the trace runs on one GPU only (asked for --gpus {args.gpus}); sharding "
              "photons over several GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.gather_probe:
        gather_probe()
        return
    if args.op_probe:
        print(json.dumps({"fp64_op_rates": fp64_op_rates(), "philox_blocks_per_s": philox_rate()}),
              flush=True)
        return
    if args.only == "ghosts":
        print(json.dumps(ghosts_only(args)), flush=True)
        return
    if args.only:
        leg = batched_leg if args.only == "batched" else gradient_leg
        print(json.dumps(leg(max(args.steps, 1))), flush=True)
        return
    import numpy as np
    import torch
    from paper_1504_06570_amd import phx
    from paper_1504_06570_amd.scene import configs as C

    n_ph = int(args.photons)
    t_setup = time.perf_counter()
    scene = C.full()
    scene.sources.n_photons[:] = n_ph
    tr = phx.Tracer(scene)
    print(f"# setup {time.perf_counter() - t_setup:.1f}s", file=sys.stderr, flush=True)
    base = int(scene.physics)
    flags = base if args.no_cull else base | phx.F_CULL
    n_surf = len(scene.prescription.surfaces)
    n_coated = sum(1 for s in scene.prescription.surfaces if s.coating >= 0)
    img = tr.new_image()
    stats = tr.new_stats()
    t_tune = time.perf_counter()
    if args.launch:
        tr.set_launch_config(**launch_shape(args.launch))
        tuned = tr.launch_config()
    elif args.no_autotune:
        tuned = tr.launch_config()
    else:
        tuned = tr.autotune(flags=flags)   # eager launches pipelined over two streams
    t_tune = time.perf_counter() - t_tune
    print(f"# autotuned {tuned} in {t_tune:.1f}s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        tr.trace(img, flags=flags, stats=stats)
    torch.cuda.synchronize()
    stats.zero_()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    tr.set_timing(True)   # HIP events around every kernel of the timed steps
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        tr.trace(img, flags=flags, stats=stats)
    ev1.record(stream)
    torch.cuda.synchronize()
    kt = tr.get_timing()
    tr.set_timing(False)
    ms = ev0.elapsed_time(ev1) / args.steps
    value = n_ph / (ms * 1e-3)
    st = stats.cpu().numpy()
    print(f"# timed {args.steps} steps: {ms:.2f} ms/step; kernels {kt}", file=sys.stderr, flush=True)
    tab = phx.stats_table(st) / args.steps
    detected = float(tab[phx.DETECTED].sum())
    traced = float(st[phx.STAT_TRACED])
    chunks = max(kt["chunks"], 1.0)
    atm = scene.atmosphere
    counts = op_counts()
    if counts is None:
        raise SystemExit(f"bench.py: {OP_COUNTS} is missing (python -m oracle.count_ops)")
    # per-launch (one chunk's kernel) figures of each stage: algorithmic work from the oracle's
    # counting build (sky: screen bytes gathered; optics + sensor: FP64 operations by outcome)
    # and, for the pre-roll, its first two Philox blocks per generated photon
    kinds = {
        "generate": dict(ms=kt["generate"] / chunks, bound="alu", unit="Tops/s", peak=PEAK_INT32_TOPS,
                         work=n_ph * args.steps * PREROLL_BLOCKS * PHILOX_INT_OPS / chunks,
                         scale=1e-12),
        "front": dict(ms=kt["front"] / chunks, bound="hbm", unit="GB/s", peak=PEAK_HBM_GBS,
                      work=traced * front_bytes_per_photon(atm.n_layers, atm.n_scales, counts) / chunks,
                      scale=1e-9),
        "back": dict(ms=kt["back"] / chunks, bound="alu", unit="TFLOP/s", peak=PEAK_FP64_TFLOPS,
                     work=back_flops(st, counts) / chunks, scale=1e-12),
    }
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    d = kinds[dom]
    achieved = d["work"] / (d["ms"] * 1e-3) * d["scale"]
    pipelined = {}
    for k, v in kinds.items():
        a_k = v["work"] / (v["ms"] * 1e-3) * v["scale"]
        pipelined[f"{k}_kernel"] = {"bound": v["bound"], "achieved": a_k, "peak": v["peak"],
                                    "unit": v["unit"], "frac": a_k / v["peak"],
                                    "launch_ms": v["ms"], "work_per_launch": v["work"]}
    implementation = {
        "front_state_write_bytes_per_launch": traced * STATE_BYTES / chunks,
        "note": "the sky stage also writes the 7-double start-plane state of each traced photon "
                "for the optics stage; that traffic comes from splitting the trace into kernels "
                "and is not in the algorithmic bytes",
    }
    stage_ms = {k: kt[k] / args.steps for k in ("generate", "compact", "front", "back")}
    extra = {}
    # The timed steps overlap each chunk's optics stage with the next chunk's sky stage, so the
    # per-launch durations above include time shared with the other kernel.  One more step with
    # the stages on a single stream gives each kernel's duration alone.
    extra["roofline_pipelined"] = pipelined
    extra["implementation_traffic"] = implementation
    if not args.no_single_stream:
        tr.set_launch_config(pipeline=0)
        iso_stats = tr.new_stats()
        tr.set_timing(True)
        tr.trace(tr.new_image(), flags=flags, stats=iso_stats)
        torch.cuda.synchronize()
        kti = tr.get_timing()
        tr.set_timing(False)
        tr.set_launch_config(pipeline=1)
        ci = max(kti["chunks"], 1.0)
        iso = {}
        for k, v in kinds.items():
            ms_k = kti[k] / ci
            a_k = v["work"] / (ms_k * 1e-3) * v["scale"]
            iso[f"{k}_kernel"] = {"bound": v["bound"], "achieved": a_k, "peak": v["peak"],
                                  "unit": v["unit"], "frac": a_k / v["peak"], "launch_ms": ms_k}
        extra["roofline_single_stream"] = iso
        extra["stage_ms_single_stream"] = {k: kti[k] for k in ("generate", "compact", "front",
                                                               "back")}
    # The optics kernel against the FP64 classes' own measured rates (division, square root and
    # transcendentals are sequences of several instructions, not one), and the whole step against
    # the sum of its stages' times at their peaks (the counted work over the measured per-class
    # rates, the screen bytes over the HBM peak, the Philox operations over the integer peak).
    rates = fp64_op_rates()
    if rates is not None:
        ops = {f: v / chunks for f, v in back_ops_by_class(st, counts).items()}
        t_back = per_class_seconds(ops, rates)
        for tab_ in (extra.get("roofline_pipelined"), extra.get("roofline_single_stream")):
            if tab_ and "back_kernel" in tab_:
                tab_["back_kernel"]["frac_per_class"] = t_back / (tab_["back_kernel"]["launch_ms"]
                                                                  * 1e-3)
        t_sky = kinds["front"]["work"] / (PEAK_HBM_GBS * 1e9)
        t_pre = kinds["generate"]["work"] / (PEAK_INT32_TOPS * 1e12)
        # the pre-roll's blocks at the measured Philox block rate
        blocks_rate = philox_rate()
        if blocks_rate:
            t_pre = kinds["generate"]["work"] / PHILOX_INT_OPS / blocks_rate
            for tab_ in (extra.get("roofline_pipelined"), extra.get("roofline_single_stream")):
                if tab_ and "generate_kernel" in tab_:
                    tab_["generate_kernel"]["frac_per_class"] = t_pre / (
                        tab_["generate_kernel"]["launch_ms"] * 1e-3)
            extra["philox_blocks_per_s"] = blocks_rate
        per_step = chunks / args.steps * 1e3   # launches per step, seconds -> ms
        t_sum = (t_sky + t_back + t_pre) * per_step
        extra["fp64_op_rates"] = {k: v for k, v in rates.items()}
        extra["fp64_ops_per_launch"] = ops
        extra["step_roofline"] = {
            "sky_ms": t_sky * per_step, "optics_ms": t_back * per_step,
            "preroll_ms": t_pre * per_step, "sum_ms": t_sum, "measured_ms": ms,
            "frac": t_sum / ms,
            "frac_max": max(t_sky, t_back, t_pre) * per_step / ms,
            "note": "each stage's counted work at its peak, summed over the step, over the "
                    "measured step time (frac); the stages run concurrently on different units, "
                    "so the largest stage alone over the step time (frac_max) is the tighter "
                    "bound"}
    if not args.no_cull and not args.no_compare:
        # the same step without the pre-roll (every photon traced until its fate)
        nc_img = tr.new_image()
        tr.trace(nc_img, flags=base)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tr.trace(nc_img, flags=base)
        e1.record(stream)
        torch.cuda.synchronize()
        nc_ms = e0.elapsed_time(e1)
        extra["value_without_preroll"] = n_ph / (nc_ms * 1e-3)
        extra["ms_per_step_without_preroll"] = nc_ms

    if not args.no_extras:
        one = tr.new_image()
        tr.trace(one, flags=flags)
        extra["readout"] = readout_leg(tr, one, max(args.steps, 1))
        del one
        fixed = bool(args.launch or args.no_autotune)   # the command fixes the launch shape
        extra["extra_physics"] = extras_leg(tr, scene, flags, max(args.steps, 1), n_ph, ms,
                                            tune=not fixed)
        extra["ghosts"] = ghost_leg(tr, flags, max(args.steps, 1), n_ph, ms, tune=not fixed)
        shape = tr.launch_config() if fixed else None
        tr.close()
        extra["hybrid_atmosphere"] = hybrid_leg(max(args.steps, 1), n_ph, ms, launch=shape)

    cpu = None
    if not args.skip_cpu:
        # the host cores that serve one GPU (at most 16 threads), then one core
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        n_cpu = int(args.cpu_sample)
        rate, dt = cpu_baseline(scene, n_cpu, threads)
        n_one = max(int(n_cpu // 16), 1)
        rate1, dt1 = cpu_baseline(scene, n_one, 1)
        cpu = {"value": rate, "unit": "photons/s", "cores": threads, "kind": "oracle",
               "sample": f"first {n_cpu:.0e} photons of the headline star, full physics, no "
                         f"pre-roll (every photon traced to its fate), {dt:.1f} s on {threads} "
                         f"host threads; one core: first {n_one:.0e} photons, {dt1:.1f} s",
               "one_core_value": rate1, "cpu_model": cpu_model(),
               "host_cpus": os.cpu_count()}
        nc = extra.get("value_without_preroll")
        if nc:
            cpu["gpu_over_oracle_equal_work"] = nc / rate
        print(f"# cpu oracle {rate:.3e} photons/s ({dt:.1f}s, {threads} threads), one core "
              f"{rate1:.3e} photons/s ({dt1:.1f}s)", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        batched = batched_leg(max(args.steps, 1))
    gradient = None
    if not args.no_gradient:
        gradient = gradient_leg(max(args.steps, 1))

    traffic = traffic_from_profiles(n_ph, f"{dom}_kernel")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "photons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "precision": "FP64 arithmetic throughout; screen gradients and coating tables are stored "
                     "as FP32 and widened on use; hardware reciprocal and reciprocal-square-root "
                     "estimates refined to about 1 ulp in the continuous geometry",
        "data": "synthetic",
        "config": {
            "workload": "full single-source trace: 1 star, 1e9 photons/step, 7 frozen-flow von "
                        "Karman layers (3 x 2048^2 screens each), TMA+camera, coatings, silicon, "
                        "diffusion, 4096^2 chip",
            "photons_per_step": n_ph,
            "preroll_cull": not args.no_cull,
            "launch_config": tuned,
            "autotune_s": t_tune,
            "detected_per_step": detected,
            "traced_per_step": traced / args.steps,
            "newton_per_traced": float(st[phx.STAT_NEWTON]) / max(traced, 1.0),
        },
        "roofline": {
            "bound": d["bound"],
            "achieved": achieved,
            "peak": d["peak"],
            "unit": d["unit"],
            "frac": achieved / d["peak"],
            "traffic": traffic,
            "kernel": f"{dom}_kernel",
            "launch_ms": d["ms"],
        },
        "stage_ms_per_step": stage_ms,
        "cpu_baseline": cpu,
        "batched": batched,
        "gradient": gradient,
        "adjoint_forward_ratio": gradient["adjoint_forward_ratio"] if gradient else None,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
