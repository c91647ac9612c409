"""Python binding of the C-ABI photon trace library (libphx.so, declared in include/phx.h).

Argument marshalling only: every step of the trace runs in the library's HIP kernels.  PyTorch
provides device memory and the stream.  Importing this module loads the library and fails
loudly if it has not been built (``python -m paper_1504_06570_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphx.so")

MAX_SURF, MAX_LAYERS, MAX_SCALES, N_THETA, N_STATUS = 16, 8, 4, 22, 12
STAT_COLS = MAX_SURF + 1
STAT_NEWTON = N_STATUS * STAT_COLS
STAT_TRACED = STAT_NEWTON + 1
STATS_LEN = STAT_TRACED + 1
MOMENT_WORDS, MOMENT_Q_LOG2 = 12, 44

F_ATMOSPHERE, F_COATINGS, F_SILICON, F_DIFFUSION = 1, 2, 4, 8
F_CULL, F_EVENTS, F_MOMENTS = 1 << 8, 1 << 9, 1 << 10
F_AEROSOL, F_DISPERSION, F_DOME, F_HALO = 1 << 4, 1 << 5, 1 << 6, 1 << 7
F_SPIDER, F_DEAD_LAYER, F_SECOND_KICK, F_FIELD_DIFFUSION = 1 << 11, 1 << 12, 1 << 13, 1 << 14
F_GHOSTS = 1 << 15
STATUS = ["DETECTED", "OFF_CHIP", "VIGNETTED", "ABSORBED", "MISSED", "NONCONV", "TIR", "ESCAPED",
          "OBSCURED", "CULLED", "EXTINCT", "DEAD"]
(DETECTED, OFF_CHIP, VIGNETTED, ABSORBED, MISSED, NONCONV, TIR, ESCAPED, OBSCURED, CULLED,
 EXTINCT, DEAD) = range(12)


class PhxError(RuntimeError):
    pass


class Surface(C.Structure):
    _fields_ = [("kind", C.c_int32), ("medium", C.c_int32), ("coating", C.c_int32),
                ("group", C.c_int32), ("z_vertex", C.c_double), ("curvature", C.c_double),
                ("conic", C.c_double), ("alpha", C.c_double * 8), ("r_inner", C.c_double),
                ("r_outer", C.c_double)]


class Prescription(C.Structure):
    _fields_ = [("n_surfaces", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("pad", C.c_int32),
                ("surf", Surface * MAX_SURF), ("pupil_r_inner", C.c_double),
                ("pupil_r_outer", C.c_double), ("z_start", C.c_double),
                ("obscuration_z", C.c_double), ("obscuration_r", C.c_double),
                ("sellmeier_b", C.c_double * 3), ("sellmeier_c", C.c_double * 3),
                ("chip_x0", C.c_double), ("chip_y0", C.c_double), ("pixel", C.c_double),
                ("si_thickness", C.c_double), ("si_temperature", C.c_double),
                ("sigma_max", C.c_double), ("group_pivot", (C.c_double * 3) * 3)]


class Atmosphere(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("n_scales", C.c_int32), ("screen_n", C.c_int32),
                ("pad", C.c_int32), ("height", C.c_double * MAX_LAYERS),
                ("wind", (C.c_double * 2) * MAX_LAYERS), ("pixel", C.c_double * MAX_SCALES),
                ("lambda_ref", C.c_double)]


class Source(C.Structure):
    _fields_ = [("xi", C.c_double), ("eta", C.c_double), ("kind", C.c_int32), ("sed", C.c_int32),
                ("lambda_lo", C.c_double), ("lambda_hi", C.c_double), ("redshift", C.c_double),
                ("sersic_n", C.c_double), ("sersic_bn", C.c_double), ("sersic_a", C.c_double),
                ("sersic_b", C.c_double), ("sersic_pa", C.c_double), ("n_photons", C.c_uint64)]


class Physics(C.Structure):
    _fields_ = [("zenith_angle", C.c_double), ("zenith_pa", C.c_double),
                ("aerosol_tau0", C.c_double), ("aerosol_gamma", C.c_double),
                ("air_pressure", C.c_double), ("air_water", C.c_double),
                ("air_temperature", C.c_double), ("dispersion_lambda0", C.c_double),
                ("dome_sigma", C.c_double), ("halo_fraction", C.c_double),
                ("halo_index", C.c_double), ("halo_r0", C.c_double), ("halo_max", C.c_double),
                ("dead_layer", C.c_double), ("spider_vanes", C.c_int32), ("pad", C.c_int32),
                ("spider_angle", C.c_double), ("spider_width", C.c_double),
                ("spider_r_inner", C.c_double), ("spider_r_outer", C.c_double),
                ("spider_z_low", C.c_double), ("spider_z_high", C.c_double),
                ("kick_r0", C.c_double), ("kick_L0", C.c_double), ("kick_kappa_crit", C.c_double),
                ("kick_kappa_max", C.c_double), ("kick_fraction", C.c_double * MAX_LAYERS),
                ("si_voltage", C.c_double), ("si_n_bulk", C.c_double), ("si_n_back", C.c_double),
                ("si_s_back", C.c_double), ("si_n_front", C.c_double), ("si_s_front", C.c_double),
                ("si_z_collect", C.c_double)]


def physics_struct(x) -> Physics:
    """phx_physics from a scene's Extras (paper_1504_06570_amd.scene.physics)."""
    P = Physics()
    P.zenith_angle, P.zenith_pa = x.zenith, x.zenith_pa
    P.aerosol_tau0, P.aerosol_gamma = x.tau0, x.gamma
    P.air_pressure, P.air_water, P.air_temperature = x.pressure, x.water, x.temperature
    P.dispersion_lambda0, P.dome_sigma = x.lam0, x.dome_sigma
    P.halo_fraction, P.halo_index, P.halo_r0, P.halo_max = x.halo_f, x.halo_n, x.halo_r0, x.halo_max
    P.dead_layer = x.dead
    P.spider_vanes, P.spider_angle, P.spider_width = x.vanes, x.vane_angle, x.vane_width
    P.spider_r_inner, P.spider_r_outer = x.vane_r_in, x.vane_r_out
    P.spider_z_low, P.spider_z_high = x.vane_z_lo, x.vane_z_hi
    P.kick_r0, P.kick_L0 = x.kick_r0, x.kick_L0
    P.kick_kappa_crit, P.kick_kappa_max = x.kick_kappa_crit, x.kick_kappa_max
    for i, f in enumerate(x.kick_fraction[:MAX_LAYERS]):
        P.kick_fraction[i] = f
    for name in ("si_voltage", "si_n_bulk", "si_n_back", "si_s_back", "si_n_front", "si_s_front",
                 "si_z_collect"):
        setattr(P, name, getattr(x, name))
    return P


MAX_AMPS = 32


class ReadoutParams(C.Structure):
    _fields_ = [("seed", C.c_uint32), ("amp_nx", C.c_int32), ("amp_ny", C.c_int32),
                ("over_x", C.c_int32), ("over_y", C.c_int32), ("pad", C.c_int32),
                ("full_well", C.c_double), ("exposure", C.c_double), ("dark_rate", C.c_double),
                ("hot_fraction", C.c_double), ("dead_fraction", C.c_double),
                ("hot_column_fraction", C.c_double), ("cte_parallel", C.c_double),
                ("cte_serial", C.c_double), ("nonlinearity", C.c_double),
                ("gain", C.c_double * MAX_AMPS), ("bias", C.c_double * MAX_AMPS),
                ("read_noise", C.c_double * MAX_AMPS), ("bit_sigma", C.c_double * 16)]


def readout_struct(rp) -> ReadoutParams:
    """phx_readout_params from a scene readout description (paper_1504_06570_amd.scene.readout)."""
    P = ReadoutParams()
    for name, _ in ReadoutParams._fields_:
        if name == "pad":
            continue
        v = getattr(rp, name)
        if name in ("gain", "bias", "read_noise", "bit_sigma"):
            for i, x in enumerate(v):
                getattr(P, name)[i] = x
        else:
            setattr(P, name, v)
    return P


class TraceArgs(C.Structure):
    _fields_ = [("seed", C.c_uint32), ("flags", C.c_uint32), ("src_begin", C.c_int32),
                ("src_end", C.c_int32), ("photon_begin", C.c_uint64), ("photon_count", C.c_uint64),
                ("exposure", C.c_double), ("pupil_margin", C.c_double),
                ("image_dev", C.c_void_p), ("stats_dev", C.c_void_p), ("moments_dev", C.c_void_p),
                ("events_dev", C.c_void_p), ("event_stride", C.c_uint64),
                ("event_capacity", C.c_uint64)]


class LaunchConfig(C.Structure):
    _fields_ = [("chunk_log2", C.c_int32), ("generate_blocks_per_cu", C.c_int32),
                ("front_blocks_per_cu", C.c_int32), ("back_blocks_per_cu", C.c_int32),
                ("dynamic_tiles", C.c_int32), ("pipeline", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


EVENT_DTYPE = np.dtype([("photon", np.uint64), ("source", np.int32), ("status", np.int32),
                        ("surface", np.int32), ("pix_i", np.int32), ("pix_j", np.int32),
                        ("newton", np.int32), ("x", np.float64), ("y", np.float64),
                        ("z", np.float64), ("xe", np.float64), ("ye", np.float64),
                        ("lam", np.float64)])
assert EVENT_DTYPE.itemsize == 80

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PhxError(f"{LIB_PATH} is missing: build it with python -m paper_1504_06570_amd.build")
        L = C.CDLL(LIB_PATH)
        L.phx_version.restype = C.c_char_p
        L.phx_create.argtypes = [C.c_int32, C.POINTER(C.c_void_p)]
        L.phx_destroy.argtypes = [C.c_void_p]
        L.phx_destroy.restype = None
        L.phx_last_error.argtypes = [C.c_void_p]
        L.phx_last_error.restype = C.c_char_p
        L.phx_load_prescription.argtypes = [C.c_void_p, C.POINTER(Prescription)]
        L.phx_set_perturbation.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32]
        L.phx_load_coatings.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_double, C.c_double, C.c_double]
        L.phx_load_screens.argtypes = [C.c_void_p, C.POINTER(Atmosphere), C.c_void_p, C.c_int64,
                                       C.c_void_p]
        L.phx_load_sources.argtypes = [C.c_void_p, C.POINTER(Source), C.c_int32, C.c_void_p,
                                       C.c_void_p, C.c_int32, C.c_int32]
        L.phx_trace.argtypes = [C.c_void_p, C.POINTER(TraceArgs), C.c_void_p]
        L.phx_load_physics.argtypes = [C.c_void_p, C.POINTER(Physics)]
        L.phx_load_reflectance.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                           C.c_int32]
        L.phx_readout.argtypes = [C.c_void_p, C.POINTER(ReadoutParams), C.c_void_p, C.c_int32,
                                  C.c_int32, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        L.phx_set_timing.argtypes = [C.c_void_p, C.c_int32]
        L.phx_get_timing.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32]
        L.phx_set_launch_config.argtypes = [C.c_void_p, C.POINTER(LaunchConfig)]
        L.phx_get_launch_config.argtypes = [C.c_void_p, C.POINTER(LaunchConfig)]
        L.phx_trace_batched.argtypes = [C.c_void_p, C.POINTER(TraceArgs), C.c_void_p]
        L.phx_trace_noalloc.argtypes = [C.c_void_p, C.POINTER(TraceArgs), C.c_void_p]
        L.phx_moments.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.phx_adjoint_moments.argtypes = [C.c_void_p, C.POINTER(TraceArgs), C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                          C.c_uint64, C.c_void_p]
        L.phx_read_image.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.phx_autotune.argtypes = [C.c_void_p, C.POINTER(TraceArgs), C.c_void_p,
                                   C.POINTER(LaunchConfig)]
        L.phx_autotune_batched.argtypes = [C.c_void_p, C.POINTER(TraceArgs), C.c_void_p,
                                           C.POINTER(LaunchConfig)]
        L.phx_adjoint.argtypes = [C.c_void_p, C.POINTER(TraceArgs), C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p]
        for f in ("phx_create", "phx_load_prescription", "phx_set_perturbation",
                  "phx_load_coatings", "phx_load_screens", "phx_load_sources", "phx_trace",
                  "phx_set_timing", "phx_get_timing", "phx_set_launch_config",
                  "phx_get_launch_config", "phx_trace_batched", "phx_autotune", "phx_adjoint",
                  "phx_load_physics", "phx_readout", "phx_load_reflectance",
                  "phx_trace_noalloc", "phx_moments", "phx_adjoint_moments",
                  "phx_read_image", "phx_autotune_batched"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def prescription_struct(p) -> Prescription:
    P = Prescription()
    P.n_surfaces = len(p.surfaces)
    if P.n_surfaces > MAX_SURF:
        raise PhxError("too many surfaces")
    P.nx, P.ny = p.chip.nx, p.chip.ny
    for k, s in enumerate(p.surfaces):
        o = P.surf[k]
        o.kind, o.medium, o.coating, o.group = s.kind, s.medium, s.coating, s.group
        o.z_vertex, o.curvature, o.conic = s.z, s.curvature, s.conic
        for i in range(8):
            o.alpha[i] = s.alpha[i]
        o.r_inner, o.r_outer = s.r_in, s.r_out
    P.pupil_r_inner, P.pupil_r_outer, P.z_start = p.pupil_r_in, p.pupil_r_out, p.z_start
    P.obscuration_z, P.obscuration_r = p.obscuration_z, p.obscuration_r
    for i in range(3):
        P.sellmeier_b[i] = p.glass_b[i]
        P.sellmeier_c[i] = p.glass_c_um2[i]
    P.chip_x0, P.chip_y0, P.pixel = p.chip.x0, p.chip.y0, p.chip.pixel
    P.si_thickness, P.si_temperature, P.sigma_max = (p.silicon.thickness, p.silicon.temperature,
                                                     p.silicon.sigma_max)
    for g in range(3):
        for i in range(3):
            P.group_pivot[g][i] = p.group_pivot[g][i]
    return P


def sources_struct(S):
    arr = (Source * len(S))()
    for i in range(len(S)):
        a = arr[i]
        a.xi, a.eta = float(S.xi[i]), float(S.eta[i])
        a.kind, a.sed = int(S.kind[i]), int(S.sed[i])
        a.lambda_lo, a.lambda_hi, a.redshift = float(S.lam_lo[i]), float(S.lam_hi[i]), float(S.redshift[i])
        a.sersic_n, a.sersic_bn = float(S.sersic_n[i]), float(S.sersic_bn[i])
        a.sersic_a, a.sersic_b, a.sersic_pa = float(S.sersic_a[i]), float(S.sersic_b[i]), float(S.sersic_pa[i])
        a.n_photons = int(S.n_photons[i])
    return arr


class Tracer:
    """A library context on one GPU with a scene (paper_1504_06570_amd.scene) loaded."""

    def __init__(self, scene, device: int = 0):
        import torch
        from .scene import coatings as coat_mod
        self.L = lib()
        self.scene = scene
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        rc = self.L.phx_create(device, C.byref(h))
        if rc != 0:
            raise PhxError(f"phx_create failed ({rc})")
        self.ctx = h
        self._check(self.L.phx_load_prescription(self.ctx, C.byref(prescription_struct(scene.prescription))))
        self.set_perturbation(scene.perturbation)
        if scene.coatings is not None:
            ct = np.ascontiguousarray(scene.coatings, np.float32)
            self._check(self.L.phx_load_coatings(self.ctx, ct.ctypes.data, ct.shape[0], ct.shape[1],
                                                 ct.shape[2], coat_mod.S_MAX, coat_mod.LAM0,
                                                 coat_mod.DLAM))
        if getattr(scene, "reflectance", None) is not None:
            rt = np.ascontiguousarray(scene.reflectance, np.float32)
            self._check(self.L.phx_load_reflectance(self.ctx, rt.ctypes.data, rt.shape[0],
                                                    rt.shape[1], rt.shape[2]))
        if scene.atmosphere is not None:
            self.load_screens(scene.atmosphere)
        if getattr(scene, "extras", None) is not None:
            self.load_physics(scene.extras)
        self.load_sources(scene.sources, scene.sed)

    def _check(self, rc):
        if rc != 0:
            msg = self.L.phx_last_error(self.ctx).decode()
            raise PhxError(f"phx error {rc}: {msg}")

    def close(self):
        if getattr(self, "ctx", None):
            self.L.phx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_perturbation(self, theta):
        th = np.ascontiguousarray(theta, np.float64)
        self._check(self.L.phx_set_perturbation(self.ctx, th.ctypes.data_as(C.POINTER(C.c_double)),
                                                th.shape[0]))

    def load_screens(self, atm):
        import torch
        A = Atmosphere()
        A.n_layers, A.n_scales, A.screen_n = atm.n_layers, atm.n_scales, atm.n
        for i in range(atm.n_layers):
            A.height[i] = atm.heights[i]
            A.wind[i][0], A.wind[i][1] = atm.wind[i]
        for s in range(atm.n_scales):
            A.pixel[s] = atm.pixels[s]
        A.lambda_ref = atm.lambda_ref
        opd = torch.from_numpy(np.ascontiguousarray(atm.opd, np.float32)).to(self.device)
        self._check(self.L.phx_load_screens(self.ctx, C.byref(A), opd.data_ptr(), opd.numel(),
                                            _stream_handle()))
        torch.cuda.current_stream().synchronize()
        del opd

    def load_physics(self, extras):
        self._check(self.L.phx_load_physics(self.ctx, C.byref(physics_struct(extras))))

    def load_sources(self, S, sed=None):
        arr = sources_struct(S)
        if sed is not None:
            e = np.ascontiguousarray(sed.lam_edges, np.float64)
            f = np.ascontiguousarray(sed.flux, np.float64)
            self._check(self.L.phx_load_sources(self.ctx, arr, len(S), e.ctypes.data, f.ctypes.data,
                                                f.shape[0], f.shape[1]))
        else:
            self._check(self.L.phx_load_sources(self.ctx, arr, len(S), None, None, 0, 0))
        self.n_sources = len(S)

    def new_image(self):
        import torch
        p = self.scene.prescription
        return torch.zeros((p.chip.ny, p.chip.nx), dtype=torch.int32, device=self.device)

    def _args(self, image, flags, seed, src_begin, src_end, photon_begin, photon_count, stats,
              moments, event_stride, events, exposure, adjoint_only=False):
        import torch
        sc = self.scene
        if image is None and not adjoint_only:
            image = self.new_image()
        if flags is None:
            flags = int(sc.physics)
        if event_stride:
            flags |= F_EVENTS
        if moments is not None:
            flags |= F_MOMENTS
        src_end = self.n_sources if src_end is None else src_end
        a = TraceArgs()
        a.seed = int(sc.seed if seed is None else seed) & 0xFFFFFFFF
        a.flags = flags
        a.src_begin, a.src_end = src_begin, src_end
        a.photon_begin, a.photon_count = int(photon_begin), int(photon_count)
        a.exposure = float(sc.exposure if exposure is None else exposure)
        a.pupil_margin = float(sc.pupil_margin)
        if image is not None:
            assert image.dtype == torch.int32 and image.is_contiguous()
            a.image_dev = image.data_ptr()
        a.stats_dev = stats.data_ptr() if stats is not None else None
        a.moments_dev = moments.data_ptr() if moments is not None else None
        if event_stride:
            if photon_count:
                total = photon_count * (src_end - src_begin)
            else:
                total = int(sc.sources.n_photons[src_begin:src_end].sum())
            cap = (total + event_stride - 1) // event_stride
            if events is None:
                events = torch.zeros(cap * EVENT_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
            a.events_dev = events.data_ptr()
            a.event_stride = event_stride
            a.event_capacity = events.numel() // EVENT_DTYPE.itemsize
        return a, image, events

    def trace(self, image=None, *, flags=None, seed=None, src_begin=0, src_end=None,
              photon_begin=0, photon_count=0, stats=None, moments=None, event_stride=0,
              events=None, stream=None, exposure=None, batched=False, noalloc=False):
        """Enqueue one trace of sources [src_begin, src_end).  `batched` replays a captured graph
        of the whole launch (phx_trace_batched); `noalloc` calls phx_trace_noalloc (the workspace
        in the library's static device array).  Returns (image, stats, moments, events) tensors
        (events as raw bytes)."""
        a, image, events = self._args(image, flags, seed, src_begin, src_end, photon_begin,
                                      photon_count, stats, moments, event_stride, events, exposure)
        fn = (self.L.phx_trace_batched if batched else
              self.L.phx_trace_noalloc if noalloc else self.L.phx_trace)
        self._check(fn(self.ctx, C.byref(a), _stream_handle(stream)))
        return image, stats, moments, events

    def adjoint(self, seeds, *, flags=None, seed=None, src_begin=0, src_end=None, photon_begin=0,
                photon_count=0, jac_stride=0, grad=None, stream=None):
        """Gradient of sum_i (xbar_i x_i + ybar_i y_i) over converted photons with respect to the
        22 perturbation parameters (phx_adjoint).  seeds: float64 device tensor [n, 8] for the
        sources [src_begin, src_end) (the coefficients of phx_adjoint; adjoint_moments forms them
        from the moment words).  With jac_stride > 0 also returns the
        per-photon Jacobians [slots, 2, 22] of every jac_stride-th photon of the launch."""
        import torch
        src_end = self.n_sources if src_end is None else src_end
        seeds = seeds.to(device=self.device, dtype=torch.float64).contiguous()
        if seeds.shape != (src_end - src_begin, 8):
            raise PhxError(f"seeds must be [{src_end - src_begin}, 8], got {tuple(seeds.shape)}")
        a, _, _ = self._args(None, flags, seed, src_begin, src_end, photon_begin, photon_count,
                             None, None, 0, None, None, adjoint_only=True)
        if grad is None:
            grad = torch.zeros(N_THETA, dtype=torch.float64, device=self.device)
        jac = None
        jp, cap = None, 0
        if jac_stride:
            if photon_count:
                total = photon_count * (src_end - src_begin)
            else:
                total = int(self.scene.sources.n_photons[src_begin:src_end].sum())
            cap = (total + jac_stride - 1) // jac_stride
            jac = torch.zeros((cap, 2, N_THETA), dtype=torch.float64, device=self.device)
            jp = jac.data_ptr()
        self._check(self.L.phx_adjoint(self.ctx, C.byref(a), seeds.data_ptr(), grad.data_ptr(), jp,
                                       int(jac_stride), int(cap), _stream_handle(stream)))
        return (grad, jac) if jac_stride else grad

    def adjoint_moments(self, words, dmom, *, flags=None, seed=None, src_begin=0, src_end=None,
                        photon_begin=0, photon_count=0, jac_stride=0, grad=None, stream=None):
        """Gradient of a loss of the per-source moments with respect to the 22 perturbation
        parameters (phx_adjoint_moments): words are the forward trace's moment words (device
        tensor [n_sources, MOMENT_WORDS]), dmom the loss gradient [src_end - src_begin, 5] with
        respect to (mean x, mean y, Ixx, Iyy, Ixy).  Returns grad (and the per-photon Jacobians
        with jac_stride > 0, as adjoint)."""
        import torch
        src_end = self.n_sources if src_end is None else src_end
        dmom = dmom.to(device=self.device, dtype=torch.float64).contiguous()
        if dmom.shape != (src_end - src_begin, 5):
            raise PhxError(f"dmom must be [{src_end - src_begin}, 5], got {tuple(dmom.shape)}")
        if words.shape != (self.n_sources, MOMENT_WORDS) or not words.is_contiguous():
            raise PhxError("words must be the contiguous [n_sources, MOMENT_WORDS] trace buffer")
        a, _, _ = self._args(None, flags, seed, src_begin, src_end, photon_begin, photon_count,
                             None, None, 0, None, None, adjoint_only=True)
        if grad is None:
            grad = torch.zeros(N_THETA, dtype=torch.float64, device=self.device)
        jac, jp, cap = None, None, 0
        if jac_stride:
            total = (photon_count * (src_end - src_begin) if photon_count else
                     int(self.scene.sources.n_photons[src_begin:src_end].sum()))
            cap = (total + jac_stride - 1) // jac_stride
            jac = torch.zeros((cap, 2, N_THETA), dtype=torch.float64, device=self.device)
            jp = jac.data_ptr()
        self._check(self.L.phx_adjoint_moments(self.ctx, C.byref(a), words.data_ptr(),
                                               dmom.data_ptr(), grad.data_ptr(), jp,
                                               int(jac_stride), int(cap), _stream_handle(stream)))
        return (grad, jac) if jac_stride else grad

    def moments(self, words, stream=None):
        """Per-source (n, mean x, mean y, Ixx, Iyy, Ixy) of moment words (device tensor
        [n, MOMENT_WORDS]) as a device float64 tensor [n, 6] (phx_moments)."""
        import torch
        assert words.is_contiguous() and words.shape[-1] == MOMENT_WORDS
        n = words.shape[0]
        out = torch.empty((n, 6), dtype=torch.float64, device=self.device)
        self._check(self.L.phx_moments(self.ctx, words.data_ptr(), n, out.data_ptr(),
                                       _stream_handle(stream)))
        return out

    def read_image(self, image, stream=None) -> np.ndarray:
        """Host copy of a trace image (phx_read_image) as uint32 [ny, nx]."""
        p = self.scene.prescription
        out = np.empty((p.chip.ny, p.chip.nx), np.uint32)
        assert image.is_contiguous()
        self._check(self.L.phx_read_image(self.ctx, image.data_ptr(), out.ctypes.data, out.size,
                                          _stream_handle(stream)))
        return out

    def launch_config(self) -> dict:
        cfg = LaunchConfig()
        self._check(self.L.phx_get_launch_config(self.ctx, C.byref(cfg)))
        return cfg.as_dict()

    def set_launch_config(self, **kw):
        """Change the launch shape; unspecified fields keep their value."""
        cfg = LaunchConfig()
        self._check(self.L.phx_get_launch_config(self.ctx, C.byref(cfg)))
        for k, v in kw.items():
            if k not in cfg.as_dict():
                raise KeyError(k)
            setattr(cfg, k, int(v))
        self._check(self.L.phx_set_launch_config(self.ctx, C.byref(cfg)))

    def autotune(self, *, flags=None, seed=None, src_begin=0, src_end=None, photon_count=0,
                 stream=None, batched=False) -> dict:
        """Pick the launch shape that traces this sample fastest (the sample's outputs go to
        scratch buffers) and keep it; returns the chosen configuration.  batched: time graph
        replays (phx_autotune_batched) in the current pipeline setting."""
        a, _, _ = self._args(self.new_image(), flags, seed, src_begin, src_end, 0, photon_count,
                             None, None, 0, None, None)
        cfg = LaunchConfig()
        f = self.L.phx_autotune_batched if batched else self.L.phx_autotune
        self._check(f(self.ctx, C.byref(a), _stream_handle(stream), C.byref(cfg)))
        return cfg.as_dict()

    def set_timing(self, on: bool):
        self._check(self.L.phx_set_timing(self.ctx, 1 if on else 0))

    def get_timing(self):
        """Accumulated kernel milliseconds since timing was switched on:
        dict(generate, front, back, chunks, compact)."""
        out = (C.c_double * 5)()
        self._check(self.L.phx_get_timing(self.ctx, out, 5))
        return dict(generate=out[0], front=out[1], back=out[2], chunks=out[3], compact=out[4])

    def readout(self, image, params, stages=False, stream=None):
        """Readout chain of an electron image (int32/uint32 tensor [ny, nx] on the device):
        returns the uint16 ADU tensor [amp, sh + over_y, sw + over_x] (as int16 storage; view it
        as uint16 on the host), and with stages=True also the electrons after defects, after the
        parallel and after the serial transfers."""
        import torch
        assert image.is_contiguous() and image.dtype == torch.int32
        ny, nx = image.shape
        na = params.amp_nx * params.amp_ny
        sw, sh = nx // params.amp_nx, ny // params.amp_ny
        ph, pw = sh + params.over_y, sw + params.over_x
        out = torch.zeros((na, ph, pw), dtype=torch.int16, device=image.device)
        bufs = [None, None, None]
        if stages:
            bufs = [torch.zeros((ny, nx), dtype=torch.int32, device=image.device),
                    torch.zeros((na, ph, sw), dtype=torch.int32, device=image.device),
                    torch.zeros((na, ph, pw), dtype=torch.int32, device=image.device)]
        ptr = lambda t: t.data_ptr() if t is not None else None
        self._check(self.L.phx_readout(self.ctx, C.byref(readout_struct(params)), image.data_ptr(),
                                       nx, ny, out.data_ptr(), out.numel(), ptr(bufs[0]),
                                       ptr(bufs[1]), ptr(bufs[2]), _stream_handle(stream)))
        return (out, *bufs) if stages else out

    def new_stats(self):
        import torch
        return torch.zeros(STATS_LEN, dtype=torch.int64, device=self.device)

    def new_moments(self):
        """Zeroed moment words [n_sources][MOMENT_WORDS] (uint64 held in int64)."""
        import torch
        return torch.zeros((self.n_sources, MOMENT_WORDS), dtype=torch.int64, device=self.device)


def moment_sums(words):
    """Moment words [n][MOMENT_WORDS] -> per source the exact integers (n, SX, SY, SXX, SYY, SXY)
    (positions in units of 2^-MOMENT_Q_LOG2 m), as Python ints."""
    if hasattr(words, "cpu"):
        words = words.cpu().numpy()
    w = np.ascontiguousarray(words).view(np.uint64).reshape(-1, MOMENT_WORDS)
    out = []
    for row in w:
        vals = [int(row[0])]
        for i in range(5):
            v = (int(row[3 + 2 * i]) << 64) | int(row[2 + 2 * i])
            vals.append(v - (1 << 128) if v >> 127 else v)
        out.append(tuple(vals))
    return out


def events_to_numpy(events) -> np.ndarray:
    return events.cpu().numpy().view(EVENT_DTYPE)


def stats_table(stats) -> np.ndarray:
    s = stats.cpu().numpy() if hasattr(stats, "cpu") else np.asarray(stats)
    return s[:STAT_NEWTON].reshape(N_STATUS, STAT_COLS)
