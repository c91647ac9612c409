"""CPU oracle for the photon trace -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import
this package.  It wraps ``phx_oracle.c`` (plain double-precision C, no code shared with the GPU
library) through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc.so")
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]

MAX_SURF, MAX_LAYERS, MAX_SCALES, N_THETA = 16, 8, 4, 22
STATUS = ["DETECTED", "OFF_CHIP", "VIGNETTED", "ABSORBED", "MISSED", "NONCONV", "TIR",
          "ESCAPED", "OBSCURED", "CULLED", "EXTINCT", "DEAD"]
DETECTED, OFF_CHIP, VIGNETTED, ABSORBED, MISSED, NONCONV, TIR, ESCAPED, OBSCURED = range(9)
EXTINCT, DEAD = 10, 11


def build() -> str:
    src = os.path.join(_HERE, "phx_oracle.c")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Surface(C.Structure):
    _fields_ = [("kind", C.c_int32), ("medium", C.c_int32), ("coating", C.c_int32),
                ("group", C.c_int32), ("z", C.c_double), ("c", C.c_double), ("kappa", C.c_double),
                ("alpha", C.c_double * 8), ("r_in", C.c_double), ("r_out", C.c_double)]


class Source(C.Structure):
    _fields_ = [("xi", C.c_double), ("eta", C.c_double), ("kind", C.c_int32), ("sed", C.c_int32),
                ("lam_lo", C.c_double), ("lam_hi", C.c_double), ("redshift", C.c_double),
                ("sersic_n", C.c_double), ("sersic_bn", C.c_double), ("sersic_a", C.c_double),
                ("sersic_b", C.c_double), ("sersic_pa", C.c_double), ("n_photons", C.c_uint64)]


class Extra(C.Structure):
    _fields_ = [("zenith", C.c_double), ("zenith_pa", C.c_double), ("tau0", C.c_double),
                ("gamma", C.c_double), ("pressure", C.c_double), ("water", C.c_double),
                ("temperature", C.c_double), ("lam0", C.c_double), ("dome_sigma", C.c_double),
                ("halo_f", C.c_double), ("halo_n", C.c_double), ("halo_r0", C.c_double),
                ("halo_max", C.c_double), ("dead", C.c_double), ("vanes", C.c_int32),
                ("pad", C.c_int32), ("vane_angle", C.c_double), ("vane_width", C.c_double),
                ("vane_r_in", C.c_double), ("vane_r_out", C.c_double), ("vane_z_lo", C.c_double),
                ("vane_z_hi", C.c_double), ("kick_r0", C.c_double), ("kick_L0", C.c_double),
                ("kick_kappa_crit", C.c_double), ("kick_kappa_max", C.c_double),
                ("kick_fraction", C.c_double * MAX_LAYERS), ("si_voltage", C.c_double),
                ("si_n_bulk", C.c_double), ("si_n_back", C.c_double), ("si_s_back", C.c_double),
                ("si_n_front", C.c_double), ("si_s_front", C.c_double),
                ("si_z_collect", C.c_double)]


class Scene(C.Structure):
    _fields_ = [
        ("n_surf", C.c_int32), ("physics", C.c_int32), ("surf", Surface * MAX_SURF),
        ("pupil_r_in", C.c_double), ("pupil_r_out", C.c_double), ("pupil_margin", C.c_double),
        ("z_start", C.c_double), ("obsc_z", C.c_double), ("obsc_r", C.c_double),
        ("glass_b", C.c_double * 3), ("glass_c", C.c_double * 3),
        ("chip_x0", C.c_double), ("chip_y0", C.c_double), ("pixel", C.c_double),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("t_si", C.c_double), ("temp_k", C.c_double), ("sigma_max", C.c_double),
        ("theta", C.c_double * N_THETA), ("pivot", (C.c_double * 3) * 3), ("zernike_r", C.c_double),
        ("n_coat", C.c_int32), ("n_s", C.c_int32), ("n_lam", C.c_int32), ("pad0", C.c_int32),
        ("s_max", C.c_double), ("lam0", C.c_double), ("dlam", C.c_double),
        ("coat", C.POINTER(C.c_float)), ("coat_r", C.POINTER(C.c_float)),
        ("n_layers", C.c_int32), ("n_scales", C.c_int32), ("screen_n", C.c_int32), ("pad1", C.c_int32),
        ("height", C.c_double * MAX_LAYERS), ("wind", (C.c_double * 2) * MAX_LAYERS),
        ("pix", C.c_double * MAX_SCALES), ("lambda_ref", C.c_double), ("opd", C.POINTER(C.c_float)),
        ("n_src", C.c_int32), ("n_sed", C.c_int32), ("sed_k", C.c_int32), ("pad2", C.c_int32),
        ("src", C.POINTER(Source)), ("sed_edges", C.POINTER(C.c_double)),
        ("sed_flux", C.POINTER(C.c_double)),
        ("seed", C.c_uint32), ("pad3", C.c_int32), ("exposure", C.c_double),
        ("ex", Extra),
        ("grad", C.POINTER(C.c_float)), ("sed_cdf", C.POINTER(C.c_double)),
        ("rot", ((C.c_double * 3) * 3) * MAX_SURF), ("trans", (C.c_double * 3) * MAX_SURF),
    ]


EVENT_DTYPE = np.dtype([("photon", np.uint64), ("source", np.int32), ("status", np.int32),
                        ("surface", np.int32), ("pix_i", np.int32), ("pix_j", np.int32),
                        ("newton", np.int32), ("x", np.float64), ("y", np.float64),
                        ("z", np.float64), ("xe", np.float64), ("ye", np.float64),
                        ("lam", np.float64), ("margin", np.float64), ("t", np.float64),
                        ("px", np.float64), ("py", np.float64), ("cond", np.float64)])

_lib = None
_lock = threading.Lock()


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build()
            L = C.CDLL(LIB_PATH)
            L.orc_prepare.argtypes = [C.POINTER(Scene)]
            L.orc_release.argtypes = [C.POINTER(Scene)]
            L.orc_trace.argtypes = [C.POINTER(Scene), C.c_int32, C.c_uint64, C.c_uint64,
                                    C.c_void_p, C.c_void_p]
            L.orc_trace_list.argtypes = [C.POINTER(Scene), C.c_int32, C.c_void_p, C.c_uint64,
                                         C.c_void_p, C.c_void_p]
            L.orc_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                     C.POINTER(C.c_uint32)]
            L.orc_u01.argtypes = [C.c_uint32]
            L.orc_u01.restype = C.c_double
            for name in ("orc_rajkanan",):
                getattr(L, name).argtypes = [C.c_double, C.c_double]
                getattr(L, name).restype = C.c_double
            L.orc_n_silicon.argtypes = [C.c_double]
            L.orc_n_silicon.restype = C.c_double
            L.orc_sellmeier.argtypes = [C.POINTER(Scene), C.c_double]
            L.orc_sellmeier.restype = C.c_double
            L.orc_zernike.argtypes = [C.c_int, C.c_double, C.c_double]
            L.orc_zernike.restype = C.c_double
            L.orc_zernike_grad.argtypes = [C.c_int, C.c_double, C.c_double,
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]
            L.orc_intersect.argtypes = [C.POINTER(Scene), C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_int)]
            L.orc_sag.argtypes = [C.POINTER(Scene), C.c_int, C.c_double, C.c_double,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
            L.orc_sag.restype = C.c_double
            L.orc_coating.argtypes = [C.POINTER(Scene), C.c_int, C.c_double, C.c_double]
            L.orc_coating.restype = C.c_double
            L.orc_screen_gradient.argtypes = [C.POINTER(Scene), C.c_int, C.c_int, C.c_double,
                                              C.c_double, C.POINTER(C.c_double),
                                              C.POINTER(C.c_double)]
            L.orc_gamma.argtypes = [C.c_uint32, C.c_int32, C.c_uint64, C.c_double,
                                    C.POINTER(C.c_double)]
            L.orc_gamma.restype = C.c_int
            L.orc_air_refractivity.argtypes = [C.c_double] * 4
            L.orc_air_refractivity.restype = C.c_double
            L.orc_halo_sample.argtypes = [C.c_uint32, C.c_int32, C.c_uint64, C.c_double,
                                          C.c_double, C.POINTER(C.c_double)]
            L.orc_halo_sample.restype = C.c_int
            L.orc_kick_variance.argtypes = [C.POINTER(Scene), C.c_int]
            L.orc_kick_variance.restype = C.c_double
            L.orc_second_kick.argtypes = [C.POINTER(Scene), C.c_int32, C.c_uint64, C.c_int,
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]
            L.orc_second_kick.restype = C.c_int
            L.orc_field.argtypes = [C.POINTER(Scene), C.c_double]
            L.orc_field.restype = C.c_double
            L.orc_mobility.argtypes = [C.c_double, C.c_double]
            L.orc_mobility.restype = C.c_double
            L.orc_field_sigma.argtypes = [C.POINTER(Scene), C.c_double]
            L.orc_field_sigma.restype = C.c_double
            L.orc_bleed.argtypes = [C.c_void_p, C.POINTER(C.c_uint32), C.c_int32, C.c_int32]
            L.orc_readout.argtypes = [C.c_void_p, C.POINTER(C.c_uint32), C.c_int32, C.c_int32,
                                      C.POINTER(C.c_uint16), C.POINTER(C.c_double),
                                      C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                      C.POINTER(C.c_uint32)]
            L.orc_jacobian.argtypes = [C.POINTER(Scene), C.c_int32, C.c_uint64, C.c_uint64,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]
            _lib = L
    return _lib


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return [int(o[i]) for i in range(4)]


class Oracle:
    """An oracle instance bound to one synthetic scene (see paper_1504_06570_amd.scene)."""

    def __init__(self, scene, theta=None):
        from paper_1504_06570_amd.scene import coatings as coat_mod
        L = lib()
        p = scene.prescription
        sc = Scene()
        self._keep = []
        sc.n_surf = len(p.surfaces)
        assert sc.n_surf <= MAX_SURF
        sc.physics = int(scene.physics)
        for k, s in enumerate(p.surfaces):
            o = sc.surf[k]
            o.kind, o.medium, o.coating, o.group = s.kind, s.medium, s.coating, s.group
            o.z, o.c, o.kappa = s.z, s.curvature, s.conic
            for i in range(8):
                o.alpha[i] = s.alpha[i]
            o.r_in, o.r_out = s.r_in, s.r_out
        sc.pupil_r_in, sc.pupil_r_out, sc.pupil_margin = p.pupil_r_in, p.pupil_r_out, scene.pupil_margin
        sc.z_start, sc.obsc_z, sc.obsc_r = p.z_start, p.obscuration_z, p.obscuration_r
        for i in range(3):
            sc.glass_b[i] = p.glass_b[i]
            sc.glass_c[i] = p.glass_c_um2[i]
        sc.chip_x0, sc.chip_y0, sc.pixel = p.chip.x0, p.chip.y0, p.chip.pixel
        sc.nx, sc.ny = p.chip.nx, p.chip.ny
        sc.t_si, sc.temp_k, sc.sigma_max = p.silicon.thickness, p.silicon.temperature, p.silicon.sigma_max
        th = np.zeros(N_THETA) if theta is None else np.asarray(theta, float)
        if theta is None and getattr(scene, "perturbation", None) is not None:
            th = np.asarray(scene.perturbation, float)
        for i in range(N_THETA):
            sc.theta[i] = th[i]
        for g in range(3):
            for i in range(3):
                sc.pivot[g][i] = p.group_pivot[g][i]
        sc.zernike_r = p.surfaces[0].r_out
        if scene.coatings is not None:
            ct = np.ascontiguousarray(scene.coatings, np.float32)
            self._keep.append(ct)
            sc.n_coat, sc.n_s, sc.n_lam = ct.shape
            sc.s_max, sc.lam0, sc.dlam = coat_mod.S_MAX, coat_mod.LAM0, coat_mod.DLAM
            sc.coat = ct.ctypes.data_as(C.POINTER(C.c_float))
            if getattr(scene, "reflectance", None) is not None:
                rt = np.ascontiguousarray(scene.reflectance, np.float32)
                assert rt.shape == ct.shape
                self._keep.append(rt)
                sc.coat_r = rt.ctypes.data_as(C.POINTER(C.c_float))
        atm = scene.atmosphere
        if atm is not None:
            opd = np.ascontiguousarray(atm.opd, np.float32)
            self._keep.append(opd)
            sc.n_layers, sc.n_scales, sc.screen_n = atm.n_layers, atm.n_scales, atm.n
            for i in range(atm.n_layers):
                sc.height[i] = atm.heights[i]
                sc.wind[i][0], sc.wind[i][1] = atm.wind[i]
            for s in range(atm.n_scales):
                sc.pix[s] = atm.pixels[s]
            sc.lambda_ref = atm.lambda_ref
            sc.opd = opd.ctypes.data_as(C.POINTER(C.c_float))
        S = scene.sources
        arr = (Source * len(S))()
        for i in range(len(S)):
            a = arr[i]
            a.xi, a.eta = float(S.xi[i]), float(S.eta[i])
            a.kind, a.sed = int(S.kind[i]), int(S.sed[i])
            a.lam_lo, a.lam_hi, a.redshift = float(S.lam_lo[i]), float(S.lam_hi[i]), float(S.redshift[i])
            a.sersic_n, a.sersic_bn = float(S.sersic_n[i]), float(S.sersic_bn[i])
            a.sersic_a, a.sersic_b, a.sersic_pa = float(S.sersic_a[i]), float(S.sersic_b[i]), float(S.sersic_pa[i])
            a.n_photons = int(S.n_photons[i])
        self._keep.append(arr)
        sc.n_src = len(S)
        sc.src = C.cast(arr, C.POINTER(Source))
        if scene.sed is not None:
            e = np.ascontiguousarray(scene.sed.lam_edges, np.float64)
            f = np.ascontiguousarray(scene.sed.flux, np.float64)
            self._keep += [e, f]
            sc.n_sed, sc.sed_k = f.shape
            sc.sed_edges = e.ctypes.data_as(C.POINTER(C.c_double))
            sc.sed_flux = f.ctypes.data_as(C.POINTER(C.c_double))
        sc.seed = int(scene.seed) & 0xFFFFFFFF
        sc.exposure = scene.exposure
        x = getattr(scene, "extras", None)
        if x is not None:
            for name, _ in Extra._fields_:
                if name == "kick_fraction":
                    for i, f in enumerate(x.kick_fraction[:MAX_LAYERS]):
                        sc.ex.kick_fraction[i] = f
                elif name != "pad":
                    setattr(sc.ex, name, getattr(x, name))
        self.sc = sc
        self.scene = scene
        if L.orc_prepare(C.byref(sc)) != 0:
            raise MemoryError("oracle prepare failed")

    def __del__(self):
        try:
            lib().orc_release(C.byref(self.sc))
        except Exception:
            pass

    @property
    def image_shape(self):
        return (self.sc.ny, self.sc.nx)

    def trace(self, src: int, begin: int, count: int, image: Optional[np.ndarray] = None,
              events: bool = True):
        ev = np.zeros(count, EVENT_DTYPE) if events else None
        img_p = image.ctypes.data if image is not None else None
        if image is not None:
            assert image.dtype == np.uint32 and image.flags.c_contiguous
        rc = lib().orc_trace(C.byref(self.sc), int(src), int(begin), int(count), img_p,
                             ev.ctypes.data if ev is not None else None)
        if rc != 0:
            raise ValueError("oracle trace failed")
        return ev

    def trace_list(self, src: int, photons, threads: int = 1):
        """Events of the given photon indices of one source (a sample of a launch), in order;
        split over `threads` Python threads (the C call releases the GIL)."""
        ph = np.ascontiguousarray(photons, np.uint64)
        ev = np.zeros(len(ph), EVENT_DTYPE)
        parts = np.array_split(np.arange(len(ph)), max(1, threads))

        def run(idx):
            if len(idx) == 0:
                return
            a, b = int(idx[0]), int(idx[-1]) + 1
            rc = lib().orc_trace_list(C.byref(self.sc), int(src), ph[a:b].ctypes.data, b - a,
                                      None, ev[a:b].ctypes.data)
            if rc != 0:
                raise ValueError("oracle trace failed")
        if threads <= 1:
            run(parts[0])
        else:
            ths = [threading.Thread(target=run, args=(p,)) for p in parts]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
        return ev

    def trace_sources(self, counts=None, begin=0, image=None, events=True, threads=1):
        """Trace photons [begin, begin + counts[s]) of every source.  Returns concatenated events.
        With threads > 1, sources/photon ranges are split over Python threads (the C call releases
        the GIL); each thread bins into its own image, summed at the end."""
        S = self.scene.sources
        n = len(S)
        counts = np.asarray(S.n_photons if counts is None else counts, np.uint64)
        counts = np.broadcast_to(counts, (n,))
        jobs = []
        for s in range(n):
            c = int(counts[s])
            if c == 0:
                continue
            chunk = max(1, (c + threads - 1) // threads) if threads > 1 else c
            for b in range(0, c, chunk):
                jobs.append((s, begin + b, min(chunk, c - b)))
        if threads <= 1:
            out = [self.trace(s, b, c, image, events) for s, b, c in jobs]
        else:
            out = [None] * len(jobs)
            imgs = [np.zeros_like(image) if image is not None else None for _ in range(threads)]
            nxt = [0]
            lk = threading.Lock()

            def worker(w):
                while True:
                    with lk:
                        i = nxt[0]
                        nxt[0] += 1
                    if i >= len(jobs):
                        return
                    s, b, c = jobs[i]
                    out[i] = self.trace(s, b, c, imgs[w], events)

            ths = [threading.Thread(target=worker, args=(w,)) for w in range(threads)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            if image is not None:
                for im in imgs:
                    image += im
        if events:
            return np.concatenate(out) if out else np.zeros(0, EVENT_DTYPE)
        return None

    def jacobian(self, src: int, begin: int, count: int, h, threads: int = 1):
        """d(xe, ye)/d(theta) of photons [begin, begin + count) of one source: Richardson-
        extrapolated central differences with steps h (22 absolute values), every decision held
        fixed.  Returns (jac [count, 2, 22], frozen [count] bool)."""
        h = np.ascontiguousarray(h, np.float64)
        assert h.shape == (N_THETA,) and np.all(h > 0)
        jac = np.zeros((count, 2, N_THETA), np.float64)
        frozen = np.zeros(count, np.int32)
        hp = h.ctypes.data_as(C.POINTER(C.c_double))

        def run(a, b):
            rc = lib().orc_jacobian(C.byref(self.sc), src, begin + a, b - a, hp,
                                    jac[a:b].ctypes.data_as(C.POINTER(C.c_double)),
                                    frozen[a:b].ctypes.data_as(C.POINTER(C.c_int32)))
            assert rc == 0

        if threads <= 1 or count < 2 * threads:
            run(0, count)
        else:
            cuts = np.linspace(0, count, threads + 1).astype(int)
            ths = [threading.Thread(target=run, args=(cuts[w], cuts[w + 1]))
                   for w in range(threads)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
        return jac, frozen.astype(bool)

    # primitives -----------------------------------------------------------------------------
    def sag(self, k, x, y):
        sx, sy = C.c_double(), C.c_double()
        s = lib().orc_sag(C.byref(self.sc), k, x, y, C.byref(sx), C.byref(sy))
        return s, sx.value, sy.value

    def intersect(self, k, q, d):
        qa = (C.c_double * 3)(*q)
        da = (C.c_double * 3)(*d)
        l, it = C.c_double(), C.c_int()
        st = lib().orc_intersect(C.byref(self.sc), k, qa, da, C.byref(l), C.byref(it))
        return st, l.value, it.value

    def field(self, z):
        return lib().orc_field(C.byref(self.sc), z)

    def field_sigma(self, depth):
        return lib().orc_field_sigma(C.byref(self.sc), depth)

    def kick_variance(self, layer):
        return lib().orc_kick_variance(C.byref(self.sc), layer)

    def second_kick(self, src, photon, layer):
        """(kx, ky, K): the second kick (radians at the reference wavelength) of one photon at
        one layer and its number of scatterings."""
        kx, ky = C.c_double(), C.c_double()
        K = lib().orc_second_kick(C.byref(self.sc), src, photon, layer, C.byref(kx), C.byref(ky))
        return kx.value, ky.value, K

    def sellmeier(self, lam):
        return lib().orc_sellmeier(C.byref(self.sc), lam)

    def coating(self, coat, s, lam):
        return lib().orc_coating(C.byref(self.sc), coat, s, lam)

    def screen_gradient(self, layer, scale, x, y):
        gx, gy = C.c_double(), C.c_double()
        lib().orc_screen_gradient(C.byref(self.sc), layer, scale, x, y, C.byref(gx), C.byref(gy))
        return gx.value, gy.value


def air_refractivity(lam, pressure, temperature, water):
    """n - 1 of air (the Filippenko formula); lam in metres, pressures in mmHg, T in deg C."""
    return lib().orc_air_refractivity(lam, pressure, temperature, water)


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


def readout_params(rp) -> ReadoutParams:
    """ctypes struct from a scene.readout.Readout description."""
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


def bleed(rp, image):
    """Saturation and bleeding of a uint32 [ny, nx] image (a copy is returned)."""
    img = np.ascontiguousarray(image, np.uint32).copy()
    ny, nx = img.shape
    P = readout_params(rp)
    assert lib().orc_bleed(C.byref(P), img.ctypes.data_as(C.POINTER(C.c_uint32)), nx, ny) == 0
    return img


def readout(rp, image):
    """The readout chain of a uint32 [ny, nx] electron image: returns (adu [amp, sh + over_y,
    sw + over_x] uint16, margin, after-defects image, after-parallel slots, after-serial slots)."""
    img = np.ascontiguousarray(image, np.uint32)
    ny, nx = img.shape
    na = rp.amp_nx * rp.amp_ny
    sw, sh = nx // rp.amp_nx, ny // rp.amp_ny
    ph, pw = sh + rp.over_y, sw + rp.over_x
    out = np.zeros((na, ph, pw), np.uint16)
    margin = np.zeros((na, ph, pw), np.float64)
    work = np.zeros_like(img)
    par = np.zeros((na, ph, sw), np.uint32)
    ser = np.zeros((na, ph, pw), np.uint32)
    P = readout_params(rp)
    u32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_uint32))
    rc = lib().orc_readout(C.byref(P), u32(img), nx, ny,
                           out.ctypes.data_as(C.POINTER(C.c_uint16)),
                           margin.ctypes.data_as(C.POINTER(C.c_double)), u32(work), u32(par),
                           u32(ser))
    if rc != 0:
        raise ValueError("oracle readout: bad geometry")
    return out, margin, work, par, ser


def mobility(E, T):
    """Electron mobility (m^2/Vs) at field E (V/m) and temperature T (K)."""
    return lib().orc_mobility(E, T)


def halo_sample(seed, src, photon, n, x_max):
    """(x, trial) of the halo sampler for one photon; trial = -1 when every trial was rejected."""
    x = C.c_double()
    t = lib().orc_halo_sample(int(seed) & 0xFFFFFFFF, int(src), int(photon), n, x_max,
                              C.byref(x))
    return x.value, t


def image_from_events(ev, shape):
    img = np.zeros(shape, np.uint32)
    d = ev[ev["status"] == DETECTED]
    np.add.at(img, (d["pix_j"], d["pix_i"]), 1)
    return img
