"""The C-ABI library loads on the CPU and exports every function include/phx.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phx_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("phx_create", "phx_destroy", "phx_load_prescription", "phx_load_screens",
              "phx_load_sources", "phx_trace", "phx_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1504_06570_amd import phx as P
    L = P.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
        assert isinstance(getattr(L, n), ctypes._CFuncPtr)
    assert P.lib().phx_version().startswith(b"phx")


def test_struct_sizes_match_header_layout():
    """The binding's ctypes structs have the header's sizes (checked against a host compile)."""
    import subprocess
    import tempfile
    from paper_1504_06570_amd import phx as P
    src = r"""
#include <stdio.h>
#include "phx.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(phx_surface),
         sizeof(phx_prescription), sizeof(phx_atmosphere), sizeof(phx_source), sizeof(phx_event),
         sizeof(phx_trace_args), offsetof(phx_trace_args, image_dev), sizeof(phx_launch_config),
         sizeof(phx_physics), offsetof(phx_physics, spider_angle), sizeof(phx_readout_params));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        got = [int(x) for x in subprocess.check_output([exe], text=True).split()]
    want = [ctypes.sizeof(P.Surface), ctypes.sizeof(P.Prescription), ctypes.sizeof(P.Atmosphere),
            ctypes.sizeof(P.Source), P.EVENT_DTYPE.itemsize, ctypes.sizeof(P.TraceArgs),
            P.TraceArgs.image_dev.offset, ctypes.sizeof(P.LaunchConfig),
            ctypes.sizeof(P.Physics), P.Physics.spider_angle.offset, ctypes.sizeof(P.ReadoutParams)]
    assert got == want


def test_create_without_gpu_is_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1504_06570_amd import phx as P
    h = ctypes.c_void_p()
    assert P.lib().phx_create(0, ctypes.byref(h)) == -1
    assert P.lib().phx_trace(None, None, None) == -1
    assert P.lib().phx_last_error(None) == b"null context"
    assert P.lib().phx_trace_batched(None, None, None) == -1
    assert P.lib().phx_autotune(None, None, None, None) == -1


def test_probe_library_exports_and_checks_arguments():
    """The benchmark's gather probe (a library of its own) loads on the CPU, and refuses invalid
    arguments before it touches a device."""
    from paper_1504_06570_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        pytest.skip("probe library not built")
    L = ctypes.CDLL(B.PROBE_LIB)
    f = L.probe_gather
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                  ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p]
    f.restype = ctypes.c_int
    assert f(None, 16, None, 1, 7, 1, 0, None) == -1        # null table and output
    assert f(16, 16, 16, 1, 7, 5, 0, None) == -1            # more than four gathers in flight
    assert f(24, 16, 16, 1, 7, 1, 0, None) == -1            # table not 16-byte aligned
    assert f(16, 1 << 33, 16, 1, 7, 1, 0, None) == -1       # more records than 32-bit indices


def test_probe_library_op_rate_entry_checks_arguments():
    """The FP64 op-rate probe refuses invalid arguments before it touches a device."""
    from paper_1504_06570_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        pytest.skip("probe library not built")
    f = ctypes.CDLL(B.PROBE_LIB).probe_fp64
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
    f.restype = ctypes.c_int
    assert f(0, None, 16, 10, None) == -1      # null output
    assert f(8, 16, 16, 10, None) == -1        # unknown class
    assert f(0, 16, 0, 10, None) == -1         # no threads
    assert f(0, 16, 16, 0, None) == -1         # no steps


def test_probe_library_philox_entry_checks_arguments():
    """The Philox block-rate probe refuses invalid arguments before it touches a device."""
    from paper_1504_06570_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        pytest.skip("probe library not built")
    f = ctypes.CDLL(B.PROBE_LIB).probe_philox
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
    f.restype = ctypes.c_int
    assert f(None, 16, 10, None) == -1         # null output
    assert f(16, 0, 10, None) == -1            # no threads
    assert f(16, 16, 0, None) == -1            # no blocks
