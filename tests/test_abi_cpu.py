"""The C-ABI library loads and exports what include/adgi.h declares (CPU only).

No compute call is made here: only argument validation, which returns before
any HIP call, is exercised.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2301_05125_amd as adgi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "adgi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(adgi_[a-z_]+)\s*\(", src)))


def test_header_declares_the_four_entry_points():
    names = _declared()
    for n in ("adgi_create_volume", "adgi_update_scene", "adgi_update_probes",
              "adgi_read_probes", "adgi_destroy_volume", "adgi_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(adgi.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def _desc(**kw):
    d = adgi.VolumeDesc()
    d.origin[:] = [0, 0, 0]
    d.spacing[:] = [1, 1, 1]
    d.dims[:] = [2, 2, 2]
    d.irr_res, d.depth_res, d.storage = 8, 16, adgi.ADGI_FP32
    d.hysteresis, d.tau_max, d.max_rays_per_frame, d.seed = 0.97, 9.8, 1024, 1
    for k, v in kw.items():
        if k in ("dims", "spacing", "origin"):
            getattr(d, k)[:] = v
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("bad", [
    {"dims": [0, 2, 2]}, {"spacing": [1, -1, 1]}, {"irr_res": 2}, {"depth_res": 35},
    {"storage": 7}, {"hysteresis": 1.0}, {"tau_max": 0.0}, {"max_rays_per_frame": 0},
    {"max_rays_per_frame": 1 << 31}, {"dims": [4096, 4096, 2]}, {"flags": 8},
])
def test_invalid_descriptor_rejected_before_any_device_call(bad):
    L = adgi.lib()
    h = C.c_void_p()
    st = L.adgi_create_volume(C.byref(_desc(**bad)), None, None, C.byref(h))
    assert st == -1
    assert h.value is None
    assert len(L.adgi_last_error()) > 0


def test_null_arguments():
    L = adgi.lib()
    assert L.adgi_create_volume(None, None, None, None) == -1
    assert L.adgi_update_scene(None, None) == -1
    assert L.adgi_update_probes(None, None, None) == -1
    assert L.adgi_read_probes(None, None) == -1
    L.adgi_destroy_volume(None)  # no-op
    assert L.adgi_state_size(None) == 0


def test_pack_channel_argument_checks():
    """adgi_pack_channel validates before any device call; count 0 is a no-op."""
    L = adgi.lib()
    x = C.c_void_p(16)  # never dereferenced: every call here returns first
    assert L.adgi_pack_channel(x, C.c_int64(-1), 0, x, x, None) == adgi.ADGI_ERR_INVALID_ARG
    assert L.adgi_pack_channel(x, C.c_int64(4), 4, x, x, None) == adgi.ADGI_ERR_INVALID_ARG
    assert L.adgi_pack_channel(x, C.c_int64(4), -1, x, x, None) == adgi.ADGI_ERR_INVALID_ARG
    assert L.adgi_pack_channel(None, C.c_int64(4), 0, x, x, None) == adgi.ADGI_ERR_INVALID_ARG
    assert L.adgi_pack_channel(x, C.c_int64(4), 0, None, None, None) == adgi.ADGI_ERR_INVALID_ARG
    assert L.adgi_pack_channel(None, C.c_int64(0), 3, None, None, None) == adgi.ADGI_OK


def test_crash_trace_prints_the_native_stack():
    """With ADGI_CRASH_TRACE set, a process that created a server (here with
    NULL arguments: no device call at all) prints the native stack on a
    segmentation fault and then hands the signal on (Python's faulthandler
    prints its stack, the process dies of SIGSEGV). The fault is a host-side
    read of address 0 in a CPU-only child process."""
    import subprocess
    import sys
    code = ("import sys, ctypes as C, faulthandler; faulthandler.enable(); "
            f"sys.path.insert(0, {ROOT!r}); import paper_2301_05125_amd as adgi; "
            "assert adgi.lib().adgi_server_create(None, None, None) == adgi.ADGI_ERR_INVALID_ARG; "
            "C.string_at(0)")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, ADGI_CRASH_TRACE="1"))
    assert r.returncode in (-11, 139), (r.returncode, r.stderr[-2000:])
    assert "adgi: native stack at the fault" in r.stderr and "libadgi.so" in r.stderr, r.stderr[-2000:]
    assert "Segmentation fault" in r.stderr
