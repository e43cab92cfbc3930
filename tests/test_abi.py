"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1508_07344_amd as sce

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(sce.library_path()):
        pytest.skip("libsce.so not built")
    return sce.load_library()


def test_header_declares_the_api():
    names = sce.exported_symbols()
    for required in ("sce_create", "sce_create_2d", "sce_create_tent", "sce_field_shape",
                     "sce_dimension", "sce_set_step_graph", "sce_set_small_step", "sce_set_options", "sce_set_particles", "sce_get_particles",
                     "sce_mode_count", "sce_modes", "sce_deposit", "sce_psi", "sce_force",
                     "sce_force_noalloc",
                     "sce_step", "sce_diagnostics", "sce_get_state", "sce_set_state", "sce_sync",
                     "sce_timing_enable", "sce_timing_read", "sce_destroy", "sce_status_string",
                     "sce_last_error", "sce_server_create", "sce_server_submit", "sce_server_tick",
                     "sce_server_poll", "sce_server_result", "sce_server_stats",
                     "sce_server_last_error", "sce_server_destroy"):
        assert required in names


def test_peak_probe_library_exports_its_header():
    """libsce_peak.so (the roofline denominators' throughput probes) exports
    every function include/sce_peak.h declares."""
    lib = os.path.join(ROOT, "paper_1508_07344_amd", "libsce_peak.so")
    if not os.path.exists(lib):
        pytest.skip("libsce_peak.so not built")
    hdr = open(os.path.join(ROOT, "include", "sce_peak.h")).read()
    declared = set(re.findall(r"^\s*int\s+(sce_peak_\w+)\s*\(", hdr, re.M))
    assert declared == {"sce_peak_mfma_f16", "sce_peak_fma_f32", "sce_peak_fma_f64"}
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True,
                         check=True).stdout
    assert declared <= set(re.findall(r"\bT (sce_peak_\w+)", out))
    ctypes.CDLL(lib)


def test_library_exports_every_declared_symbol():
    _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", sce.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sce_\w+)", out))
    missing = set(sce.exported_symbols()) - exported
    assert not missing, missing
    lib = ctypes.CDLL(sce.library_path())
    for name in sce.exported_symbols():
        assert hasattr(lib, name)


def test_invalid_create_arguments_are_rejected_on_host():
    lib = _lib()
    h = ctypes.c_void_p()
    bad = [(-1.0, 8, 1, 0.05), (float("nan"), 8, 1, 0.05), (float("inf"), 8, 1, 0.05),
           (1.0, 0, 1, 0.05), (1.0, 65, 1, 0.05), (1.0, 8, 7, 0.05), (1.0, 8, 1, -0.1),
           (1.0, 8, 1, float("nan"))]
    for args in bad:
        assert lib.sce_create(*args, ctypes.byref(h)) == sce.SCE_EINVAL, args
        assert not h.value
    assert lib.sce_create(1.0, 8, 1, 0.05, None) == sce.SCE_EINVAL
    for args in bad:
        assert lib.sce_create_2d(*args, ctypes.byref(h)) == sce.SCE_EINVAL, args
        assert not h.value
    assert lib.sce_create_2d(1.0, 8, 1, 0.05, None) == sce.SCE_EINVAL
    d = ctypes.c_int32()
    assert lib.sce_dimension(None, ctypes.byref(d)) == sce.SCE_EINVAL
    for L, n, dim in [(-1.0, 8, 3), (float("nan"), 8, 3), (1.0, 0, 3), (1.0, 65, 2), (1.0, 8, 1),
                      (1.0, 8, 4)]:
        assert lib.sce_create_tent(L, n, dim, ctypes.byref(h)) == sce.SCE_EINVAL, (L, n, dim)
        assert not h.value
    assert lib.sce_create_tent(1.0, 8, 3, None) == sce.SCE_EINVAL
    assert lib.sce_field_shape(None, ctypes.byref(d)) == sce.SCE_EINVAL


def test_null_context_is_rejected():
    lib = _lib()
    assert lib.sce_sync(None) == sce.SCE_EINVAL
    assert lib.sce_step(None, 1e-3, 1) == sce.SCE_EINVAL
    assert lib.sce_set_step_graph(None, 8) == sce.SCE_EINVAL
    assert lib.sce_set_small_step(None, 0) == sce.SCE_EINVAL
    assert lib.sce_deposit(None, None, 0) == sce.SCE_EINVAL
    lib.sce_destroy(None)  # no-op


def test_status_strings():
    lib = _lib()
    for s in range(-6, 1):
        assert lib.sce_status_string(s).decode()


def test_server_arguments_are_rejected_on_host():
    from paper_1508_07344_amd.sce import _ServerOpts
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.sce_server_create(None, None) == sce.SCE_EINVAL
    for prec, max_active, want in [(sce.PREC["split_f16"], 0, sce.SCE_ENOTSUP), (7, 0, sce.SCE_ENOTSUP),
                                   (sce.PREC["fp32"], -1, sce.SCE_EINVAL)]:
        o = _ServerOpts(0, prec, max_active, 0, None)
        assert lib.sce_server_create(ctypes.byref(o), ctypes.byref(h)) == want
        assert not h.value
    n = ctypes.c_int32()
    assert lib.sce_server_tick(None, None, None) == sce.SCE_EINVAL
    assert lib.sce_server_submit(None, None, None) == sce.SCE_EINVAL
    assert lib.sce_server_poll(None, None, 0, ctypes.byref(n)) == sce.SCE_EINVAL
    assert lib.sce_server_result(None, 1, None, None, None, None, None) == sce.SCE_EINVAL
    assert lib.sce_server_stats(None, None) == sce.SCE_EINVAL
    assert lib.sce_server_last_error(None).decode()
    lib.sce_server_destroy(None)  # no-op
