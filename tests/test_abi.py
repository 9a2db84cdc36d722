"""The C-ABI library builds, loads and exports every entry point declared in
include/wl.h; host-side argument checks that never reach the device.  CPU
only (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wl.h")
LIB = os.path.join(ROOT, "paper_1407_7486_amd", "libwl.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"\b(wl_[a-z_]+)\s*\(", txt))


@pytest.fixture(scope="module")
def wl():
    if not os.path.exists(LIB):
        pytest.fail("libwl.so not built: run __graft_entry__.build()")
    import paper_1407_7486_amd as wl
    return wl


def test_header_declares_the_entry_points():
    names = declared()
    assert {"wl_create", "wl_ensemble_upload", "wl_average", "wl_per_loop"} <= names


def test_library_exports_every_declared_symbol(wl):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], stdout=subprocess.PIPE,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (wl_\w+)", out))
    missing = declared() - exported
    assert not missing, missing
    assert set(wl.EXPORTS) == declared()
    for n in declared():
        assert wl.raw_function(n) is not None


def test_static_strings(wl):
    assert "gfx950" in wl.wl_version()
    assert wl.wl_strerror(wl.WL_EINVAL) == "invalid argument"
    assert wl.wl_strerror(12345) == "unknown error code"


def test_null_arguments_are_rejected_without_a_device(wl):
    lib = ctypes.CDLL(LIB)
    lib.wl_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert lib.wl_create(None, 0, None) == wl.WL_EINVAL
    lib.wl_destroy.argtypes = [ctypes.c_void_p]
    assert lib.wl_destroy(None) == wl.WL_OK
    lib.wl_ensemble_free.argtypes = [ctypes.c_void_p]
    assert lib.wl_ensemble_free(None) == wl.WL_OK
    lib.wl_ensemble_info.argtypes = [ctypes.c_void_p] * 4
    assert lib.wl_ensemble_info(None, None, None, None) == wl.WL_EINVAL
    for fn in ("wl_average", "wl_average_async", "wl_average_async_noalloc",
               "wl_per_loop", "wl_ensemble_upload"):
        f = getattr(lib, fn)
        f.restype = ctypes.c_int
        # a NULL context is rejected before anything else is read
        assert f(None, None, None, None, 0, None, 0, 0, 0, None, None, None) \
            == wl.WL_EINVAL
    lib.wl_discretisation.restype = ctypes.c_int
    assert lib.wl_discretisation(None, None, None, None, 0, None, 0, 0, 0, 0, None, None,
                                 None, None) == wl.WL_EINVAL
    lib.wl_subloop_per_loop.restype = ctypes.c_int
    assert lib.wl_subloop_per_loop(None, None, None, None, 0, None, 0, 0, 0, 0,
                                   ctypes.c_int64(0), ctypes.c_int64(0), None, None,
                                   None) == wl.WL_EINVAL
    lib.wl_action.restype = ctypes.c_int
    assert lib.wl_action(None, None, None, 0, None, 0, ctypes.c_int64(0), 0, None) \
        == wl.WL_EINVAL
    lib.wl_action_grids.restype = ctypes.c_int
    assert lib.wl_action_grids(None, None, None) == wl.WL_EINVAL
    lib.wl_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    assert lib.wl_set_timing(None, 1) == wl.WL_EINVAL
    lib.wl_last_kernel_ms.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.wl_last_kernel_ms(None, None) == wl.WL_EINVAL


def test_noalloc_scratch_size_matches_the_header(wl):
    txt = open(HEADER).read()
    m = re.search(r"#define WL_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    assert m, "WL_NOALLOC_SCRATCH_BYTES not found"
    assert wl.WL_NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))


def test_binding_constants_match_the_header(wl):
    """Every integer #define of include/wl.h that the binding also names
    (precision modes, field kinds, flags, error codes) has the same value."""
    txt = open(HEADER).read()
    defs = {n: int(v) for n, v in re.findall(r"#define (WL_[A-Z0-9_]+) (-?\d+)\b", txt)}
    shared = {n for n in defs if hasattr(wl, n)}
    assert {"WL_FP32C", "WL_FP32", "WL_FP64", "WL_FP32K", "WL_SECH2"} <= shared
    bad = {n: (defs[n], getattr(wl, n)) for n in shared if getattr(wl, n) != defs[n]}
    assert not bad, bad


def test_no_device_is_reported_cleanly(wl):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    with pytest.raises(wl.WLError) as ei:
        wl.wl_create(0, None)
    assert ei.value.code == wl.WL_ENODEV


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The product package has no CPU fallback: importing it from a copy
    without libwl.so raises ImportError."""
    import shutil
    import sys
    pkg = tmp_path / "paper_1407_7486_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1407_7486_amd", "__init__.py"), pkg)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n import paper_1407_7486_amd\nexcept ImportError as e:\n"
            " print('IMPORTERROR', e)\n" % str(tmp_path))
    out = subprocess.run([sys.executable, "-c", code], stdout=subprocess.PIPE,
                         text=True).stdout
    assert "IMPORTERROR" in out and "not been built" in out


def test_action_grids_match_the_oracle(wl):
    """Host logic of the C ABI (no device): the action grids equal the
    oracle's, and invalid specs are refused."""
    import numpy as np

    import oracle
    for args in [(1.0, 0.05, 1.0, 32, 1.0, 16), (0.3, 0.01, 3.0, 64, 2.5, 40)]:
        m2, a, Tm, nT, rm, nr = args
        T, rho = wl.wl_action_grids(wl.action_spec(m2, a, Tm, nT, rm, nr))
        To, ro = oracle.action_grids(a, Tm, nT, rm, nr)
        np.testing.assert_allclose(T, To, rtol=1e-15)
        np.testing.assert_allclose(rho, ro, rtol=1e-15)
    for bad in [(1.0, 0.05, 1.0, 31, 1.0, 16), (1.0, 0.0, 1.0, 32, 1.0, 16),
                (1.0, 0.05, 1.0, 32, 1.0, 0)]:
        with pytest.raises(wl.WLError):
            wl.wl_action_grids(wl.action_spec(*bad))
