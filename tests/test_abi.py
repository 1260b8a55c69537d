"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the device."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fc.h")


@pytest.fixture(scope="module")
def fcmod():
    import paper_2002_07858_amd.fc as fc
    if not os.path.exists(fc.LIB_PATH):
        from paper_2002_07858_amd import build
        build.build()
    return fc


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fc_build_grid", "fc_build_covariance", "fc_scan", "fc_critical_value",
              "fc_grid_destroy", "fc_grid_device_bytes", "fc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(fcmod):
    lib = ctypes.CDLL(fcmod.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(fcmod.EXPORTED)


def test_status_codes_match_header(fcmod):
    text = open(HEADER).read()
    for name in ("FC_OK", "FC_ERR_INVALID_ARG", "FC_ERR_NOT_PD", "FC_ERR_NOMEM",
                 "FC_ERR_DEVICE", "FC_ERR_STATE", "FC_ERR_UNSUPPORTED", "FC_FORM_FP64",
                 "FC_FORM_FP32", "FC_FORM_SPLIT_BF16", "FC_FORM_SPLIT_FP16", "FC_STAT_PEARSON",
                 "FC_STAT_FIXED", "FC_MAX_BINS"):
        m = re.search(rf"\b{name}\s*=?\s*(-?\d+)", text)
        assert m, name
        assert int(m.group(1)) == getattr(fcmod, name), name


def _call_build_grid(fcmod, D, lens, vals, N, S):
    out = ctypes.c_void_p()
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    rc = fcmod.lib().fc_build_grid(ctypes.byref(out), D, lens.ctypes.data_as(ctypes.c_void_p),
                                   vals.ctypes.data_as(ctypes.c_void_p), N,
                                   S.ctypes.data_as(ctypes.c_void_p), None, None)
    return rc, out.value


def test_build_grid_rejects_bad_arguments_on_host(fcmod):
    S = np.ones((4, 3))
    assert _call_build_grid(fcmod, 0, [4], [0, 1, 2, 3], 3, S)[0] == fcmod.FC_ERR_INVALID_ARG
    assert _call_build_grid(fcmod, 1, [0], [0.0], 3, S)[0] == fcmod.FC_ERR_INVALID_ARG
    assert _call_build_grid(fcmod, 1, [4], [0, 1, 2, 3], 0, S)[0] == fcmod.FC_ERR_INVALID_ARG
    S65 = np.ones((4, 65))
    rc, h = _call_build_grid(fcmod, 1, [4], [0, 1, 2, 3], 65, S65)
    assert rc == fcmod.FC_ERR_UNSUPPORTED and h is None
    Sbad = np.ones((4, 3))
    Sbad[2, 1] = np.nan
    rc, _ = _call_build_grid(fcmod, 1, [4], [0, 1, 2, 3], 3, Sbad)
    assert rc == fcmod.FC_ERR_INVALID_ARG
    assert "non-finite" in fcmod.fc_last_error()
    rc, _ = _call_build_grid(fcmod, 2, [1 << 16, 1 << 16], np.zeros(1 << 17), 3, S)
    assert rc == fcmod.FC_ERR_INVALID_ARG


def test_calls_on_null_grid_fail_cleanly(fcmod):
    L = fcmod.lib()
    F = np.eye(3)
    bad = np.zeros(1, dtype=np.int64)
    assert L.fc_build_covariance(None, F.ctypes.data_as(ctypes.c_void_p), 0, None, 2,
                                 bad.ctypes.data_as(ctypes.c_void_p), None) == \
        fcmod.FC_ERR_INVALID_ARG
    assert L.fc_scan(None, 2, 10, None, None, None, None, None, None, None) == \
        fcmod.FC_ERR_INVALID_ARG
    assert L.fc_grid_inverse_cov(None, 0, 1, None, None) == fcmod.FC_ERR_INVALID_ARG
    assert L.fc_grid_info(None, None, None, None, None) == fcmod.FC_ERR_INVALID_ARG
    assert L.fc_grid_device_bytes(None) == 0
    L.fc_grid_destroy(None)


def test_critical_value_validation(fcmod):
    L = fcmod.lib()
    a = np.array([0.9])
    ap = a.ctypes.data_as(ctypes.c_void_p)
    assert L.fc_critical_value(-1, None, None, 1, ap, None, 10, 5.0, None, None) == \
        fcmod.FC_ERR_INVALID_ARG
    assert L.fc_critical_value(1, None, None, 0, ap, None, 10, 5.0, None, None) == \
        fcmod.FC_ERR_INVALID_ARG
    a0 = np.array([0.0])
    assert L.fc_critical_value(1, None, None, 1, a0.ctypes.data_as(ctypes.c_void_p), None, 10,
                               5.0, None, None) == fcmod.FC_ERR_INVALID_ARG
    # zero segments: nothing to do, no device work
    assert L.fc_critical_value(0, None, None, 1, ap, None, 10, 5.0, None, None) == fcmod.FC_OK
    # a segment but NULL device pointers
    assert L.fc_critical_value(1, None, None, 1, ap, None, 10, 5.0, None, None) == \
        fcmod.FC_ERR_INVALID_ARG


def test_binding_refuses_host_arrays(fcmod):
    with pytest.raises(TypeError):
        fcmod._dev(np.zeros(3), "f64", "d")


def test_slice_entry_points_validate_on_host(fcmod):
    """Grid-sliced scans: argument errors are reported before any device work."""
    L = fcmod.lib()
    assert L.fc_scan_state_init(-1, None, None, None) == fcmod.FC_ERR_INVALID_ARG
    assert L.fc_scan_state_init((1 << 30) + 1, None, None, None) == fcmod.FC_ERR_INVALID_ARG
    assert L.fc_scan_state_init(0, None, None, None) == fcmod.FC_OK        # nothing to do
    assert L.fc_scan_state_init(5, None, None, None) == fcmod.FC_ERR_INVALID_ARG
    assert L.fc_scan_slice(None, 2, 10, None, None, 0, 1, None, None, None) == \
        fcmod.FC_ERR_INVALID_ARG
    assert "grid is NULL" in fcmod.fc_last_error()
    assert L.fc_scan_points_slice(None, 2, 1, None, None, 10, None, 0, 1, None, 0, None, None,
                                  None) == fcmod.FC_ERR_INVALID_ARG
    b = ctypes.c_size_t(7)
    assert L.fc_scan_points_slice_workspace(None, 2, 1, 10, 1, ctypes.byref(b)) == \
        fcmod.FC_ERR_INVALID_ARG
    assert L.fc_scan_state_finalize(None, 10, None, None, None, None, None, None, None) == \
        fcmod.FC_ERR_INVALID_ARG


def test_bench_refuses_several_gpus():
    """The benchmark runs on one GPU; asked for more it exits with a message."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_checks_sizes_before_the_library(fcmod):
    """Tensors too short for the call are refused in the binding: the kernels
    would read or write past their ends."""
    torch = pytest.importorskip("torch")
    g = fcmod.Grid(0)
    g._shape = (57, 100)  # N, G of a grid that is never touched
    d = torch.zeros((10, 57), dtype=torch.float64)
    p = torch.zeros(10, dtype=torch.int64)
    out = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match=r"\[K\]\[57\]"):
        fcmod.fc_scan(g, 2, torch.zeros((10, 56), dtype=torch.float64), p, out)
    with pytest.raises(ValueError, match="p_idx"):
        fcmod.fc_scan(g, 2, d, p[:9], out)
    with pytest.raises(ValueError, match="chi2_p"):
        fcmod.fc_scan(g, 2, d, p, out, chi2_p=out[:5])
    with pytest.raises(ValueError, match="seg_off"):
        fcmod.fc_scan_points(g, 2, p[:2], p[:2], d, out)
    with pytest.raises(ValueError, match="crit"):
        fcmod.fc_critical_value(p[:3], out, [0.9, 0.95], out[:3])
    with pytest.raises(ValueError, match="keys"):
        fcmod.fc_scan_slice(g, 2, d, p, 0, 10, p[:4], out)


def test_profile_calls_validate(fcmod):
    L = fcmod.lib()
    assert L.fc_profile_read(None, None, None) == fcmod.FC_ERR_INVALID_ARG
    assert L.fc_profile_enable(0) == fcmod.FC_OK
    n = ctypes.c_int64(-1)
    ms = ctypes.c_double(-1.0)
    assert L.fc_profile_read(b"k_scan_f64m", ctypes.byref(n), ctypes.byref(ms)) == fcmod.FC_OK
    assert n.value == 0 and ms.value == 0.0
