"""The C-ABI library loads, exports every entry point its header declares, and
rejects bad descriptors with the documented status codes before touching a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1705_01893_amd import mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:mm_status|const char\s*\*)\s*(mm_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("mm_plan", "mm_plan_destroy", "mm_plan_workspace_bytes", "mm_plan_hits", "mm_messenger_iter",
                 "mm_solve", "mm_cg_solve", "mm_chi2", "mm_status_str", "mm_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = mm.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_status_strings():
    assert mm.mm_status_str(0) == "ok"
    assert "length" in mm.mm_status_str(2)
    assert mm.mm_status_str(99) == "unknown status"


def _desc(**over):
    n = over.pop("lengths", [64, 64])
    off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    nch = len(n)
    arr = dict(fs=np.full(nch, 10.0), sig=np.ones(nch), fk=np.ones(nch), al=np.full(nch, -2.0), off=off)
    arr.update(over.pop("arrays", {}))
    d = mm._Desc()
    d.ncomp = over.pop("ncomp", 1)
    d.precision = over.pop("precision", 0)
    d.npix = over.pop("npix", 16)
    d.nx = over.pop("nx", 4)
    d.nchunk = nch
    d.chunk_off = arr["off"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.fsample = arr["fs"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.sigma = arr["sig"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.fknee = arr["fk"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.alpha = arr["al"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if "tau" in arr:
        d.tau = arr["tau"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # a non-null placeholder: every case below fails validation before the pointer is used
    d.pix = over.pop("pix", 0x1000)
    d.psi = over.pop("psi", None)
    d.psi_kind = over.pop("psi_kind", 0)
    d.map_access = over.pop("map_access", 0)
    d.tune = over.pop("tune", 0)
    d.binning = over.pop("binning", 0)
    d.with_adjoint = over.pop("with_adjoint", 0)
    d.tile_pixels = over.pop("tile_pixels", 0)
    d.pix_b = over.pop("pix_b", None)
    d.psi_b = over.pop("psi_b", None)
    d.weight_a = over.pop("weight_a", 1.0)
    d.weight_b = over.pop("weight_b", -1.0)
    d.with_gapfill = over.pop("with_gapfill", 0)
    assert not over
    return d, arr


@pytest.mark.parametrize("case, status", [
    (dict(ncomp=2), mm.MM_E_ARG),
    (dict(precision=7), mm.MM_E_ARG),
    (dict(map_access=3), mm.MM_E_ARG),
    (dict(tune=2), mm.MM_E_ARG),
    (dict(binning=2), mm.MM_E_ARG),
    (dict(with_adjoint=2), mm.MM_E_ARG),
    (dict(tile_pixels=8), mm.MM_E_ARG),
    (dict(tile_pixels=4096), mm.MM_E_ARG),
    (dict(npix=0), mm.MM_E_ARG),
    (dict(npix=15, nx=4), mm.MM_E_ARG),
    (dict(pix=None), mm.MM_E_ARG),
    (dict(lengths=[64, 63]), mm.MM_E_LEN),       # odd length
    (dict(lengths=[64, 2 * 7 * 8]), mm.MM_E_LEN),  # half length has a factor 7
    (dict(ncomp=3), mm.MM_E_ARG),                 # I/Q/U without angles
    (dict(arrays=dict(sig=np.array([1.0, -1.0]))), mm.MM_E_ARG),
    (dict(arrays=dict(tau=np.array([1.0, 1.5]))), mm.MM_E_ARG),  # tau above sigma^2
    (dict(arrays=dict(off=np.array([1, 65, 129], np.int64))), mm.MM_E_ARG),
    # composite pointing: second angles, finite weights, projected access and sorted binning required
    (dict(ncomp=3, psi=0x2000, psi_kind=1, pix_b=0x3000), mm.MM_E_ARG),
    (dict(pix_b=0x3000, weight_b=float("nan")), mm.MM_E_ARG),
    (dict(pix_b=0x3000, weight_a=float("inf")), mm.MM_E_ARG),
    (dict(pix_b=0x3000, map_access=1), mm.MM_E_ARG),
    (dict(pix_b=0x3000, binning=1), mm.MM_E_ARG),
    # gap filling: a flag, single-beam pointing, projected access
    (dict(with_gapfill=2), mm.MM_E_ARG),
    (dict(with_gapfill=1, pix_b=0x3000), mm.MM_E_ARG),
    (dict(with_gapfill=1, map_access=1), mm.MM_E_ARG),
])
def test_plan_validation(case, status):
    """Both the workspace query and the plan reject the description before any device work."""
    d, keep = _desc(**case)
    h = ctypes.c_void_p()
    st = mm.lib().mm_plan(ctypes.byref(d), None, 0, None, ctypes.byref(h))
    assert st == status, mm.lib().mm_last_error()
    assert h.value is None
    assert len(mm.lib().mm_last_error()) > 0
    v = ctypes.c_size_t(12345)
    st = mm.lib().mm_plan_workspace_bytes(ctypes.byref(d), None, ctypes.byref(v))
    assert st == status, mm.lib().mm_last_error()
    assert v.value == 12345


def test_null_plan_is_rejected():
    lib = mm.lib()
    assert lib.mm_plan_destroy(None) == mm.MM_E_ARG
    v = ctypes.c_size_t()
    assert lib.mm_plan_workspace_bytes(None, None, ctypes.byref(v)) == mm.MM_E_ARG
    assert lib.mm_plan_binning_stats(None, None) == mm.MM_E_ARG
    assert lib.mm_messenger_iter(None, None, 1.0, None, None, None, None) == mm.MM_E_ARG
