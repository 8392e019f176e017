"""ctypes binding of libmm (include/mm.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: it checks tensor devices, dtypes and shapes, passes raw
pointers and the current HIP stream, and turns status codes into exceptions.
The library must be built (``python -m paper_1705_01893_amd.build``); there is
no fallback path.
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmm.so")

MM_FP64, MM_MIXED = 0, 1
MM_PSI_NONE, MM_PSI_F64, MM_PSI_F32, MM_PSI_U16 = 0, 1, 2, 3
MM_MAP_AUTO, MM_MAP_GATHER, MM_MAP_PROJECTED = 0, 1, 2
MM_TUNE_MEASURE, MM_TUNE_STATIC, MM_TUNE_PICK0 = 0, 1, 16
MM_BIN_SORTED, MM_BIN_ATOMIC = 0, 1
MM_OK, MM_E_ARG, MM_E_LEN, MM_E_NOMEM, MM_E_HIP, MM_E_SINGULAR, MM_E_NONFINITE = range(7)
_STATUS_NAMES = {0: "MM_OK", 1: "MM_E_ARG", 2: "MM_E_LEN", 3: "MM_E_NOMEM", 4: "MM_E_HIP",
                 5: "MM_E_SINGULAR", 6: "MM_E_NONFINITE"}


class MMError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {_STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ncomp", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("npix", ctypes.c_int64), ("nx", ctypes.c_int64), ("nchunk", ctypes.c_int64),
        ("chunk_off", ctypes.POINTER(ctypes.c_int64)),
        ("fsample", ctypes.POINTER(ctypes.c_double)), ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("fknee", ctypes.POINTER(ctypes.c_double)), ("alpha", ctypes.POINTER(ctypes.c_double)),
        ("tau", ctypes.POINTER(ctypes.c_double)),
        ("pix", ctypes.c_void_p), ("psi", ctypes.c_void_p),
        ("psi_kind", ctypes.c_int32), ("map_access", ctypes.c_int32),
        ("psi_table", ctypes.POINTER(ctypes.c_float)), ("psi_table_len", ctypes.c_int64),
        ("tune", ctypes.c_int32), ("binning", ctypes.c_int32), ("with_adjoint", ctypes.c_int32),
        ("tile_pixels", ctypes.c_int32),
        ("pix_b", ctypes.c_void_p), ("psi_b", ctypes.c_void_p),
        ("weight_a", ctypes.c_double), ("weight_b", ctypes.c_double),
        ("with_gapfill", ctypes.c_int32), ("pad_", ctypes.c_int32),
    ]


class _Sched(ctypes.Structure):
    _fields_ = [("nlevel", ctypes.c_int32), ("first_inf", ctypes.c_int32),
                ("lambda_", ctypes.POINTER(ctypes.c_double)), ("iters", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmm.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1705_01893_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.mm_plan_workspace_bytes.argtypes = [ctypes.POINTER(_Desc), vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mm_plan_workspace_bytes_noalloc.argtypes = [ctypes.POINTER(_Desc), vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mm_plan.argtypes = [ctypes.POINTER(_Desc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.mm_plan_destroy.argtypes = [vp]
    L.mm_plan_binning_stats.argtypes = [vp, ctypes.POINTER(i64)]
    L.mm_plan_hits.argtypes = [vp, vp, vp]
    L.mm_plan_solvable.argtypes = [vp, vp, vp]
    L.mm_plan_nsolvable.argtypes = [vp, ctypes.POINTER(i64)]
    L.mm_plan_map_access.argtypes = [vp, ctypes.POINTER(i32)]
    L.mm_plan_chunk_layout.argtypes = [vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.mm_messenger_iter.argtypes = [vp, vp, dbl, vp, vp, vp, vp]
    L.mm_solve.argtypes = [vp, vp, vp, ctypes.POINTER(_Sched), vp, vp, vp, vp]
    L.mm_solve_mapsized.argtypes = [vp, vp, ctypes.POINTER(_Sched), vp, vp, vp]
    L.mm_solve_gapfill.argtypes = [vp, vp, vp, ctypes.POINTER(_Sched), vp, vp, vp, vp]
    L.mm_cooling_levels.argtypes = [vp, i32, dbl, ctypes.POINTER(dbl)]
    L.mm_cg_solve.argtypes = [vp, vp, vp, i32, dbl, vp, vp, vp, vp, ctypes.POINTER(i32), vp]
    L.mm_chi2.argtypes = [vp, vp, vp, dbl, ctypes.POINTER(dbl), vp, vp]
    L.mm_apply.argtypes = [vp, i32, dbl, vp, vp, vp, vp]
    L.mm_chi2_modes.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(i64), i32, vp, vp, i32, vp]
    L.mm_lift_rhs.argtypes = [vp, vp, vp, vp]
    L.mm_plan_set_noise.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                     ctypes.POINTER(dbl), vp]
    L.mm_tod_apply.argtypes = [vp, i32, dbl, vp, vp, vp]
    L.mm_noise_grad.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mm_set_timing.argtypes = [vp, i32]
    L.mm_get_timing.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    for name in ("mm_plan_set_noise", "mm_tod_apply", "mm_noise_grad", "mm_set_timing", "mm_get_timing", "mm_plan", "mm_plan_destroy", "mm_plan_workspace_bytes", "mm_plan_workspace_bytes_noalloc",
                 "mm_plan_binning_stats", "mm_plan_hits", "mm_plan_solvable",
                 "mm_plan_nsolvable", "mm_plan_map_access", "mm_plan_chunk_layout", "mm_messenger_iter", "mm_solve", "mm_solve_mapsized",
                 "mm_solve_gapfill", "mm_cooling_levels", "mm_cg_solve",
                 "mm_chi2", "mm_chi2_modes", "mm_apply", "mm_lift_rhs"):
        getattr(L, name).restype = ctypes.c_int
    L.mm_status_str.argtypes = [ctypes.c_int]
    L.mm_status_str.restype = ctypes.c_char_p
    L.mm_last_error.argtypes = []
    L.mm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st: int, where: str) -> None:
    if st != MM_OK:
        raise MMError(st, where, lib().mm_last_error().decode(errors="replace"))


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor], name: str, dtype=None, numel: Optional[int] = None) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _host_f64(x, n, name):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    if a.size != n:
        raise ValueError(f"{name} must have {n} entries")
    return a


class Plan:
    """A built plan: owns the C handle and the workspace tensor, keeps the pointing tensors alive."""

    def __init__(self, handle: int, desc_arrays: dict, ncomp: int, npix: int, nchunk: int, nsamp: int,
                 precision: int, tensors: list, workspace: torch.Tensor):
        self.handle = ctypes.c_void_p(handle)
        self._keep = (desc_arrays, tensors)
        self.workspace = workspace
        self.ncomp, self.npix, self.nchunk, self.nsamp, self.precision = ncomp, npix, nchunk, nsamp, precision
        # messenger variance per chunk as last given to the library (None: its default sigma^2)
        self.tau = desc_arrays.get("tau")

    @property
    def tod_dtype(self):
        return torch.float64 if self.precision == MM_FP64 else torch.float32

    @property
    def map_shape(self):
        return (self.ncomp, self.npix)

    def close(self):
        if self.handle:
            lib().mm_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_desc(*, ncomp: int, npix: int, chunk_off, fsample, sigma, fknee, alpha, pix: torch.Tensor,
              psi: Optional[torch.Tensor] = None, psi_table=None, tau=None, nx: int = 0,
              precision: int = MM_FP64, map_access: int = MM_MAP_AUTO, tune: int = MM_TUNE_MEASURE,
              binning: int = MM_BIN_SORTED, with_adjoint: bool = False, tile_pixels: int = 0,
              pix_b: Optional[torch.Tensor] = None, psi_b: Optional[torch.Tensor] = None,
              weights=(1.0, -1.0), with_gapfill: bool = False):
    """The mm_plan_desc of a problem and the host arrays it points to (keep both alive together).
    pix (int32) and psi (float64 / float32 / uint16) are device tensors.  pix_b / psi_b (same
    types) add the second component of a composite pointing P = w_a P_A + w_b P_B with
    weights = (w_a, w_b); they are ignored without pix_b."""
    off = np.ascontiguousarray(np.asarray(chunk_off, dtype=np.int64).reshape(-1))
    nchunk = off.size - 1
    nsamp = int(off[-1])
    arrs = {k: _host_f64(v, nchunk, k) for k, v in
            dict(fsample=fsample, sigma=sigma, fknee=fknee, alpha=alpha).items()}
    if tau is not None:
        arrs["tau"] = _host_f64(tau, nchunk, "tau")
    arrs["off"] = off
    d = _Desc()
    d.ncomp, d.precision, d.npix, d.nx, d.nchunk = ncomp, precision, npix, nx, nchunk
    d.map_access = map_access
    d.tune = tune
    d.binning = binning
    d.with_adjoint = int(bool(with_adjoint))
    d.tile_pixels = int(tile_pixels)
    d.with_gapfill = int(bool(with_gapfill))
    d.chunk_off = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    for k in ("fsample", "sigma", "fknee", "alpha"):
        setattr(d, k, arrs[k].ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    d.tau = arrs["tau"].ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if tau is not None else None
    d.pix = _ptr(pix, "pix", torch.int32, nsamp)
    kind = MM_PSI_NONE
    if psi is not None:
        kind = {torch.float64: MM_PSI_F64, torch.float32: MM_PSI_F32, torch.uint16: MM_PSI_U16}.get(psi.dtype)
        if kind is None:
            raise TypeError("psi must be float64, float32 or uint16")
        d.psi = _ptr(psi, "psi", None, nsamp)
    d.psi_kind = kind
    if psi_table is not None:
        tab = np.ascontiguousarray(np.asarray(psi_table, dtype=np.float32).reshape(-1))
        arrs["psi_table"] = tab
        d.psi_table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        d.psi_table_len = tab.size
    if pix_b is not None:
        d.pix_b = _ptr(pix_b, "pix_b", torch.int32, nsamp)
        if psi_b is not None:
            if psi is None or psi_b.dtype != psi.dtype:
                raise TypeError("psi_b must have the type of psi")
            d.psi_b = _ptr(psi_b, "psi_b", None, nsamp)
        d.weight_a, d.weight_b = float(weights[0]), float(weights[1])
    return d, arrs


def mm_plan_workspace_bytes(stream=None, **kw) -> int:
    """Workspace bytes of the plan the keyword arguments (those of mm_plan) describe."""
    d, arrs = plan_desc(**kw)
    v = ctypes.c_size_t()
    _check(lib().mm_plan_workspace_bytes(ctypes.byref(d), _stream(stream), ctypes.byref(v)),
           "mm_plan_workspace_bytes")
    return v.value


def mm_plan(*, stream=None, **kw) -> Plan:
    """Build a plan (mm_plan) in a workspace tensor sized by mm_plan_workspace_bytes (torch owns the
    device memory).  Keyword arguments: those of plan_desc."""
    d, arrs = plan_desc(**kw)
    st = _stream(stream)
    v = ctypes.c_size_t()
    _check(lib().mm_plan_workspace_bytes(ctypes.byref(d), st, ctypes.byref(v)), "mm_plan_workspace_bytes")
    pix, psi = kw["pix"], kw.get("psi")
    ws = torch.empty(max(int(v.value), 1), dtype=torch.uint8, device=pix.device)
    h = ctypes.c_void_p()
    _check(lib().mm_plan(ctypes.byref(d), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), st,
                         ctypes.byref(h)), "mm_plan")
    nsamp = int(arrs["off"][-1])
    return Plan(h.value, arrs, kw["ncomp"], kw["npix"], arrs["off"].size - 1, nsamp,
                kw.get("precision", MM_FP64), [pix, psi, kw.get("pix_b"), kw.get("psi_b")], ws)


def mm_plan_binning_stats(plan: Plan) -> dict:
    """Pixel tiles, tile width and height, sub-batches, segments, sorted entries and workspace bytes in use."""
    out = (ctypes.c_int64 * 7)()
    _check(lib().mm_plan_binning_stats(plan.handle, out), "mm_plan_binning_stats")
    keys = ("tiles", "tile_w", "tile_h", "sub_batches", "segments", "sorted_entries", "workspace_used")
    return {k: int(v) for k, v in zip(keys, out)}


def mm_plan_hits(plan: Plan, hits: torch.Tensor, stream=None) -> None:
    _check(lib().mm_plan_hits(plan.handle, _ptr(hits, "hits", torch.int32, plan.npix), _stream(stream)),
           "mm_plan_hits")


def mm_plan_solvable(plan: Plan, mask: torch.Tensor, stream=None) -> None:
    _check(lib().mm_plan_solvable(plan.handle, _ptr(mask, "mask", torch.uint8, plan.npix), _stream(stream)),
           "mm_plan_solvable")


def mm_plan_nsolvable(plan: Plan) -> int:
    v = ctypes.c_int64()
    _check(lib().mm_plan_nsolvable(plan.handle, ctypes.byref(v)), "mm_plan_nsolvable")
    return v.value


def mm_plan_map_access(plan: Plan) -> int:
    v = ctypes.c_int32()
    _check(lib().mm_plan_map_access(plan.handle, ctypes.byref(v)), "mm_plan_map_access")
    return v.value


def mm_plan_chunk_layout(plan: Plan, chunk: int) -> dict:
    """Transform layout of one chunk: M1, M2, cb, the chosen candidate and the candidate count."""
    m1, m2 = ctypes.c_int64(), ctypes.c_int64()
    cb, pick, ncand = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mm_plan_chunk_layout(plan.handle, chunk, ctypes.byref(m1), ctypes.byref(m2), ctypes.byref(cb),
                                      ctypes.byref(pick), ctypes.byref(ncand)), "mm_plan_chunk_layout")
    return {"M1": m1.value, "M2": m2.value, "cb": cb.value, "pick": pick.value, "ncand": ncand.value}


def _map_ptr(plan, t, name):
    return _ptr(t, name, torch.float64, plan.ncomp * plan.npix)


def mm_messenger_iter(plan: Plan, d: torch.Tensor, lam: float, m_in: torch.Tensor, m_out: torch.Tensor,
                      chi2: Optional[torch.Tensor] = None, stream=None) -> None:
    _check(lib().mm_messenger_iter(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp), float(lam),
                                   _map_ptr(plan, m_in, "m_in"), _map_ptr(plan, m_out, "m_out"),
                                   _ptr(chi2, "chi2", torch.float64, 1), _stream(stream)), "mm_messenger_iter")


def mm_cooling_levels(plan: Plan, nlevel: int, lambda_max: float = 0.0) -> list:
    out = (ctypes.c_double * nlevel)()
    _check(lib().mm_cooling_levels(plan.handle, int(nlevel), float(lambda_max), out), "mm_cooling_levels")
    return list(out)


def mm_solve(plan: Plan, d: Optional[torch.Tensor], lambdas: Sequence[float], iters: Sequence[int],
             m_out: torch.Tensor, first_inf: bool = True, m0: Optional[torch.Tensor] = None,
             chi2_hist: Optional[torch.Tensor] = None, rhs_map: Optional[torch.Tensor] = None, stream=None) -> None:
    """Cooled messenger solve on the data d, or (d None) on a map right-hand side rhs_map."""
    lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
    its = np.ascontiguousarray(np.asarray(iters, dtype=np.int32))
    if lam.size != its.size:
        raise ValueError("lambdas and iters must have equal length")
    sc = _Sched()
    sc.nlevel, sc.first_inf = lam.size, int(bool(first_inf))
    sc.lambda_ = lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    sc.iters = its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    nh = int(bool(first_inf)) + int(its.sum()) + 1
    _check(lib().mm_solve(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp), _map_ptr(plan, rhs_map, "rhs_map"),
                          ctypes.byref(sc), _map_ptr(plan, m0, "m0"), _map_ptr(plan, m_out, "m_out"),
                          _ptr(chi2_hist, "chi2_hist", torch.float64, nh), _stream(stream)), "mm_solve")


def mm_solve_mapsized(plan: Plan, d: torch.Tensor, lambdas: Sequence[float], iters: Sequence[int],
                      m_out: torch.Tensor, first_inf: bool = True, m0: Optional[torch.Tensor] = None,
                      stream=None) -> None:
    """Cooled messenger solve in the map-sized form m <- m_d(lambda) + F(lambda) m."""
    lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
    its = np.ascontiguousarray(np.asarray(iters, dtype=np.int32))
    if lam.size != its.size:
        raise ValueError("lambdas and iters must have equal length")
    sc = _Sched()
    sc.nlevel, sc.first_inf = lam.size, int(bool(first_inf))
    sc.lambda_ = lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    sc.iters = its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(lib().mm_solve_mapsized(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp), ctypes.byref(sc),
                                   _map_ptr(plan, m0, "m0"), _map_ptr(plan, m_out, "m_out"), _stream(stream)),
           "mm_solve_mapsized")


def mm_solve_gapfill(plan: Plan, d: torch.Tensor, gaps: torch.Tensor, lambdas: Sequence[float], iters: Sequence[int],
                     m_out: torch.Tensor, first_inf: bool = True, m0: Optional[torch.Tensor] = None,
                     d0_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """Cooled solve with gap filling (composite noise N = N_0 + N_1); gaps: device uint8 per sample
    (nonzero: unusable data); d0_out receives the gap-filled TOD."""
    lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
    its = np.ascontiguousarray(np.asarray(iters, dtype=np.int32))
    if lam.size != its.size:
        raise ValueError("lambdas and iters must have equal length")
    sc = _Sched()
    sc.nlevel, sc.first_inf = lam.size, int(bool(first_inf))
    sc.lambda_ = lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    sc.iters = its.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(lib().mm_solve_gapfill(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp),
                                  _ptr(gaps, "gaps", torch.uint8, plan.nsamp), ctypes.byref(sc),
                                  _map_ptr(plan, m0, "m0"), _map_ptr(plan, m_out, "m_out"),
                                  _ptr(d0_out, "d0_out", plan.tod_dtype, plan.nsamp), _stream(stream)),
           "mm_solve_gapfill")


def mm_cg_solve(plan: Plan, m_out: torch.Tensor, maxiter: int, d: Optional[torch.Tensor] = None,
                rhs_map: Optional[torch.Tensor] = None, rtol: float = 0.0, m0: Optional[torch.Tensor] = None,
                chi2_hist: Optional[torch.Tensor] = None, rz_hist: Optional[torch.Tensor] = None,
                stream=None) -> int:
    it = ctypes.c_int32()
    _check(lib().mm_cg_solve(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp),
                             _map_ptr(plan, rhs_map, "rhs_map"), int(maxiter), float(rtol),
                             _map_ptr(plan, m0, "m0"), _map_ptr(plan, m_out, "m_out"),
                             _ptr(chi2_hist, "chi2_hist", torch.float64, maxiter + 1),
                             _ptr(rz_hist, "rz_hist", torch.float64, maxiter + 1),
                             ctypes.byref(it), _stream(stream)), "mm_cg_solve")
    return it.value


def mm_chi2(plan: Plan, d: torch.Tensor, m: torch.Tensor, lam: float = 1.0,
            per_chunk: Optional[torch.Tensor] = None, stream=None) -> float:
    v = ctypes.c_double()
    _check(lib().mm_chi2(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp), _map_ptr(plan, m, "m"),
                         float(lam), ctypes.byref(v), _ptr(per_chunk, "per_chunk", torch.float64, plan.nchunk),
                         _stream(stream)), "mm_chi2")
    return v.value


def chi2_modes_nbins(plan: Plan, chunks, per_octave: int) -> int:
    """Number of log-spaced bins mm_chi2_modes fills for these chunks (its documented rule)."""
    maxm = max(int(plan._keep[0]["off"][c + 1] - plan._keep[0]["off"][c]) // 2 for c in chunks)
    return 1 + per_octave * (maxm.bit_length())


def mm_chi2_modes(plan: Plan, d: torch.Tensor, m: torch.Tensor, chunks, per_octave: int = 4, lam: float = 1.0,
                  stream=None):
    """Per-mode chi^2 terms of the listed chunks (concatenated, n_i/2 + 1 each) and their log-binned
    sums [nsel, nbins, 2] (sum of terms, number of real modes)."""
    ch = np.ascontiguousarray(np.asarray(chunks, dtype=np.int64).reshape(-1))
    off = plan._keep[0]["off"]
    nmodes = int(sum((off[c + 1] - off[c]) // 2 + 1 for c in ch))
    nb = chi2_modes_nbins(plan, ch, per_octave)
    modes = torch.empty(nmodes, dtype=torch.float64, device=d.device)
    bins = torch.empty((ch.size, nb, 2), dtype=torch.float64, device=d.device)
    _check(lib().mm_chi2_modes(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp), _map_ptr(plan, m, "m"),
                               float(lam), int(ch.size), ch.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               int(per_octave), modes.data_ptr(), bins.data_ptr(), int(nb), _stream(stream)),
           "mm_chi2_modes")
    return modes, bins


def mm_apply(plan: Plan, which: int, out: torch.Tensor, x: Optional[torch.Tensor] = None,
             d: Optional[torch.Tensor] = None, lam: float = 1.0, stream=None) -> None:
    _check(lib().mm_apply(plan.handle, int(which), float(lam), _map_ptr(plan, x, "x"),
                          _ptr(d, "d", plan.tod_dtype, plan.nsamp), _map_ptr(plan, out, "out"),
                          _stream(stream)), "mm_apply")


def mm_lift_rhs(plan: Plan, g: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    _check(lib().mm_lift_rhs(plan.handle, _map_ptr(plan, g, "g"), _ptr(out, "out", plan.tod_dtype, plan.nsamp),
                             _stream(stream)), "mm_lift_rhs")


def mm_plan_set_noise(plan: Plan, sigma, fknee, alpha, tau=None, stream=None) -> None:
    n = plan.nchunk
    arrs = [_host_f64(v, n, k) for k, v in (("sigma", sigma), ("fknee", fknee), ("alpha", alpha))]
    t = _host_f64(tau, n, "tau") if tau is not None else None
    P = ctypes.POINTER(ctypes.c_double)
    _check(lib().mm_plan_set_noise(plan.handle, *[a.ctypes.data_as(P) for a in arrs],
                                   t.ctypes.data_as(P) if t is not None else None, _stream(stream)),
           "mm_plan_set_noise")
    plan.tau = t


def mm_tod_apply(plan: Plan, which: int, x: torch.Tensor, out: torch.Tensor, lam: float = 1.0, stream=None) -> None:
    _check(lib().mm_tod_apply(plan.handle, int(which), float(lam), _map_ptr(plan, x, "x"),
                              _ptr(out, "out", plan.tod_dtype, plan.nsamp), _stream(stream)), "mm_tod_apply")


def mm_noise_grad(plan: Plan, d: torch.Tensor, m: torch.Tensor, z: torch.Tensor, grad: torch.Tensor,
                  stream=None) -> None:
    _check(lib().mm_noise_grad(plan.handle, _ptr(d, "d", plan.tod_dtype, plan.nsamp), _map_ptr(plan, m, "m"),
                               _map_ptr(plan, z, "z"), _ptr(grad, "grad", torch.float64, 3 * plan.nchunk),
                               _stream(stream)), "mm_noise_grad")


def mm_set_timing(plan: Plan, enable: bool) -> None:
    _check(lib().mm_set_timing(plan.handle, int(bool(enable))), "mm_set_timing")


def mm_get_timing(plan: Plan):
    """(milliseconds[5], launches[5]) per pass A, B, C, D, projection since the last call."""
    ms = (ctypes.c_double * 5)()
    n = (ctypes.c_int64 * 5)()
    _check(lib().mm_get_timing(plan.handle, ms, n), "mm_get_timing")
    return list(ms), list(n)


def mm_status_str(status: int) -> str:
    return lib().mm_status_str(int(status)).decode()
