"""The allocation-free workspace query against the allocating one, through the C ABI.

mm_plan_workspace_bytes_noalloc keeps its counters and chunk table in a fixed device array of
the library instead of a buffer it allocates; its result must equal mm_plan_workspace_bytes'
exactly (an integer), call after call, also when a smaller problem follows a larger one (the
array keeps the previous call's contents)."""

import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1705_01893_amd import mm  # noqa: E402
from tests.tiny_inputs import tiny_problem  # noqa: E402

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _query(fn, d):
    v = ctypes.c_size_t(0)
    st = fn(ctypes.byref(d), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(v))
    return st, v.value


def _desc(t, dev, **over):
    kw = dict(ncomp=t.ncomp, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample, sigma=t.sigma,
              fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(np.ascontiguousarray(t.pix)).to(dev),
              psi=torch.from_numpy(t.psi).to(dev) if t.ncomp == 3 else None)
    kw.update(over)
    d, keep = mm.plan_desc(**kw)
    return d, (keep, kw)


def test_noalloc_query_matches_allocating_query(dev):
    lib = mm.lib()
    lib.mm_plan_workspace_bytes_noalloc.argtypes = lib.mm_plan_workspace_bytes.argtypes
    lib.mm_plan_workspace_bytes_noalloc.restype = ctypes.c_int
    cases = [
        ("large", tiny_problem(4201, ncomp=3, lengths=(6000, 4096, 2 * 1250, 3 * 1024, 512), nx=32), {}),
        ("smaller", tiny_problem(4202, ncomp=3, lengths=(256, 192), nx=8), {}),
        ("temperature, adjoint", tiny_problem(4203, ncomp=1, lengths=(2 * 3 * 5 * 8, 128), nx=8),
         dict(with_adjoint=True)),
    ]
    for name, t, over in cases:
        d, keep = _desc(t, dev, **over)
        for rep in range(2):
            st0, b0 = _query(lib.mm_plan_workspace_bytes, d)
            st1, b1 = _query(lib.mm_plan_workspace_bytes_noalloc, d)
            say(f"[no-alloc query] {name} call {rep}: {b1} bytes (allocating query: {b0})")
            assert st0 == mm.MM_OK and st1 == mm.MM_OK, lib.mm_last_error()
            assert b1 == b0 > 0
        # a plan in a workspace of exactly that size works
        ws = torch.empty(b1, dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        st = lib.mm_plan(ctypes.byref(d), ctypes.c_void_p(ws.data_ptr()), b1,
                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
        assert st == mm.MM_OK, lib.mm_last_error()
        assert lib.mm_plan_destroy(h) == mm.MM_OK
    # the same rejection of a bad pointing as the allocating query
    t = tiny_problem(4204, ncomp=3, lengths=(64, 64), nx=4)
    pix = t.pix.copy()
    pix[3] = t.npix
    d, keep = _desc(t, dev, pix=torch.from_numpy(pix).to(dev))
    assert _query(lib.mm_plan_workspace_bytes_noalloc, d)[0] == mm.MM_E_ARG
    assert _query(lib.mm_plan_workspace_bytes, d)[0] == mm.MM_E_ARG


def test_noalloc_query_rejects_more_chunks_than_its_array_holds(dev):
    """131039 chunks fit the fixed 1 MiB array; one more is refused with MM_E_ARG."""
    lib = mm.lib()
    lib.mm_plan_workspace_bytes_noalloc.argtypes = lib.mm_plan_workspace_bytes.argtypes
    lib.mm_plan_workspace_bytes_noalloc.restype = ctypes.c_int
    for nch, ok in ((131039, True), (131040, False)):
        off = np.arange(nch + 1, dtype=np.int64) * 2
        pix = torch.zeros(2 * nch, dtype=torch.int32, device=dev)
        ones = np.ones(nch)
        d, keep = mm.plan_desc(ncomp=1, npix=4, nx=2, chunk_off=off, fsample=ones, sigma=ones, fknee=ones,
                               alpha=-ones, pix=pix)
        st, b = _query(lib.mm_plan_workspace_bytes_noalloc, d)
        say(f"[no-alloc query] {nch} chunks: status {st}")
        if ok:
            assert st == mm.MM_OK, lib.mm_last_error()
            assert b == _query(lib.mm_plan_workspace_bytes, d)[1]
        else:
            assert st == mm.MM_E_ARG
            assert b"131039" in lib.mm_last_error()
