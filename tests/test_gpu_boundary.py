"""The boundary's workspace contract on the GPU: the size query, plans in caller memory,
a short workspace, the buffers that only with_adjoint reserves, the map right-hand side of
mm_solve, and the device-built binning lists against a host count of the same rule."""

import bisect
import ctypes
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.messenger import make_setup, messenger_step  # noqa: E402
from paper_1705_01893_amd import mm  # noqa: E402
from tests.tiny_inputs import random_map, tiny_problem  # noqa: E402

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _kw(t, dev, **over):
    kw = dict(ncomp=t.ncomp, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample, sigma=t.sigma,
              fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(np.ascontiguousarray(t.pix)).to(dev),
              psi=torch.from_numpy(t.psi).to(dev) if t.ncomp == 3 else None)
    kw.update(over)
    return kw


def test_query_is_reproducible_and_plan_fits(dev):
    say("[ws query]")
    t = tiny_problem(3101, ncomp=3, lengths=(512, 256, 1024), nx=16)
    kw = _kw(t, dev)
    b1 = mm.mm_plan_workspace_bytes(**kw)
    b2 = mm.mm_plan_workspace_bytes(**kw)
    assert b1 == b2 > 0
    plan = mm.mm_plan(**kw)
    st = mm.mm_plan_binning_stats(plan)
    assert plan.workspace.numel() == b1
    assert 0 < st["workspace_used"] <= b1
    # the adjoint buffer adds one TOD-sized buffer (at least nsamp values of the TOD type)
    b3 = mm.mm_plan_workspace_bytes(**_kw(t, dev, with_adjoint=True))
    assert b3 >= b1 + t.nsamp * 8
    plan.close()


def test_short_workspace_is_rejected(dev):
    say("[ws short]")
    t = tiny_problem(3102, ncomp=3, lengths=(256, 256), nx=8)
    kw = _kw(t, dev)
    need = mm.mm_plan_workspace_bytes(**kw)
    d, keep = mm.plan_desc(**kw)
    for have in (need - 256, 1024):
        ws = torch.empty(have, dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        st = mm.lib().mm_plan(ctypes.byref(d), ctypes.c_void_p(ws.data_ptr()), have,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
        assert st == mm.MM_E_NOMEM, mm.lib().mm_last_error()
        assert h.value is None
    # misaligned workspace
    ws = torch.empty(need + 512, dtype=torch.uint8, device=dev)
    h = ctypes.c_void_p()
    st = mm.lib().mm_plan(ctypes.byref(d), ctypes.c_void_p(ws.data_ptr() + 8), need,
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    assert st == mm.MM_E_ARG


def test_bad_pointing_is_rejected(dev):
    say("[ws bad pointing]")
    t = tiny_problem(3103, ncomp=3, lengths=(64, 64), nx=4)
    pix = t.pix.copy()
    pix[17] = t.npix  # one past the map
    with pytest.raises(mm.MMError) as e:
        mm.mm_plan_workspace_bytes(**_kw(t, dev, pix=torch.from_numpy(pix).to(dev)))
    assert e.value.status == mm.MM_E_ARG
    psi = t.psi.copy()
    psi[5] = np.inf
    with pytest.raises(mm.MMError) as e:
        mm.mm_plan(**_kw(t, dev, psi=torch.from_numpy(psi).to(dev)))
    assert e.value.status == mm.MM_E_ARG


def test_adjoint_buffer_needed(dev):
    say("[ws adjoint]")
    t = tiny_problem(3104, ncomp=3, lengths=(256, 128), nx=8)
    plan = mm.mm_plan(**_kw(t, dev))
    m = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    g = torch.zeros((plan.nchunk, 3), dtype=torch.float64, device=dev)
    with pytest.raises(mm.MMError) as e:
        mm.mm_noise_grad(plan, torch.from_numpy(t.d).to(dev), m, m, g)
    assert e.value.status == mm.MM_E_ARG
    with pytest.raises(mm.MMError) as e:
        mm.mm_solve(plan, None, [1.0], [2], m, rhs_map=m.clone())
    assert e.value.status == mm.MM_E_ARG
    plan.close()


@pytest.mark.parametrize("ncomp", [1, 3])
def test_solve_with_map_rhs_equals_lifted_data(dev, ncomp):
    """mm_solve(rhs_map = g) runs the schedule on N T^-1 P W^-1 g: the same maps and chi^2 history as
    mm_solve on the TOD that mm_lift_rhs writes, whose right-hand side P^T N^-1 d is g."""
    say(f"[rhs_map] ncomp={ncomp}")
    t = tiny_problem(3105, ncomp=ncomp, lengths=(2 * 3 * 5 * 8, 2 * 64), nx=8, alpha=(-1.2, -1.0),
                     fknee=(0.3, 0.5))
    plan = mm.mm_plan(**_kw(t, dev, with_adjoint=True))
    g = torch.from_numpy(random_map(77, ncomp, t.npix)).to(dev)
    lams, its = [40.0, 6.0, 1.0], [2, 2, 3]
    nh = 1 + sum(its) + 1
    z1 = torch.zeros_like(g)
    h1 = torch.zeros(nh, dtype=torch.float64, device=dev)
    mm.mm_solve(plan, None, lams, its, z1, chi2_hist=h1, rhs_map=g)
    dg = torch.empty(t.nsamp, dtype=torch.float64, device=dev)
    mm.mm_lift_rhs(plan, g, dg)
    z2 = torch.zeros_like(g)
    h2 = torch.zeros(nh, dtype=torch.float64, device=dev)
    mm.mm_solve(plan, dg, lams, its, z2, chi2_hist=h2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    assert torch.equal(h1, h2)
    # the lifted data carry g as their right-hand side: P^T N^-1 (N T^-1 P W^-1 g) = g on solvable pixels
    b = torch.zeros_like(g)
    mm.mm_apply(plan, 0, b, d=dg)
    torch.cuda.synchronize()
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, ncomp)
    ref = g.cpu().numpy().copy()
    ref[:, ~S.solvable] = 0.0
    got = b.cpu().numpy()
    got[:, ~S.solvable] = 0.0
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10
    plan.close()


# The binning lists follow one rule (per pixel tile, the tile's on-map samples in time order cut
# into sub-batches of at most 4096 samples and 512 time-contiguous segments inside one chunk);
# the device builds them by slab walks and prefix sums.  Their counts against a host walk of
# the same rule: integers, so exactly equal.
def _host_counts(pix, off, nxm, tw, th):
    ns = len(pix)
    ntx = (nxm + tw - 1) // tw
    ok = pix >= 0
    p = pix[ok]
    tiles = (p // nxm // th) * ntx + (p % nxm) // tw
    js = np.nonzero(ok)[0]
    order = np.argsort(tiles, kind="stable")
    nsb = nseg = nsort = 0
    bounds = np.searchsorted(np.sort(tiles), np.arange(tiles.max() + 2))
    for t in range(len(bounds) - 1):
        o = js[order[bounds[t]:bounds[t + 1]]]
        i = 0
        while i < len(o):
            b0, cur_end, chunk_end, k = i, -1, -1, 0
            while i < len(o) and i - b0 < 4096:
                j = int(o[i])
                if not (j == cur_end and j < chunk_end):
                    if k == 512:
                        break
                    chunk_end = off[bisect.bisect_right(off, j)]
                    k += 1
                cur_end = j + 1
                i += 1
            nsb += 1
            nseg += k
            nsort += (i - b0 + 15) // 16 * 16
    return nsb, nseg, nsort


@pytest.mark.parametrize("walk", [True, False])
def test_binning_lists_match_host_count(dev, walk):
    say(f"[ws lists] walk={walk}")
    t = tiny_problem(3106, ncomp=3, lengths=(6000, 4096, 2 * 1250, 3 * 1024), nx=32, walk=walk)
    plan = mm.mm_plan(**_kw(t, dev))
    st = mm.mm_plan_binning_stats(plan)
    tw, th = st["tile_w"], st["tile_h"]
    assert st["tiles"] == ((32 + tw - 1) // tw) * ((32 + th - 1) // th)
    ref = _host_counts(t.pix, list(t.chunk_off), 32, tw, th)
    assert (st["sub_batches"], st["segments"], st["sorted_entries"]) == ref
    plan.close()
