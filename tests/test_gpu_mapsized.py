"""The map-sized form of the cooled solve (Section 2.1, eqns. md and F; Section 4.1) on the GPU
against the oracle's map-sized iteration m <- m_d(lambda) + F(lambda) m, schedule for schedule,
and against the residual form (equal in exact arithmetic by the Woodbury identity)."""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.messenger import make_setup, messenger_step, messenger_step_mapsized  # noqa: E402
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


SHAPES = {"pow2": dict(lengths=(256, 512, 128), nx=8),
          "mixed_radix": dict(lengths=(2 * 3 * 5 * 8, 2 * 45, 2 * 27 * 4, 2 * 125), nx=8)}


@pytest.mark.parametrize("access", [mm.MM_MAP_GATHER, mm.MM_MAP_PROJECTED])
@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_mapsized_schedule_fp64(dev, shape, ncomp, access):
    say(f"[mapsized] shape={shape} ncomp={ncomp} access={access}")
    t = tiny_problem(5301, ncomp=ncomp, **SHAPES[shape])
    psi = torch.from_numpy(t.psi).to(dev) if ncomp == 3 else None
    plan = mm.mm_plan(ncomp=ncomp, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample, sigma=t.sigma,
                      fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(t.pix).to(dev), psi=psi, map_access=access)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, ncomp)
    lams, its = [60.0, 7.0, 1.0], [2, 3, 2]
    seq = [math.inf] + [lv for lv, k in zip(lams, its) for _ in range(k)]
    d = torch.from_numpy(t.d).to(dev)
    m = torch.zeros((ncomp, t.npix), dtype=torch.float64, device=dev)
    mm.mm_solve_mapsized(plan, d, lams, its, m)
    m2 = torch.zeros_like(m)
    mm.mm_solve_mapsized(plan, d, lams, its, m2)  # graph replay
    torch.cuda.synchronize()
    assert torch.equal(m, m2)
    ref = np.zeros((ncomp, t.npix))
    res = np.zeros((ncomp, t.npix))
    for lam in seq:
        ref = messenger_step_mapsized(S, t.d, ref, lam)
        res = messenger_step(S, t.d, res, lam)
    e, er = rel(m.cpu().numpy(), ref), rel(m.cpu().numpy(), res)
    say(f"  vs oracle map-sized {e:.2e}, vs oracle residual form {er:.2e}")
    assert e < 1e-10 and er < 1e-10
    # from a given start map, without the lambda = inf step
    m0 = random_map(9, ncomp, t.npix)
    m0[:, ~S.solvable] = 0.0
    mg = torch.from_numpy(m0).to(dev)
    mo = torch.zeros_like(mg)
    mm.mm_solve_mapsized(plan, d, [5.0, 1.0], [1, 2], mo, first_inf=False, m0=mg)
    torch.cuda.synchronize()
    ref = m0
    for lam in (5.0, 1.0, 1.0):
        ref = messenger_step_mapsized(S, t.d, ref, lam)
    assert rel(mo.cpu().numpy(), ref) < 1e-10
    plan.close()


def test_mapsized_mixed(dev):
    say("[mapsized mixed]")
    t = tiny_problem(5302, ncomp=3, psi_dtype=np.float32, tod_dtype=np.float32, **SHAPES["mixed_radix"])
    plan = mm.mm_plan(ncomp=3, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample, sigma=t.sigma,
                      fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(t.pix).to(dev),
                      psi=torch.from_numpy(t.psi).to(dev), precision=mm.MM_MIXED)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    lams, its = [40.0, 1.0], [3, 3]
    m = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    mm.mm_solve_mapsized(plan, torch.from_numpy(t.d).to(dev), lams, its, m)
    torch.cuda.synchronize()
    ref = np.zeros((3, t.npix))
    for lam in [math.inf] + [40.0] * 3 + [1.0] * 3:
        ref = messenger_step_mapsized(S, t.d.astype(np.float64), ref, lam)
    e = rel(m.cpu().numpy(), ref)
    say(f"  mixed vs oracle map-sized {e:.2e}")
    assert e < 1e-5
    plan.close()
