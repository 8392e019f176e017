"""GPU parity of the atomic binning (MM_BIN_ATOMIC, the measured alternative to the sorted
segmented reduction): FP64 atomic adds in time order, so only the rounding order differs.
Same oracle and bars as the sorted binning."""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.cg import pcg_solve  # noqa: E402
from oracle.messenger import chi2, cooling_schedule, make_setup, messenger_solve, messenger_step  # noqa: E402
from paper_1705_01893_amd import mm  # noqa: E402
from tests.tiny_inputs import random_map, tiny_problem  # noqa: E402

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
MIX_TOL = 1e-5
MIX_CHI2 = 1e-6
SHAPES = {
    "pow2": dict(lengths=(256, 512, 128), nx=8),
    "mixed_radix": dict(lengths=(2 * 3 * 5 * 8, 2 * 45, 2 * 27 * 4, 2 * 125), nx=8),
    "long": dict(lengths=(2 * 4096, 2 * 6000), nx=16),
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def plan_for(t, dev, precision=mm.MM_FP64, access=mm.MM_MAP_AUTO):
    psi = torch.from_numpy(np.ascontiguousarray(t.psi)).to(dev) if t.ncomp == 3 else None
    return mm.mm_plan(ncomp=t.ncomp, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample, sigma=t.sigma,
                      fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(t.pix).to(dev), psi=psi,
                      precision=precision, map_access=access, binning=mm.MM_BIN_ATOMIC)


def setup(t):
    return make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, t.ncomp)


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("lam", [math.inf, 1.0, 37.5])
def test_one_iteration(dev, shape, ncomp, lam):
    say(f"[atomic iter] shape={shape} ncomp={ncomp} lam={lam}")
    t = tiny_problem(202, ncomp=ncomp, **SHAPES[shape])
    plan = plan_for(t, dev)
    S = setup(t)
    m0 = random_map(5, ncomp, t.npix)
    m0[:, ~S.solvable] = 0.0
    mo = torch.zeros((ncomp, t.npix), dtype=torch.float64, device=dev)
    c2 = torch.zeros(1, dtype=torch.float64, device=dev)
    mm.mm_messenger_iter(plan, torch.from_numpy(t.d).to(dev), lam, torch.from_numpy(m0).to(dev), mo, c2)
    torch.cuda.synchronize()
    assert rel(mo.cpu().numpy(), messenger_step(S, t.d, m0, lam)) < F64_TOL
    assert c2.item() == pytest.approx(chi2(S, t.d, m0), rel=F64_TOL)


@pytest.mark.parametrize("access", [mm.MM_MAP_GATHER, mm.MM_MAP_PROJECTED])
def test_full_schedule(dev, access):
    say(f"[atomic solve] access={access}")
    t = tiny_problem(313, ncomp=3, **SHAPES["long"])
    plan = plan_for(t, dev, access=access)
    S = setup(t)
    lmax, nlev, per = 40.0, 3, 3
    lams = cooling_schedule(nlev, per, lmax)
    m = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    hist = torch.zeros(len(lams) + 1, dtype=torch.float64, device=dev)
    mm.mm_solve(plan, torch.from_numpy(t.d).to(dev), [lmax ** ((nlev - 1 - l) / (nlev - 1)) for l in range(nlev)],
                [per] * nlev, m, chi2_hist=hist)
    torch.cuda.synchronize()
    m_ref, h_ref = messenger_solve(S, t.d, lams)
    assert rel(m.cpu().numpy(), m_ref) < F64_TOL
    np.testing.assert_allclose(hist.cpu().numpy(), h_ref, rtol=F64_TOL)


def test_cg(dev):
    say("[atomic cg]")
    t = tiny_problem(606, ncomp=3, **SHAPES["pow2"])
    plan = plan_for(t, dev)
    S = setup(t)
    m = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    n = mm.mm_cg_solve(plan, m, 25, d=torch.from_numpy(t.d).to(dev))
    torch.cuda.synchronize()
    assert n == 25
    m_ref, _ = pcg_solve(S, t.d, 25)
    assert rel(m.cpu().numpy(), m_ref) < 1e-9


def test_mixed_precision(dev):
    say("[atomic mixed]")
    t = tiny_problem(505, ncomp=3, psi_dtype=np.float32, tod_dtype=np.float32, **SHAPES["mixed_radix"])
    plan = plan_for(t, dev, precision=mm.MM_MIXED)
    S = setup(t)
    lams = cooling_schedule(3, 3, 50.0)
    m = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    hist = torch.zeros(len(lams) + 1, dtype=torch.float64, device=dev)
    mm.mm_solve(plan, torch.from_numpy(t.d).to(dev), [50.0, 50.0 ** 0.5, 1.0], [3, 3, 3], m, chi2_hist=hist)
    torch.cuda.synchronize()
    m_ref, h_ref = messenger_solve(S, t.d.astype(np.float64), lams)
    assert rel(m.cpu().numpy(), m_ref) < MIX_TOL
    np.testing.assert_allclose(hist.cpu().numpy(), h_ref, rtol=MIX_CHI2)
