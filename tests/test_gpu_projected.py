"""GPU parity of the projected map access (MM_MAP_PROJECTED, the mode large maps take):
P m is written in pixel-tile order into a time-ordered buffer by the binning pass or a
projection pass, and the time-domain sweeps read it instead of gathering the map.
Forced here on small problems and checked against the CPU FP64 oracle (same bars as
the gather mode) and against the gather mode on identical inputs."""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.cg import apply_A, pcg_solve, rhs  # noqa: E402
from oracle.grad import data_grad, noise_param_grad  # noqa: E402
from oracle.messenger import (chi2, chi2_of_residual, cooling_schedule, make_setup,  # noqa: E402
                              messenger_solve, messenger_step)
from paper_1705_01893_amd import mm  # noqa: E402
from tests.tiny_inputs import random_map, tiny_problem  # noqa: E402

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
MIX_TOL = 1e-5
MIX_CHI2 = 1e-6

SHAPES = {
    "pow2": dict(lengths=(256, 512, 128), nx=8),
    "mixed_radix": dict(lengths=(2 * 3 * 5 * 8, 2 * 45, 2 * 27 * 4, 2 * 125), nx=8),
    "odd_half": dict(lengths=(30, 18, 50), nx=4),
    "long": dict(lengths=(2 * 4096, 2 * 6000), nx=16),
    "tiny_chunks": dict(lengths=(2, 4, 6, 10, 16), nx=4),
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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def plan_for(t, dev, access=mm.MM_MAP_PROJECTED, precision=mm.MM_FP64):
    psi = torch.from_numpy(np.ascontiguousarray(t.psi)).to(dev) if t.ncomp == 3 else None
    return mm.mm_plan(ncomp=t.ncomp, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample,
                      sigma=t.sigma, fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(t.pix).to(dev), psi=psi,
                      precision=precision, map_access=access, with_adjoint=True)


def setup(t):
    return make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, t.ncomp)


def tod(t, dev, precision=mm.MM_FP64):
    dt = np.float64 if precision == mm.MM_FP64 else np.float32
    return torch.from_numpy(np.ascontiguousarray(t.d.astype(dt))).to(dev)


def test_access_mode_is_reported(dev):
    t = tiny_problem(1, ncomp=3, **SHAPES["pow2"])
    assert mm.mm_plan_map_access(plan_for(t, dev, mm.MM_MAP_AUTO)) == mm.MM_MAP_GATHER  # 64 pixels
    assert mm.mm_plan_map_access(plan_for(t, dev, mm.MM_MAP_GATHER)) == mm.MM_MAP_GATHER
    assert mm.mm_plan_map_access(plan_for(t, dev)) == mm.MM_MAP_PROJECTED


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("lam", [math.inf, 1.0, 37.5])
def test_one_iteration(dev, shape, ncomp, lam):
    """A single iteration from a map that is non-zero on unsolvable pixels too
    (the projection pass must include them, as the gather does)."""
    say(f"[proj iter] shape={shape} ncomp={ncomp} lam={lam}")
    t = tiny_problem(202, ncomp=ncomp, **SHAPES[shape])
    plan = plan_for(t, dev)
    S = setup(t)
    m0 = random_map(5, ncomp, t.npix)
    mi = torch.from_numpy(m0).to(dev)
    mo = torch.zeros_like(mi)
    c2 = torch.zeros(1, dtype=torch.float64, device=dev)
    mm.mm_messenger_iter(plan, tod(t, dev), lam, mi, mo, c2)
    torch.cuda.synchronize()
    assert rel(mo.cpu().numpy(), messenger_step(S, t.d, m0, lam)) < F64_TOL
    assert c2.item() == pytest.approx(chi2(S, t.d, m0), rel=F64_TOL)


@pytest.mark.parametrize("shape", ["pow2", "mixed_radix", "long", "tiny_chunks"])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_full_schedule_chains_the_projection(dev, shape, ncomp):
    """mm_solve reuses the P m written by each iteration's binning pass in the next one:
    the whole schedule and its chi^2 history must match the oracle."""
    say(f"[proj solve] shape={shape} ncomp={ncomp}")
    t = tiny_problem(313, ncomp=ncomp, **SHAPES[shape])
    plan = plan_for(t, dev)
    S = setup(t)
    lmax, nlev, per = 40.0, 4, 3
    lams = cooling_schedule(nlev, per, lmax)
    levels = [lmax ** ((nlev - 1 - l) / (nlev - 1)) for l in range(nlev)]
    m = torch.zeros((ncomp, t.npix), dtype=torch.float64, device=dev)
    hist = torch.zeros(len(lams) + 1, dtype=torch.float64, device=dev)
    mm.mm_solve(plan, tod(t, dev), levels, [per] * nlev, m, chi2_hist=hist)
    torch.cuda.synchronize()
    m_ref, h_ref = messenger_solve(S, t.d, lams)
    assert rel(m.cpu().numpy(), m_ref) < F64_TOL
    np.testing.assert_allclose(hist.cpu().numpy(), h_ref, rtol=F64_TOL)
    # a second call replays the captured schedule and must give identical bits
    m2 = torch.zeros_like(m)
    hist2 = torch.zeros_like(hist)
    mm.mm_solve(plan, tod(t, dev), levels, [per] * nlev, m2, chi2_hist=hist2)
    torch.cuda.synchronize()
    assert torch.equal(m, m2) and torch.equal(hist, hist2)


@pytest.mark.parametrize("shape", ["pow2", "long"])
def test_projected_equals_gather(dev, shape):
    """Same inputs through both access modes: the same arithmetic up to summation order of P m."""
    say(f"[proj vs gather] shape={shape}")
    t = tiny_problem(414, ncomp=3, **SHAPES[shape])
    outs = []
    for access in (mm.MM_MAP_GATHER, mm.MM_MAP_PROJECTED):
        plan = plan_for(t, dev, access)
        m = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
        hist = torch.zeros(1 + 9 + 1, dtype=torch.float64, device=dev)
        mm.mm_solve(plan, tod(t, dev), [30.0, 30.0 ** 0.5, 1.0], [3, 3, 3], m, chi2_hist=hist)
        torch.cuda.synchronize()
        outs.append((m.cpu().numpy(), hist.cpu().numpy()))
    assert rel(outs[1][0], outs[0][0]) < 1e-13
    np.testing.assert_allclose(outs[1][1], outs[0][1], rtol=1e-13)


@pytest.mark.parametrize("shape", ["pow2", "mixed_radix"])
def test_mixed_precision_schedule(dev, shape):
    say(f"[proj mixed] shape={shape}")
    t = tiny_problem(505, ncomp=3, psi_dtype=np.float32, tod_dtype=np.float32, **SHAPES[shape])
    plan = plan_for(t, dev, precision=mm.MM_MIXED)
    S = setup(t)
    lams = cooling_schedule(3, 3, 50.0)
    m = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    hist = torch.zeros(len(lams) + 1, dtype=torch.float64, device=dev)
    mm.mm_solve(plan, tod(t, dev, mm.MM_MIXED), [50.0, 50.0 ** 0.5, 1.0], [3, 3, 3], m, chi2_hist=hist)
    torch.cuda.synchronize()
    m_ref, h_ref = messenger_solve(S, t.d.astype(np.float64), lams)
    assert rel(m.cpu().numpy(), m_ref) < MIX_TOL
    np.testing.assert_allclose(hist.cpu().numpy(), h_ref, rtol=MIX_CHI2)


@pytest.mark.parametrize("lam", [1.0, 12.0])
def test_chi2_per_chunk(dev, lam):
    say(f"[proj chi2] lam={lam}")
    t = tiny_problem(303, ncomp=3, **SHAPES["mixed_radix"])
    plan = plan_for(t, dev)
    S = setup(t)
    m = random_map(6, 3, t.npix)
    per = torch.zeros(plan.nchunk, dtype=torch.float64, device=dev)
    v = mm.mm_chi2(plan, tod(t, dev), torch.from_numpy(m).to(dev), lam, per)
    ref = chi2_of_residual(S, t.d - S.pointing.project(m), lam, per_chunk=True)
    np.testing.assert_allclose(per.cpu().numpy(), ref, rtol=F64_TOL)
    assert v == pytest.approx(ref.sum(), rel=F64_TOL)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_cg(dev, ncomp):
    say(f"[proj cg] ncomp={ncomp}")
    t = tiny_problem(606, ncomp=ncomp, **SHAPES["pow2"])
    plan = plan_for(t, dev)
    S = setup(t)
    m = torch.zeros((ncomp, t.npix), dtype=torch.float64, device=dev)
    maxit = 25
    ch = torch.zeros(maxit + 1, dtype=torch.float64, device=dev)
    n = mm.mm_cg_solve(plan, m, maxit, d=tod(t, dev), chi2_hist=ch)
    torch.cuda.synchronize()
    assert n == maxit
    m_ref, info = pcg_solve(S, t.d, maxit, record_chi2=True)
    assert rel(m.cpu().numpy(), m_ref) < 1e-9
    np.testing.assert_allclose(ch.cpu().numpy(), info["chi2"], rtol=1e-9)


def test_apply_and_tod_apply(dev):
    say("[proj apply]")
    t = tiny_problem(808, ncomp=3, **SHAPES["mixed_radix"])
    plan = plan_for(t, dev)
    S = setup(t)
    x = random_map(8, 3, t.npix)
    x[:, ~S.solvable] = 0
    out = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    mm.mm_apply(plan, 0, out, x=torch.from_numpy(x).to(dev))
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), apply_A(S, x)) < F64_TOL
    mm.mm_apply(plan, 0, out, d=tod(t, dev))
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), rhs(S, t.d)) < F64_TOL
    z = random_map(3, 3, t.npix)
    tout = torch.zeros(t.nsamp, dtype=torch.float64, device=dev)
    mm.mm_tod_apply(plan, 0, torch.from_numpy(z).to(dev), tout)
    torch.cuda.synchronize()
    assert rel(tout.cpu().numpy(), data_grad(S, z)) < F64_TOL


@pytest.mark.parametrize("ncomp", [1, 3])
def test_noise_grad(dev, ncomp):
    say(f"[proj noise_grad] ncomp={ncomp}")
    t = tiny_problem(41, ncomp=ncomp, lengths=(256, 512, 128), nx=8)
    plan = plan_for(t, dev)
    S = setup(t)
    m = random_map(1, ncomp, t.npix)
    z = random_map(2, ncomp, t.npix)
    out = torch.zeros((plan.nchunk, 3), dtype=torch.float64, device=dev)
    mm.mm_noise_grad(plan, tod(t, dev), torch.from_numpy(m).to(dev), torch.from_numpy(z).to(dev), out)
    torch.cuda.synchronize()
    ref = noise_param_grad(S, t.d, m, z, t.fsample, t.sigma, t.fknee, t.alpha)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
