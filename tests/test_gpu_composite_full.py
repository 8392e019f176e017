"""GPU parity of composite pointing at the full differential-beam workloads, as the benchmark
runs them: diff256 (16 x 2^20 samples, 256 x 256 temperature map, FP64) and diff512 (64 x 2^20,
512 x 512 I/Q/U, FP32 TOD), each in both forms, against the CPU FP64 oracle on every pixel:
hit counts and the solvable mask (bit-exact), the lambda = inf step from zero (the first weighted
Jacobi step), one lambda = 1 step and one mid-schedule step from the oracle's state, and chi^2.
Bars: FP64 rel-L2 1e-10, FP32-mixed 1e-5 (chi^2 1e-10 / 1e-6)."""

import math
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.composite import make_composite_setup  # noqa: E402
from oracle.messenger import chi2, messenger_step  # noqa: E402
from paper_1705_01893_amd import mm  # noqa: E402
from synth import config_by_name, make_problem  # noqa: E402

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


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["diff256", "diff512"])
def test_full_differential_workload(dev, name):
    cfg = config_by_name(name)
    t0 = time.perf_counter()
    p = make_problem(cfg, workers=16)
    say(f"[{name}] generated {int(p.chunk_off[-1])} samples in {time.perf_counter() - t0:.1f} s")
    S = make_composite_setup(p.chunk_off, p.fsample, p.sigma, p.fknee, p.alpha, p.pix, p.psi, p.pix_b, p.psi_b,
                             p.npix, p.ncomp, w_a=p.weights[0], w_b=p.weights[1])
    on = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    pix, pix_b = on(p.pix), on(p.pix_b)
    for form in ("fp64", "mixed"):
        prec = mm.MM_FP64 if form == "fp64" else mm.MM_MIXED
        dt = np.float64 if form == "fp64" else np.float32
        tol, ctol = (1e-10, 1e-10) if form == "fp64" else (1e-5, 1e-6)
        psi = None if p.psi is None else on(p.psi.astype(dt))
        psi_b = None if p.psi_b is None else on(p.psi_b.astype(dt))
        d_host = p.d.astype(dt)
        d = on(d_host)
        d64 = d_host.astype(np.float64)
        # the oracle sees the angles the form stores
        So = S if p.psi is None or p.psi.dtype == dt else make_composite_setup(
            p.chunk_off, p.fsample, p.sigma, p.fknee, p.alpha, p.pix, p.psi.astype(dt), p.pix_b, p.psi_b.astype(dt),
            p.npix, p.ncomp, w_a=p.weights[0], w_b=p.weights[1])
        plan = mm.mm_plan(ncomp=p.ncomp, npix=p.npix, nx=cfg.nx, chunk_off=p.chunk_off, fsample=p.fsample,
                          sigma=p.sigma, fknee=p.fknee, alpha=p.alpha, pix=pix, psi=psi, pix_b=pix_b, psi_b=psi_b,
                          weights=p.weights, precision=prec)
        hits = torch.zeros(p.npix, dtype=torch.int32, device=dev)
        mask = torch.zeros(p.npix, dtype=torch.uint8, device=dev)
        mm.mm_plan_hits(plan, hits)
        mm.mm_plan_solvable(plan, mask)
        torch.cuda.synchronize()
        assert np.array_equal(hits.cpu().numpy().astype(np.int64), So.hits)
        assert np.array_equal(mask.cpu().numpy().astype(bool), So.solvable)
        # lambda = inf from zero, then lambda = 1 and lambda = 40 from the oracle's iterate
        m = torch.zeros((p.ncomp, p.npix), dtype=torch.float64, device=dev)
        mm.mm_messenger_iter(plan, d, math.inf, m, m)
        torch.cuda.synchronize()
        r_inf = messenger_step(So, d64, np.zeros((p.ncomp, p.npix)), math.inf)
        e_inf = rel(m.cpu().numpy(), r_inf)
        src = torch.from_numpy(r_inf).to(dev)
        errs = {}
        for lam in (1.0, 40.0):
            out = torch.zeros_like(src)
            c2 = torch.zeros(1, dtype=torch.float64, device=dev)
            mm.mm_messenger_iter(plan, d, lam, src, out, c2)
            torch.cuda.synchronize()
            errs[lam] = rel(out.cpu().numpy(), messenger_step(So, d64, r_inf, lam))
            if lam == 1.0:
                want = chi2(So, d64, r_inf)
                errs["chi2"] = abs(c2.item() - want) / want
        say(f"[{name}] {form}: lambda=inf {e_inf:.2e}, lambda=1 {errs[1.0]:.2e}, lambda=40 {errs[40.0]:.2e}, "
            f"chi2 {errs['chi2']:.2e}")
        assert e_inf < tol and errs[1.0] < tol and errs[40.0] < tol and errs["chi2"] < ctol
        plan.close()
        del plan, d
        torch.cuda.empty_cache()
