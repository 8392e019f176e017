"""Batching form: many detector chunks of uneven 5-smooth lengths processed in one
launch per pass, in FP64 and FP32-mixed, against the oracle (the uneven-length workload's
recipe at a reduced size: 24 detectors, lengths log-uniform in [2^12, 2^15], 128x128 map)."""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.messenger import cooling_schedule, messenger_solve, setup_from_problem  # noqa: E402
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


@pytest.fixture(scope="module")
def prob():
    cfg = config_by_name("batched1024").scaled("batched-small", ndet=24, nsamp=1 << 15, nx=128,
                                                nsamp_min=1 << 12)
    return make_problem(cfg)


def test_lengths_are_uneven_and_transform_friendly(prob):
    n = np.diff(prob.chunk_off)
    assert len(set(n.tolist())) > 10
    for v in n:
        m = int(v) // 2
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        assert m == 1 and v % 2 == 0


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_batched_solve(dev, prob, form):
    say(f"[batched] form={form}")
    mixed = form == "mixed"
    tod = prob.d.astype(np.float32 if mixed else np.float64)
    psi = prob.psi.astype(np.float32 if mixed else np.float64)
    plan = mm.mm_plan(ncomp=3, npix=prob.npix, nx=prob.cfg.nx, chunk_off=prob.chunk_off, fsample=prob.fsample,
                      sigma=prob.sigma, fknee=prob.fknee, alpha=prob.alpha, pix=torch.from_numpy(prob.pix).to(dev),
                      psi=torch.from_numpy(psi).to(dev), precision=mm.MM_MIXED if mixed else mm.MM_FP64)
    hits = torch.zeros(prob.npix, dtype=torch.int32, device=dev)
    mm.mm_plan_hits(plan, hits)
    levels = mm.mm_cooling_levels(plan, 3, 0.0)
    m = torch.zeros((3, prob.npix), dtype=torch.float64, device=dev)
    h = torch.zeros(1 + 9 + 1, dtype=torch.float64, device=dev)
    mm.mm_solve(plan, torch.from_numpy(tod).to(dev), levels, [3, 3, 3], m, chi2_hist=h)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(hits.cpu().numpy(), np.bincount(prob.pix[prob.pix >= 0], minlength=prob.npix))
    from oracle.messenger import make_setup
    S = make_setup(prob.chunk_off, prob.fsample, prob.sigma, prob.fknee, prob.alpha, prob.pix, psi, prob.npix, 3)
    lams = [math.inf] + [lv for lv in levels for _ in range(3)]
    m_ref, h_ref = messenger_solve(S, tod.astype(np.float64), lams)
    rel = np.linalg.norm(m.cpu().numpy() - m_ref) / np.linalg.norm(m_ref)
    tol_m, tol_c = (1e-5, 1e-6) if mixed else (1e-10, 1e-10)
    assert rel < tol_m, rel
    np.testing.assert_allclose(h.cpu().numpy(), h_ref, rtol=tol_c)
    plan.close()
