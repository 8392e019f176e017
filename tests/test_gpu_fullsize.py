"""Parity at the benchmark workload's full size (16 detectors x 2^20 samples, 256x256 I/Q/U,
FP64), in the launch configuration bench.py times: the binned map (lambda = inf step), one
lambda = 1 iteration from it and chi^2, against the oracle on every pixel."""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.messenger import binned_map, chi2, messenger_step, setup_from_problem  # noqa: E402
from paper_1705_01893_amd import mm  # noqa: E402
from synth import config_by_name, make_problem  # noqa: E402

pytestmark = pytest.mark.gpu


def test_iqu256_full_size_iteration():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    print("[fullsize] generating iqu256", flush=True)
    prob = make_problem(config_by_name("iqu256"))
    plan = mm.mm_plan(ncomp=3, npix=prob.npix, nx=prob.cfg.nx, chunk_off=prob.chunk_off, fsample=prob.fsample,
                      sigma=prob.sigma, fknee=prob.fknee, alpha=prob.alpha, pix=torch.from_numpy(prob.pix).to(dev),
                      psi=torch.from_numpy(prob.psi).to(dev))
    d = torch.from_numpy(prob.d).to(dev)
    m0 = torch.zeros((3, prob.npix), dtype=torch.float64, device=dev)
    m1 = torch.zeros_like(m0)
    m2 = torch.zeros_like(m0)
    c2 = torch.zeros(1, dtype=torch.float64, device=dev)
    mm.mm_messenger_iter(plan, d, math.inf, m0, m1)
    mm.mm_messenger_iter(plan, d, 1.0, m1, m2, c2)
    torch.cuda.synchronize()
    print("[fullsize] oracle", flush=True)
    S = setup_from_problem(prob)
    r1 = binned_map(S, prob.d)
    assert np.linalg.norm(m1.cpu().numpy() - r1) / np.linalg.norm(r1) < 1e-10
    r2 = messenger_step(S, prob.d, r1, 1.0)
    assert np.linalg.norm(m2.cpu().numpy() - r2) / np.linalg.norm(r2) < 1e-10
    assert c2.item() == pytest.approx(chi2(S, prob.d, r1), rel=1e-10)
    plan.close()
