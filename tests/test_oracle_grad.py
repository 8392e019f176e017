"""Pins for the gradient oracle: the implicit-gradient formulas against brute-force
central differences of the dense minimum-variance map (no GPU)."""

import numpy as np
import pytest

from oracle import dense
from oracle.grad import data_grad, noise_param_grad, spectrum_derivatives
from oracle.messenger import make_setup
from tests.tiny_inputs import random_map, tiny_problem


def _setup(t, sigma=None, fknee=None, alpha=None):
    return make_setup(t.chunk_off, t.fsample, t.sigma if sigma is None else sigma,
                      t.fknee if fknee is None else fknee, t.alpha if alpha is None else alpha,
                      t.pix, t.psi, t.npix, t.ncomp)


def _loss(S, d, m_ref):
    m = dense.gls(S, d)
    return float(np.sum((m - m_ref) ** 2)), m


def _adjoint(S, g):
    cols = np.concatenate([np.nonzero(S.solvable)[0] + q * S.npix for q in range(S.ncomp)])
    A = dense.normal_matrix(S)
    z = np.zeros(S.ncomp * S.npix)
    z[cols] = np.linalg.solve(A, g.reshape(-1)[cols])
    return z.reshape(S.ncomp, S.npix)


def test_spectrum_derivatives_against_differences():
    n, fs, s, fk, al = 32, 10.0, 1.3, 0.7, -1.8
    N0 = spectrum_derivatives(n, fs, s, fk, al)
    h = 1e-6
    for i, (ds, dfk, dal) in enumerate([(h, 0, 0), (0, h, 0), (0, 0, h)]):
        up = spectrum_derivatives(n, fs, s + ds, fk + dfk, al + dal)[0]
        dn = spectrum_derivatives(n, fs, s - ds, fk - dfk, al - dal)[0]
        np.testing.assert_allclose((up - dn) / (2 * h), N0[1 + i], rtol=1e-6)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_noise_param_gradient_matches_central_differences(ncomp):
    t = tiny_problem(31, ncomp=ncomp, lengths=(48, 40), nx=3)
    S = _setup(t)
    m_ref = random_map(3, ncomp, t.npix)
    L0, m = _loss(S, t.d, m_ref)
    z = _adjoint(S, 2.0 * (m - m_ref))
    grad = noise_param_grad(S, t.d, m, z, t.fsample, t.sigma, t.fknee, t.alpha)
    for c in range(len(t.sigma)):
        for j, name in enumerate(("sigma", "fknee", "alpha")):
            base = {"sigma": t.sigma.copy(), "fknee": t.fknee.copy(), "alpha": t.alpha.copy()}
            h = 1e-5 * max(abs(base[name][c]), 1.0)
            up = {k: v.copy() for k, v in base.items()}
            dn = {k: v.copy() for k, v in base.items()}
            up[name][c] += h
            dn[name][c] -= h
            fd = (_loss(_setup(t, **up), t.d, m_ref)[0] - _loss(_setup(t, **dn), t.d, m_ref)[0]) / (2 * h)
            assert grad[c, j] == pytest.approx(fd, rel=2e-5, abs=1e-9 * abs(L0)), (c, name)


def test_data_gradient_matches_central_differences():
    t = tiny_problem(32, ncomp=3, lengths=(40, 36), nx=3)
    S = _setup(t)
    m_ref = random_map(4, 3, t.npix)
    _, m = _loss(S, t.d, m_ref)
    gd = data_grad(S, _adjoint(S, 2.0 * (m - m_ref)))
    rng = np.random.default_rng(5)
    for j in rng.choice(t.nsamp, size=6, replace=False):
        h = 1e-5
        d1, d2 = t.d.copy(), t.d.copy()
        d1[j] += h
        d2[j] -= h
        fd = (_loss(S, d1, m_ref)[0] - _loss(S, d2, m_ref)[0]) / (2 * h)
        assert gd[j] == pytest.approx(fd, rel=1e-6, abs=1e-10)
