"""Pins of the gap-filling oracle (composite noise N = N_0 + N_1, Appendix C).

* the fixed point of the four updates is the generalised least-squares map of the samples
  outside the gaps with their noise covariance restricted to them, and d_0 there is the
  conditional mean of the data in the gaps (dense matrices, tiny problems);
* every single update minimises chi^2_1 over its field (chi^2_1 never rises, and no small
  change of the updated field lowers it);
* the data inside the gaps are never read; noise-free data make the sky map a fixed point;
* lambda = inf gives t_0 = d_0 and the map of the binned d_0;
* with no gaps the map's fixed point is the plain GLS map.
"""

import math

import numpy as np
import pytest

from oracle import dense
from oracle.gapfill import (augmented_chi2, gap_init, gap_solve, gap_step, make_gap_setup, update_d0, update_m,
                            update_t0, update_t1)
from oracle.messenger import binned_map
from tests.tiny_inputs import gap_mask, random_map, tiny_problem


def setup(t, gaps, eps_frac=0.2):
    eps = eps_frac * t.sigma ** 2
    return make_gap_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, t.ncomp, gaps, eps)


def dense_N(G):
    """The chunks' noise covariance N as an explicit block-circulant matrix (eigenvalues N_k)."""
    ns = int(G.S.noise.chunk_off[-1])
    out = np.zeros((ns, ns))
    for c in range(G.S.noise.nchunk):
        a, b = int(G.S.noise.chunk_off[c]), int(G.S.noise.chunk_off[c + 1])
        out[a:b, a:b] = dense.circulant_inverse(1.0 / G.S.noise.spectra[c], b - a)
    return out


def gap_gls(G, d):
    """The GLS map of the samples outside the gaps (their N restricted), over the solvable pixels,
    and the conditional mean of d_0 given it."""
    S = G.S
    n = ~G.gaps
    N = dense_N(G)
    Sig = N[np.ix_(n, n)]
    cols = np.concatenate([np.nonzero(S.solvable)[0] + q * S.npix for q in range(S.ncomp)])
    P = dense.pointing_matrix(S)[:, cols]
    Pn = P[n]
    A = Pn.T @ np.linalg.solve(Sig, Pn)
    x = np.linalg.solve(A, Pn.T @ np.linalg.solve(Sig, np.asarray(d, np.float64)[n]))
    m = np.zeros(S.ncomp * S.npix)
    m[cols] = x
    m = m.reshape(S.ncomp, S.npix)
    Pm = S.pointing.project(m)
    r = (np.asarray(d, np.float64) - Pm)[n]
    N0_cols = N[:, n] - np.diag(G.per_sample(G.eps))[:, n]     # N_0 = N - eps I
    d0 = Pm + N0_cols @ np.linalg.solve(Sig, r)
    return m, d0


@pytest.mark.parametrize("ncomp", [1, 3])
def test_fixed_point_is_the_gap_aware_gls_map(ncomp):
    t = tiny_problem(71, ncomp=ncomp, lengths=(96, 80), nx=4, flag_frac=0.0)
    gaps = gap_mask(5, t.chunk_off, 0.12, 5)
    G = setup(t, gaps)
    m, d0 = gap_gls(G, t.d)
    t0 = update_t0(G, d0, m, 1.0)
    m1, d1, t1 = gap_step(G, t.d, m, d0, t0, 1.0)
    assert np.linalg.norm(m1 - m) <= 1e-10 * np.linalg.norm(m)
    assert np.linalg.norm(d1 - d0) <= 1e-10 * np.linalg.norm(d0)
    assert np.linalg.norm(t1 - t0) <= 1e-10 * np.linalg.norm(t0)
    # and the iteration from the start heads there (temperature: on this I/Q/U problem a pixel
    # whose Q and U the samples outside the gaps barely separate converges far more slowly)
    if ncomp == 1:
        mk, _, _ = gap_solve(G, t.d, [1.0] * 3000)
        assert np.linalg.norm(mk - m) <= 1e-6 * np.linalg.norm(m)


def test_without_gaps_the_map_fixed_point_is_plain_gls():
    t = tiny_problem(72, ncomp=3, lengths=(64, 48), nx=4, flag_frac=0.0)
    G = setup(t, np.zeros(t.nsamp, dtype=bool))
    m = dense.gls(G.S, t.d)
    d0 = np.asarray(t.d, np.float64) - np.diag(G.per_sample(G.eps)) @ np.linalg.solve(
        dense_N(G), np.asarray(t.d, np.float64) - G.S.pointing.project(m))
    t0 = update_t0(G, d0, m, 1.0)
    m1, _, _ = gap_step(G, t.d, m, d0, t0, 1.0)
    assert np.linalg.norm(m1 - m) <= 1e-10 * np.linalg.norm(m)


@pytest.mark.parametrize("lam", [1.0, 7.0])
def test_every_update_minimises_the_augmented_chi2(lam):
    t = tiny_problem(73, ncomp=3, lengths=(64, 48), nx=4, flag_frac=0.0)
    gaps = gap_mask(6, t.chunk_off, 0.15, 4)
    G = setup(t, gaps)
    rng = np.random.default_rng(3)
    d = np.asarray(t.d, np.float64)
    m = random_map(4, 3, t.npix)
    m[:, ~G.S.solvable] = 0.0
    d0 = d + rng.standard_normal(len(d))
    t0 = d + rng.standard_normal(len(d))
    t1 = update_t1(G, d, d0)
    prev = augmented_chi2(G, d, m, d0, t0, t1, lam)

    def check(field_name, fields, value):
        nonlocal prev
        cur = augmented_chi2(G, d, *fields, lam)
        assert cur <= prev * (1 + 1e-12)
        prev = cur
        # stationary: a small change of the updated field (free entries only) does not lower it
        for sgn in (1.0, -1.0):
            delta = sgn * 1e-4 * rng.standard_normal(value.shape)
            if field_name == "t1":
                delta[~G.gaps] = 0.0          # fixed to the data outside the gaps
            if field_name == "m":
                delta[:, ~G.S.solvable] = 0.0  # unsolvable pixels are held at zero
            pert = dict(zip(("m", "d0", "t0", "t1"), fields))
            pert[field_name] = value + delta
            assert augmented_chi2(G, d, pert["m"], pert["d0"], pert["t0"], pert["t1"], lam) >= cur * (1 - 1e-12)

    for _ in range(3):
        t1 = update_t1(G, d, d0)
        check("t1", (m, d0, t0, t1), t1)
        d0 = update_d0(G, t0, t1)
        check("d0", (m, d0, t0, t1), d0)
        t0 = update_t0(G, d0, m, lam)
        check("t0", (m, d0, t0, t1), t0)
        m = update_m(G, t0)
        check("m", (m, d0, t0, t1), m)


def test_data_inside_the_gaps_are_never_read():
    t = tiny_problem(74, ncomp=3, lengths=(64, 48), nx=4)
    gaps = gap_mask(7, t.chunk_off, 0.2, 3)
    G = setup(t, gaps)
    d2 = np.asarray(t.d, np.float64).copy()
    d2[gaps] = 1e9
    a = gap_solve(G, t.d, [math.inf, 30.0, 30.0, 1.0, 1.0])
    b = gap_solve(G, d2, [math.inf, 30.0, 30.0, 1.0, 1.0])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_noise_free_sky_is_a_fixed_point():
    t = tiny_problem(75, ncomp=3, lengths=(64, 48), nx=4)
    gaps = gap_mask(8, t.chunk_off, 0.2, 3)
    G = setup(t, gaps)
    m_true = random_map(9, 3, t.npix, 4.0)
    m_true[:, ~G.S.solvable] = 0.0
    d = G.S.pointing.project(m_true)
    d[gaps] = -7.0e3
    Pm = G.S.pointing.project(m_true)
    for lam in (math.inf, 3.0, 1.0):
        m1, d1, t1 = gap_step(G, d, m_true, Pm, Pm, lam)
        assert np.linalg.norm(m1 - m_true) <= 1e-12 * np.linalg.norm(m_true)
        assert np.linalg.norm(d1 - Pm) <= 1e-12 * np.linalg.norm(Pm)


def test_lambda_inf_bins_the_gap_filled_data():
    t = tiny_problem(76, ncomp=3, lengths=(64, 48), nx=4)
    gaps = gap_mask(10, t.chunk_off, 0.2, 3)
    G = setup(t, gaps)
    d0, t0 = gap_init(G, t.d)
    assert np.array_equal(d0[gaps], np.zeros(int(gaps.sum())))
    m, d1, t1 = gap_step(G, t.d, random_map(1, 3, t.npix), d0, t0, math.inf)
    assert np.array_equal(t1, d1)
    assert np.linalg.norm(m - binned_map(G.S, d1)) <= 1e-13 * np.linalg.norm(m)
