"""Pins that tie the CPU oracle to the paper and to mathematics (no GPU).

Each test checks the oracle against something other than itself: exact values
(golden files), closed forms, invariants the paper states, textbook special
cases, or brute-force dense linear algebra on tiny inputs.
"""

import math
import os

import numpy as np
import pytest

import oracle
from oracle import dense
from oracle.cg import pcg_solve, apply_A
from oracle.messenger import (make_setup, messenger_step, messenger_step_two_equation,
                              messenger_step_mapsized, binned_map, chi2, chi2_lambda,
                              chi2_of_residual, cooling_schedule, messenger_solve, lambda_max_rule)
from oracle.noise import noise_psd, chi2_weights, NoiseModel
from oracle.pointing import Pointing, invert_blocks
from tests.tiny_inputs import tiny_problem, random_map

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def _setup(t, **kw):
    return make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, t.ncomp, **kw)


# ------------------------------------------------------------------------------------------------
# exact values

def test_polarization_response_golden():
    """Section 2: P carries I, Q, U weights.  Exact responses at multiples of pi/8."""
    g = _golden("polarization_response.txt")
    psi = g[:, 0] * np.pi
    pt = Pointing(np.zeros(len(psi), np.int32), psi, npix=1, ncomp=3)
    out = pt.project(np.array([[1.0], [2.0], [3.0]]))
    np.testing.assert_allclose(out, g[:, 1], rtol=0, atol=1e-14)


def test_noise_psd_golden():
    """Section 2.3 power law at exact bins, DC bin clamped to f_1."""
    g = _golden("noise_psd.txt")
    N = noise_psd(16, 8.0, 2.0, 1.0, -2.0)
    np.testing.assert_allclose(N[g[:, 0].astype(int)], g[:, 1], rtol=1e-15)


def test_cooling_schedule_levels():
    """Section 3.1: one very-high-lambda step, then geometric levels ending at exactly lambda = 1."""
    lams = cooling_schedule(10, 5, 1e4)
    assert math.isinf(lams[0]) and len(lams) == 1 + 50
    levels = np.array(lams[1::5])
    assert levels[0] == 1e4 and levels[-1] == 1.0
    ratios = levels[:-1] / levels[1:]
    np.testing.assert_allclose(ratios, 10 ** (4 / 9), rtol=1e-13)


@pytest.mark.parametrize("tau0, expect", [(None, 3.0), (0.5, 4.0)])
def test_lambda_max_rule_hand_values(tau0, expect):
    """Section 3.1: the top level puts lambda tau at the largest noise power of any chunk.

    Two chunks of n = 8 samples at f_s = 8 Hz (bins f_k = k Hz, k = 0..4, f_0 clamped to f_1):
      chunk 0: sigma = 1, f_knee = 1, alpha = -2: N = 1 + f^-2 -> 2, 2, 1.25, 1.111, 1.0625;
               largest 2 at the low end, tau = sigma^2 = 1 (or 0.5) -> ratio 2 (or 4);
      chunk 1: sigma = 2, f_knee = 2, alpha = +1: N = 4 (1 + f/2) -> 6, 6, 8, 10, 12;
               largest 12 at Nyquist, tau = 4 -> ratio 3.
    The rule takes the larger ratio: 3 (or 4 when chunk 0 has tau = 0.5).  Taking the smaller,
    dividing by tau twice or reading only one end of the spectrum all give another value."""
    off = np.array([0, 8, 16])
    tau = None if tau0 is None else np.array([tau0, 4.0])
    S = make_setup(off, np.array([8.0, 8.0]), np.array([1.0, 2.0]), np.array([1.0, 2.0]),
                   np.array([-2.0, 1.0]), np.zeros(16, np.int32), None, 1, 1, tau=tau)
    assert lambda_max_rule(S) == pytest.approx(expect, rel=1e-15)


# ------------------------------------------------------------------------------------------------
# closed forms for the noise operator and chi^2

@pytest.mark.parametrize("n", [16, 15])
def test_chi2_of_fourier_modes_closed_form(n):
    """x^T N^-1 x for a pure cosine at bin k0 is (n/2)/N_k0 (0 < k0 < n/2), n/N_0 for a
    constant and n/N_{n/2} for the alternating sequence: pins the bin multiplicities."""
    N = noise_psd(n, 5.0, 1.1, 0.7, -1.7)
    nm = NoiseModel(chunk_off=np.array([0, n]), spectra=[N], tau=np.array([1.1 ** 2]))
    pt = Pointing(np.full(n, -1, np.int32), None, npix=1, ncomp=1)
    S = oracle.Setup(pointing=pt, noise=nm, W=np.zeros((1, 1, 1)), W_inv=np.zeros((1, 1, 1)),
                     solvable=np.zeros(1, bool), hits=np.zeros(1, np.int64))
    j = np.arange(n)
    for k0 in range(1, (n - 1) // 2 + 1):
        x = np.cos(2 * np.pi * k0 * j / n)
        assert chi2_of_residual(S, x) == pytest.approx((n / 2) / N[k0], rel=1e-12)
        assert x @ nm.apply_inverse(x) == pytest.approx((n / 2) / N[k0], rel=1e-12)
    assert chi2_of_residual(S, np.ones(n)) == pytest.approx(n / N[0], rel=1e-12)
    if n % 2 == 0:
        alt = (-1.0) ** j
        assert chi2_of_residual(S, alt) == pytest.approx(n / N[n // 2], rel=1e-12)


def test_fft_noise_inverse_matches_explicit_circulant():
    """N^-1 via rfft/irfft equals the explicit cosine-sum circulant matrix."""
    for n in (8, 9, 20):
        N = noise_psd(n, 3.0, 0.9, 0.4, -2.5)
        nm = NoiseModel(chunk_off=np.array([0, n]), spectra=[N], tau=np.array([0.81]))
        C = dense.circulant_inverse(N, n)
        x = np.random.default_rng(n).standard_normal(n)
        np.testing.assert_allclose(nm.apply_inverse(x), C @ x, rtol=1e-12, atol=1e-13)
        # naive O(n^2) DFT of the eigenvalue relation: C applied to a Fourier vector scales it
        k = 2
        v = np.exp(2j * np.pi * k * np.arange(n) / n)
        np.testing.assert_allclose(C @ v, v / N[k], rtol=1e-12, atol=1e-13)


def test_chi2_weights():
    assert list(chi2_weights(6)) == [1, 2, 2, 1]
    assert list(chi2_weights(7)) == [1, 2, 2, 2]


# ------------------------------------------------------------------------------------------------
# closed forms for the iteration

def _identity_problem(n=32, tau_scale=1.0, psd=None):
    """P = I: every sample its own pixel.  The GLS map is the data itself."""
    pix = np.arange(n, dtype=np.int32)
    N = noise_psd(n, 4.0, 1.2, 0.8, -2.0)
    S = make_setup(np.array([0, n]), [4.0], [1.2], [0.8], [-2.0], pix, None, npix=n, ncomp=1,
                   tau=None if psd is None else [min(psd)], psd=None if psd is None else [psd])
    return S, N


def test_identity_pointing_messenger_closed_form():
    """With P = I the error of every Fourier mode contracts by N-bar_k / (lambda tau + N-bar_k)
    per iteration (Section 2.1): after K steps from zero, m-hat = d-hat (1 - rho_k^K)."""
    n = 32
    S, N = _identity_problem(n)
    tau = S.noise.tau[0]
    d = np.random.default_rng(1).standard_normal(n)
    for lam in (1.0, 7.5, 300.0):
        m = np.zeros((1, n))
        K = 6
        for _ in range(K):
            m = messenger_step(S, d, m, lam)
        nbar = N - tau
        rho = nbar / (lam * tau + nbar)
        expect = np.fft.irfft(np.fft.rfft(d) * (1 - rho ** K), n)
        np.testing.assert_allclose(m[0], expect, rtol=1e-12, atol=1e-12)


def test_single_pixel_closed_form():
    """One pixel, one chunk: the GLS map is the sample mean (the constant vector is the
    DC eigenvector of N^-1) and each iteration removes a fraction lambda tau / (lambda tau + N-bar_0)
    of the remaining error."""
    n = 24
    pix = np.zeros(n, np.int32)
    S = make_setup(np.array([0, n]), [2.0], [0.9], [0.3], [-2.2], pix, None, npix=1, ncomp=1)
    d = np.random.default_rng(2).standard_normal(n) + 5
    tau = S.noise.tau[0]
    nbar0 = S.noise.spectra[0][0] - tau
    lam = 40.0
    m = np.array([[0.0]])
    err = 0.0 - d.mean()
    for _ in range(5):
        m = messenger_step(S, d, m, lam)
        err *= nbar0 / (lam * tau + nbar0)
        assert m[0, 0] - d.mean() == pytest.approx(err, rel=1e-10, abs=1e-13)
    np.testing.assert_allclose(dense.gls(S, d)[0, 0], d.mean(), rtol=1e-12)


def test_two_chunk_single_pixel_gls_weighting():
    """Two chunks on one pixel: the GLS map weights each chunk's mean by n_c / N_{c,0}."""
    lens = (20, 30)
    pix = np.zeros(sum(lens), np.int32)
    off = np.array([0, 20, 50])
    S = make_setup(off, [2.0, 2.0], [0.9, 1.4], [0.3, 0.5], [-2.0, -1.0], pix, None, npix=1, ncomp=1)
    d = np.random.default_rng(3).standard_normal(50)
    w = np.array([lens[c] / S.noise.spectra[c][0] for c in range(2)])
    means = np.array([d[:20].mean(), d[20:].mean()])
    np.testing.assert_allclose(dense.gls(S, d)[0, 0], (w * means).sum() / w.sum(), rtol=1e-12)


def test_white_noise_one_step_is_gls():
    """All noise in T (N = T): the messenger converges in one step (Section 4.2), to the binned
    map, which is then the minimum-variance map, from any starting map and at any lambda."""
    t = tiny_problem(4, lengths=(40, 56), nx=3)
    psd = [np.full(int(n) // 2 + 1, s * s) for n, s in zip(np.diff(t.chunk_off), t.sigma)]
    S = _setup(t, psd=psd, tau=t.sigma ** 2)
    m_gls = dense.gls(S, t.d)
    for lam in (1.0, 3.0, math.inf):
        m1 = messenger_step(S, t.d, random_map(9, 3, t.npix), lam)
        np.testing.assert_allclose(m1, m_gls, rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(binned_map(S, t.d), m_gls, rtol=1e-10, atol=1e-11)


def test_lambda_inf_step_is_binned_map():
    """Very large lambda: F = 0 and the next map is W^-1 P^T T^-1 d whatever the current map."""
    t = tiny_problem(5)
    S = _setup(t)
    mb = binned_map(S, t.d)
    for seed in (0, 1):
        m0 = random_map(seed, 3, t.npix, 5.0)
        np.testing.assert_allclose(messenger_step(S, t.d, m0, math.inf), mb, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(messenger_step(S, t.d, m0, 1e14), mb, rtol=1e-6, atol=1e-6)


# ------------------------------------------------------------------------------------------------
# invariants and brute force

@pytest.mark.parametrize("lam", [1.0, 5.0, 1e3, math.inf])
def test_three_forms_agree(lam):
    """Residual, two-equation and map-sized forms are equal (Woodbury, Section 2.1)."""
    t = tiny_problem(6, lengths=(64, 50, 36))
    S = _setup(t)
    m = random_map(3, 3, t.npix)
    a = messenger_step(S, t.d, m, lam)
    b = messenger_step_two_equation(S, t.d, m, lam)
    c = messenger_step_mapsized(S, t.d, m, lam)
    scale = np.abs(a).max()
    assert np.abs(a - b).max() <= 1e-12 * scale
    assert np.abs(a - c).max() <= 1e-12 * scale


def test_residual_form_matches_dense_operator():
    """One step equals m + W^-1 P^T G P-restricted algebra built from explicit matrices."""
    t = tiny_problem(7, lengths=(30, 26), nx=3)
    S = _setup(t)
    m = random_map(4, 3, t.npix)
    m[:, ~S.solvable] = 0
    lam = 12.0
    P = dense.pointing_matrix(S)
    G = np.zeros((t.nsamp, t.nsamp))
    for c in range(S.noise.nchunk):
        a, b = int(t.chunk_off[c]), int(t.chunk_off[c + 1])
        tau = S.noise.tau[c]
        G[a:b, a:b] = dense.circulant_inverse((S.noise.spectra[c] - tau) / lam + tau, b - a)
    W = P.T @ (P / np.repeat(S.noise.tau, np.diff(t.chunk_off))[:, None])
    cols = np.concatenate([np.nonzero(S.solvable)[0] + q * t.npix for q in range(3)])
    upd = np.linalg.solve(W[np.ix_(cols, cols)], (P.T @ G @ (t.d - P @ m.reshape(-1)))[cols])
    expect = m.reshape(-1).copy()
    expect[cols] += upd
    np.testing.assert_allclose(messenger_step(S, t.d, m, lam).reshape(-1), expect, rtol=1e-10, atol=1e-12)


def test_gls_limit_well_conditioned():
    """Many lambda = 1 iterations converge to the dense minimum-variance map (eqn. mapmaking)."""
    t = tiny_problem(8, lengths=(40, 40), nx=3, fknee=(0.3, 0.2), alpha=(-1.0, -1.0), fs=20.0)
    S = _setup(t)
    m_gls = dense.gls(S, t.d)
    m = np.zeros((3, t.npix))
    for _ in range(400):
        m = messenger_step(S, t.d, m, 1.0)
    rel = np.linalg.norm(m - m_gls) / np.linalg.norm(m_gls)
    assert rel < 1e-10


def test_fixed_points():
    """The GLS map is fixed under a lambda = 1 step; m(lambda) (eqn. mlambda) under a lambda step."""
    t = tiny_problem(9)
    S = _setup(t)
    m_gls = dense.gls(S, t.d)
    np.testing.assert_allclose(messenger_step(S, t.d, m_gls, 1.0), m_gls, rtol=1e-9, atol=1e-9 * np.abs(m_gls).max())
    for lam in (4.0, 100.0):
        ml = dense.m_lambda(S, t.d, lam)
        np.testing.assert_allclose(messenger_step(S, t.d, ml, lam), ml, rtol=1e-9, atol=1e-9 * np.abs(ml).max())


@pytest.mark.parametrize("lam", [1.0, 30.0])
def test_F_spectrum_and_error_recursion(lam):
    """eps_{i+1} = F(lambda) eps_i with the eigenvalues of F in [0, 1) (Section 2.1)."""
    t = tiny_problem(10, lengths=(48, 40), nx=3)
    S = _setup(t)
    F = dense.F_matrix(S, lam)
    ev = np.linalg.eigvals(F)
    assert np.all(np.abs(ev.imag) < 1e-9)
    assert ev.real.min() > -1e-10 and ev.real.max() < 1.0
    ml = dense.m_lambda(S, t.d, lam)
    cols = np.concatenate([np.nonzero(S.solvable)[0] + q * t.npix for q in range(3)])
    m0 = random_map(11, 3, t.npix)
    m0[:, ~S.solvable] = 0
    m1 = messenger_step(S, t.d, m0, lam)
    eps0 = (m0 - ml).reshape(-1)[cols]
    eps1 = (m1 - ml).reshape(-1)[cols]
    np.testing.assert_allclose(eps1, F @ eps0, rtol=1e-8, atol=1e-9 * np.abs(eps0).max())


def test_noise_free_iterates_are_unbiased():
    """d = P m_true: after the lambda = inf step every iterate equals m_true at any lambda
    (Sections 2.1 and 3.1: an unbiased iterate stays unbiased)."""
    t = tiny_problem(12)
    S = _setup(t)
    m_true = random_map(13, 3, t.npix, 4.0)
    m_true[:, ~S.solvable] = 0
    d = S.pointing.project(m_true)
    m = random_map(14, 3, t.npix)
    for lam in cooling_schedule(4, 3, 500.0):
        m = messenger_step(S, d, m, lam)
        np.testing.assert_allclose(m, m_true, rtol=0, atol=1e-12 * np.abs(m_true).max())


def test_chi2_decreases_under_cooling():
    """chi^2(m, lambda) is non-increasing within a level and chi^2(m) non-increasing at lambda = 1."""
    t = tiny_problem(15, lengths=(64, 64), nx=4)
    S = _setup(t)
    lams = cooling_schedule(5, 6, lambda_max_rule(S))
    m = np.zeros((3, t.npix))
    prev = None
    for i, lam in enumerate(lams):
        m_new = messenger_step(S, t.d, m, lam)
        if i > 0 and lams[i - 1] == lam and not math.isinf(lam):
            c_old = chi2_lambda(S, t.d, m, lam)
            c_new = chi2_lambda(S, t.d, m_new, lam)
            assert c_new <= c_old * (1 + 1e-12)
        m = m_new
    # final level at lambda = 1: plain chi^2 non-increasing
    tail = [chi2(S, t.d, m)]
    for _ in range(5):
        m = messenger_step(S, t.d, m, 1.0)
        tail.append(chi2(S, t.d, m))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(tail, tail[1:]))


def test_chi2_matches_dense_quadratic_form():
    t = tiny_problem(16, lengths=(20, 17), nx=3)
    S = _setup(t)
    m = random_map(17, 3, t.npix)
    r = t.d - dense.pointing_matrix(S) @ m.reshape(-1)
    expect = r @ dense.noise_inverse_dense(S) @ r
    assert chi2(S, t.d, m) == pytest.approx(expect, rel=1e-12)
    for lam in (3.0, 50.0):
        expect_l = r @ dense.noise_inverse_dense(S, lam - 1.0) @ r
        assert chi2_lambda(S, t.d, m, lam) == pytest.approx(expect_l, rel=1e-12)


def test_weight_blocks_and_solvability():
    """W = P^T T^-1 P per pixel; a pixel seen at a single angle cannot separate Q from U."""
    n = 12
    pix = np.array([0] * 6 + [1] * 6, np.int32)
    psi = np.array([0.3] * 6 + [0.0, 0.5, 1.0, 1.5, 2.0, 2.5])
    pt = Pointing(pix, psi, npix=2, ncomp=3)
    W = pt.weight_blocks(np.full(n, 0.5))
    P = np.zeros((n, 6))
    for j in range(n):
        P[j, [pix[j], 2 + pix[j], 4 + pix[j]]] = [1, np.cos(2 * psi[j]), np.sin(2 * psi[j])]
    full = P.T @ (0.5 * P)
    for p in range(2):
        idx = [p, 2 + p, 4 + p]
        np.testing.assert_allclose(W[p], full[np.ix_(idx, idx)], rtol=1e-14, atol=1e-15)
    Winv, ok = invert_blocks(W, pt.hits())
    assert not ok[0] and ok[1]
    np.testing.assert_allclose(Winv[1] @ W[1], np.eye(3), atol=1e-12)
    assert np.all(Winv[0] == 0)


# ------------------------------------------------------------------------------------------------
# the comparison solver

def test_pcg_reaches_gls():
    t = tiny_problem(18, lengths=(40, 44), nx=3)
    S = _setup(t)
    m_gls = dense.gls(S, t.d)
    m, info = pcg_solve(S, t.d, maxiter=200, rtol=1e-14)
    assert np.linalg.norm(m - m_gls) / np.linalg.norm(m_gls) < 1e-9


def test_pcg_terminates_in_distinct_eigenvalue_count():
    """P = I, a spectrum with three distinct values and M^-1 = tau I: CG is exact after 3 steps."""
    n = 32
    vals = np.array([1.0, 4.0, 9.0])
    psd = vals[np.arange(n // 2 + 1) % 3]
    S, _ = _identity_problem(n, psd=psd)
    d = np.random.default_rng(19).standard_normal(n)
    m, info = pcg_solve(S, d, maxiter=3)
    np.testing.assert_allclose(m[0], d, rtol=1e-10, atol=1e-10)


def test_pcg_operator_is_symmetric():
    t = tiny_problem(20)
    S = _setup(t)
    x, y = random_map(1, 3, t.npix), random_map(2, 3, t.npix)
    x[:, ~S.solvable] = 0
    y[:, ~S.solvable] = 0
    assert np.sum(x * apply_A(S, y)) == pytest.approx(np.sum(y * apply_A(S, x)), rel=1e-11)


# ------------------------------------------------------------------------------------------------
# chi^2 per Fourier mode (the diagnostic of Section 3.1)

def test_mode_bin_hand_values():
    """Two bins per octave: k = 0 | 1 | (empty) | 2 | 3 | 4, 5 | 6, 7 | 8 ..."""
    from oracle.messenger import mode_bin
    got = [mode_bin(k, 2) for k in range(10)]
    assert got == [0, 1, 3, 4, 5, 5, 6, 6, 7, 7]
    assert [mode_bin(k, 1) for k in (1, 2, 3, 4, 7, 8, 1023, 1024)] == [1, 2, 2, 3, 3, 4, 10, 11]


def test_chi2_modes_pure_cosine_closed_form():
    """A residual that is one cosine at bin k0 puts all of chi^2 in bin(k0), with the closed form
    A^2 n / (2 N_k0) (n/2 from the rfft amplitude, a multiplicity of 2); the bins' mode counts add
    up to n."""
    from oracle.messenger import chi2_modes, mode_bin
    n, k0, A = 64, 11, 1.7
    N = noise_psd(n, 5.0, 1.1, 0.7, -1.7)
    nm = NoiseModel(chunk_off=np.array([0, n]), spectra=[N], tau=np.array([1.1 ** 2]))
    pt = Pointing(np.full(n, -1, np.int32), None, npix=1, ncomp=1)
    S = oracle.Setup(pointing=pt, noise=nm, W=np.zeros((1, 1, 1)), W_inv=np.zeros((1, 1, 1)),
                     solvable=np.zeros(1, bool), hits=np.zeros(1, np.int64))
    d = A * np.cos(2 * np.pi * k0 * np.arange(n) / n)
    terms, bins = chi2_modes(S, d, np.zeros((1, 1)), [0], per_octave=3)
    expect = A * A * n / (2 * N[k0])
    assert terms[0][k0] == pytest.approx(expect, rel=1e-12)
    assert bins[0, mode_bin(k0, 3), 0] == pytest.approx(expect, rel=1e-12)
    assert bins[0, :, 0].sum() == pytest.approx(expect, rel=1e-12)
    assert bins[0, :, 1].sum() == n


def test_chi2_modes_unit_mean_for_white_noise():
    """Data that are white noise of the modelled variance (N = sigma^2 at every bin when f_knee is
    far below f_1): every bin's mean term is 1 within 5 standard errors (each real mode's term is
    chi^2 with one degree of freedom: variance 2 per mode)."""
    from oracle.messenger import chi2_modes
    rng = np.random.default_rng(4)
    n = 4096
    nm = NoiseModel.from_params(np.array([0, n]), [100.0], [1.3], [1e-9], [-1.0])
    pt = Pointing(np.full(n, -1, np.int32), None, npix=1, ncomp=1)
    S = oracle.Setup(pointing=pt, noise=nm, W=np.zeros((1, 1, 1)), W_inv=np.zeros((1, 1, 1)),
                     solvable=np.zeros(1, bool), hits=np.zeros(1, np.int64))
    d = rng.standard_normal(n) * 1.3
    _, bins = chi2_modes(S, d, np.zeros((1, 1)), [0], per_octave=2)
    for s, cnt in bins[0]:
        if cnt >= 8:
            assert abs(s / cnt - 1.0) < 5 * np.sqrt(2.0 / cnt)
