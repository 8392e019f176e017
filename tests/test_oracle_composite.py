"""Pins of the composite-pointing oracle (Section 2.2, Section 3.2, Appendix B).

Each pin ties ``oracle.composite`` to something outside it: the dense matrices of the
definitions (P entry by entry, the circulant filter, the block matrix W_AB), the closed forms
the paper names (P_B = 0 gives back the single beam; the lambda = inf step is a weighted
Jacobi step), the brute-force pseudo-inverse of Section 3.2 (only the mean of a differential
map is unconstrained), the fixed points, and the monotone chi^2 that the split
T_A = T_B = T/2 guarantees.
"""

import math

import numpy as np
import pytest

from oracle import dense
from oracle.cg import pcg_solve
from oracle.composite import (composite_pointing_matrix, composite_step_mapsized, make_composite_setup,
                              normal_matrix_by_columns, pinv_solve)
from oracle.messenger import binned_map, chi2, chi2_lambda, make_setup, messenger_step
from synth import config_by_name, make_problem
from tests.tiny_inputs import random_map, tiny_composite

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def comp_setup(t, pix_b, psi_b, w, tau=None):
    return make_composite_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, pix_b, psi_b,
                                t.npix, t.ncomp, w_a=w[0], w_b=w[1], tau=tau)


def single_setup(t, tau=None):
    return make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, t.ncomp, tau=tau)


def dense_filter(S, lam):
    """(lambda^-1 N-bar + T)^-1 as an explicit block-circulant matrix (T^-1 at lambda = inf)."""
    ns = int(S.noise.chunk_off[-1])
    G = np.zeros((ns, ns))
    for c in range(S.noise.nchunk):
        a, b = int(S.noise.chunk_off[c]), int(S.noise.chunk_off[c + 1])
        tau = S.noise.tau[c]
        if math.isinf(lam):
            G[a:b, a:b] = np.eye(b - a) / tau
        else:
            G[a:b, a:b] = dense.circulant_inverse((S.noise.spectra[c] - tau) / lam + tau, b - a)
    return G


def dense_component(t, pix, psi, ncomp, npix):
    """One single-pixel component as a dense matrix, straight from the pointing weights
    (1, cos 2 psi, sin 2 psi)."""
    P = np.zeros((len(pix), ncomp * npix))
    for j, p in enumerate(pix):
        if p < 0:
            continue
        P[j, p] = 1.0
        if ncomp == 3:
            P[j, npix + p] = math.cos(2.0 * float(psi[j]))
            P[j, 2 * npix + p] = math.sin(2.0 * float(psi[j]))
    return P


@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("w", [(1.0, -1.0), (0.7, 1.3)])
@pytest.mark.parametrize("lam", [math.inf, 6.5, 1.0])
def test_step_matches_dense_definitions(ncomp, w, lam):
    t, pb, sb, _ = tiny_composite(3 + ncomp, ncomp=ncomp, weights=w)
    S = comp_setup(t, pb, sb, w)
    npix = t.npix
    PA = dense_component(t, t.pix, t.psi, ncomp, npix)
    PB = dense_component(t, pb, sb, ncomp, npix)
    P = w[0] * PA + w[1] * PB
    assert np.allclose(composite_pointing_matrix(S), P, rtol=0, atol=1e-15)
    tau = np.repeat(S.noise.tau, np.diff(S.noise.chunk_off))
    Ta_inv = np.diag(2.0 / tau)                  # T_A = T_B = T / 2
    W_AB = (w[0] * PA).T @ Ta_inv @ (w[0] * PA) + (w[1] * PB).T @ Ta_inv @ (w[1] * PB)
    # the oracle's per-pixel blocks are the diagonal blocks of the dense W_AB (which has no others)
    for p in range(npix):
        idx = [q * npix + p for q in range(ncomp)]
        assert np.allclose(S.W[p], W_AB[np.ix_(idx, idx)], rtol=1e-13, atol=1e-13)
    cols = np.concatenate([np.nonzero(S.solvable)[0] + q * npix for q in range(ncomp)])
    m0 = random_map(11, ncomp, npix)
    m0[:, ~S.solvable] = 0.0
    d = np.asarray(t.d, dtype=np.float64)
    G = dense_filter(S, lam)
    upd = np.linalg.solve(W_AB[np.ix_(cols, cols)], P[:, cols].T @ G @ (d - P @ m0.reshape(-1)))
    want = m0.reshape(-1).copy()
    want[cols] += upd
    got = messenger_step(S, t.d, m0, lam).reshape(-1)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    # the map-sized form of Appendix B gives the same step (Woodbury)
    got2 = composite_step_mapsized(S, t.d, m0, lam).reshape(-1)
    assert np.linalg.norm(got2 - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_no_second_component_is_the_single_beam_with_half_tau(ncomp):
    """P_B = 0: at lambda = 1 the composite step equals the single-beam step with messenger
    covariance T_A = T/2 (end of Appendix B)."""
    t, pb, sb, w = tiny_composite(21, b_mode="none", ncomp=ncomp, weights=(1.0, -1.0))
    S = comp_setup(t, pb, sb, w)
    tau = t.sigma ** 2 * 0.8
    S = comp_setup(t, pb, sb, w, tau=tau)
    S1 = single_setup(t, tau=tau / 2)
    assert np.array_equal(S.solvable, S1.solvable) and np.array_equal(S.hits, S1.hits)
    m0 = random_map(5, ncomp, t.npix)
    a = messenger_step(S, t.d, m0, 1.0)
    b = messenger_step(S1, t.d, m0, 1.0)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_no_second_component_lambda_inf_is_half_weight_jacobi(ncomp):
    """P_B = 0: W_AB = 2 P^T T^-1 P, so K lambda = inf steps give m_bin + 2^-K (m_0 - m_bin)."""
    t, pb, sb, w = tiny_composite(22, b_mode="none", ncomp=ncomp)
    S = comp_setup(t, pb, sb, w)
    m_bin = binned_map(single_setup(t), t.d)
    m = random_map(6, ncomp, t.npix)
    m[:, ~S.solvable] = 0.0
    m0 = m.copy()
    for K in range(1, 6):
        m = messenger_step(S, t.d, m, math.inf)
        want = m_bin + 2.0 ** -K * (m0 - m_bin)
        assert np.linalg.norm(m - want) <= 1e-13 * np.linalg.norm(want)


@pytest.mark.parametrize("ncomp", [1, 3])
def test_identical_components_lambda_inf_gives_half_the_binned_map(ncomp):
    """P_B = P_A with weights (1, 1): P = 2 P_A and W_AB = P^T T^-1 P, so F(inf) = 0 and one
    lambda = inf step gives (P^T T^-1 P)^-1 P^T T^-1 d = m_bin(P_A) / 2 from any start."""
    t, pb, sb, w = tiny_composite(23, b_mode="same", ncomp=ncomp, weights=(1.0, 1.0))
    S = comp_setup(t, pb, sb, w)
    m_bin = binned_map(single_setup(t), t.d)
    got = messenger_step(S, t.d, random_map(7, ncomp, t.npix, 5.0), math.inf)
    assert np.linalg.norm(got - 0.5 * m_bin) <= 1e-13 * np.linalg.norm(m_bin)


def test_differential_fixed_points_are_the_pseudo_inverse_solutions():
    """Differential (w = +1, -1) temperature map: the mean is a null mode of P^T N^-1 P.  The
    least-norm solutions of Section 3.2's brute force, m(lambda) = (P^T N'^-1 P)^+ P^T N'^-1 d,
    are fixed points of the iteration at lambda (lambda = 1: the GLS map)."""
    t, pb, sb, w = tiny_composite(31, ncomp=1, flag_b=0.0, flag_frac=0.0, lengths=(96, 64))
    S = comp_setup(t, pb, sb, w)
    cols = np.nonzero(S.solvable)[0]
    d = np.asarray(t.d, dtype=np.float64)
    P = composite_pointing_matrix(S)[:, cols]
    for lam in (1.0, 5.0):
        Ninv = dense.noise_inverse_dense(S, lam - 1.0)
        A = P.T @ Ninv @ P
        x, kept = pinv_solve(A, P.T @ Ninv @ d, 1e-10)
        assert kept == len(cols) - 1          # only the mean is lost
        m = np.zeros((1, t.npix))
        m[0, cols] = x
        step = messenger_step(S, t.d, m, lam)
        assert np.linalg.norm(step - m) <= 1e-10 * np.linalg.norm(m)


def test_noise_free_differential_map_is_a_fixed_point_and_jacobi_converges_to_it():
    """d = P m_true: m_true is a fixed point at every lambda, and repeated lambda = inf steps from
    zero approach m_true up to the unconstrained mean (Section 2.2: a weighted Jacobi method
    toward the binned solution)."""
    t, pb, sb, w = tiny_composite(32, ncomp=1, flag_b=0.0, flag_frac=0.0, lengths=(96, 64))
    S = comp_setup(t, pb, sb, w)
    m_true = random_map(8, 1, t.npix, 3.0)
    m_true[:, ~S.solvable] = 0.0
    d = S.pointing.project(m_true)
    for lam in (math.inf, 20.0, 1.0):
        assert np.linalg.norm(messenger_step(S, d, m_true, lam) - m_true) <= 1e-13 * np.linalg.norm(m_true)
    m = np.zeros_like(m_true)
    for _ in range(3000):
        m = messenger_step(S, d, m, math.inf)
    e = (m - m_true)[:, S.solvable]
    e -= e.mean()
    assert np.linalg.norm(e) <= 1e-8 * np.linalg.norm(m_true)


@pytest.mark.parametrize("lam", [40.0, 4.0, 1.0])
def test_chi2_never_increases_inside_a_level(lam):
    """With T_A = T_B = T/2, A_lambda <= P^T T^-1 P <= W_AB ((a+b)^2 <= 2a^2 + 2b^2), so the
    argument of the single beam applies: chi^2(m_i, lambda) is non-increasing inside a level."""
    t, pb, sb, w = tiny_composite(33, ncomp=3, weights=(1.0, -1.0))
    S = comp_setup(t, pb, sb, w)
    m = random_map(9, 3, t.npix, 10.0)
    prev = chi2_lambda(S, t.d, m, lam)
    for _ in range(12):
        m = messenger_step(S, t.d, m, lam)
        cur = chi2_lambda(S, t.d, m, lam)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_brute_force_rank_on_the_differential_scan():
    """Section 3.2's low-resolution brute force on the synthetic differential scan: tabulating
    P^T N^-1 P over the observed pixels leaves exactly one poorly constrained mode, the mean."""
    cfg = config_by_name("diff256").scaled("diff_rank", ndet=4, nsamp=1 << 13, nx=24, diff_sep=2.0)
    pr = make_problem(cfg)
    S = make_composite_setup(pr.chunk_off, pr.fsample, pr.sigma, pr.fknee, pr.alpha, pr.pix, None, pr.pix_b, None,
                             pr.npix, 1, w_a=pr.weights[0], w_b=pr.weights[1])
    cols = np.nonzero(S.solvable)[0]
    A = normal_matrix_by_columns(S, cols)
    ev, V = np.linalg.eigh(A)
    assert np.sum(ev > 1e-9 * ev.max()) == len(cols) - 1
    null = V[:, 0]
    assert abs(null.sum()) / (np.linalg.norm(null) * math.sqrt(len(cols))) > 1 - 1e-9


def test_pcg_on_the_composite_operator_reaches_the_least_squares_chi2():
    t, pb, sb, w = tiny_composite(34, ncomp=1, flag_b=0.0, flag_frac=0.0, lengths=(96, 64))
    S = comp_setup(t, pb, sb, w)
    cols = np.nonzero(S.solvable)[0]
    d = np.asarray(t.d, dtype=np.float64)
    P = composite_pointing_matrix(S)[:, cols]
    Ninv = dense.noise_inverse_dense(S)
    x, _ = pinv_solve(P.T @ Ninv @ P, P.T @ Ninv @ d, 1e-10)
    m_ls = np.zeros((1, t.npix))
    m_ls[0, cols] = x
    m, _ = pcg_solve(S, t.d, 200, rtol=1e-14)
    c_ls, c_cg = chi2(S, t.d, m_ls), chi2(S, t.d, m)
    assert abs(c_cg - c_ls) <= 1e-10 * c_ls
