"""Messenger mapmaking with a composite pointing matrix P = P_A + P_B (Section 2.2, Appendix B).

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Every sample j sees the sky through two single-pixel components (a differential
instrument: the two sides of a differencing assembly):

    (P m)_j = w_A a(psi_A,j) . m[p_A,j]  +  w_B a(psi_B,j) . m[p_B,j],

a(psi) = (1, cos 2 psi, sin 2 psi) (the first entry alone for temperature maps), and one
scalar weight per component (w_A = +1, w_B = -1 for a pure difference).  A component whose
pixel index is negative is absent from that sample (its row of P_A or P_B is zero).

The messenger covariance is split T_A = T_B = T / 2, the choice the paper tests
(Section 3.2): the block-diagonal matrix the update inverts is then

    W_AB = P_A^T T_A^-1 P_A + P_B^T T_B^-1 P_B = 2 (P_A^T T^-1 P_A + P_B^T T^-1 P_B),

one ncomp x ncomp block per pixel, and one iteration in the compact form (eqn. mdiffcompact) is

    m_{i+1} = m_i + W_AB^-1 P^T (lambda^-1 N-bar + T)^-1 (d - P m_i).

Unlike the single beam, F(lambda) = I - W_AB^-1 P^T (lambda^-1 N-bar + T)^-1 P does not vanish
at lambda = inf: the lambda = inf step, where the filter is T^-1, is a weighted Jacobi step
toward the binned solution (P^T T^-1 P)^-1 P^T T^-1 d (Section 2.2).

``CompositePointing`` has the interface of ``pointing.Pointing`` (project, back, hits), and
``make_composite_setup`` returns a ``messenger.Setup`` whose W / W_inv are W_AB and its
inverse, so the residual form, chi^2 and CG of ``messenger`` and ``cg`` apply unchanged.
The map-sized form (Appendix B) has its own functions here, since the single-beam ones use
W^-1 P^T T^-1 P = I, which W_AB does not satisfy.
"""

from __future__ import annotations

import math

import numpy as np

from .messenger import Setup, _hold_unsolvable, weighted_solve
from .noise import NoiseModel
from .pointing import Pointing, invert_blocks


class CompositePointing:
    """P = w_A P_A + w_B P_B with single-pixel components P_A, P_B (``Pointing``)."""

    def __init__(self, pix_a, psi_a, pix_b, psi_b, npix: int, ncomp: int, w_a: float = 1.0, w_b: float = -1.0):
        self.a = Pointing(pix_a, psi_a, npix, ncomp)
        self.b = Pointing(pix_b, psi_b, npix, ncomp)
        if self.a.nsamp != self.b.nsamp:
            raise ValueError("the two components must cover the same samples")
        self.w_a, self.w_b = float(w_a), float(w_b)
        self.npix, self.ncomp = int(npix), int(ncomp)

    @property
    def nsamp(self) -> int:
        return self.a.nsamp

    def project(self, m: np.ndarray) -> np.ndarray:
        return self.w_a * self.a.project(m) + self.w_b * self.b.project(m)

    def back(self, y: np.ndarray) -> np.ndarray:
        return self.w_a * self.a.back(y) + self.w_b * self.b.back(y)

    def hits(self) -> np.ndarray:
        """Pointing entries per pixel: the samples of either component that fall on it."""
        return self.a.hits() + self.b.hits()

    def split_weight_blocks(self, inv_var_per_sample: np.ndarray) -> np.ndarray:
        """W_AB = P_A^T (T/2)^-1 P_A + P_B^T (T/2)^-1 P_B for T^-1 = diag(inv_var_per_sample)."""
        v = 2.0 * np.asarray(inv_var_per_sample, dtype=np.float64)
        return self.w_a ** 2 * self.a.weight_blocks(v) + self.w_b ** 2 * self.b.weight_blocks(v)


def make_composite_setup(chunk_off, fsample, sigma, fknee, alpha, pix_a, psi_a, pix_b, psi_b, npix: int,
                         ncomp: int, w_a: float = 1.0, w_b: float = -1.0, tau=None, psd=None,
                         rcond_min: float = 1e-8) -> Setup:
    """A ``Setup`` for P = w_A P_A + w_B P_B with W = W_AB (T_A = T_B = T/2).  A pixel is solvable
    when it has pointing entries and its W_AB block passes the test of ``invert_blocks``."""
    noise = NoiseModel.from_params(chunk_off, fsample, sigma, fknee, alpha, tau=tau, psd=psd)
    pt = CompositePointing(pix_a, psi_a, pix_b, psi_b, npix, ncomp, w_a, w_b)
    if pt.nsamp != int(noise.chunk_off[-1]):
        raise ValueError("pointing and chunk table disagree on the number of samples")
    W = pt.split_weight_blocks(1.0 / noise.tau_per_sample())
    hits = pt.hits()
    W_inv, solvable = invert_blocks(W, hits, rcond_min)
    return Setup(pointing=pt, noise=noise, W=W, W_inv=W_inv, solvable=solvable, hits=hits)


def _gains(S: Setup, lam: float):
    """Per-chunk bin gains 1 / ((N_k - tau) / lambda + tau) of (lambda^-1 N-bar + T)^-1."""
    out = []
    for c in range(S.noise.nchunk):
        tau = float(S.noise.tau[c])
        nbar = S.noise.spectra[c] - tau
        out.append(1.0 / (nbar / lam + tau))
    return out


def _filter(S: Setup, x: np.ndarray, lam: float) -> np.ndarray:
    """(lambda^-1 N-bar + T)^-1 x (T^-1 x at lambda = inf)."""
    if math.isinf(lam):
        return np.asarray(x, dtype=np.float64) / S.noise.tau_per_sample()
    return S.noise.apply_spectral(np.asarray(x, dtype=np.float64), _gains(S, lam))


def composite_md(S: Setup, d: np.ndarray, lam: float) -> np.ndarray:
    """m_d(lambda) = W_AB^-1 P^T (lambda^-1 N-bar + T)^-1 d (Appendix B)."""
    return _hold_unsolvable(S, weighted_solve(S, S.pointing.back(_filter(S, d, lam))))


def composite_F(S: Setup, m: np.ndarray, lam: float) -> np.ndarray:
    """F(lambda) m = m - W_AB^-1 P^T (lambda^-1 N-bar + T)^-1 P m (Appendix B)."""
    m = np.asarray(m, dtype=np.float64).reshape(S.ncomp, S.npix)
    return m - weighted_solve(S, S.pointing.back(_filter(S, S.pointing.project(m), lam)))


def composite_step_mapsized(S: Setup, d: np.ndarray, m: np.ndarray, lam: float) -> np.ndarray:
    """m_{i+1} = m_d(lambda) + F(lambda) m_i, the map-sized form of Appendix B."""
    return _hold_unsolvable(S, composite_md(S, d, lam) + composite_F(S, m, lam))


# ---------------------------------------------------------------------------------------------
# explicit matrices for tiny problems (the brute-force route of Section 3.2)

def composite_pointing_matrix(S: Setup) -> np.ndarray:
    """P = w_A P_A + w_B P_B with one row per sample and column q * npix + p, entry by entry."""
    pt = S.pointing
    P = np.zeros((pt.nsamp, pt.ncomp * pt.npix))
    for comp, w in ((pt.a, pt.w_a), (pt.b, pt.w_b)):
        rows = np.nonzero(comp.on)[0]
        for q in range(pt.ncomp):
            np.add.at(P, (rows, q * pt.npix + comp.pix[rows]), w * comp.A[rows, q])
    return P


def normal_matrix_by_columns(S: Setup, cols: np.ndarray, extra_tau_factor: float = 0.0) -> np.ndarray:
    """P^T N'^-1 P restricted to the map entries ``cols`` (q * npix + p), one column at a time
    through the operators (N' = N + extra_tau_factor T), for problems too long for a dense N^-1."""
    gains = [1.0 / (S.noise.spectra[c] + extra_tau_factor * S.noise.tau[c]) for c in range(S.noise.nchunk)]
    out = np.empty((len(cols), len(cols)))
    for i, col in enumerate(cols):
        e = np.zeros(S.ncomp * S.npix)
        e[col] = 1.0
        y = S.noise.apply_spectral(S.pointing.project(e.reshape(S.ncomp, S.npix)), gains)
        out[:, i] = S.pointing.back(y).reshape(-1)[cols]
    return out


def pinv_solve(A: np.ndarray, b: np.ndarray, rtol: float):
    """Least-norm solution of A x = b keeping the eigenmodes of A above rtol * max (Section 3.2);
    returns (x, number of modes kept)."""
    w, V = np.linalg.eigh(A)
    keep = w > rtol * w.max()
    return V[:, keep] @ ((V[:, keep].T @ b) / w[keep]), int(keep.sum())
