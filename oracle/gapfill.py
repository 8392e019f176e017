"""Messenger mapmaking with composite timestream noise N = N_0 + N_1: gap filling (Appendix C).

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The noise is split into a stationary part N_0 (diagonal in the Fourier domain) and a part N_1
diagonal in the time domain with infinite variance in the gaps (samples whose data are
unusable) and a small variance eps_c elsewhere.  Reading used here (the paper leaves the split
open): N_0 = N - eps_c I with N the chunk's usual noise law, so that outside the gaps
N_0 + N_1 = N and the fixed point is the generalised least-squares map of the samples outside
the gaps, with their noise covariance N restricted to them.

Four fields are iterated, each set to its conditional mean given the others, in the order the
appendix lists them (eqns. 2mess_t1, 2mess_d0, 2mess_t0, 2mess_m):

    t_1 = (N-bar_1^-1 + T_1^-1)^-1 (N-bar_1^-1 d + T_1^-1 d_0)
    d_0 = (N-bar_0^-1 + T_1^-1)^-1 (N-bar_0^-1 t_0 + T_1^-1 t_1)
    t_0 = (N-bar_0^-1 + (lambda T_0)^-1)^-1 (N-bar_0^-1 d_0 + (lambda T_0)^-1 P m)
    m   = (P^T T_0^-1 P)^-1 P^T T_0^-1 t_0

with N-bar_i = N_i - T_i.  They are the block-coordinate minimisers of

    chi^2_1 = (d - t_1)^T N-bar_1^-1 (d - t_1) + (t_1 - d_0)^T T_1^-1 (t_1 - d_0)
            + (d_0 - t_0)^T N-bar_0^-1 (d_0 - t_0) + (t_0 - P m)^T (lambda T_0)^-1 (t_0 - P m),

whose marginal over t_1, d_0 and t_0 is the mapmaking chi^2 with N'(lambda) = N + (lambda - 1) T_0
(lambda enters as in Section 2.1, on the messenger covariance next to the map).  Choices:

* T_1 = eps_c I, the largest allowed (N-bar_1 = N_1 - T_1 >= 0): N-bar_1 is then zero outside the
  gaps and infinite inside, and the t_1 update is the selection t_1 = d outside the gaps,
  t_1 = d_0 inside;
* T_0 = tau_0 I with tau_0 = sigma_c^2 - eps_c, the largest allowed (N-bar_0 >= 0): N-bar_0 is then
  the power-law part sigma^2 (f/f_knee)^alpha of the spectrum (the DC bin clamped as elsewhere);
* start: d_0 = d outside the gaps and 0 inside, t_0 = d_0.

d_0 is the gap-filled time-ordered data: inside the gaps it converges to the prediction of the
data there from the map and the samples around them.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .messenger import Setup, _hold_unsolvable, make_setup, weighted_solve


@dataclass
class GapSetup:
    S: Setup                # pointing, noise N, W_0 = P^T T_0^-1 P (tau = tau_0 = sigma^2 - eps)
    gaps: np.ndarray        # bool [N_s]
    eps: np.ndarray         # float64 [nchunk]
    sigma2: np.ndarray      # float64 [nchunk]

    def per_sample(self, v) -> np.ndarray:
        return np.repeat(np.asarray(v, dtype=np.float64), np.diff(self.S.noise.chunk_off))

    def nbar0(self, c: int) -> np.ndarray:
        """N-bar_0 = N_0 - T_0 = N - sigma^2 at the real bins of chunk c."""
        return self.S.noise.spectra[c] - self.sigma2[c]


def make_gap_setup(chunk_off, fsample, sigma, fknee, alpha, pix, psi, npix: int, ncomp: int, gaps, eps) -> GapSetup:
    sigma = np.asarray(sigma, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    if np.any(eps <= 0) or np.any(eps >= sigma ** 2):
        raise ValueError("eps must lie in (0, sigma^2)")
    S = make_setup(chunk_off, fsample, sigma, fknee, alpha, pix, psi, npix, ncomp, tau=sigma ** 2 - eps)
    return GapSetup(S=S, gaps=np.asarray(gaps, dtype=bool), eps=eps, sigma2=sigma ** 2)


def gap_init(G: GapSetup, d: np.ndarray):
    """The starting messenger fields (d_0, t_0)."""
    d0 = np.where(G.gaps, 0.0, np.asarray(d, dtype=np.float64))
    return d0, d0.copy()


def _spectral(G: GapSetup, x: np.ndarray, gain_of_chunk) -> np.ndarray:
    return G.S.noise.apply_spectral(x, [gain_of_chunk(c) for c in range(G.S.noise.nchunk)])


def update_t1(G: GapSetup, d: np.ndarray, d0: np.ndarray) -> np.ndarray:
    """t_1: the data outside the gaps, d_0 inside (N-bar_1 = 0 outside, infinite inside)."""
    return np.where(G.gaps, d0, np.asarray(d, dtype=np.float64))


def update_d0(G: GapSetup, t0: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """d_0: per Fourier bin the weights N-bar_0^-1 and T_1^-1 = 1/eps, written as
    eps / (eps + N-bar_0) on t_0 and N-bar_0 / (eps + N-bar_0) on t_1."""
    return (_spectral(G, t0, lambda c: G.eps[c] / (G.eps[c] + G.nbar0(c)))
            + _spectral(G, t1, lambda c: G.nbar0(c) / (G.eps[c] + G.nbar0(c))))


def update_t0(G: GapSetup, d0: np.ndarray, m: np.ndarray, lam: float) -> np.ndarray:
    """t_0: the weights N-bar_0^-1 and (lambda tau_0)^-1; at lambda = inf the map side drops out."""
    if math.isinf(lam):
        return d0.copy()
    S = G.S
    lt = lam * S.noise.tau
    return (_spectral(G, d0, lambda c: lt[c] / (lt[c] + G.nbar0(c)))
            + _spectral(G, S.pointing.project(m), lambda c: G.nbar0(c) / (lt[c] + G.nbar0(c))))


def update_m(G: GapSetup, t0: np.ndarray) -> np.ndarray:
    """m: the binned t_0 with weights 1 / tau_0."""
    S = G.S
    return _hold_unsolvable(S, weighted_solve(S, S.pointing.back(t0 / S.noise.tau_per_sample())))


def gap_step(G: GapSetup, d: np.ndarray, m: np.ndarray, d0: np.ndarray, t0: np.ndarray, lam: float):
    """One pass over the four updates in the appendix's order; returns (m, d_0, t_0)."""
    t1 = update_t1(G, d, d0)
    d0 = update_d0(G, t0, t1)
    t0 = update_t0(G, d0, m, lam)
    return update_m(G, t0), d0, t0


def gap_solve(G: GapSetup, d: np.ndarray, lambdas, m0=None):
    """Iterate over the lambda sequence from the starting fields; returns (m, d_0, t_0)."""
    S = G.S
    m = np.zeros((S.ncomp, S.npix)) if m0 is None else np.asarray(m0, dtype=np.float64).reshape(S.ncomp, S.npix)
    d0, t0 = gap_init(G, d)
    for lam in lambdas:
        m, d0, t0 = gap_step(G, d, m, d0, t0, lam)
    return m, d0, t0


def augmented_chi2(G: GapSetup, d, m, d0, t0, t1, lam: float) -> float:
    """chi^2_1 of the four fields (the N-bar_1 term is zero for t_1 equal to d outside the gaps and
    is the constraint that fixes it there; finite lambda)."""
    S = G.S
    d64 = np.asarray(d, dtype=np.float64)
    if np.any(t1[~G.gaps] != d64[~G.gaps]):
        return math.inf
    e = G.per_sample(G.eps)
    out = float(np.sum((t1 - d0) ** 2 / e))
    r = d0 - t0
    for c in range(S.noise.nchunk):
        a, b = int(S.noise.chunk_off[c]), int(S.noise.chunk_off[c + 1])
        n = b - a
        rh = np.fft.rfft(r[a:b])
        w = np.full(n // 2 + 1, 2.0)
        w[0] = 1.0
        if n % 2 == 0:
            w[-1] = 1.0
        out += float(np.sum(w * (rh.real ** 2 + rh.imag ** 2) / G.nbar0(c)) / n)
    q = t0 - S.pointing.project(m)
    out += float(np.sum(q ** 2 / (lam * S.noise.tau_per_sample())))
    return out
