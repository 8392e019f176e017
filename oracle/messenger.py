"""The messenger-field mapmaking iteration (Section 2.1) and its chi^2 (Section 2).

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Notation follows the paper: d data, P pointing, m map, N noise covariance,
T = tau I per chunk the messenger covariance, N-bar = N - T, lambda the
cooling parameter, W = P^T T^-1 P (block diagonal, one block per pixel).

Three algebraically equal forms of one iteration are implemented:

* ``messenger_step``            compact residual form, eqn. (mcompact):
      m_{i+1} = m_i + W^-1 P^T (lambda^-1 N-bar + T)^-1 (d - P m_i)
* ``messenger_step_two_equation`` the two-equation form that opens Section 2.1:
      t_i = (N-bar^-1 + (lambda T)^-1)^-1 (N-bar^-1 d + (lambda T)^-1 P m_i),
      m_{i+1} = W^-1 P^T T^-1 t_i
* ``messenger_step_mapsized``   the map-sized form, eqns. (mapsized), (md) and the
      first line of (F): m_{i+1} = m_d(lambda) + F(lambda) m_i

Unsolvable pixels (see ``pointing.invert_blocks``) are held at zero by all
three.  The residual form is the one the library computes; the other two are
cross-checks.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from .noise import NoiseModel, chi2_weights, messenger_filter
from .pointing import Pointing, invert_blocks


@dataclass
class Setup:
    pointing: Pointing
    noise: NoiseModel
    W: np.ndarray            # [npix, ncomp, ncomp]  P^T T^-1 P
    W_inv: np.ndarray        # [npix, ncomp, ncomp]  zero blocks where unsolvable
    solvable: np.ndarray     # bool [npix]
    hits: np.ndarray         # int64 [npix]

    @property
    def ncomp(self) -> int:
        return self.pointing.ncomp

    @property
    def npix(self) -> int:
        return self.pointing.npix


def make_setup(chunk_off, fsample, sigma, fknee, alpha, pix, psi, npix: int, ncomp: int,
               tau=None, psd=None, rcond_min: float = 1e-8) -> Setup:
    noise = NoiseModel.from_params(chunk_off, fsample, sigma, fknee, alpha, tau=tau, psd=psd)
    pt = Pointing(pix, psi, npix, ncomp)
    if pt.nsamp != int(noise.chunk_off[-1]):
        raise ValueError("pointing and chunk table disagree on the number of samples")
    W = pt.weight_blocks(1.0 / noise.tau_per_sample())
    hits = pt.hits()
    W_inv, solvable = invert_blocks(W, hits, rcond_min)
    return Setup(pointing=pt, noise=noise, W=W, W_inv=W_inv, solvable=solvable, hits=hits)


def setup_from_problem(prob, tau=None, psd=None) -> Setup:
    """Convenience: build a Setup from a ``synth.Problem``'s arrays."""
    return make_setup(prob.chunk_off, prob.fsample, prob.sigma, prob.fknee, prob.alpha, prob.pix,
                      prob.psi_values(), prob.npix, prob.ncomp, tau=tau, psd=psd)


# ---------------------------------------------------------------------------------------------
# building blocks

def weighted_solve(S: Setup, b: np.ndarray) -> np.ndarray:
    """W^-1 b pixel by pixel (zero where unsolvable)."""
    b = np.asarray(b, dtype=np.float64).reshape(S.ncomp, S.npix)
    return np.einsum("pqr,rp->qp", S.W_inv, b)


def residual(S: Setup, d: np.ndarray, m: np.ndarray) -> np.ndarray:
    """d - P m, with d promoted to float64 from whatever type it is stored in."""
    return np.asarray(d, dtype=np.float64) - S.pointing.project(m)


def apply_filter(S: Setup, x: np.ndarray, lam: float) -> np.ndarray:
    """(lambda^-1 N-bar + T)^-1 x, chunk by chunk in the Fourier domain."""
    gains = [messenger_filter(S.noise.spectra[c], float(S.noise.tau[c]), lam) for c in range(S.noise.nchunk)]
    if math.isinf(lam):
        return np.asarray(x, dtype=np.float64) / S.noise.tau_per_sample()
    return S.noise.apply_spectral(x, gains)


def chi2_of_residual(S: Setup, r: np.ndarray, lam: float = 1.0, per_chunk: bool = False):
    """r^T N'(lambda)^-1 r as a sum over Fourier modes, N' = N + (lambda - 1) T (Section 2.1).

    With the unnormalised rfft r-hat of each chunk of length n:
        chi^2 = sum_c (1/n_c) sum_k omega_k |r-hat_{c,k}|^2 / N'_{c,k},
    omega_k the bin multiplicity.  lambda = 1 gives eqn. (chi2).
    """
    out = np.empty(S.noise.nchunk)
    for c in range(S.noise.nchunk):
        a, b = int(S.noise.chunk_off[c]), int(S.noise.chunk_off[c + 1])
        n = b - a
        rh = np.fft.rfft(np.asarray(r[a:b], dtype=np.float64))
        Np = S.noise.spectra[c] + (lam - 1.0) * S.noise.tau[c]
        out[c] = np.sum(chi2_weights(n) * (rh.real ** 2 + rh.imag ** 2) / Np) / n
    return out if per_chunk else float(out.sum())


def mode_bin(k: int, per_octave: int) -> int:
    """Log-spaced bin of real Fourier bin k: 0 for k = 0, else 1 + s*o + floor(s*(k - 2^o)/2^o)
    with o = floor(log2 k) and s bins per octave."""
    if k == 0:
        return 0
    o = k.bit_length() - 1
    return 1 + per_octave * o + (per_octave * (k - (1 << o))) // (1 << o)


def chi2_modes(S: Setup, d: np.ndarray, m: np.ndarray, chunks, per_octave: int, lam: float = 1.0):
    """chi^2 mode by mode for the listed chunks (Section 3.1 examines it per Fourier mode: each
    term |r-hat_k|^2 / (n N'_k) has unit mean under the right noise model).

    Returns (terms, bins): terms[i] = omega_k |r-hat_k|^2 / (n N'_k) for k = 0..n/2 of chunk i
    (they sum to its chi^2), and bins [len(chunks), nbins, 2] with the sum of the terms in each
    log-spaced bin (mode_bin) and the number of real modes they stand for (sum of omega_k).
    """
    r = residual(S, d, m)
    nm = max(int(S.noise.chunk_off[c + 1] - S.noise.chunk_off[c]) // 2 for c in chunks)
    nbins = 1 + per_octave * nm.bit_length()
    terms, bins = [], np.zeros((len(chunks), nbins, 2))
    for i, c in enumerate(chunks):
        a, b = int(S.noise.chunk_off[c]), int(S.noise.chunk_off[c + 1])
        n = b - a
        rh = np.fft.rfft(r[a:b])
        w = chi2_weights(n)
        t = w * (rh.real ** 2 + rh.imag ** 2) / (n * (S.noise.spectra[c] + (lam - 1.0) * S.noise.tau[c]))
        terms.append(t)
        for k in range(n // 2 + 1):
            j = mode_bin(k, per_octave)
            bins[i, j, 0] += t[k]
            bins[i, j, 1] += w[k]
    return terms, bins


def chi2(S: Setup, d: np.ndarray, m: np.ndarray, per_chunk: bool = False):
    """chi^2(m) = (d - P m)^T N^-1 (d - P m), eqn. (chi2), evaluated over Fourier modes."""
    return chi2_of_residual(S, residual(S, d, m), 1.0, per_chunk)


def chi2_lambda(S: Setup, d: np.ndarray, m: np.ndarray, lam: float) -> float:
    """chi^2(m, lambda) with N'(lambda) = N + (lambda - 1) T (Section 2.1)."""
    return chi2_of_residual(S, residual(S, d, m), lam)


def _hold_unsolvable(S: Setup, m: np.ndarray) -> np.ndarray:
    m = m.copy()
    m[:, ~S.solvable] = 0.0
    return m


# ---------------------------------------------------------------------------------------------
# the iteration

def messenger_step(S: Setup, d: np.ndarray, m: np.ndarray, lam: float) -> np.ndarray:
    """One iteration of the compact residual form, eqn. (mcompact)."""
    m = np.asarray(m, dtype=np.float64).reshape(S.ncomp, S.npix)
    r = residual(S, d, m)                     # d - P m_i
    y = apply_filter(S, r, lam)               # (lambda^-1 N-bar + T)^-1 (d - P m_i)
    b = S.pointing.back(y)                    # P^T ...
    return _hold_unsolvable(S, m + weighted_solve(S, b))


def messenger_step_two_equation(S: Setup, d: np.ndarray, m: np.ndarray, lam: float) -> np.ndarray:
    """One iteration of the two-equation form (messenger field t, then the map).

    Per Fourier bin the first equation weights the data and the projected map by
    (1/N-bar) / (1/N-bar + 1/(lambda tau)) and (1/(lambda tau)) / (1/N-bar + 1/(lambda tau));
    both are written with numerator and denominator multiplied by N-bar lambda tau so
    that a bin with N-bar = 0 (all noise in T) gives t = d there.
    """
    m = np.asarray(m, dtype=np.float64).reshape(S.ncomp, S.npix)
    Pm = S.pointing.project(m)
    d64 = np.asarray(d, dtype=np.float64)
    if math.isinf(lam):
        t = d64.copy()
    else:
        wd, wm = [], []
        for c in range(S.noise.nchunk):
            nbar = S.noise.spectra[c] - S.noise.tau[c]
            lt = lam * S.noise.tau[c]
            wd.append(lt / (nbar + lt))
            wm.append(nbar / (nbar + lt))
        t = S.noise.apply_spectral(d64, wd) + S.noise.apply_spectral(Pm, wm)
    b = S.pointing.back(t / S.noise.tau_per_sample())   # P^T T^-1 t
    return _hold_unsolvable(S, weighted_solve(S, b))


def messenger_step_mapsized(S: Setup, d: np.ndarray, m: np.ndarray, lam: float) -> np.ndarray:
    """m_d(lambda) + F(lambda) m with m_d from eqn. (md) (first line) and F from eqn. (F) (second line)."""
    m = np.asarray(m, dtype=np.float64).reshape(S.ncomp, S.npix)
    return _hold_unsolvable(S, mapsized_md(S, d, lam) + mapsized_F(S, m, lam))


def mapsized_md(S: Setup, d: np.ndarray, lam: float) -> np.ndarray:
    """m_d(lambda) = W^-1 P^T T^-1 (N-bar^-1 + (lambda T)^-1)^-1 N-bar^-1 d."""
    d64 = np.asarray(d, dtype=np.float64)
    if math.isinf(lam):
        t = d64
    else:
        gains = []
        for c in range(S.noise.nchunk):
            nbar = S.noise.spectra[c] - S.noise.tau[c]
            lt = lam * S.noise.tau[c]
            gains.append(lt / (nbar + lt))          # (N-bar^-1 + (lambda tau)^-1)^-1 N-bar^-1 per bin
        t = S.noise.apply_spectral(d64, gains)
    return weighted_solve(S, S.pointing.back(t / S.noise.tau_per_sample()))


def mapsized_F(S: Setup, m: np.ndarray, lam: float) -> np.ndarray:
    """F(lambda) m = W^-1 P^T T^-1 (I + lambda T N-bar^-1)^-1 P m."""
    if math.isinf(lam):
        return np.zeros_like(m)
    Pm = S.pointing.project(m)
    gains = []
    for c in range(S.noise.nchunk):
        nbar = S.noise.spectra[c] - S.noise.tau[c]
        lt = lam * S.noise.tau[c]
        gains.append(nbar / (nbar + lt))             # (I + lambda tau N-bar^-1)^-1 per bin
    t = S.noise.apply_spectral(Pm, gains)
    return weighted_solve(S, S.pointing.back(t / S.noise.tau_per_sample()))


def binned_map(S: Setup, d: np.ndarray) -> np.ndarray:
    """W^-1 P^T T^-1 d, the large-lambda limit of Section 2.1 (a weighted co-addition)."""
    b = S.pointing.back(np.asarray(d, dtype=np.float64) / S.noise.tau_per_sample())
    return _hold_unsolvable(S, weighted_solve(S, b))


# ---------------------------------------------------------------------------------------------
# cooling schedule and the full solve

def lambda_max_rule(S: Setup) -> float:
    """Top cooling level: lambda tau reaches the largest noise power (Section 3.1)."""
    return float(max((S.noise.spectra[c].max() / S.noise.tau[c]) for c in range(S.noise.nchunk)))


def cooling_schedule(nlevel: int, iters_per_level: int, lambda_max: float, first_inf: bool = True) -> List[float]:
    """One lambda = inf step, then nlevel levels with lambda tau log-spaced from lambda_max tau
    down to tau (lambda = 1 last), iters_per_level iterations each (Section 3.1)."""
    lams: List[float] = [math.inf] if first_inf else []
    for j in range(nlevel):
        if nlevel == 1:
            lam = 1.0
        else:
            lam = lambda_max ** ((nlevel - 1 - j) / (nlevel - 1))
        lams.extend([lam] * iters_per_level)
    return lams


def messenger_solve(S: Setup, d: np.ndarray, lambdas: Sequence[float], m0: Optional[np.ndarray] = None,
                    record_chi2: bool = True):
    """Iterate the residual form over the given lambda sequence.

    Returns (m, chi2_history) where chi2_history[i] = chi^2(m_i) for the map that entered
    iteration i, plus chi^2 of the final map as the last entry.
    """
    m = np.zeros((S.ncomp, S.npix)) if m0 is None else np.asarray(m0, dtype=np.float64).reshape(S.ncomp, S.npix).copy()
    hist = []
    for lam in lambdas:
        if record_chi2:
            hist.append(chi2(S, d, m))
        m = messenger_step(S, d, m, lam)
    if record_chi2:
        hist.append(chi2(S, d, m))
    return m, np.array(hist)
