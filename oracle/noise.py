"""Noise model, messenger covariance and the spectral filters of the iteration.

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Readings of the paper used here (each also listed with the design notes):

* The noise covariance of one detector chunk is taken to be exactly circulant,
  i.e. diagonal in the discrete Fourier basis of that chunk (Section 2 treats
  stationary noise as nearly so).  Its eigenvalue at rfft
  bin k is N_k, in per-sample-variance units: white noise of per-sample
  standard deviation sigma has N_k = sigma^2 at every k.
* The power law is the one of the simulation section (Section 2.3),
  N(f) = sigma^2 (1 + (f / f_knee)^alpha), with the slope alpha a per-chunk
  parameter (the paper fixes it at -2).  f_k = k f_s / n.  The f = 0 bin, where
  the law diverges, takes the value at the first nonzero frequency f_1.
* The messenger covariance is T = tau_c I on chunk c (Section 2.1, and
  piecewise per detector in Section 4.2).  Its default is tau_c = sigma_c^2,
  the minimum of the chunk's noise spectrum, so N-bar = N - T stays positive
  semidefinite (Section 2.1 requires tau not to exceed the minimum noise).
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np


def noise_psd(n: int, fs: float, sigma: float, fknee: float, alpha: float) -> np.ndarray:
    """N_k for k = 0 .. n//2 from the Section 2.3 power law, DC bin clamped to f_1."""
    if n < 2:
        raise ValueError("chunk too short")
    f = np.arange(n // 2 + 1, dtype=np.float64) * (fs / n)
    f[0] = f[1]
    return sigma * sigma * (1.0 + (f / fknee) ** alpha)


def chi2_weights(n: int) -> np.ndarray:
    """Multiplicity of each rfft bin in the full length-n spectrum.

    The bins k and n-k of a real signal carry the same power, so every bin
    counts twice except k = 0 and, for even n, k = n/2.
    """
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    return w


def messenger_filter(N: np.ndarray, tau: float, lam: float) -> np.ndarray:
    """Eigenvalues of (lambda^-1 N-bar + T)^-1 with N-bar = N - T (Section 2.1, eqn. mcompact).

    lambda = inf gives T^-1 (the limit of Section 2.1 where F vanishes).
    """
    if math.isinf(lam):
        return np.full_like(N, 1.0 / tau)
    nbar = N - tau
    return 1.0 / (nbar / lam + tau)


@dataclass
class NoiseModel:
    """Per-chunk noise spectra and messenger variances."""
    chunk_off: np.ndarray            # int64 [nchunk+1]
    spectra: List[np.ndarray]        # N_k per chunk, k = 0..n_c//2
    tau: np.ndarray                  # float64 [nchunk]

    @classmethod
    def from_params(cls, chunk_off, fsample, sigma, fknee, alpha, tau=None, psd: Optional[Sequence] = None):
        chunk_off = np.asarray(chunk_off, dtype=np.int64)
        nchunk = len(chunk_off) - 1
        spectra = []
        for c in range(nchunk):
            n = int(chunk_off[c + 1] - chunk_off[c])
            if psd is not None and psd[c] is not None:
                spec = np.asarray(psd[c], dtype=np.float64)
                if spec.shape != (n // 2 + 1,):
                    raise ValueError("tabulated spectrum has the wrong length")
            else:
                spec = noise_psd(n, float(fsample[c]), float(sigma[c]), float(fknee[c]), float(alpha[c]))
            spectra.append(spec)
        if tau is None:
            if psd is None:
                tau = np.asarray(sigma, dtype=np.float64) ** 2
            else:
                tau = np.array([s.min() for s in spectra])
        tau = np.asarray(tau, dtype=np.float64)
        for c in range(nchunk):
            if tau[c] <= 0 or tau[c] > spectra[c].min() * (1 + 1e-12):
                raise ValueError("messenger variance must be positive and not exceed the noise minimum")
        return cls(chunk_off=chunk_off, spectra=spectra, tau=tau)

    @property
    def nchunk(self) -> int:
        return len(self.chunk_off) - 1

    def lengths(self) -> np.ndarray:
        return np.diff(self.chunk_off)

    def tau_per_sample(self) -> np.ndarray:
        return np.repeat(self.tau, self.lengths())

    def apply_spectral(self, x: np.ndarray, gains: List[np.ndarray]) -> np.ndarray:
        """Per chunk: irfft(rfft(x_c) * gains_c).  A circulant operator diagonal in Fourier space."""
        out = np.empty(len(x), dtype=np.float64)
        for c in range(self.nchunk):
            a, b = int(self.chunk_off[c]), int(self.chunk_off[c + 1])
            n = b - a
            out[a:b] = np.fft.irfft(np.fft.rfft(np.asarray(x[a:b], dtype=np.float64)) * gains[c], n)
        return out

    def apply_inverse(self, x: np.ndarray) -> np.ndarray:
        """N^-1 x."""
        return self.apply_spectral(x, [1.0 / s for s in self.spectra])
