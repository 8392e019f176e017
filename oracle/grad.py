"""Gradients of a loss of the solved map (implicit differentiation of eqn. mapmaking).

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The solved map is the minimum-variance map m = A^-1 P^T N^-1 d with
A = P^T N^-1 P (Section 2).  For a loss L(m) with g = dL/dm and the adjoint
map z = A^-1 g:

* dL/dd = N^-1 P z;
* dm = A^-1 P^T (dN^-1) r with r = d - P m, so
  dL/dtheta = (P z)^T (dN^-1/dtheta) r, and with N circulant per chunk,
  dN^-1 has eigenvalues -dN_k / N_k^2:
      dL/dtheta_c = -(1/n_c) sum_k omega_k Re(conj(zhat_k) rhat_k) (dN_k/dtheta_c) / N_k^2
  (zhat, rhat the rfft of chunk c of P z and r, omega_k the bin multiplicity).

For the power law N = sigma^2 (1 + (f/fknee)^alpha) (DC bin at f_1):
dN/dsigma = 2 N / sigma, dN/dfknee = -alpha sigma^2 (f/fknee)^alpha / fknee,
dN/dalpha = sigma^2 (f/fknee)^alpha ln(f/fknee).
"""

from __future__ import annotations

import numpy as np

from .messenger import Setup
from .noise import chi2_weights


def spectrum_derivatives(n: int, fs: float, sigma: float, fknee: float, alpha: float):
    """(N_k, dN/dsigma, dN/dfknee, dN/dalpha) at the rfft bins, DC bin at f_1."""
    f = np.arange(n // 2 + 1, dtype=np.float64) * (fs / n)
    f[0] = f[1]
    x = (f / fknee) ** alpha
    N = sigma * sigma * (1.0 + x)
    return N, 2.0 * N / sigma, -alpha * sigma * sigma * x / fknee, sigma * sigma * x * np.log(f / fknee)


def noise_param_grad(S: Setup, d: np.ndarray, m: np.ndarray, z: np.ndarray, fsample, sigma, fknee, alpha):
    """dL/d(sigma, fknee, alpha) per chunk, [nchunk, 3], from the solved map m and adjoint map z."""
    r = np.asarray(d, dtype=np.float64) - S.pointing.project(m)
    Pz = S.pointing.project(z)
    out = np.zeros((S.noise.nchunk, 3))
    for c in range(S.noise.nchunk):
        a, b = int(S.noise.chunk_off[c]), int(S.noise.chunk_off[c + 1])
        n = b - a
        rh = np.fft.rfft(r[a:b])
        zh = np.fft.rfft(Pz[a:b])
        N, dsig, dfk, dal = spectrum_derivatives(n, fsample[c], sigma[c], fknee[c], alpha[c])
        cross = chi2_weights(n) * (zh.real * rh.real + zh.imag * rh.imag) / (N * N)
        out[c] = -np.array([np.sum(cross * dsig), np.sum(cross * dfk), np.sum(cross * dal)]) / n
    return out


def data_grad(S: Setup, z: np.ndarray) -> np.ndarray:
    """dL/dd = N^-1 P z."""
    return S.noise.apply_inverse(S.pointing.project(z))
