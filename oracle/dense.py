"""Explicit matrices for tiny problems: the limits the iteration approaches.

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Everything here is built entry by entry and solved by dense linear algebra, as
in the brute-force check of Section 3.2 (tabulate P^T N^-1 P, decompose, and
keep only well-constrained modes in a pseudo-inverse):

* ``circulant_inverse``  N_c^-1 of one chunk from its eigenvalues, as the real
  symmetric matrix (1/n) sum_k cos(2 pi k (j - j') / n) / N_k over the full
  length-n spectrum (N_{n-k} = N_k);
* ``pointing_matrix``    P with one row per sample, column q * npix + p;
* ``gls``                m = (P^T N^-1 P)^-1 P^T N^-1 d over the solvable pixels (eqn. mapmaking);
* ``m_lambda``           m(lambda) with N'(lambda) = N + (lambda - 1) T (eqn. mlambda);
* ``F_matrix``           F(lambda) = I - W^-1 P^T (lambda^-1 N-bar + T)^-1 P (eqn. F, last line).
"""

from __future__ import annotations

import math
from typing import Optional

import numpy as np
import scipy.linalg

from .messenger import Setup


def circulant_inverse(N_half: np.ndarray, n: int) -> np.ndarray:
    full = np.empty(n)
    for k in range(n):
        full[k] = N_half[min(k, n - k)]
    j = np.arange(n)
    lag = (j[:, None] - j[None, :]) % n
    k = np.arange(n)
    # C[lag] = (1/n) sum_k cos(2 pi k lag / n) / N_k
    table = (np.cos(2.0 * np.pi * np.outer(np.arange(n), k) / n) / full[None, :]).sum(axis=1) / n
    return table[lag]


def noise_inverse_dense(S: Setup, extra_tau_factor: float = 0.0) -> np.ndarray:
    """Block-diagonal N'^-1 with N' = N + extra_tau_factor * T (0 gives N^-1)."""
    ns = int(S.noise.chunk_off[-1])
    out = np.zeros((ns, ns))
    for c in range(S.noise.nchunk):
        a, b = int(S.noise.chunk_off[c]), int(S.noise.chunk_off[c + 1])
        spec = S.noise.spectra[c] + extra_tau_factor * S.noise.tau[c]
        out[a:b, a:b] = circulant_inverse(spec, b - a)
    return out


def pointing_matrix(S: Setup) -> np.ndarray:
    pt = S.pointing
    P = np.zeros((pt.nsamp, pt.ncomp * pt.npix))
    rows = np.nonzero(pt.on)[0]
    for q in range(pt.ncomp):
        P[rows, q * pt.npix + pt.pix[rows]] = pt.A[rows, q]
    return P


def _solvable_columns(S: Setup) -> np.ndarray:
    return np.concatenate([np.nonzero(S.solvable)[0] + q * S.npix for q in range(S.ncomp)])


def _solve_spd(A: np.ndarray, b: np.ndarray, pinv_rtol: Optional[float]) -> np.ndarray:
    if pinv_rtol is None:
        c, low = scipy.linalg.cho_factor(A)
        return scipy.linalg.cho_solve((c, low), b)
    # Section 3.2: eigen-decomposition, keep only the well-constrained modes
    w, V = np.linalg.eigh(A)
    keep = w > pinv_rtol * w.max()
    return V[:, keep] @ ((V[:, keep].T @ b) / w[keep])


def gls(S: Setup, d: np.ndarray, pinv_rtol: Optional[float] = None, extra_tau_factor: float = 0.0) -> np.ndarray:
    """Minimum-variance map (eqn. mapmaking) restricted to solvable pixels."""
    Ninv = noise_inverse_dense(S, extra_tau_factor)
    P = pointing_matrix(S)[:, _solvable_columns(S)]
    A = P.T @ Ninv @ P
    b = P.T @ (Ninv @ np.asarray(d, dtype=np.float64))
    x = _solve_spd(A, b, pinv_rtol)
    m = np.zeros(S.ncomp * S.npix)
    m[_solvable_columns(S)] = x
    return m.reshape(S.ncomp, S.npix)


def m_lambda(S: Setup, d: np.ndarray, lam: float, pinv_rtol: Optional[float] = None) -> np.ndarray:
    """Fixed point of the iteration at cooling parameter lambda (eqn. mlambda)."""
    return gls(S, d, pinv_rtol, extra_tau_factor=lam - 1.0)


def normal_matrix(S: Setup) -> np.ndarray:
    """P^T N^-1 P over the solvable pixels."""
    P = pointing_matrix(S)[:, _solvable_columns(S)]
    return P.T @ noise_inverse_dense(S) @ P


def F_matrix(S: Setup, lam: float) -> np.ndarray:
    """F(lambda) restricted to the solvable pixels, built entry by entry."""
    cols = _solvable_columns(S)
    P = pointing_matrix(S)[:, cols]
    ns = P.shape[0]
    G = np.zeros((ns, ns))
    for c in range(S.noise.nchunk):
        a, b = int(S.noise.chunk_off[c]), int(S.noise.chunk_off[c + 1])
        tau = S.noise.tau[c]
        if math.isinf(lam):
            G[a:b, a:b] = np.eye(b - a) / tau
        else:
            # (lambda^-1 N-bar + T)^-1 has eigenvalues 1 / ((N_k - tau)/lambda + tau)
            spec = (S.noise.spectra[c] - tau) / lam + tau
            G[a:b, a:b] = circulant_inverse(spec, b - a)
    W = P.T @ (P / np.repeat(S.noise.tau, np.diff(S.noise.chunk_off))[:, None])
    return np.eye(len(cols)) - np.linalg.solve(W, P.T @ G @ P)
