"""Diagonal-preconditioned conjugate gradients on the mapmaking equation.

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The comparison solver of Sections 1, 2 and 3.1: textbook preconditioned CG on
(P^T N^-1 P) m = P^T N^-1 d, started from zero (Section 3.1).  The paper
calls its CG diagonal-preconditioned without defining the preconditioner; the reading used here
is the per-pixel block P^T diag(1/tau) P, i.e. the same W^-1 blocks the
messenger iteration uses, which with the default tau_c = sigma_c^2 is the
white-noise weight map (diagonal for temperature-only maps, 3x3 blocks for
I, Q, U).  Unsolvable pixels are excluded (zero preconditioner block).
"""

from __future__ import annotations

from typing import Optional

import numpy as np

from .messenger import Setup, chi2, weighted_solve


def apply_A(S: Setup, x: np.ndarray) -> np.ndarray:
    """P^T N^-1 P x."""
    return S.pointing.back(S.noise.apply_inverse(S.pointing.project(x)))


def rhs(S: Setup, d: np.ndarray) -> np.ndarray:
    """P^T N^-1 d."""
    return S.pointing.back(S.noise.apply_inverse(np.asarray(d, dtype=np.float64)))


def pcg_solve(S: Setup, d: Optional[np.ndarray], maxiter: int, m0: Optional[np.ndarray] = None,
              b: Optional[np.ndarray] = None, record_chi2: bool = False, rtol: float = 0.0):
    """Preconditioned CG.  Returns (m, info) with info['chi2'] (chi^2 of every iterate, when
    asked for and d is given) and info['rz'] (r^T M^-1 r per iteration)."""
    if b is None:
        b = rhs(S, d)
    b = np.asarray(b, dtype=np.float64).reshape(S.ncomp, S.npix)
    x = np.zeros_like(b) if m0 is None else np.asarray(m0, dtype=np.float64).reshape(b.shape).copy()
    r = b - apply_A(S, x)
    z = weighted_solve(S, r)
    p = z.copy()
    rz = float(np.sum(r * z))
    rz0 = rz
    chi2s = [chi2(S, d, x)] if (record_chi2 and d is not None) else []
    rzs = [rz]
    it = 0
    for it in range(1, maxiter + 1):
        q = apply_A(S, p)
        alpha = rz / float(np.sum(p * q))
        x += alpha * p
        r -= alpha * q
        z = weighted_solve(S, r)
        rz_new = float(np.sum(r * z))
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        rzs.append(rz)
        if record_chi2 and d is not None:
            chi2s.append(chi2(S, d, x))
        if rtol > 0 and rz <= rtol * rtol * rz0:
            break
    return x, {"chi2": np.array(chi2s), "rz": np.array(rzs), "iters": it}
