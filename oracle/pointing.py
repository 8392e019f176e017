"""Pointing matrix P, its transpose, hit counts and the weight blocks P^T T^-1 P.

TEST INFRASTRUCTURE (oracle): used only by tests, the smoke check and the
benchmark's CPU-baseline leg.

Section 2 defines P as the matrix that carries each sample's weight on the map
pixels in temperature and polarization; Section 2.2 restricts the single
pencil beam to one pixel (or one polarized pixel block) per sample.  Reading
used here: sample j at pixel p_j with angle psi_j sees
    (P m)_j = I[p_j] + Q[p_j] cos 2 psi_j + U[p_j] sin 2 psi_j
(T-only maps keep the first term).  A negative pixel index means the sample is
off the map: its row of P is zero, but it still belongs to its chunk's noise
filter and chi^2.

Map layout: float64 [ncomp, npix].
"""

from __future__ import annotations

import numpy as np


class Pointing:
    def __init__(self, pix: np.ndarray, psi, npix: int, ncomp: int):
        if ncomp not in (1, 3):
            raise ValueError("ncomp must be 1 or 3")
        self.npix = int(npix)
        self.ncomp = int(ncomp)
        self.pix = np.asarray(pix).astype(np.int64)
        if np.any(self.pix >= npix):
            raise ValueError("pixel index beyond the map")
        self.on = self.pix >= 0
        self.pix_on = self.pix[self.on]
        n = len(self.pix)
        # weights a_j, zero rows for samples off the map
        self.A = np.zeros((n, ncomp), dtype=np.float64)
        self.A[self.on, 0] = 1.0
        if ncomp == 3:
            two_psi = 2.0 * np.asarray(psi).astype(np.float64)   # the stored angle, promoted
            self.A[self.on, 1] = np.cos(two_psi[self.on])
            self.A[self.on, 2] = np.sin(two_psi[self.on])

    @property
    def nsamp(self) -> int:
        return len(self.pix)

    def project(self, m: np.ndarray) -> np.ndarray:
        """(P m)_j = sum_q a_jq m[q, p_j]; zero off the map."""
        m = np.asarray(m, dtype=np.float64).reshape(self.ncomp, self.npix)
        out = np.zeros(self.nsamp, dtype=np.float64)
        for q in range(self.ncomp):
            out[self.on] += self.A[self.on, q] * m[q][self.pix_on]
        return out

    def back(self, y: np.ndarray) -> np.ndarray:
        """(P^T y)[q, p] = sum over samples j at pixel p of a_jq y_j."""
        y = np.asarray(y, dtype=np.float64)
        b = np.empty((self.ncomp, self.npix), dtype=np.float64)
        for q in range(self.ncomp):
            b[q] = np.bincount(self.pix_on, weights=self.A[self.on, q] * y[self.on], minlength=self.npix)
        return b

    def hits(self) -> np.ndarray:
        """Number of samples per pixel (int)."""
        return np.bincount(self.pix_on, minlength=self.npix).astype(np.int64)

    def weight_blocks(self, inv_var_per_sample: np.ndarray) -> np.ndarray:
        """P^T diag(v) P as one ncomp x ncomp block per pixel, [npix, ncomp, ncomp]."""
        v = np.asarray(inv_var_per_sample, dtype=np.float64)[self.on]
        W = np.empty((self.npix, self.ncomp, self.ncomp), dtype=np.float64)
        for q in range(self.ncomp):
            for r in range(q, self.ncomp):
                w = np.bincount(self.pix_on, weights=self.A[self.on, q] * self.A[self.on, r] * v,
                                minlength=self.npix)
                W[:, q, r] = w
                W[:, r, q] = w
        return W


def invert_blocks(W: np.ndarray, hits: np.ndarray, rcond_min: float = 1e-8):
    """Invert the per-pixel blocks of P^T T^-1 P.

    A pixel is solvable when it has hits and, for 3x3 blocks, the determinant of
    the block normalised by its diagonal, det(W) / (W_00 W_11 W_22), is at least
    ``rcond_min``.  (With weights (1, cos 2psi, sin 2psi), W_11 + W_22 = W_00, so
    this number measures how well the pixel's angles separate Q from U; it is 1
    for evenly spread angles and 0 for a single angle.  Unlike a condition number
    computed from the inverse it stays near 0 for exactly singular blocks whose
    determinant is rounding noise.)  Unsolvable pixels get a zero block (their map
    values are held at zero).  Returns (W_inv, solvable).
    """
    npix, nc, _ = W.shape
    solvable = hits > 0
    Winv = np.zeros_like(W)
    if nc == 1:
        solvable = solvable & (W[:, 0, 0] > 0)
        Winv[solvable, 0, 0] = 1.0 / W[solvable, 0, 0]
        return Winv, solvable
    idx = np.nonzero(solvable)[0]
    blocks = W[idx]
    diag = blocks[:, 0, 0] * blocks[:, 1, 1] * blocks[:, 2, 2]
    dets = np.linalg.det(blocks)
    good = diag > 0
    good[good] = dets[good] / diag[good] >= rcond_min
    solvable = np.zeros(npix, dtype=bool)
    solvable[idx[good]] = True
    Winv[idx[good]] = np.linalg.inv(blocks[good])
    return Winv, solvable
