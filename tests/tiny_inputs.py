"""Seeded tiny inputs shared by the oracle pins and the GPU parity tests.

Input generation only (random pointing, noise parameters and data); no part of
the mapmaking method lives here.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class Tiny:
    chunk_off: np.ndarray
    fsample: np.ndarray
    sigma: np.ndarray
    fknee: np.ndarray
    alpha: np.ndarray
    pix: np.ndarray
    psi: Optional[np.ndarray]
    d: np.ndarray
    npix: int
    ncomp: int
    nx: int = 0

    @property
    def nsamp(self) -> int:
        return int(self.chunk_off[-1])


def tiny_problem(seed: int, lengths=(64, 48), nx: int = 4, ncomp: int = 3, fknee=(0.5, 2.0),
                 alpha=(-2.0, -1.5), sigma=(1.0, 1.3), fs: float = 10.0, flag_frac: float = 0.05,
                 psi_dtype=np.float64, tod_dtype=np.float64, walk: bool = True) -> Tiny:
    """A few short chunks scanning a small nx*nx map.

    With ``walk`` the pointing follows a random walk (so neighbouring samples share
    pixels, like a scan); otherwise pixels are drawn uniformly.  A fraction of samples
    is flagged off the map.  Angles are uniform in [0, pi).
    """
    rng = np.random.default_rng(seed)
    lengths = np.asarray(lengths, dtype=np.int64)
    nchunk = len(lengths)
    chunk_off = np.zeros(nchunk + 1, dtype=np.int64)
    np.cumsum(lengths, out=chunk_off[1:])
    ns = int(chunk_off[-1])
    npix = nx * nx
    if walk:
        x = np.empty(ns, np.int64)
        y = np.empty(ns, np.int64)
        cx, cy = nx // 2, nx // 2
        for j in range(ns):
            step = rng.integers(0, 5)
            if step == 1:
                cx = (cx + 1) % nx
            elif step == 2:
                cx = (cx - 1) % nx
            elif step == 3:
                cy = (cy + 1) % nx
            elif step == 4:
                cy = (cy - 1) % nx
            x[j], y[j] = cx, cy
        pix = (y * nx + x).astype(np.int32)
    else:
        pix = rng.integers(0, npix, size=ns).astype(np.int32)
    if flag_frac > 0:
        pix[rng.random(ns) < flag_frac] = -1
    psi = rng.uniform(0.0, np.pi, size=ns).astype(psi_dtype) if ncomp == 3 else None
    sig = np.resize(np.asarray(sigma, dtype=np.float64), nchunk)
    fk = np.resize(np.asarray(fknee, dtype=np.float64), nchunk)
    al = np.resize(np.asarray(alpha, dtype=np.float64), nchunk)
    d = (rng.standard_normal(ns) * 3.0).astype(tod_dtype)
    return Tiny(chunk_off=chunk_off, fsample=np.full(nchunk, fs), sigma=sig, fknee=fk, alpha=al,
                pix=pix, psi=psi, d=d, npix=npix, ncomp=ncomp, nx=nx)


def random_map(seed: int, ncomp: int, npix: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal((ncomp, npix)) * scale


def tiny_composite(seed: int, b_mode: str = "shift", lengths=(64, 48), nx: int = 5, ncomp: int = 3,
                   weights=(1.0, -1.0), flag_b: float = 0.1, **kw):
    """A ``tiny_problem`` plus a second pointing component for P = w_A P_A + w_B P_B.

    b_mode: "shift" (beam B two pixels to the right of beam A in even chunks and one pixel
    below it in odd ones, wrapping, so that the differences link every pixel; a fraction
    ``flag_b`` of B's entries off the map), "none" (P_B = 0: every B index -1), "same"
    (B = A: the same pixels and angles).  B's angles are drawn independently for "shift".
    Returns (tiny, pix_b, psi_b, weights)."""
    t = tiny_problem(seed, lengths=lengths, nx=nx, ncomp=ncomp, **kw)
    rng = np.random.default_rng(seed + 1000)
    if b_mode == "none":
        pix_b = np.full_like(t.pix, -1)
        psi_b = None if t.psi is None else t.psi.copy()
    elif b_mode == "same":
        pix_b = t.pix.copy()
        psi_b = None if t.psi is None else t.psi.copy()
    else:
        on = t.pix >= 0
        x, y = t.pix % nx, t.pix // nx
        odd = (np.searchsorted(t.chunk_off, np.arange(len(t.pix)), side="right") - 1) % 2 == 1
        pix_b = np.where(on, np.where(odd, ((y + 1) % nx) * nx + x, y * nx + (x + 2) % nx), -1).astype(np.int32)
        pix_b[rng.random(len(pix_b)) < flag_b] = -1
        psi_b = None if t.psi is None else rng.uniform(0.0, np.pi, size=len(pix_b)).astype(t.psi.dtype)
    return t, pix_b, psi_b, tuple(float(w) for w in weights)


def gap_mask(seed: int, chunk_off, frac: float = 0.1, run: int = 6) -> np.ndarray:
    """Gaps as runs of `run` consecutive samples placed at random, about `frac` of the samples."""
    rng = np.random.default_rng(seed)
    ns = int(chunk_off[-1])
    g = np.zeros(ns, dtype=bool)
    nrun = max(1, int(frac * ns / run))
    for s0 in rng.integers(0, max(1, ns - run), size=nrun):
        g[s0:s0 + run] = True
    return g
