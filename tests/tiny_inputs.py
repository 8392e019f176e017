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
