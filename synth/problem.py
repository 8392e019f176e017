"""Build one synthetic observation: sky, pointing, noise and time-ordered data.

Recipe (every random draw is seeded from one SeedSequence tree, so a problem
is reproducible and each chunk's noise does not depend on how many chunks are
generated before it):

* seed tree: child ``cfg.index`` of ``SeedSequence(170501893)`` (spawned five or more at
  once: the first five children do not depend on how many are spawned) and then its
  children, in order: sky, noise parameters, chunk lengths, detector offsets,
  then one child per chunk for that chunk's noise realisation;
* sky: flat-sky Gaussian random field on the nx*nx grid with power falling as
  the inverse square of the wavenumber, zero mean, scaled to the requested rms
  (Q and U are independent fields);
* pointing: see ``scans.py``; nearest-pixel, int32 pixel index, -1 off the map;
* noise: per chunk, a white unit-variance draw shaped in Fourier space by the
  square root of the power law sigma^2 (1 + (f/fknee)^alpha) of the paper's
  simulation section, with the f=0 bin given the value at the first nonzero
  frequency; the realisation therefore has that power spectrum exactly;
* data: signal read off the sky along the pointing (I + Q cos 2psi + U sin 2psi)
  plus the noise, stored in the workload's TOD type.
"""

from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .configs import WorkloadConfig
from .scans import chunk_pointing, chunk_pointing_differential

ROOT_SEED = 170501893


@dataclass
class Problem:
    """Plain arrays describing one observation.  No solver state."""
    cfg: WorkloadConfig
    chunk_off: np.ndarray          # int64 [nchunk+1] sample offsets
    fsample: np.ndarray            # float64 [nchunk]
    sigma: np.ndarray              # float64 [nchunk] white-noise std per sample
    fknee: np.ndarray              # float64 [nchunk]
    alpha: np.ndarray              # float64 [nchunk]
    pix: np.ndarray                # int32 [N_s]; -1 = off the map
    psi: Optional[np.ndarray]      # float64 / float32 [N_s] polarization angle, or None
    psi_index: Optional[np.ndarray] = None   # uint16 [N_s] index into psi_table (psi_kind == "u16")
    psi_table: Optional[np.ndarray] = None   # float32 [ntable]
    d: Optional[np.ndarray] = None           # float64 / float32 [N_s]
    m_true: Optional[np.ndarray] = None      # float64 [ncomp, npix]
    noise: Optional[np.ndarray] = None       # float64 [N_s] (kept only when asked for)
    # differential pointing (Section 3.2): the second beam's pixels and angles, and the weights
    # of the two beams in each sample (None for a single beam)
    pix_b: Optional[np.ndarray] = None
    psi_b: Optional[np.ndarray] = None
    weights: Optional[tuple] = None
    extra: dict = field(default_factory=dict)

    @property
    def nchunk(self) -> int:
        return len(self.chunk_off) - 1

    @property
    def nsamp_total(self) -> int:
        return int(self.chunk_off[-1])

    @property
    def npix(self) -> int:
        return self.cfg.npix

    @property
    def ncomp(self) -> int:
        return self.cfg.ncomp

    def psi_values(self) -> Optional[np.ndarray]:
        """Per-sample angle as stored (table lookups resolved), or None for T-only."""
        if self.psi is not None:
            return self.psi
        if self.psi_index is not None:
            return self.psi_table[self.psi_index]
        return None

    def chunk(self, c: int) -> slice:
        return slice(int(self.chunk_off[c]), int(self.chunk_off[c + 1]))


def _seed_tree(cfg: WorkloadConfig):
    top = np.random.SeedSequence(ROOT_SEED).spawn(max(5, cfg.index + 1))[cfg.index]
    kids = top.spawn(4 + cfg.ndet)
    return kids[0], kids[1], kids[2], kids[3], kids[4:]


def _five_smooth_leq(x: int) -> int:
    """Largest 2^a 3^b 5^c that does not exceed x (x >= 1)."""
    best = 1
    p5 = 1
    while p5 <= x:
        p3 = p5
        while p3 <= x:
            v = p3
            while v * 2 <= x:
                v *= 2
            best = max(best, v)
            p3 *= 3
        p5 *= 5
    return best


def chunk_lengths(cfg: WorkloadConfig, ss_len) -> np.ndarray:
    """Chunk lengths.  Equal lengths, or log-uniform in [nsamp_min, nsamp] snapped down
    to n = 2*M with M a 5-smooth number (only transform-friendly lengths, no padding)."""
    if cfg.nsamp_min == cfg.nsamp:
        return np.full(cfg.ndet, cfg.nsamp, dtype=np.int64)
    rng = np.random.default_rng(ss_len)
    u = rng.uniform(math.log(cfg.nsamp_min), math.log(cfg.nsamp), size=cfg.ndet)
    raw = np.floor(np.exp(u)).astype(np.int64)
    return np.array([2 * _five_smooth_leq(int(v) // 2) for v in raw], dtype=np.int64)


def noise_params(cfg: WorkloadConfig, ss_par):
    rng = np.random.default_rng(ss_par)
    sigma = rng.uniform(cfg.sig_lo, cfg.sig_hi, size=cfg.ndet)
    fknee = rng.uniform(cfg.fk_lo, cfg.fk_hi, size=cfg.ndet)
    alpha = rng.uniform(cfg.al_lo, cfg.al_hi, size=cfg.ndet)
    if cfg.frac_high_knee > 0:
        nhigh = int(round(cfg.frac_high_knee * cfg.ndet))
        sel = rng.choice(cfg.ndet, size=nhigh, replace=False)
        fknee[sel] = cfg.fknee_high
    if cfg.sig_lo == cfg.sig_hi:
        sigma[:] = cfg.sig_lo
    if cfg.fk_lo == cfg.fk_hi:
        fknee[:] = cfg.fk_lo
    if cfg.al_lo == cfg.al_hi:
        alpha[:] = cfg.al_lo
    return sigma, fknee, alpha


def gaussian_sky(cfg: WorkloadConfig, ss_sky) -> np.ndarray:
    """Flat-sky Gaussian random fields with power ~ k^-2, zero mean, given rms."""
    rng = np.random.default_rng(ss_sky)
    n = cfg.nx
    kx = np.fft.fftfreq(n) * n
    ky = np.fft.rfftfreq(n) * n
    k2 = kx[:, None] ** 2 + ky[None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = 1.0 / np.sqrt(k2[nz])          # sqrt of a k^-2 power law
    out = np.empty((cfg.ncomp, n * n), dtype=np.float64)
    for q in range(cfg.ncomp):
        white = rng.standard_normal((n, n))
        field_ = np.fft.irfft2(np.fft.rfft2(white) * amp, s=(n, n))
        field_ -= field_.mean()
        rms = cfg.rms_t if q == 0 else cfg.rms_p
        field_ *= rms / max(field_.std(), 1e-300)
        out[q] = field_.reshape(-1)          # pixel p = y * nx + x
    return out


def _noise_shape(n: int, fs: float, sigma: float, fknee: float, alpha: float) -> np.ndarray:
    """Square root of the simulation power law at the rfft bins (input recipe, Section 2.3)."""
    f = np.arange(n // 2 + 1, dtype=np.float64) * (fs / n)
    f[0] = f[1]
    return sigma * np.sqrt(1.0 + (f / fknee) ** alpha)


def chunk_noise(n: int, fs: float, sigma: float, fknee: float, alpha: float, ss) -> np.ndarray:
    rng = np.random.default_rng(ss)
    white = rng.standard_normal(n)
    return np.fft.irfft(np.fft.rfft(white) * _noise_shape(n, fs, sigma, fknee, alpha), n)


def _signal(m_true: np.ndarray, pix: np.ndarray, psi: Optional[np.ndarray]) -> np.ndarray:
    """Sky read off along the pointing: I + Q cos 2psi + U sin 2psi (0 off the map)."""
    on = pix >= 0
    p = np.where(on, pix, 0)
    s = m_true[0][p].copy()
    if m_true.shape[0] == 3:
        two = 2.0 * psi.astype(np.float64)
        s += m_true[1][p] * np.cos(two) + m_true[2][p] * np.sin(two)
    s[~on] = 0.0
    return s


def make_problem(cfg: WorkloadConfig, with_noise: bool = True, noise_scale: float = 1.0,
                 keep_noise: bool = False, workers: int = 8) -> Problem:
    """Generate the observation described by ``cfg``.

    ``noise_scale`` multiplies the noise realisation (0 gives noise-free data for
    unbiasedness checks); ``keep_noise`` stores the realisation in ``Problem.noise``.
    With ``cfg.diff_sep > 0`` every sample is the difference of two beams (weights +1 and -1,
    same angle): d = sky(beam A) - sky(beam B) + noise.
    """
    diff = cfg.diff_sep > 0
    ss_sky, ss_par, ss_len, ss_off, ss_chunks = _seed_tree(cfg)
    lengths = chunk_lengths(cfg, ss_len)
    chunk_off = np.zeros(cfg.ndet + 1, dtype=np.int64)
    np.cumsum(lengths, out=chunk_off[1:])
    ns = int(chunk_off[-1])
    sigma, fknee, alpha = noise_params(cfg, ss_par)
    fsample = np.full(cfg.ndet, cfg.fsample, dtype=np.float64)
    offsets = np.random.default_rng(ss_off).uniform(0.0, 1.0, size=(cfg.ndet, 2))
    m_true = gaussian_sky(cfg, ss_sky)

    pix = np.empty(ns, dtype=np.int32)
    psi_store = None
    psi_index = None
    psi_table = None
    if cfg.psi_kind == "f64":
        psi_store = np.empty(ns, dtype=np.float64)
    elif cfg.psi_kind == "f32":
        psi_store = np.empty(ns, dtype=np.float32)
    elif cfg.psi_kind == "u16":
        psi_index = np.empty(ns, dtype=np.uint16)
        # one angle per (detector, scan half)
        base = np.pi * np.arange(cfg.ndet, dtype=np.float64) / cfg.ndet
        psi_table = np.stack([base, base + np.pi / 4], axis=1).reshape(-1).astype(np.float32)
    tod_dtype = np.float64 if cfg.tod_dtype == "f64" else np.float32
    d = np.empty(ns, dtype=tod_dtype)
    noise_all = np.empty(ns, dtype=np.float64) if keep_noise else None
    if diff and cfg.psi_kind == "u16":
        raise ValueError("differential workloads store their angles directly")
    pix_b = np.empty(ns, dtype=np.int32) if diff else None
    psi_b = np.empty_like(psi_store) if (diff and psi_store is not None) else None

    def work(c: int):
        sl = slice(int(chunk_off[c]), int(chunk_off[c + 1]))
        n = int(lengths[c])
        if diff:
            cpix, cpix_b, cpsi, chalf = chunk_pointing_differential(cfg, c, n, offsets[c])
            pix_b[sl] = cpix_b
        else:
            cpix, cpsi, chalf = chunk_pointing(cfg, c, n, offsets[c])
        pix[sl] = cpix
        psi_used = None
        if cfg.psi_kind in ("f64", "f32"):
            psi_store[sl] = cpsi
            psi_used = psi_store[sl]
            if diff:
                psi_b[sl] = cpsi
        elif cfg.psi_kind == "u16":
            idx = (2 * c + chalf).astype(np.uint16)
            psi_index[sl] = idx
            psi_used = psi_table[idx]
        sig = _signal(m_true, cpix, psi_used)
        if diff:
            sig = sig - _signal(m_true, cpix_b, psi_used)
        if with_noise and noise_scale != 0.0:
            nz = chunk_noise(n, float(fsample[c]), float(sigma[c]), float(fknee[c]), float(alpha[c]),
                             ss_chunks[c]) * noise_scale
        else:
            nz = np.zeros(n)
        if keep_noise:
            noise_all[sl] = nz
        d[sl] = (sig + nz).astype(tod_dtype)

    if workers > 1 and cfg.ndet > 1:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(work, range(cfg.ndet)))
    else:
        for c in range(cfg.ndet):
            work(c)

    return Problem(cfg=cfg, chunk_off=chunk_off, fsample=fsample, sigma=sigma, fknee=fknee,
                   alpha=alpha, pix=pix, psi=psi_store, psi_index=psi_index, psi_table=psi_table,
                   d=d, m_true=m_true, noise=noise_all, pix_b=pix_b, psi_b=psi_b,
                   weights=(1.0, -1.0) if diff else None)
