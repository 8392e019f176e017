"""Workload definitions.

Each workload fixes the shapes of a synthetic observation: number of detector
chunks and their lengths, sample rate, map size, Stokes components, the noise
law of every detector and the numeric type of the time-ordered data.  The
cooling-schedule fields record how many levels and iterations a solve runs;
how the levels are placed is the solver's business.

The named workloads mirror the simulations of Section 2.3 of the paper
(cross-linked rasters, 1/f plus white noise, polarized detectors; two of them
with the differencing beams of Section 3.2) at the sizes used for parity and
throughput measurement.  ``scaled`` derives small variants
with the same structure for tests that must finish in seconds.
"""

from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import Optional


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    index: int                 # position in the seed tree (0..4); scaled variants reuse their parent's
    ndet: int                  # number of detector chunks
    nsamp: int                 # samples per chunk (upper end of the range when uneven)
    nsamp_min: int             # lower end of the length range (== nsamp when all chunks are equal)
    fsample: float             # Hz
    nx: int                    # map is nx * nx pixels
    ncomp: int                 # 1 = temperature only, 3 = I, Q, U
    tod_dtype: str             # "f64" or "f32"
    psi_kind: str              # "none", "f64", "f32" or "u16" (index into an angle table)
    scan: str                  # "boustrophedon64" (the fixed T-only raster) or "crossed"
    # noise law per detector: sigma ~ U(sig_lo, sig_hi), fknee ~ U(fk_lo, fk_hi), alpha ~ U(al_lo, al_hi)
    sig_lo: float = 1.0
    sig_hi: float = 1.0
    fk_lo: float = 1.0
    fk_hi: float = 1.0
    al_lo: float = -2.0
    al_hi: float = -2.0
    frac_high_knee: float = 0.0  # fraction of detectors forced to fknee_high
    fknee_high: float = 5.0
    # cooling schedule: nlevel geometric levels of iters_per_level iterations after one lambda=inf step
    nlevel: int = 10
    iters_per_level: int = 5
    lambda_max: Optional[float] = None  # None => the solver's own rule
    # sky amplitudes (rms of the temperature and of each polarization component)
    rms_t: float = 10.0
    rms_p: float = 1.0
    # differential pointing: separation (pixels) of the second beam, 0 for a single beam
    diff_sep: float = 0.0

    @property
    def npix(self) -> int:
        return self.nx * self.nx

    def scaled(self, name: str, ndet: int, nsamp: int, nx: int, nsamp_min: Optional[int] = None,
               **kw) -> "WorkloadConfig":
        """Same structure, smaller sizes (for tests)."""
        return dataclasses.replace(self, name=name, ndet=ndet, nsamp=nsamp,
                                   nsamp_min=nsamp if nsamp_min is None else nsamp_min, nx=nx, **kw)


CONFIGS = [
    # Temperature-only plain solve: one detector, 65536 samples at 100 Hz on a 64x64 map,
    # horizontal then vertical boustrophedon (32768 samples each), white sigma=1 plus 1/f with
    # fknee=1 Hz and slope -2, lambda cooled from 1e4 to 1 over 10 levels of 5 iterations.
    WorkloadConfig(name="t64", index=0, ndet=1, nsamp=65536, nsamp_min=65536, fsample=100.0, nx=64,
                   ncomp=1, tod_dtype="f64", psi_kind="none", scan="boustrophedon64",
                   nlevel=10, iters_per_level=5, lambda_max=1e4),
    # I/Q/U FP64: 16 detectors x 2^20 samples at 200 Hz, 256x256 map, crossed rasters.
    WorkloadConfig(name="iqu256", index=1, ndet=16, nsamp=1 << 20, nsamp_min=1 << 20, fsample=200.0,
                   nx=256, ncomp=3, tod_dtype="f64", psi_kind="f64", scan="crossed",
                   sig_lo=0.8, sig_hi=1.2, fk_lo=0.1, fk_hi=2.0, al_lo=-3.0, al_hi=-1.0,
                   nlevel=10, iters_per_level=10),
    # Batched FP32-mixed: 512 detectors of uneven length log-uniform in [2^18, 2^21], 1024x1024 map.
    WorkloadConfig(name="batched1024", index=2, ndet=512, nsamp=1 << 21, nsamp_min=1 << 18,
                   fsample=200.0, nx=1024, ncomp=3, tod_dtype="f32", psi_kind="f32", scan="crossed",
                   sig_lo=0.8, sig_hi=1.2, fk_lo=0.1, fk_hi=2.0, al_lo=-3.0, al_hi=-1.0,
                   nlevel=10, iters_per_level=10),
    # Differentiation workload: 64 detectors x 2^20, 512x512, FP32-mixed.
    WorkloadConfig(name="grad512", index=3, ndet=64, nsamp=1 << 20, nsamp_min=1 << 20, fsample=200.0,
                   nx=512, ncomp=3, tod_dtype="f32", psi_kind="f32", scan="crossed",
                   sig_lo=0.8, sig_hi=1.2, fk_lo=0.1, fk_hi=2.0, al_lo=-3.0, al_hi=-1.0,
                   nlevel=10, iters_per_level=5),
    # Large single-GPU share: 1024 detectors x 2^22, 2048x2048, FP32 TOD, uint16 angle-table index,
    # 5% of detectors at fknee = 5 Hz, 15 cooling levels.
    WorkloadConfig(name="large2048", index=4, ndet=1024, nsamp=1 << 22, nsamp_min=1 << 22,
                   fsample=200.0, nx=2048, ncomp=3, tod_dtype="f32", psi_kind="u16", scan="crossed",
                   sig_lo=0.8, sig_hi=1.2, fk_lo=0.1, fk_hi=2.0, al_lo=-3.0, al_hi=-1.0,
                   frac_high_knee=0.05, fknee_high=5.0, nlevel=15, iters_per_level=5),
    # Differential beams (Section 3.2): two beams 8 pixels apart (the paper's 18 arcmin on a
    # 600-pixel map, scaled to 256), each sample their difference; temperature only, FP64,
    # 16 detectors x 2^20 on the crossed rasters, a 16 x 10 schedule.
    WorkloadConfig(name="diff256", index=5, ndet=16, nsamp=1 << 20, nsamp_min=1 << 20, fsample=200.0,
                   nx=256, ncomp=1, tod_dtype="f64", psi_kind="none", scan="crossed",
                   sig_lo=0.8, sig_hi=1.2, fk_lo=0.1, fk_hi=2.0, al_lo=-3.0, al_hi=-1.0,
                   nlevel=16, iters_per_level=10, diff_sep=8.0),
    # Differential I/Q/U, FP32-mixed: 64 detectors x 2^20 on a 512 x 512 map, beams 16 pixels apart.
    WorkloadConfig(name="diff512", index=6, ndet=64, nsamp=1 << 20, nsamp_min=1 << 20, fsample=200.0,
                   nx=512, ncomp=3, tod_dtype="f32", psi_kind="f32", scan="crossed",
                   sig_lo=0.8, sig_hi=1.2, fk_lo=0.1, fk_hi=2.0, al_lo=-3.0, al_hi=-1.0,
                   nlevel=16, iters_per_level=10, diff_sep=16.0),
]


def config_by_name(name: str) -> WorkloadConfig:
    for c in CONFIGS:
        if c.name == name:
            return c
    raise KeyError(name)
