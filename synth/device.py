"""The synthetic workloads generated on the GPU (for the 4.3e9-sample workload).

Same recipe and seed tree as ``problem.py`` (sky, noise parameters, chunk lengths, detector
offsets and the scan from ``scans.py``), with two differences that keep generation of
billions of samples to seconds:

* each chunk's white noise is drawn by torch's device generator (Philox), seeded with the
  first 64-bit word of the chunk's SeedSequence child, and shaped by torch's FFT on the GPU;
  the realisation therefore differs from the host generator's, but it is again exactly the
  power law sigma^2 (1 + (f/fknee)^alpha) (f_0 at f_1) per chunk, and it does not depend on
  which other chunks are generated;
* the pointing is the same float64 arithmetic as ``scans.py`` evaluated by torch on the GPU.

Like the rest of ``synth``, this is input generation only: it holds no part of the mapmaking
method.  Whatever consumes the data (the library on the GPU, the CPU oracle on copies of
chosen chunks) reads the stored arrays.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

from .configs import WorkloadConfig
from .problem import _seed_tree, chunk_lengths, gaussian_sky, noise_params


@dataclass
class DeviceProblem:
    cfg: WorkloadConfig
    chunks: np.ndarray             # detector indices held (a subset keeps each chunk's own data)
    chunk_off: np.ndarray          # int64 [nchunk+1]
    fsample: np.ndarray
    sigma: np.ndarray
    fknee: np.ndarray
    alpha: np.ndarray
    pix: torch.Tensor              # int32 [N_s] on the device, -1 off the map
    psi: Optional[torch.Tensor]    # uint16 index into psi_table, or float32 / float64 angles
    psi_table: Optional[np.ndarray]
    d: torch.Tensor                # TOD in the workload's type
    m_true: np.ndarray             # float64 [ncomp, npix] (host)
    # differential pointing: second beam's pixels / angles on the device, beam weights (or None)
    pix_b: Optional[torch.Tensor] = None
    psi_b: Optional[torch.Tensor] = None
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

    def chunk(self, c: int) -> slice:
        return slice(int(self.chunk_off[c]), int(self.chunk_off[c + 1]))

    def host_chunks(self, idx: Sequence[int]):
        """pix, stored angle values (table lookups resolved, float32/64) and d of the given chunks,
        copied to the host, with their chunk table: the inputs the oracle reads (and the second
        beam's pix_b / psi_b for differential pointing)."""
        sl = [self.chunk(c) for c in idx]
        pix = np.concatenate([self.pix[s].cpu().numpy() for s in sl])
        d = np.concatenate([self.d[s].cpu().numpy() for s in sl])
        psi = None
        if self.psi is not None:
            raw = np.concatenate([self.psi[s].cpu().numpy() for s in sl])
            psi = self.psi_table[raw.view(np.uint16)] if self.psi_table is not None else raw
        lens = np.array([s.stop - s.start for s in sl], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        ix = np.asarray(idx)
        out = dict(chunk_off=off, fsample=self.fsample[ix], sigma=self.sigma[ix], fknee=self.fknee[ix],
                   alpha=self.alpha[ix], pix=pix, psi=psi, d=d)
        if self.pix_b is not None:
            out["pix_b"] = np.concatenate([self.pix_b[s].cpu().numpy() for s in sl])
            out["psi_b"] = (None if self.psi_b is None else
                            np.concatenate([self.psi_b[s].cpu().numpy() for s in sl]))
        return out


def _raster_positions(nh: int, w: int, rotate: bool, dev):
    s = torch.arange(nh, dtype=torch.int64, device=dev)
    line = (s * w) // nh
    a = ((s * w) % nh).to(torch.float64) / nh
    x = torch.where(line % 2 == 1, (1.0 - a) * w, a * w)
    y = line.to(torch.float64) + 0.5
    if rotate:
        c = math.cos(math.pi / 4)
        xc, yc = x - 0.5 * w, y - 0.5 * w
        x = c * xc - c * yc + 0.5 * w
        y = c * xc + c * yc + 0.5 * w
    return x, y


def make_problem_device(cfg: WorkloadConfig, dev, chunks: Optional[Sequence[int]] = None,
                        noise_scale: float = 1.0, batch: int = 16) -> DeviceProblem:
    """Generate the workload (or the given detector chunks of it) directly in device memory."""
    if cfg.scan != "crossed":
        raise ValueError("the device generator draws the crossed raster")
    ss_sky, ss_par, ss_len, ss_off, ss_chunks = _seed_tree(cfg)
    lengths_all = chunk_lengths(cfg, ss_len)
    sig_all, fk_all, al_all = noise_params(cfg, ss_par)
    offsets = np.random.default_rng(ss_off).uniform(0.0, 1.0, size=(cfg.ndet, 2))
    m_true = gaussian_sky(cfg, ss_sky)
    idx = np.arange(cfg.ndet) if chunks is None else np.asarray(chunks, dtype=np.int64)
    lengths = lengths_all[idx]
    off = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    ns = int(off[-1])
    w = cfg.nx
    pix = torch.empty(ns, dtype=torch.int32, device=dev)
    psi = None
    psi_table = None
    if cfg.psi_kind == "u16":
        psi = torch.empty(ns, dtype=torch.uint16, device=dev)
        base = np.pi * np.arange(cfg.ndet, dtype=np.float64) / cfg.ndet
        psi_table = np.stack([base, base + np.pi / 4], axis=1).reshape(-1).astype(np.float32)
        tab_dev = torch.from_numpy(psi_table).to(dev)
    elif cfg.psi_kind in ("f32", "f64"):
        psi = torch.empty(ns, dtype=torch.float32 if cfg.psi_kind == "f32" else torch.float64, device=dev)
    tod_t = torch.float32 if cfg.tod_dtype == "f32" else torch.float64
    d = torch.empty(ns, dtype=tod_t, device=dev)
    sky = torch.from_numpy(m_true).to(dev)
    cache = {}
    for b0 in range(0, len(idx), batch):
        for k in range(b0, min(b0 + batch, len(idx))):
            c = int(idx[k])
            n = int(lengths[k])
            sl = slice(int(off[k]), int(off[k + 1]))
            if n not in cache:
                nh0 = n // 2
                x0, y0 = _raster_positions(nh0, w, False, dev)
                x1, y1 = _raster_positions(n - nh0, w, True, dev)
                f = torch.arange(n // 2 + 1, dtype=torch.float64, device=dev) * (cfg.fsample / n)
                f[0] = f[1]
                half = torch.cat([torch.zeros(nh0, dtype=torch.int64, device=dev),
                                  torch.ones(n - nh0, dtype=torch.int64, device=dev)])
                cache = {n: (torch.cat([x0, x1]), torch.cat([y0, y1]), f, half)}
            xb, yb, f, half = cache[n]
            x = xb + (float(offsets[c, 0]) - 0.5)
            y = yb + (float(offsets[c, 1]) - 0.5)
            ix = torch.floor(x).to(torch.int64)
            iy = torch.floor(y).to(torch.int64)
            on = (ix >= 0) & (ix < w) & (iy >= 0) & (iy < w)
            p = torch.where(on, iy * w + ix, torch.full_like(ix, -1))
            pix[sl] = p.to(torch.int32)
            pc = torch.where(on, p, torch.zeros_like(p))
            sig = sky[0][pc]
            if cfg.ncomp == 3:
                if cfg.psi_kind == "u16":
                    ti = (2 * c + half).to(torch.int32)
                    psi[sl] = ti.to(torch.uint16)
                    ang = tab_dev[ti].to(torch.float64)
                else:
                    base = math.pi * c / cfg.ndet
                    a64 = base + (math.pi / 4) * half.to(torch.float64)
                    a_st = a64.to(torch.float32) if cfg.psi_kind == "f32" else a64
                    psi[sl] = a_st
                    ang = a_st.to(torch.float64)
                two = 2.0 * ang
                sig = sig + sky[1][pc] * torch.cos(two) + sky[2][pc] * torch.sin(two)
            sig = torch.where(on, sig, torch.zeros_like(sig))
            if noise_scale != 0.0:
                seed = int(ss_chunks[c].generate_state(1, np.uint64)[0])
                g = torch.Generator(device=dev)
                g.manual_seed(seed)
                white = torch.randn(n, generator=g, dtype=torch.float64, device=dev)
                shape = float(sig_all[c]) * torch.sqrt(1.0 + (f / float(fk_all[c])) ** float(al_all[c]))
                noise = torch.fft.irfft(torch.fft.rfft(white) * shape, n=n)
                sig = sig + noise * noise_scale
            d[sl] = sig.to(tod_t)
    return DeviceProblem(cfg=cfg, chunks=idx, chunk_off=off, fsample=np.full(len(idx), cfg.fsample),
                         sigma=sig_all[idx], fknee=fk_all[idx], alpha=al_all[idx], pix=pix, psi=psi,
                         psi_table=psi_table, d=d, m_true=m_true)
