"""Scan patterns (pointing) for the synthetic workloads.

Positions are continuous pixel coordinates: pixel (x, y) covers
[x, x+1) x [y, y+1) and has index p = y * nx + x.  Pointing is nearest-pixel
(the pixel containing the position), so the sky is constant inside a pixel and
the data carry no sub-pixel signal.  Samples that land outside the map get
index -1.

``boustrophedon64``: the fixed temperature-only raster.  The first half of the
chunk sweeps rows left-right / right-left (each pixel gets the same number of
consecutive samples), the second half sweeps columns the same way, so every
pixel is hit equally often from two orthogonal directions.

``crossed``: each detector's chunk is split in two halves.  The first half is a
horizontal boustrophedon with one line per map row; the second half is the same
pattern rotated by 45 degrees about the map centre, so its corners leave the
map.  Each detector carries a fixed offset inside one pixel, and its
polarization angle is pi*c/ndet in the first half and pi*c/ndet + pi/4 in the
second.  The octagonal centre is cross-linked, the corners are not.
"""

from __future__ import annotations

import numpy as np


def _boustrophedon64(n: int, nx: int):
    half = n // 2
    per_row = half // nx
    per_pix = per_row // nx
    if per_pix * nx * nx != half or 2 * half != n:
        raise ValueError("boustrophedon64 needs n = 2 * nx * nx * k")
    s = np.arange(half, dtype=np.int64)
    row = s // per_row
    col = (s % per_row) // per_pix
    col = np.where(row % 2 == 1, nx - 1 - col, col)
    p_h = row * nx + col            # horizontal sweep: (x=col, y=row)
    p_v = col * nx + row            # vertical sweep: x and y swapped
    pix = np.concatenate([p_h, p_v]).astype(np.int32)
    halfid = np.concatenate([np.zeros(half, np.int8), np.ones(half, np.int8)])
    return pix, halfid


def _raster_positions(nh: int, w: int, rotate: bool):
    s = np.arange(nh, dtype=np.int64)
    line = (s * w) // nh
    a = ((s * w) % nh).astype(np.float64) / nh
    x = np.where(line % 2 == 1, (1.0 - a) * w, a * w)
    y = line.astype(np.float64) + 0.5
    if rotate:
        c = np.cos(np.pi / 4)
        xc, yc = x - 0.5 * w, y - 0.5 * w
        x = c * xc - c * yc + 0.5 * w
        y = c * xc + c * yc + 0.5 * w
    return x, y


def chunk_pointing(cfg, c: int, n: int, offset):
    """Pixel index (int32), stored angle (or None) and scan-half id (int8) of chunk ``c``."""
    w = cfg.nx
    if cfg.scan == "boustrophedon64":
        pix, halfid = _boustrophedon64(n, w)
        return pix, None, halfid
    if cfg.scan != "crossed":
        raise ValueError(cfg.scan)
    nh0 = n // 2
    nh1 = n - nh0
    x0, y0 = _raster_positions(nh0, w, rotate=False)
    x1, y1 = _raster_positions(nh1, w, rotate=True)
    x = np.concatenate([x0, x1]) + (offset[0] - 0.5)
    y = np.concatenate([y0, y1]) + (offset[1] - 0.5)
    ix = np.floor(x).astype(np.int64)
    iy = np.floor(y).astype(np.int64)
    on = (ix >= 0) & (ix < w) & (iy >= 0) & (iy < w)
    pix = np.where(on, iy * w + ix, -1).astype(np.int32)
    halfid = np.concatenate([np.zeros(nh0, np.int8), np.ones(nh1, np.int8)])
    psi = None
    if cfg.ncomp == 3:
        base = np.pi * c / cfg.ndet
        psi64 = base + (np.pi / 4) * halfid.astype(np.float64)
        psi = psi64.astype(np.float32) if cfg.psi_kind in ("f32", "u16") else psi64
    return pix, psi, halfid
