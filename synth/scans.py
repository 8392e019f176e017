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

``chunk_pointing_differential``: the same scan carrying a pair of beams a fixed
distance apart, as the differencing assemblies of Section 3.2.
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


def _crossed_positions(cfg, n: int, offset):
    w = cfg.nx
    nh0 = n // 2
    x0, y0 = _raster_positions(nh0, w, rotate=False)
    x1, y1 = _raster_positions(n - nh0, w, rotate=True)
    x = np.concatenate([x0, x1]) + (offset[0] - 0.5)
    y = np.concatenate([y0, y1]) + (offset[1] - 0.5)
    halfid = np.concatenate([np.zeros(nh0, np.int8), np.ones(n - nh0, np.int8)])
    return x, y, halfid


def _nearest(x, y, w):
    ix = np.floor(x).astype(np.int64)
    iy = np.floor(y).astype(np.int64)
    on = (ix >= 0) & (ix < w) & (iy >= 0) & (iy < w)
    return np.where(on, iy * w + ix, -1)


def _angles(cfg, c: int, halfid):
    if cfg.ncomp != 3:
        return None
    base = np.pi * c / cfg.ndet
    psi64 = base + (np.pi / 4) * halfid.astype(np.float64)
    return psi64.astype(np.float32) if cfg.psi_kind in ("f32", "u16") else psi64


def chunk_pointing(cfg, c: int, n: int, offset):
    """Pixel index (int32), stored angle (or None) and scan-half id (int8) of chunk ``c``."""
    w = cfg.nx
    if cfg.scan == "boustrophedon64":
        pix, halfid = _boustrophedon64(n, w)
        return pix, None, halfid
    if cfg.scan != "crossed":
        raise ValueError(cfg.scan)
    x, y, halfid = _crossed_positions(cfg, n, offset)
    return _nearest(x, y, w).astype(np.int32), _angles(cfg, c, halfid), halfid


def chunk_pointing_differential(cfg, c: int, n: int, offset):
    """Two beams of chunk ``c`` on the crossed rasters: beam A as in ``chunk_pointing``, beam B
    ``cfg.diff_sep`` pixels away along the direction 2 pi c / ndet (turned by 45 degrees with the
    rotated half of the scan, so the pair keeps its orientation relative to the scan lines).  A
    sample with either beam off the map is flagged in both (index -1): a difference needs both
    ends.  Returns (pix_a, pix_b, angle, halfid); both beams share the angle."""
    if cfg.scan != "crossed":
        raise ValueError("differential beams ride the crossed rasters")
    w = cfg.nx
    x, y, halfid = _crossed_positions(cfg, n, offset)
    theta = 2.0 * np.pi * c / cfg.ndet + (np.pi / 4) * halfid.astype(np.float64)
    pa = _nearest(x, y, w)
    pb = _nearest(x + cfg.diff_sep * np.cos(theta), y + cfg.diff_sep * np.sin(theta), w)
    both = (pa >= 0) & (pb >= 0)
    pa = np.where(both, pa, -1).astype(np.int32)
    pb = np.where(both, pb, -1).astype(np.int32)
    return pa, pb, _angles(cfg, c, halfid), halfid
