"""The CPU oracle over large workloads, chunk group by chunk group, in a pool of host threads.

Test infrastructure: it calls the oracle's own functions on slices of the workload's chunks
and adds up what is a sum over chunks (P^T y, the weight blocks P^T T^-1 P, hit counts, chi^2);
the per-pixel solves use the oracle's functions on the summed blocks.  `get_chunks(idx)` returns
the host arrays of the listed chunks with their own chunk table (keys chunk_off, fsample, sigma,
fknee, alpha, pix, psi (stored angle values or None), d)."""

from __future__ import annotations

import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
from oracle.messenger import _hold_unsolvable, apply_filter, chi2_of_residual, weighted_solve
from oracle.noise import NoiseModel
from oracle.pointing import Pointing, invert_blocks


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def group_setup(get_chunks, idx, npix, ncomp):
    h = get_chunks(idx)
    pt = Pointing(h["pix"], h["psi"], npix, ncomp)
    nm = NoiseModel.from_params(h["chunk_off"], h["fsample"], h["sigma"], h["fknee"], h["alpha"])
    return oracle.Setup(pointing=pt, noise=nm, W=None, W_inv=None, solvable=None, hits=None), h


def sweep(nchunk, get_chunks, npix, ncomp, fn, nacc, group=4, threads=16, label="oracle"):
    """Sum over chunk groups of fn(S_group, h_group) (a tuple of nacc arrays)."""
    groups = [list(range(g, min(g + group, nchunk))) for g in range(0, nchunk, group)]
    accs, lock = {}, threading.Lock()  # one accumulator per worker thread

    def work(idx):
        key = threading.get_ident()
        with lock:
            acc = accs.setdefault(key, [None])
        S, h = group_setup(get_chunks, idx, npix, ncomp)
        out = fn(S, h)
        if acc[0] is None:
            acc[0] = [np.array(o, dtype=np.float64, copy=True) for o in out]
        else:
            for a, o in zip(acc[0], out):
                a += o
        return len(idx)

    done, t0, step = 0, time.perf_counter(), max(1, nchunk // 4)
    with ThreadPoolExecutor(threads) as ex:
        for n in ex.map(work, groups):
            mark = done // step
            done += n
            if done // step != mark:
                say(f"  {label}: {done}/{nchunk} chunks, {time.perf_counter() - t0:.0f} s")
    return [sum(a[0][i] for a in accs.values() if a[0] is not None) for i in range(nacc)]


class Binned:
    """Hits, weight blocks and their inverses, and the binned map W^-1 P^T T^-1 d (Section 2.1)."""

    def __init__(self, nchunk, get_chunks, npix, ncomp, **kw):
        def fn(S, h):
            inv_tau = 1.0 / S.noise.tau_per_sample()
            W = S.pointing.weight_blocks(inv_tau)
            b = S.pointing.back(np.asarray(h["d"], dtype=np.float64) * inv_tau)
            return S.pointing.hits().astype(np.float64), W, b

        hits, W, b = sweep(nchunk, get_chunks, npix, ncomp, fn, 3, label="oracle binned map", **kw)
        self.hits = hits.astype(np.int64)
        Winv, solvable = invert_blocks(W, self.hits)
        self.S = oracle.Setup(pointing=Pointing(np.zeros(0, np.int64), np.zeros(0), npix, ncomp), noise=None,
                              W=W, W_inv=Winv, solvable=solvable, hits=self.hits)
        self.solvable = solvable
        self.m_bin = _hold_unsolvable(self.S, weighted_solve(self.S, b))
        self.nchunk, self.get_chunks, self.npix, self.ncomp, self.kw = nchunk, get_chunks, npix, ncomp, kw

    def chi2(self, m):
        """chi^2(m) of eqn. (chi2), summed over all chunks."""
        def fn(S, h):
            r = np.asarray(h["d"], dtype=np.float64) - S.pointing.project(m)
            return (np.atleast_1d(chi2_of_residual(S, r, 1.0)),)

        return float(sweep(self.nchunk, self.get_chunks, self.npix, self.ncomp, fn, 1, label="oracle chi^2",
                           **self.kw)[0][0])

    def step(self, m, lam):
        """One iteration of eqn. (mcompact) from m at lambda (finite), and chi^2(m) of eqn. (chi2)."""
        def fn(S, h):
            r = np.asarray(h["d"], dtype=np.float64) - S.pointing.project(m)
            chi = np.atleast_1d(chi2_of_residual(S, r, 1.0))
            return S.pointing.back(apply_filter(S, r, lam)), chi

        b, chi = sweep(self.nchunk, self.get_chunks, self.npix, self.ncomp, fn, 2,
                       label=f"oracle iteration at lambda={lam:g}", **self.kw)
        return _hold_unsolvable(self.S, m + weighted_solve(self.S, b)), float(chi[0])


def problem_chunks(prob):
    """get_chunks for a host-generated synth.Problem (stored angle values, table lookups resolved)."""
    off = prob.chunk_off
    psi = prob.psi_values()

    def get(idx):
        sl = [slice(int(off[c]), int(off[c + 1])) for c in idx]
        lens = np.array([s.stop - s.start for s in sl], dtype=np.int64)
        ix = np.asarray(idx)
        cat = lambda a: np.concatenate([a[s] for s in sl])  # noqa: E731
        return dict(chunk_off=np.concatenate([[0], np.cumsum(lens)]), fsample=prob.fsample[ix],
                    sigma=prob.sigma[ix], fknee=prob.fknee[ix], alpha=prob.alpha[ix], pix=cat(prob.pix),
                    psi=None if psi is None else cat(psi), d=cat(prob.d))

    return get
