"""The chunk-group sweep used by the large parity tests gives the oracle's whole-problem results
(sums over chunks taken group by group in threads).  The groups' partial sums are added in an
order that depends on thread scheduling, and the 3x3 solves of pixels whose angles barely
separate Q from U amplify that rounding, hence 1e-11 rather than a few ulps."""

import numpy as np

from oracle.messenger import binned_map, chi2, make_setup, messenger_step
from tests.oracle_sweeps import Binned
from tests.tiny_inputs import tiny_problem


def test_group_sweep_equals_whole_problem():
    t = tiny_problem(9001, ncomp=3, lengths=(64, 48, 96, 32, 80, 64, 40), nx=6)
    off = t.chunk_off

    def get_chunks(idx):
        sl = [slice(int(off[c]), int(off[c + 1])) for c in idx]
        lens = np.array([s.stop - s.start for s in sl], dtype=np.int64)
        ix = np.asarray(idx)
        cat = lambda a: np.concatenate([a[s] for s in sl])  # noqa: E731
        return dict(chunk_off=np.concatenate([[0], np.cumsum(lens)]), fsample=t.fsample[ix], sigma=t.sigma[ix],
                    fknee=t.fknee[ix], alpha=t.alpha[ix], pix=cat(t.pix), psi=cat(t.psi), d=cat(t.d))

    S = make_setup(off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    B = Binned(len(off) - 1, get_chunks, t.npix, 3, group=2, threads=3)
    assert np.array_equal(B.hits, S.hits)
    assert np.array_equal(B.solvable, S.solvable)
    ref = binned_map(S, t.d)
    assert np.linalg.norm(B.m_bin - ref) / np.linalg.norm(ref) < 1e-11
    m1, c0 = B.step(ref, 7.0)
    r1 = messenger_step(S, t.d, ref, 7.0)
    assert np.linalg.norm(m1 - r1) / np.linalg.norm(r1) < 1e-11
    assert abs(c0 - chi2(S, t.d, ref)) / chi2(S, t.d, ref) < 1e-12
