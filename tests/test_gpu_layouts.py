"""GPU parity of the transform layouts: every candidate layout (split M = M1 M2, column-block
width, radix order) of several chunk lengths, selected with MM_TUNE_PICK0 + i, against the CPU
FP64 oracle; and the layout the plan-time tuner picks."""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.messenger import chi2, chi2_of_residual, make_setup, messenger_step  # noqa: E402
from paper_1705_01893_amd import mm  # noqa: E402
from tests.tiny_inputs import random_map, tiny_problem  # noqa: E402

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10
MIX_TOL = 1e-5

# chunk lengths n = 2M: a power of two, and mixed radix-2/3/5 half lengths
LENGTHS = {
    "pow2": (2 ** 15, 2 ** 14),
    "mixed": (2 * 3 * 5 * 2 ** 8, 2 * 27 * 25 * 4),
}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def wave_local_inverse(lay):
    """Whether a plan with these layouts (not FP64 power-of-two) runs the inverse column pass
    in the wave-local LDS layout: every class holds at least one column per wave (8 waves)."""
    return all(l["cb"] >= 8 for l in lay)


def plan_for(t, dev, tune, precision=mm.MM_FP64):
    psi = torch.from_numpy(np.ascontiguousarray(t.psi)).to(dev)
    return mm.mm_plan(ncomp=3, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample, sigma=t.sigma,
                      fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(t.pix).to(dev), psi=psi,
                      precision=precision, tune=tune)


@pytest.mark.parametrize("shape", list(LENGTHS))
def test_every_layout_fp64(dev, shape):
    t = tiny_problem(77, ncomp=3, lengths=LENGTHS[shape], nx=16)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    m0 = random_map(7, 3, t.npix)
    m0[:, ~S.solvable] = 0
    ref = {lam: messenger_step(S, t.d, m0, lam) for lam in (1.0, 37.5)}
    c2ref = chi2(S, t.d, m0)
    d = torch.from_numpy(t.d).to(dev)
    ncand = mm.mm_plan_chunk_layout(plan_for(t, dev, mm.MM_TUNE_STATIC), 0)["ncand"]
    seen = set()
    kinds = set()
    for pick in range(max(ncand, mm.mm_plan_chunk_layout(plan_for(t, dev, mm.MM_TUNE_STATIC), 1)["ncand"])):
        plan = plan_for(t, dev, mm.MM_TUNE_PICK0 + pick)
        lay = [mm.mm_plan_chunk_layout(plan, c) for c in range(plan.nchunk)]
        key = tuple((l["M1"], l["M2"], l["cb"], l["pick"]) for l in lay)
        say(f"[layout] shape={shape} pick={pick} {key}")
        assert all(l["M1"] * l["M2"] * 2 == n for l, n in zip(lay, LENGTHS[shape]))
        seen.add(key)
        kinds.add(wave_local_inverse(lay))
        mi = torch.from_numpy(m0).to(dev)
        for lam, r in ref.items():
            mo = torch.zeros_like(mi)
            c2 = torch.zeros(1, dtype=torch.float64, device=dev)
            mm.mm_messenger_iter(plan, d, lam, mi, mo, c2)
            torch.cuda.synchronize()
            assert rel(mo.cpu().numpy(), r) < F64_TOL, (pick, lam)
            assert c2.item() == pytest.approx(c2ref, rel=F64_TOL)
    assert len(seen) >= 3  # several distinct layouts were exercised
    if shape == "mixed":  # both LDS layouts of the inverse column pass were exercised
        assert kinds == {True, False}


@pytest.mark.parametrize("shape", list(LENGTHS))
def test_every_layout_mixed(dev, shape):
    t = tiny_problem(78, ncomp=3, lengths=LENGTHS[shape], nx=16, psi_dtype=np.float32, tod_dtype=np.float32)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    m0 = random_map(8, 3, t.npix)
    m0[:, ~S.solvable] = 0
    ref = messenger_step(S, t.d.astype(np.float64), m0, 1.0)
    d = torch.from_numpy(t.d).to(dev)
    n0 = mm.mm_plan_chunk_layout(plan_for(t, dev, mm.MM_TUNE_STATIC, mm.MM_MIXED), 0)["ncand"]
    kinds = set()
    for pick in range(n0):
        say(f"[layout mixed] pick={pick}")
        plan = plan_for(t, dev, mm.MM_TUNE_PICK0 + pick, mm.MM_MIXED)
        kinds.add(wave_local_inverse([mm.mm_plan_chunk_layout(plan, c) for c in range(plan.nchunk)]))
        mi = torch.from_numpy(m0).to(dev)
        mo = torch.zeros_like(mi)
        mm.mm_messenger_iter(plan, d, 1.0, mi, mo)
        torch.cuda.synchronize()
        assert rel(mo.cpu().numpy(), ref) < MIX_TOL, pick
    if shape == "mixed":
        assert kinds == {True, False}


def test_register_column_transform_mixed(dev):
    """A 2^21-sample chunk under its 1024 x 1024 split with 8-column blocks, whose inverse column
    pass transforms each 1024-point column in one wave's registers (lane shuffles between the
    radix-2 levels); FP32-mixed iterations at lambda = 1 and 37.5 and chi^2 against the FP64
    oracle."""
    t = tiny_problem(84, ncomp=3, lengths=(2 ** 21, 2 ** 15), nx=16, psi_dtype=np.float32, tod_dtype=np.float32,
                     walk=False)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    ncand = mm.mm_plan_chunk_layout(plan_for(t, dev, mm.MM_TUNE_STATIC, mm.MM_MIXED), 0)["ncand"]
    plan = None
    for pick in range(ncand):
        cand = plan_for(t, dev, mm.MM_TUNE_PICK0 + pick, mm.MM_MIXED)
        lay = mm.mm_plan_chunk_layout(cand, 0)
        if (lay["M2"], lay["cb"]) == (1024, 8):
            plan = cand
            break
    say(f"[register columns] {lay}")
    assert plan is not None
    m0 = random_map(11, 3, t.npix)
    m0[:, ~S.solvable] = 0
    d64 = t.d.astype(np.float64)
    d = torch.from_numpy(t.d).to(dev)
    for lam in (1.0, 37.5):
        mo = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
        c2 = torch.zeros(1, dtype=torch.float64, device=dev)
        mm.mm_messenger_iter(plan, d, lam, torch.from_numpy(m0).to(dev), mo, c2)
        torch.cuda.synchronize()
        assert rel(mo.cpu().numpy(), messenger_step(S, d64, m0, lam)) < MIX_TOL, lam
        assert c2.item() == pytest.approx(chi2(S, d64, m0), rel=1e-6)


def test_inverse_pass_layout_per_class(dev):
    """Two chunk lengths whose static layouts differ in the inverse column pass's LDS layout
    (2^22 complex values: 4 columns per item, interleaved; 2^16: 16 columns, wave-local), so the
    pass picks the layout per transform class; FP32-mixed against the FP64 oracle."""
    t = tiny_problem(80, ncomp=3, lengths=(2 ** 23, 2 ** 17), nx=16, psi_dtype=np.float32, tod_dtype=np.float32,
                     walk=False)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    plan = plan_for(t, dev, mm.MM_TUNE_STATIC, mm.MM_MIXED)
    lay = [mm.mm_plan_chunk_layout(plan, c) for c in range(plan.nchunk)]
    say(f"[layout per class] {lay}")
    assert lay[0]["cb"] < 8 <= lay[1]["cb"]
    m0 = random_map(10, 3, t.npix)
    m0[:, ~S.solvable] = 0
    mo = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    mm.mm_messenger_iter(plan, torch.from_numpy(t.d).to(dev), 2.0, torch.from_numpy(m0).to(dev), mo)
    torch.cuda.synchronize()
    assert rel(mo.cpu().numpy(), messenger_step(S, t.d.astype(np.float64), m0, 2.0)) < MIX_TOL


def test_tuner_picks_a_valid_layout(dev):
    """Chunks long enough to be tuned: the measured choice is one of the candidates and the
    iteration it runs matches the oracle."""
    t = tiny_problem(79, ncomp=3, lengths=(2 ** 16, 2 * 3 * 5 * 2 ** 12), nx=16)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    plan = plan_for(t, dev, mm.MM_TUNE_MEASURE)
    for c in range(plan.nchunk):
        lay = mm.mm_plan_chunk_layout(plan, c)
        say(f"[tuned] chunk {c}: {lay}")
        assert 0 <= lay["pick"] < lay["ncand"]
        assert 2 * lay["M1"] * lay["M2"] == int(t.chunk_off[c + 1] - t.chunk_off[c])
    assert mm.mm_plan_chunk_layout(plan_for(t, dev, mm.MM_TUNE_STATIC), 0)["pick"] == 0
    m0 = random_map(9, 3, t.npix)
    m0[:, ~S.solvable] = 0
    mo = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
    mm.mm_messenger_iter(plan, torch.from_numpy(t.d).to(dev), 4.0, torch.from_numpy(m0).to(dev), mo)
    torch.cuda.synchronize()
    assert rel(mo.cpu().numpy(), messenger_step(S, t.d, m0, 4.0)) < F64_TOL


def test_tuner_choice_persisted(dev, tmp_path, monkeypatch):
    """MM_TUNE_CACHE: a measured choice is written to the file, one line per key ending with the
    chosen index, and a later plan reading a file (a new path, so the in-process cache misses)
    takes the index it finds there instead of timing the candidates."""
    t = tiny_problem(83, ncomp=3, lengths=(2 * 3 * 5 * 2 ** 11,), nx=16)
    first = tmp_path / "tune_a.txt"
    monkeypatch.setenv("MM_TUNE_CACHE", str(first))
    lay = mm.mm_plan_chunk_layout(plan_for(t, dev, mm.MM_TUNE_MEASURE), 0)
    say(f"[tune cache] measured: {lay}")
    assert lay["ncand"] > 1
    lines = first.read_text().splitlines()
    assert len(lines) == 1
    tok = lines[0].split()
    assert len(tok) == 8 and int(tok[7]) == lay["pick"]
    # the key: device, runtime, build, M, precision, the TOD streams pass A reads (this small map
    # is gathered: d alone) and the number of candidates timed
    ntimed = int(tok[6])
    assert int(tok[3]) == 2 * 3 * 5 * 2 ** 10 and tok[4] == "f64" and tok[5] == "a1"
    assert 1 < ntimed <= lay["ncand"]
    other = (lay["pick"] + 1) % ntimed
    second = tmp_path / "tune_b.txt"
    second.write_text("not a choice\n" + " ".join(tok[:7] + [str(other)]) + "\n")
    monkeypatch.setenv("MM_TUNE_CACHE", str(second))
    lay2 = mm.mm_plan_chunk_layout(plan_for(t, dev, mm.MM_TUNE_MEASURE), 0)
    say(f"[tune cache] read back: {lay2}")
    assert lay2["pick"] == other
    # projected map access: pass A reads d and P m, so the timing does too, under a key of its own
    third = tmp_path / "tune_c.txt"
    monkeypatch.setenv("MM_TUNE_CACHE", str(third))
    psi = torch.from_numpy(np.ascontiguousarray(t.psi)).to(dev)
    plan3 = mm.mm_plan(ncomp=3, npix=t.npix, nx=t.nx, chunk_off=t.chunk_off, fsample=t.fsample, sigma=t.sigma,
                       fknee=t.fknee, alpha=t.alpha, pix=torch.from_numpy(t.pix).to(dev), psi=psi,
                       precision=mm.MM_FP64, tune=mm.MM_TUNE_MEASURE, map_access=mm.MM_MAP_PROJECTED)
    lay3 = mm.mm_plan_chunk_layout(plan3, 0)
    tok3 = third.read_text().split()
    say(f"[tune cache] projected: {lay3} {tok3}")
    assert len(tok3) == 8 and tok3[5] == "a2" and tok3[:5] == tok[:5] and int(tok3[7]) == lay3["pick"]


def test_long_chunks_mixed(dev):
    """Two 2^22-sample chunks (the large workload's chunk length) under its 2048 x 1024 split with
    8-column blocks: FP32-mixed iterations at lambda = 1 and 37.5 and chi^2 with the iteration
    and on its own (per chunk, lambda = 5) against the FP64 oracle.  (At these lengths the FP32
    transforms' rounding, carried by the 1/f power the filter passes at large lambda, puts one
    iteration from a random map at 1.6e-6 relative at lambda = 1 and 8.8e-6 at 37.5.)"""
    t = tiny_problem(85, ncomp=3, lengths=(2 ** 22, 2 ** 22), nx=16, psi_dtype=np.float32, tod_dtype=np.float32,
                     walk=False)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    plan = plan_for(t, dev, mm.MM_TUNE_STATIC, mm.MM_MIXED)
    lay = [mm.mm_plan_chunk_layout(plan, c) for c in range(plan.nchunk)]
    say(f"[long chunks] {lay}")
    assert all((l["M1"], l["M2"], l["cb"]) == (2048, 1024, 8) for l in lay)
    m0 = random_map(12, 3, t.npix)
    m0[:, ~S.solvable] = 0
    d64 = t.d.astype(np.float64)
    d = torch.from_numpy(t.d).to(dev)
    mi = torch.from_numpy(m0).to(dev)
    for lam in (1.0, 37.5):
        mo = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
        c2 = torch.zeros(1, dtype=torch.float64, device=dev)
        mm.mm_messenger_iter(plan, d, lam, mi, mo, c2)
        torch.cuda.synchronize()
        assert rel(mo.cpu().numpy(), messenger_step(S, d64, m0, lam)) < MIX_TOL, lam
        assert c2.item() == pytest.approx(chi2(S, d64, m0), rel=1e-6)
    per = torch.zeros(plan.nchunk, dtype=torch.float64, device=dev)
    v = mm.mm_chi2(plan, d, mi, 5.0, per)
    ref = chi2_of_residual(S, d64 - S.pointing.project(m0), 5.0, per_chunk=True)
    assert v == pytest.approx(float(np.sum(ref)), rel=1e-6)
    assert np.allclose(per.cpu().numpy(), ref, rtol=1e-6, atol=0)


def test_long_chunks_fp64(dev):
    """Two 2^22-sample chunks under the FP64 split of that length (1024-point rows in pairs,
    2048-point columns in blocks of two: the compiled-in radix schedules, whose first and last
    stages read and write the work buffer): FP64 iterations at lambda = 1 and 37.5 and chi^2
    against the FP64 oracle."""
    t = tiny_problem(86, ncomp=3, lengths=(2 ** 22, 2 ** 22), nx=16, walk=False)
    S = make_setup(t.chunk_off, t.fsample, t.sigma, t.fknee, t.alpha, t.pix, t.psi, t.npix, 3)
    plan = plan_for(t, dev, mm.MM_TUNE_STATIC)
    lay = [mm.mm_plan_chunk_layout(plan, c) for c in range(plan.nchunk)]
    say(f"[long chunks fp64] {lay}")
    assert all((l["M1"], l["M2"], l["cb"]) == (1024, 2048, 2) for l in lay)
    m0 = random_map(13, 3, t.npix)
    m0[:, ~S.solvable] = 0
    d = torch.from_numpy(t.d).to(dev)
    mi = torch.from_numpy(m0).to(dev)
    for lam in (1.0, 37.5):
        mo = torch.zeros((3, t.npix), dtype=torch.float64, device=dev)
        c2 = torch.zeros(1, dtype=torch.float64, device=dev)
        mm.mm_messenger_iter(plan, d, lam, mi, mo, c2)
        torch.cuda.synchronize()
        assert rel(mo.cpu().numpy(), messenger_step(S, t.d, m0, lam)) < F64_TOL, lam
        assert c2.item() == pytest.approx(chi2(S, t.d, m0), rel=F64_TOL)
