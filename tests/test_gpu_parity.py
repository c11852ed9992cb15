"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Decisions (extrema count k, mask length L, step count m, number of IMFs)
must be identical, with no tie escape.  IMFs: FP64 entry points within
||d|| <= 1e-12 ||IMF|| + 1e-15 ||s||; FP32 entry points within 1e-5 relative
L2 per IMF.  At the benchmark sizes every signal's decisions are compared with
the oracle decisions stored by tests/golden/make_golden.py.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import siggen
from oracle import dif
from oracle import fif_spectral as fs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1802_01359_amd as fif  # noqa: E402

from parity_util import check, golden_equal, load_golden, record  # noqa: E402


def oracle_many(signals, delta, max_imfs, **kw):
    """Oracle decompositions in parallel threads (the C oracle releases the GIL)."""
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        futs = [ex.submit(dif.decompose, s, delta, max_imfs, **kw) for s in signals]
        return [f.result() for f in futs]


def _check(ref, s, imfs, rem, info, n, delta, fp64, lam_abs=None, config=None):
    check(ref, s, imfs, rem, info, n, delta, fp64, lam_abs, config)


def _signal(N, seed):
    if N < 64:
        return np.random.default_rng(seed).standard_normal(N)
    f = (max(1.0, N / 700.0), max(2.0, N / 90.0), N / 9.0)
    return siggen.tones3(N=N, freqs=f, seed_index=seed)


@pytest.mark.parametrize("N", [2, 3, 8, 30, 105, 360, 1000, 2048, 4096, 6000, 8192,
                               10000, 16384, 20736, 65536, 131072, 196608])
def test_fp64_single_matches_oracle(N):
    s = _signal(N, N)
    max_imfs = 6
    ref = dif.decompose(s, 1e-3, max_imfs)
    x = torch.tensor(s, dtype=torch.float64, device="cuda")
    print("case fp64 single N=%d" % N, flush=True)
    res = fif.decompose(x, 1e-3, max_imfs)
    torch.cuda.synchronize()
    imfs = np.zeros((max_imfs, N))
    imfs[:res.n_imfs] = res.imfs.cpu().numpy()
    _check(ref, s, imfs, res.remainder.cpu().numpy(), res.info, res.n_imfs, 1e-3, True,
           config="single-signal fp64 lengths 2..196608")


def test_three_tone_workload_fp64():
    """N = 4096, three AM tones at 8/40/200 cycles, delta 1e-3, 8 IMFs,
    against the literal time-domain iteration (folded taps)."""
    s = siggen.tones3()
    ref = dif.decompose(s, 1e-3, 8, inner_form=0)
    x = torch.tensor(s, dtype=torch.float64, device="cuda")
    res = fif.decompose(x, 1e-3, 8)
    torch.cuda.synchronize()
    imfs = np.zeros((8, 4096))
    imfs[:res.n_imfs] = res.imfs.cpu().numpy()
    _check(ref, s, imfs, res.remainder.cpu().numpy(), res.info, res.n_imfs, 1e-3, True,
           config="tones3-1x4096 fp64 (literal oracle)")


def _run_batch(lengths, sigs, delta, max_imfs, dtype, **opt):
    plan = fif.Plan(lengths, max_imfs, fif.Options(**opt))
    packed = torch.tensor(np.concatenate(sigs), dtype=dtype, device="cuda")
    out = plan.run(packed, delta)
    torch.cuda.synchronize()
    return plan, packed, out


@pytest.mark.parametrize("delta,lengths", [
    (1e-3, [4096, 1000, 8192, 16384, 6000, 2, 3, 30000, 65536, 12288, 360]),
    (1e-4, [4096, 1000, 2, 3, 360, 2048]),
])
def test_fp32_batch_mixed_lengths(delta, lengths):
    sigs = [_signal(N, 100 + i).astype(np.float32) for i, N in enumerate(lengths)]
    max_imfs = 7
    print("case fp32 batch delta=%g" % delta, flush=True)
    plan, packed, out = _run_batch(lengths, sigs, delta, max_imfs, torch.float32)
    info = out.info()
    n = out.n_imfs.cpu().numpy()
    assert np.all(out.sig_status.cpu().numpy() == 0)
    print("  oracle for %d signals" % len(lengths), flush=True)
    refs = oracle_many([s.astype(np.float64) for s in sigs], delta, max_imfs)
    for b, N in enumerate(lengths):
        s64 = sigs[b].astype(np.float64)
        ref = refs[b]
        imfs = out.imfs_of(b).cpu().numpy().astype(np.float64)
        rem = out.remainder_of(b).cpu().numpy().astype(np.float64)
        _check(ref, s64, imfs, rem, info[b], int(n[b]), delta, False, config="mixed-length fp32 batches")


def test_batch_is_independent_of_composition_and_deterministic():
    lengths = [4096, 65536, 1000, 16384, 4096]
    sigs = [_signal(N, 7 + i) for i, N in enumerate(lengths)]
    plan, packed, out = _run_batch(lengths, sigs, 1e-3, 6, torch.float64)
    out2 = plan.run(packed, 1e-3)
    torch.cuda.synchronize()
    assert torch.equal(out.imfs, out2.imfs) and torch.equal(out.remainders, out2.remainders)
    info = out.info()
    for b in (0, 1, 2):
        x = torch.tensor(sigs[b], dtype=torch.float64, device="cuda")
        res = fif.decompose(x, 1e-3, 6)
        torch.cuda.synchronize()
        k = res.n_imfs
        assert k == int(out.n_imfs[b])
        assert torch.equal(res.imfs, out.imfs_of(b)[:k])
        assert torch.equal(res.remainder, out.remainder_of(b))
        assert np.array_equal(res.info, info[b][:k])
    # permuted batch gives the same bits per signal
    perm = [2, 0, 4, 1, 3]
    p2, _, o2 = _run_batch([lengths[i] for i in perm], [sigs[i] for i in perm], 1e-3, 6, torch.float64)
    for nb, ob in enumerate(perm):
        assert torch.equal(o2.imfs_of(nb), out.imfs_of(ob))


def test_edge_cases():
    N = 512
    x = siggen.grid(N)
    cases = {
        "constant": np.full(N, 2.5),
        "zero": np.zeros(N),
        "ramp": x * x,
        "nan": np.where(np.arange(N) == 17, np.nan, np.cos(2 * np.pi * 9 * x)),
        "inf": np.where(np.arange(N) == 3, np.inf, np.cos(2 * np.pi * 9 * x)),
        "tones": siggen.tones3(N=N, freqs=(3, 17, 60)),
    }
    names = list(cases)
    plan, packed, out = _run_batch([N] * len(names), [cases[k] for k in names], 1e-3, 5, torch.float64)
    st = out.sig_status.cpu().numpy()
    n = out.n_imfs.cpu().numpy()
    for b, k in enumerate(names):
        s = cases[k]
        rem = out.remainder_of(b).cpu().numpy()
        imfs = out.imfs_of(b).cpu().numpy()
        if k in ("nan", "inf"):
            assert st[b] == fif._binding.FIF_ERR_NONFINITE and n[b] == 0
            assert np.array_equal(rem, s, equal_nan=True) and np.all(imfs == 0)
            continue
        assert st[b] == 0
        ref = dif.decompose(s, 1e-3, 5)
        assert n[b] == ref.n_imfs, k
        if ref.n_imfs == 0:
            assert np.all(imfs == 0)
            assert np.max(np.abs(rem - s)) <= 1e-15 * max(1.0, np.max(np.abs(s)))
    xs = torch.tensor(cases["nan"], dtype=torch.float64, device="cuda")
    with pytest.raises(fif.FifError):
        fif.decompose(xs, 1e-3, 4)


def test_cap_on_a_pure_tone():
    N = 256
    s = np.cos(2 * np.pi * 8 * np.arange(N) / N)
    ref = dif.decompose(s, 1e-6, 1, max_inner=50)
    x = torch.tensor(s, dtype=torch.float64, device="cuda")
    res = fif.decompose(x, 1e-6, 1, fif.Options(max_inner=50))
    assert int(res.info["m"][0]) == 50 == ref.m[0]
    assert res.info["flags"][0] & fif.IMF_CAP
    assert abs(res.info["sd"][0] - ref.sd[0]) < 1e-13


@pytest.mark.parametrize("N,k0", [(256, 8), (65536, 700), (131072, 1400)])
def test_pure_tone_runs_to_the_default_cap(N, k0):
    """A pure tone whose lambda exceeds delta has SD_m = lambda for every m:
    the answer is the cap (10^6, far past the step where the tone's weight
    underflows FP64), with SD = lambda, on both sides.  N = 65536 takes the
    deferred check in pass 1, which fails there and sends the step to the
    exact search; N = 131072 the multi-workgroup search."""
    s = np.cos(2 * np.pi * k0 * np.arange(N) / N + 0.3)
    delta = 5e-4
    ref = fs.decompose(s, delta, 1, mask_rule=1, search="bisect")
    assert ref.m[0] == 1_000_000 and ref.flags[0] & 1
    x = torch.tensor(s, dtype=torch.float64, device="cuda")
    print("pure tone N=%d k0=%d" % (N, k0), flush=True)
    res = fif.decompose(x, delta, 1, fif.Options(mask_rule=1))
    torch.cuda.synchronize()
    assert int(res.info["L"][0]) == ref.L[0]
    assert int(res.info["m"][0]) == 1_000_000
    assert res.info["flags"][0] & fif.IMF_CAP
    assert res.info["sd"][0] == pytest.approx(ref.sd[0], rel=1e-9)
    imf = res.imfs[0].cpu().numpy()
    assert np.linalg.norm(imf - ref.imfs[0]) <= 1e-12 * np.linalg.norm(s)


@pytest.mark.parametrize("N", [4096, 65536])
def test_mask_rule_paper_constant(N):
    s = _signal(N, 3)
    ref = dif.decompose(s, 1e-3, 5, mask_rule=1, nu=1.6)
    x = torch.tensor(s, dtype=torch.float64, device="cuda")
    res = fif.decompose(x, 1e-3, 5, fif.Options(mask_rule=1, nu=1.6))
    imfs = np.zeros((5, N))
    imfs[:res.n_imfs] = res.imfs.cpu().numpy()
    _check(ref, s, imfs, res.remainder.cpu().numpy(), res.info, res.n_imfs, 1e-3, True)


def test_large_lengths_multi_workgroup_scan():
    """Signals with more bins than one scan workgroup holds (N/2 > 32768)
    mixed with small ones in one FP32 batch."""
    lengths = [262144, 4096, 131072, 100000, 81920]
    sigs = [_signal(N, 500 + i).astype(np.float32) for i, N in enumerate(lengths)]
    plan, packed, out = _run_batch(lengths, sigs, 1e-3, 6, torch.float32)
    info = out.info()
    n = out.n_imfs.cpu().numpy()
    assert np.all(info["flags"][:, :] & 4 == 0)  # never out of search rounds
    print("  oracle for %d signals" % len(lengths), flush=True)
    refs = oracle_many([s.astype(np.float64) for s in sigs], 1e-3, 6)
    for b, ref in enumerate(refs):
        s64 = sigs[b].astype(np.float64)
        _check(ref, s64, out.imfs_of(b).cpu().numpy().astype(np.float64),
               out.remainder_of(b).cpu().numpy().astype(np.float64), info[b], int(n[b]), 1e-3, False)


def test_chirp_batch_full_size():
    """1024 signals of N = 65536 (2-6 AM chirps, 30 dB noise), FP32,
    delta 1e-3, 12 IMFs: the benchmark's configuration.  Every signal's IMF
    count and (k, L, m) equal the time-domain oracle's stored decisions; the
    IMFs of eight signals are compared with the time-domain oracle; every
    signal reconstructs."""
    B, N, J = 1024, 65536, 12
    gold = load_golden("chirps")
    assert len(gold) == B
    print("case chirp batch B=%d N=%d" % (B, N), flush=True)
    sigs = [siggen.chirps(i).astype(np.float32) for i in range(B)]
    plan, packed, out = _run_batch([N] * B, sigs, 1e-3, J, torch.float32)
    assert int(out.sig_status.abs().sum()) == 0
    n = out.n_imfs.cpu().numpy()
    info = out.info()
    for b in range(B):
        golden_equal(gold[b], info[b], int(n[b]), 1e-3, "chirps signal %d" % b)
    # reconstruction of every signal (sum of IMF rows + remainder = signal)
    im = out.imfs.view(B, J, N).double()
    recon = im.sum(1) + out.remainders.view(B, N).double()
    err = (recon - packed.view(B, N).double()).norm(dim=1) / packed.view(B, N).double().norm(dim=1)
    assert float(err.max()) < 1e-6
    picks = (0, 1, 170, 341, 512, 682, 853, 1023)
    print("  oracle for signals %s" % (picks,), flush=True)
    refs = oracle_many([sigs[b].astype(np.float64) for b in picks], 1e-3, J)
    for b, ref in zip(picks, refs):
        s64 = sigs[b].astype(np.float64)
        _check(ref, s64, out.imfs_of(b).cpu().numpy().astype(np.float64),
               out.remainder_of(b).cpu().numpy().astype(np.float64), info[b], int(n[b]), 1e-3, False,
               config="chirps-1024x65536 fp32")


def _spectral_many(signals, delta, max_imfs):
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        futs = [ex.submit(fs.decompose, s, delta, max_imfs, search="bisect") for s in signals]
        return [f.result() for f in futs]


def test_uneven_batch_full_size():
    """The benchmark's uneven configuration: 4096 FP32 signals, 7-smooth
    lengths log-uniform in [1024, 262144], delta 1e-4, 12 IMFs.  The stored
    time-domain oracle decisions of a 64-signal sample stratified by length
    must be met exactly; every signal reconstructs; the IMFs of eight of the
    sampled signals are compared with the spectral oracle (bisection search:
    its m is pinned to the linear scan's)."""
    L = [int(n) for n in siggen.uneven_lengths(4096)]
    gold = load_golden("uneven")
    print("case uneven batch B=%d total=%d" % (len(L), sum(L)), flush=True)
    sigs = [siggen.uneven_signal(i, n).astype(np.float32) for i, n in enumerate(L)]
    plan, packed, out = _run_batch(L, sigs, 1e-4, 12, torch.float32)
    assert int(out.sig_status.abs().sum()) == 0
    info = out.info()
    n = out.n_imfs.cpu().numpy()
    assert np.all(info["flags"] & 4 == 0)
    for b, g in gold.items():
        assert g["N"] == L[b]
        golden_equal(g, info[b], int(n[b]), 1e-4, "uneven signal %d (N=%d)" % (b, L[b]))
    worst = 0.0
    for b in range(len(L)):
        x = packed[int(out.offsets[b]):int(out.offsets[b + 1])].double()
        rec = out.imfs_of(b).double().sum(0) + out.remainder_of(b).double()
        worst = max(worst, float((rec - x).norm() / x.norm()))
    assert worst < 1e-6, worst
    keys = sorted(gold, key=lambda b: L[b])
    picks = [keys[i] for i in (0, 9, 18, 27, 36, 45, 54, 63)]
    print("  spectral oracle for signals %s lengths %s" % (picks, [L[b] for b in picks]), flush=True)
    refs = _spectral_many([sigs[b].astype(np.float64) for b in picks], 1e-4, 12)
    for b, ref in zip(picks, refs):
        s64 = sigs[b].astype(np.float64)
        _check(ref, s64, out.imfs_of(b).cpu().numpy().astype(np.float64),
               out.remainder_of(b).cpu().numpy().astype(np.float64), info[b], int(n[b]), 1e-4, False,
               config="uneven-4096x[1024,262144] fp32")


@pytest.mark.timeout(900)
def test_long_signal_full_size():
    """The benchmark's long configuration: one FP32 signal of 2^24 samples,
    delta 1e-3, 20 IMFs.  Every IMF's (k, L, m) and the IMF count equal the
    stored decisions of the direct-form oracle (linear scan); every IMF is
    compared with the oracle's IMF, rebuilt from those decisions by the
    direct form; reconstruction and zero-mean IMFs."""
    s = siggen.long_drift().astype(np.float32)
    N = s.size
    g = load_golden("long")[0]
    print("case long N=%d" % N, flush=True)
    plan, packed, out = _run_batch([N], [s], 1e-3, 20, torch.float32)
    info = out.info()[0]
    nn = int(out.n_imfs.cpu().numpy()[0])
    assert np.all(info["flags"] & 4 == 0)
    golden_equal(g, info, nn, 1e-3, "long signal")
    im = out.imfs_of(0).double()
    rec = im.sum(0) + out.remainder_of(0).double()
    x = packed.double()
    assert float((rec - x).norm() / x.norm()) < 1e-6
    means = im[:nn].mean(1).abs().cpu().numpy()
    assert np.all(means <= 1e-6 * float(x.abs().max()))
    print("  oracle IMFs from the stored decisions, %d IMFs" % nn, flush=True)
    ref, _ = fs.imfs_at(s.astype(np.float64), g["L"], g["m"])
    imfs = out.imfs_of(0).cpu().numpy()
    for j in range(nn):
        a = ref[j]
        err = np.linalg.norm(a - imfs[j].astype(np.float64)) / np.linalg.norm(a)
        assert err <= 1e-5, (j, err)
        record("long-1x16777216 fp32", err)
    record("long-1x16777216 fp32", 0.0, imfs=0, signals=1)


# with a one-pass length (4096) beside the four-step ones, and without: a
# group whose one-workgroup scan list holds only four-step signals runs the
# 1024-thread scan kernel without the FP64 search
REDO_LENGTHS = {"mixed": [65536, 65536, 16384, 4096, 12000, 10125, 131072, 98415],
                "four_step": [65536, 16384, 12000, 10125, 131072, 98415]}


@pytest.mark.parametrize("kind", sorted(REDO_LENGTHS))
@pytest.mark.parametrize("shift", [1, -1])
def test_deferred_check_redo_path(shift, kind, monkeypatch):
    """The FP64 check of m for four-step signals runs inside pass 1; when it
    fails the step is redone (exact search, pass 1 again; for signals of the
    multi-workgroup search its FP64 rounds). A host-side hook shifts every
    deferred estimate so that every check fails: decisions must equal the
    unshifted run's and the oracle's, and every IMF is flagged as refined
    (but m = 1 shifted down, which stays 1 and passes).  Lengths: paired and
    unpaired four-step plans (10125 = 3^4 5^3), and the multi-workgroup search
    with paired (131072) and unpaired (98415 = 3^9 5) plans."""
    lengths = REDO_LENGTHS[kind]
    sigs = [siggen.chirps(i).astype(np.float32) if N == 65536 else _signal(N, 900 + i).astype(np.float32)
            for i, N in enumerate(lengths)]
    print("case deferred check shift=%d lengths %s" % (shift, lengths), flush=True)
    plan0, packed, ref = _run_batch(lengths, sigs, 1e-3, 6, torch.float32)
    monkeypatch.setenv("FIF_DEBUG_MT_SHIFT", str(shift))
    plan1, _, out = _run_batch(lengths, sigs, 1e-3, 6, torch.float32)
    i0, i1 = ref.info(), out.info()
    n0, n1 = ref.n_imfs.cpu().numpy(), out.n_imfs.cpu().numpy()
    assert np.array_equal(n0, n1)
    for key in ("k", "L", "m"):
        assert np.array_equal(i0[key], i1[key]), key
    for b, N in enumerate(lengths):
        four_step = N > 8192
        valid = np.arange(6) < n1[b]
        if four_step:
            refined = (i1["flags"][b][valid] & fif.IMF_REFINED) != 0
            assert np.all(refined | ((shift < 0) & (i1["m"][b][valid] == 1))), (N, i1["flags"][b][valid])
        a = ref.imfs_of(b).double()
        c = out.imfs_of(b).double()
        assert float((a - c).norm()) <= 1e-6 * float(a.norm())
    refs = oracle_many([s.astype(np.float64) for s in sigs[:2]], 1e-3, 6)
    for b, r in enumerate(refs):
        _check(r, sigs[b].astype(np.float64), out.imfs_of(b).cpu().numpy().astype(np.float64),
               out.remainder_of(b).cpu().numpy().astype(np.float64), i1[b], int(n1[b]), 1e-3, False)
