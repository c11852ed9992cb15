"""The FP32 lane (fif_options.precision = FIF_PREC_FP32): transforms, stored
spectra and the four-step intermediate in FP32; lambda, the powers and the
stop-test sums FP64.  It carries no parity claim -- an FP32-synthesised
residual can gain or lose extrema -- so these tests check what must hold
anyway and report how often its decisions differ from the FP64 path's:

* every signal still decomposes exactly: IMFs plus remainder give back the
  input to FP32 rounding (each IMF is a spectral part of the residual);
* while a signal's decisions (k, L, m) agree with the FP64 path's, its IMFs
  agree with the FP64 path's to the error of an FP32 transform;
* the decision-mismatch rate on the chirp batch against the stored oracle
  decisions (all 1024 signals), printed.
"""
from __future__ import annotations

import numpy as np
import pytest

import siggen
from parity_util import load_golden
from test_gpu_parity import _signal  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1802_01359_amd as fif  # noqa: E402


def _run(lengths, x, delta, J, precision):
    plan = fif.Plan(lengths, J, fif.Options(precision=precision))
    out = plan.run(x, delta)
    torch.cuda.synchronize()
    return out


def _first_difference(ia, ib, na, nb, b):
    """Index of the first IMF of signal b whose (k, L, m) or presence differ."""
    n = min(na[b], nb[b])
    for j in range(n):
        if (ia["k"][b][j], ia["L"][b][j], ia["m"][b][j]) != (ib["k"][b][j], ib["L"][b][j], ib["m"][b][j]):
            return j
    return n


def test_fp32_lane_reconstructs_and_tracks_the_fp64_path():
    lengths = [4096, 1000, 12000, 65536, 65536, 10125, 131072, 98415]
    sigs = [(siggen.chirps(i) if N == 65536 else _signal(N, 1100 + i)).astype(np.float32)
            for i, N in enumerate(lengths)]
    x = torch.tensor(np.concatenate(sigs), device="cuda")
    J = 8
    print("FP32 lane: lengths %s" % lengths, flush=True)
    a = _run(lengths, x, 1e-3, J, fif.PREC_FP32)
    b = _run(lengths, x, 1e-3, J, fif.PREC_MIXED)
    assert np.all(a.sig_status.cpu().numpy() == 0)
    ia, ib = a.info(), b.info()
    na, nb = a.n_imfs.cpu().numpy(), b.n_imfs.cpu().numpy()
    same_imfs = 0
    for s, N in enumerate(lengths):
        sig = sigs[s].astype(np.float64)
        ima = a.imfs_of(s).cpu().numpy().astype(np.float64)
        rem = a.remainder_of(s).cpu().numpy().astype(np.float64)
        recon = ima[:na[s]].sum(axis=0) + rem
        err = np.linalg.norm(recon - sig) / np.linalg.norm(sig)
        assert err <= 1e-5, (N, err)
        imb = b.imfs_of(s).cpu().numpy().astype(np.float64)
        jd = _first_difference(ia, ib, na, nb, s)
        for j in range(jd):
            e = np.linalg.norm(ima[j] - imb[j]) / max(np.linalg.norm(imb[j]), 1e-300)
            # FP32 transforms of the residual, N up to 2^17: a few 1e-6
            assert e <= 1e-4 + 1e-5 * np.linalg.norm(sig) / max(np.linalg.norm(imb[j]), 1e-300), (N, j, e)
        same_imfs += jd
        print("  N=%6d IMFs %d/%d, decisions equal for the first %d, reconstruction %.2e" % (
            N, na[s], nb[s], jd, err), flush=True)
    assert same_imfs > 0


def test_fp32_lane_mismatch_rate_on_the_chirp_batch():
    gold = load_golden("chirps")
    B, N, J = 1024, 65536, 12
    x = torch.tensor(np.concatenate([siggen.chirps(i) for i in range(B)]).astype(np.float32), device="cuda")
    out = _run([N] * B, x, 1e-3, J, fif.PREC_FP32)
    info = out.info()
    n = out.n_imfs.cpu().numpy()
    # an IMF counts as agreeing while every decision of the signal up to it
    # agrees (after a difference the residuals differ)
    sig_same = imf_same = imf_total = 0
    for s in range(B):
        g = gold[s]
        imf_total += g["n_imfs"]
        j = 0
        while j < min(n[s], g["n_imfs"]) and \
                (info["k"][s][j], info["L"][s][j], info["m"][s][j]) == (g["k"][j], g["L"][j], g["m"][j]):
            j += 1
        imf_same += j
        sig_same += (j == g["n_imfs"] and n[s] == g["n_imfs"])
    print("FP32 lane on the chirp batch: %d of %d signals and %d of %d IMFs with the oracle's decisions"
          % (sig_same, B, imf_same, imf_total), flush=True)
    assert 0 < imf_same <= imf_total
