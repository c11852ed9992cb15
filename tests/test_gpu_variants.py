"""Parity of the HIP path's method variants with the spectral oracle, through
the C ABI: the absolute stop criterion, the a-priori N0 of Theorem 5, the
thresholded IMF and the spectral-peak mask length.

Same bar as the plain method: identical (k, L, m) unless the oracle's margin
certifies a tie; IMFs within 1e-12 (FP64 entry points) or 1e-5 (FP32) in
relative L2.
"""
from __future__ import annotations

import numpy as np
import pytest

import siggen
from oracle import fif_spectral as fs
from test_gpu_parity import _check, _signal  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1802_01359_amd as fif  # noqa: E402

SMALL = [4096, 1000, 30, 8192, 12000, 65536]
LARGE = [4096, 131072, 262144]


def _sigs(lengths):
    return [siggen.chirps(i) if N == 65536 else _signal(N, 300 + i) for i, N in enumerate(lengths)]


def _batch_vs_oracle(lengths, delta, max_imfs, dtype, oracle_kw, lam_abs=None, **opt):
    sigs = _sigs(lengths)
    if dtype == torch.float32:
        sigs = [s.astype(np.float32) for s in sigs]
    print("variant %s lengths %s dtype %s" % (opt, lengths, dtype), flush=True)
    plan = fif.Plan(lengths, max_imfs, fif.Options(**opt))
    out = plan.run(torch.tensor(np.concatenate(sigs), dtype=dtype, device="cuda"), delta)
    torch.cuda.synchronize()
    info = out.info()
    n = out.n_imfs.cpu().numpy()
    assert np.all(out.sig_status.cpu().numpy() == 0)
    for b, N in enumerate(lengths):
        s64 = np.asarray(sigs[b], dtype=np.float64)
        ref = fs.decompose(s64, delta, max_imfs, **oracle_kw)
        imfs = out.imfs_of(b).cpu().numpy().astype(np.float64)
        rem = out.remainder_of(b).cpu().numpy().astype(np.float64)
        _check(ref, s64, imfs, rem, info[b], int(n[b]), delta, dtype == torch.float64, lam_abs)
    return info, n


@pytest.mark.parametrize("dtype,lengths,imfs", [(torch.float64, SMALL, 5), (torch.float32, SMALL, 5),
                                                (torch.float32, LARGE, 3)])
def test_absolute_stop(dtype, lengths, imfs):
    """LARGE: 131072 and 262144 samples take the multi-workgroup search, with
    Theorem 5's N0 as its upper bracket."""
    info, n = _batch_vs_oracle(lengths, 1e-2, imfs, dtype, dict(stop="abs"), stop_mode=1)
    assert np.all(info["m"][n > 0][:, 0] >= 1) if n.max() > 0 else True


def test_absolute_stop_small_signal_takes_one_step():
    """A residual whose first step ||s_1 - s_0|| is already below delta: the
    smallest m >= 1 with ||s_{m+1} - s_m|| < delta is 1 (there is no m = 0),
    on both sides."""
    lengths = [4096, 1000, 8192, 65536]
    sigs = [2e-5 * _signal(N, 700 + i) for i, N in enumerate(lengths)]
    plan = fif.Plan(lengths, 3, fif.Options(stop_mode=1))
    out = plan.run(torch.tensor(np.concatenate(sigs), dtype=torch.float64, device="cuda"), 1e-2)
    torch.cuda.synchronize()
    info = out.info()
    n = out.n_imfs.cpu().numpy()
    for b, N in enumerate(lengths):
        ref = fs.decompose(sigs[b], 1e-2, 3, stop="abs")
        assert ref.n_imfs >= 1 and ref.m[0] == 1 and ref.sd_prev[0] < 1e-2
        _check(ref, sigs[b], out.imfs_of(b).cpu().numpy(), out.remainder_of(b).cpu().numpy(), info[b], int(n[b]),
               1e-2, True)


def test_apriori_n0():
    info, n = _batch_vs_oracle([4096, 1000, 30, 8192, 65536, 131072, 262144], 1e-3, 3, torch.float64,
                               dict(stop="apriori"), stop_mode=2)
    # no search: evals record one FP64 pass and no FP32 pass
    ev = info["evals"][np.arange(3)[None, :] < n[:, None]]
    assert np.all((ev & 0xffff) == 0) and np.all((ev >> 16) == 1)


@pytest.mark.parametrize("dtype,lengths", [(torch.float64, SMALL), (torch.float32, LARGE)])
def test_thresholded_imf(dtype, lengths):
    _batch_vs_oracle(lengths, 1e-3, 5, dtype, dict(gamma=1e-2), gamma=1e-2)


@pytest.mark.parametrize("dtype,lengths", [(torch.float64, SMALL), (torch.float32, LARGE)])
def test_spectral_peak_mask_rule(dtype, lengths):
    _batch_vs_oracle(lengths, 1e-3, 5, dtype, dict(mask_rule=2, peak_rho=0.1), mask_rule=2, peak_rho=0.1)


def test_variants_in_the_single_signal_form():
    s = siggen.tones3()
    x = torch.tensor(s, dtype=torch.float64, device="cuda")
    for opt, kw in ((dict(stop_mode=1), dict(stop="abs")), (dict(gamma=0.05), dict(gamma=0.05)),
                    (dict(mask_rule=2), dict(mask_rule=2))):
        print("single variant %s" % opt, flush=True)
        res = fif.decompose(x, 1e-3, 6, fif.Options(**opt))
        torch.cuda.synchronize()
        ref = fs.decompose(s, 1e-3, 6, **kw)
        imfs = np.zeros((6, s.size))
        imfs[:res.n_imfs] = res.imfs.cpu().numpy()
        _check(ref, s, imfs, res.remainder.cpu().numpy(), res.info, res.n_imfs, 1e-3, True)
