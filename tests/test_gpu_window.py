"""Parity of the HIP path's sampled window shapes with the spectral oracle,
through the C ABI: each outer step tabulates lambda_j = (DFT(h)_j / sum h)^2
of the folded taps on the GPU (Section 4: the direct method needs only the
eigenvalues of W, which any window provides).

Same bar as the plain method: identical (k, L, m) unless the oracle's margin
certifies a tie; IMFs within 1e-12 (FP64 entry points) or 1e-5 (FP32) in
relative L2, plus, in FP64, the eigenvalue term below.  The triangle shape
{1, 0} must reproduce the closed-form path.

Eigenvalue term: here both sides take lambda from an FFT (the closed form
agrees to an ulp, this does not).  With |dH| <= ~1.8e-15 per side (sum of
the normalised taps 1, log2 N <= 16 passes), lambda = H^2 differs by
3.6e-15 sqrt(lambda); the gain error m (1-lambda)^(m-1) dlambda peaks near
lambda = 1/(2m) at about 1.6e-15 sqrt(m); so ||IMF error|| may grow by
2e-15 (1 + sqrt(m)) ||s|| (the residual is never larger than s).
"""
from __future__ import annotations

import numpy as np
import pytest

import siggen
from oracle import fif_spectral as fs
from test_gpu_parity import _check
from test_gpu_variants import LARGE, SMALL, _batch_vs_oracle, _sigs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1802_01359_amd as fif  # noqa: E402

def LAM_ABS(m):
    return 2e-15 * (1.0 + float(m) ** 0.5)


# raised cosine on 33 samples, a flat top with a linear edge, a non-monotone shape
RAISED_COS = list(0.5 * (1.0 + np.cos(np.pi * np.arange(33) / 32)))
FLAT_TOP = [1.0, 1.0, 0.0]
BUMPY = [0.6, 1.0, 0.3, 0.5, 0.0]


@pytest.mark.parametrize("shape", [RAISED_COS, FLAT_TOP, BUMPY])
def test_window_shape_fp64(shape):
    _batch_vs_oracle(SMALL, 1e-3, 5, torch.float64, dict(window=shape), LAM_ABS, window=shape)


@pytest.mark.parametrize("shape", [RAISED_COS, BUMPY])
def test_window_shape_fp32_large(shape):
    # 131072 and 262144 take the multi-workgroup search
    _batch_vs_oracle(LARGE, 1e-3, 4, torch.float32, dict(window=shape), LAM_ABS, window=shape)


def test_window_shape_with_other_variants():
    _batch_vs_oracle(SMALL, 1e-2, 4, torch.float64, dict(window=RAISED_COS, stop="abs", gamma=1e-2), LAM_ABS,
                     window=RAISED_COS, stop_mode=1, gamma=1e-2)
    # on the 30-sample noise signal the peak rule gives L = 2: the flat top is
    # then a 3-tap box whose spectrum has exact zeros, and after the first IMF
    # every bin left has lambda > delta, so SD_m cannot reach delta: the later
    # IMFs run to the cap on both sides (the oracle bisects, which its pins
    # tie to the linear scan)
    _batch_vs_oracle(SMALL, 1e-3, 4, torch.float64, dict(window=FLAT_TOP, mask_rule=2, search="bisect"),
                     LAM_ABS, window=FLAT_TOP, mask_rule=2)


def test_triangle_shape_reproduces_the_closed_form_path():
    lengths = [65536] * 4 + [4096, 1000]
    sigs = _sigs(lengths)
    x = torch.tensor(np.concatenate(sigs), dtype=torch.float64, device="cuda")
    outs = []
    for opt in (fif.Options(), fif.Options(window=[1.0, 0.0])):
        print("triangle as %s" % ("closed form" if opt.window is None else "sampled shape"), flush=True)
        plan = fif.Plan(lengths, 8, opt)
        out = plan.run(x, 1e-3)
        torch.cuda.synchronize()
        outs.append(out)
    a, b = outs
    ia, ib = a.info(), b.info()
    na, nb = a.n_imfs.cpu().numpy(), b.n_imfs.cpu().numpy()
    for s in range(len(lengths)):
        n = min(na[s], nb[s])
        same = all(np.array_equal(ia[k][s, :n], ib[k][s, :n]) for k in ("k", "L", "m"))
        if not (same and na[s] == nb[s]):
            # a tie of the FP64 decisions is the only admissible difference
            ref = fs.decompose(np.asarray(sigs[s], dtype=np.float64), 1e-3, 8)
            _check(ref, sigs[s], b.imfs_of(s).cpu().numpy(), b.remainder_of(s).cpu().numpy(), ib[s], int(nb[s]),
                   1e-3, True, LAM_ABS)
            continue
        da = a.imfs_of(s)[:n].cpu().numpy()
        db = b.imfs_of(s)[:n].cpu().numpy()
        scale = np.linalg.norm(sigs[s])
        tol = sum(LAM_ABS(m) for m in ia["m"][s, :n]) + 1e-12
        assert np.linalg.norm(da - db) <= tol * scale


def test_window_shape_single_signal_form():
    s = siggen.tones3()
    x = torch.tensor(s, dtype=torch.float64, device="cuda")
    print("single form, raised cosine", flush=True)
    res = fif.decompose(x, 1e-3, 6, fif.Options(window=RAISED_COS))
    torch.cuda.synchronize()
    ref = fs.decompose(s, 1e-3, 6, window=RAISED_COS)
    imfs = np.zeros((6, s.size))
    imfs[:res.n_imfs] = res.imfs.cpu().numpy()
    _check(ref, s, imfs, res.remainder.cpu().numpy(), res.info, res.n_imfs, 1e-3, True, LAM_ABS)
