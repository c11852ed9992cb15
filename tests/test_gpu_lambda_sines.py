"""lambda_j's sines read from the per-length tables or evaluated in place
(FIF_LAMBDA_SINES=table|sin|both) give the same decomposition bit for bit:
the in-place evaluation is the table fill's own expression.  One plan covers
every kind of length (one LDS pass, paired and unpaired four-step, the
multi-workgroup search), and the in-place form is also checked against the
spectral oracle (Section 4 direct form)."""
from __future__ import annotations

import os

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

# 4096: one LDS pass; 65536: paired four-step; 10125 = 3^4 5^3 and
# 98415 = 3^9 5: unpaired four-step (odd factors); 131072: paired, searched
# by the multi-workgroup scan; 98415 too
LENGTHS = [4096, 65536, 10125, 98415, 131072]
DELTA = 1e-3
J = 6


def _sigs():
    return [(siggen.chirps(i) if N == 65536 else _signal(N, 700 + i)).astype(np.float32)
            for i, N in enumerate(LENGTHS)]


def _run(mode, x):
    os.environ["FIF_LAMBDA_SINES"] = mode
    try:
        plan = fif.Plan(LENGTHS, J)
    finally:
        del os.environ["FIF_LAMBDA_SINES"]
    out = plan.run(x, DELTA)
    torch.cuda.synchronize()
    return out


def test_sines_in_place_equal_tables():
    sigs = _sigs()
    x = torch.tensor(np.concatenate(sigs), device="cuda")
    print("lambda sines: lengths %s" % LENGTHS, flush=True)
    outs = {m: _run(m, x) for m in ("table", "sin", "both")}
    ref = outs["table"]
    ir = ref.info()
    for mode in ("sin", "both"):
        o = outs[mode]
        io = o.info()
        assert torch.equal(o.n_imfs, ref.n_imfs), mode
        assert torch.equal(o.sig_status, ref.sig_status), mode
        for key in ("k", "L", "m"):
            assert np.array_equal(io[key], ir[key]), (mode, key)
        for b in range(len(LENGTHS)):
            assert torch.equal(o.imfs_of(b), ref.imfs_of(b)), (mode, b)
            assert torch.equal(o.remainder_of(b), ref.remainder_of(b)), (mode, b)
    # the in-place form against the oracle on the four-step lengths
    o = outs["both"]
    info = o.info()
    n = o.n_imfs.cpu().numpy()
    for b in (1, 2):
        s64 = sigs[b].astype(np.float64)
        r = fs.decompose(s64, DELTA, J)
        _check(r, s64, o.imfs_of(b).cpu().numpy().astype(np.float64),
               o.remainder_of(b).cpu().numpy().astype(np.float64), info[b], int(n[b]), DELTA, False)
