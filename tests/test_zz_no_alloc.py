"""fif_decompose_batched_static (the entry point that allocates nothing)
against fif_decompose_batched, through the C ABI.

Both run the same kernels on the same inputs; the static entry point only
takes its workspace from the library's fixed array and issues every kernel on
the caller's stream.  Results must be identical bit for bit: IMF counts,
(k, L, m, SD), IMFs, remainders.  Two calls in a row, the second with a
smaller batch (the array keeps the first call's contents), then a plan too
large for the array, which must be refused.
"""
from __future__ import annotations

import numpy as np
import pytest

import siggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1802_01359_amd as fif  # noqa: E402
from paper_1802_01359_amd import _binding  # noqa: E402


def _signals(lengths, seed0):
    out = []
    for i, N in enumerate(lengths):
        if N == 65536:
            out.append(siggen.chirps(seed0 + i))
        else:
            out.append(siggen.tones3(N=N, freqs=(max(1.0, N / 700.0), max(2.0, N / 90.0), N / 9.0),
                                     seed_index=seed0 + i))
    return torch.tensor(np.concatenate(out), dtype=torch.float32, device="cuda")


def _same(a, b):
    assert torch.equal(a.n_imfs, b.n_imfs)
    assert torch.equal(a.sig_status, b.sig_status)
    assert torch.equal(a.info_raw, b.info_raw)
    assert torch.equal(a.imfs, b.imfs)
    assert torch.equal(a.remainders, b.remainders)


@pytest.mark.parametrize("lengths,seed0", [
    ([65536, 4096, 12000, 1000, 8192, 131072, 30], 40),     # first call: larger batch
    ([2048, 360, 16384], 60),                               # second call: smaller batch
])
def test_static_workspace_matches_batched(lengths, seed0):
    print("static workspace: lengths %s" % (lengths,), flush=True)
    plan = fif.Plan(lengths, 6)
    assert plan.workspace_bytes <= fif.STATIC_WORKSPACE_BYTES
    x = _signals(lengths, seed0)
    ref = plan.run(x, 1e-3)
    got = plan.run_static(x, 1e-3)
    torch.cuda.synchronize()
    _same(ref, got)
    assert int(got.n_imfs.min()) >= 1


def test_static_workspace_twice_in_a_row_then_smaller():
    """Two calls in a row on the same array, the second with a smaller batch
    and a different delta: each equals its workspace-argument twin."""
    big = [65536, 65536, 20736]
    small = [4096, 1000]
    pb, ps = fif.Plan(big, 8), fif.Plan(small, 8)
    xb, xs = _signals(big, 70), _signals(small, 80)
    rb = pb.run(xb, 1e-3)
    rs = ps.run(xs, 1e-4)
    gb = pb.run_static(xb, 1e-3)
    gs = ps.run_static(xs, 1e-4)
    torch.cuda.synchronize()
    _same(rb, gb)
    _same(rs, gs)


def test_static_workspace_refuses_large_plans():
    plan = fif.Plan([1 << 22], 4)
    assert plan.workspace_bytes > fif.STATIC_WORKSPACE_BYTES
    x = torch.zeros(1 << 22, dtype=torch.float32, device="cuda")
    with pytest.raises(fif.FifError) as e:
        plan.run_static(x, 1e-3)
    assert e.value.status == _binding.FIF_ERR_CAPACITY
