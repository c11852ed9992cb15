"""The step-count proposal network on the GPU, through the C ABI.

Forward outputs, loss and every parameter gradient of the BF16 MFMA kernels
are compared with the CPU reference run in its bfloat16 mode (the same
roundings, FP64 elsewhere); the feature kernel with the reference features
of the FFT of the input; and a decomposition that uses proposals with the
plain one (decisions and IMFs bitwise identical, whatever the proposals).
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import siggen
from oracle import proposal_net as pn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1802_01359_amd as fif  # noqa: E402


def _params(seed, scale=0.12):
    rng = np.random.default_rng(seed)
    P = pn.unpack(rng.normal(0.0, scale, pn.n_params()))
    P["W0"][:, 2:, :] = 0.0
    for l in range(pn.NLAYERS):
        P[f"b{l}"] = rng.uniform(0.0, 0.1, pn.CH)
    return pn.pack(P).astype(np.float32).astype(np.float64)


def _feats(B, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((B, pn.NFEAT, pn.CIN0))
    x[:, :, 0] = rng.normal(-1.5, 0.6, (B, pn.NFEAT))
    x[:, :, 1] = rng.uniform(0.1, 0.9, (B, 1))
    return pn.bf16_round(x)


def _to_dev(x):
    return torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("B", [1, 37, 300])
def test_forward_matches_reference(B):
    print("net forward B=%d" % B, flush=True)
    flat = _params(1)
    x = _feats(B, 2)
    m = fif.Model(flat, max_batch=max(B, 64))
    y = m.forward(_to_dev(x)).cpu().numpy().astype(np.float64)
    y_ref, _ = pn.forward(flat, x, bf16=True)
    assert _rel(y, y_ref) <= 2e-3, _rel(y, y_ref)


@pytest.mark.parametrize("B", [5, 64])
def test_gradient_matches_reference(B):
    print("net gradient B=%d" % B, flush=True)
    flat = _params(3)
    x = _feats(B, 4)
    t = np.random.default_rng(5).uniform(0.2, 0.8, (B, 2))
    m = fif.Model(flat, max_batch=64)
    loss, g = m.grad(_to_dev(x), torch.tensor(t, dtype=torch.float32).cuda())
    torch.cuda.synchronize()
    loss = float(loss.cpu()[0])
    g = g.cpu().numpy().astype(np.float64)
    l_ref, g_ref = pn.loss_and_grad(flat, x, t, bf16=True)
    assert abs(loss - l_ref) <= 1e-3 * l_ref, (loss, l_ref)
    assert _rel(g, g_ref) <= 1e-2, _rel(g, g_ref)
    for name, shape, off in pn.param_layout():
        n = int(np.prod(shape))
        gs, rs = g[off:off + n], g_ref[off:off + n]
        if np.linalg.norm(rs) > 0:
            assert _rel(gs, rs) <= 3e-2, (name, _rel(gs, rs))
        else:
            assert np.all(gs == 0), name


def test_training_fits_a_fixed_batch_and_params_roundtrip(tmp_path):
    print("net training", flush=True)
    B = 64
    flat = _params(7, scale=0.05)
    x = _to_dev(_feats(B, 8))
    t = torch.tensor(np.random.default_rng(9).uniform(0.2, 0.8, (B, 2)), dtype=torch.float32).cuda()
    m = fif.Model(flat, max_batch=B)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    m.train_step(x, t, 1e-3, loss)
    torch.cuda.synchronize()
    first = float(loss.cpu()[0])
    for _ in range(150):
        m.train_step(x, t, 1e-3, loss)
    torch.cuda.synchronize()
    last = float(loss.cpu()[0])
    assert last < 0.2 * first, (first, last)
    p = m.get_params()
    P = pn.unpack(p)
    assert np.all(P["W0"][:, 2:, :] == 0)   # padded channels never receive gradient
    path = str(tmp_path / "net.fifnet")
    m.save(path)
    m2 = fif.Model(path=path, max_batch=B)
    assert np.array_equal(m2.get_params(), p)
    y1 = m.forward(x)
    y2 = m2.forward(x)
    assert torch.equal(y1, y2)


def test_features_of_the_first_step_match_reference():
    lengths = [65536, 4096, 1000, 262144, 30]
    sig = [siggen.uneven_signal(i, n) for i, n in enumerate(lengths)]
    print("features lengths %s" % lengths, flush=True)
    max_imfs = 3
    plan = fif.Plan(lengths, max_imfs)
    feats = torch.zeros(len(lengths) * max_imfs, 1024, 8, dtype=torch.bfloat16, device="cuda")
    plan.record_features(feats)
    x = torch.tensor(np.concatenate(sig), dtype=torch.float64).cuda()
    out = plan.run(x, 1e-3)
    torch.cuda.synchronize()
    info = out.info()
    f = feats.float().cpu().numpy().reshape(len(lengths), max_imfs, 1024, 8)
    for b, s in enumerate(sig):
        L = int(info[b, 0]["L"])
        ref = pn.bf16_round(pn.features(np.fft.rfft(s), L))
        got = f[b, 0]
        assert np.all(got[:, 2:] == 0)
        assert np.all(got[:, 1] == ref[:, 1])
        d = np.abs(got[:, 0] - ref[:, 0])
        assert np.all(d <= 2.0 ** -7 * np.abs(ref[:, 0]) + 1e-6), (b, float(d.max()))


def _const_model(m_hat):
    """A network whose output is the constant log2(m_hat)/16."""
    P = pn.unpack(np.zeros(pn.n_params()))
    P["bh"] = np.array([np.log2(m_hat) / 16.0, 0.5])
    return fif.Model(pn.pack(P), max_batch=64)


@pytest.mark.parametrize("proposal", ["random", 1, 100, 5000, 1 << 40])
def test_proposal_keeps_the_decomposition(proposal):
    lengths = [65536] * 6 + [4096, 1000, 131072, 262144, 8192, 30]
    sig = [siggen.chirps(i) if n == 65536 else siggen.uneven_signal(i, n) for i, n in enumerate(lengths)]
    print("proposal %s lengths %s" % (proposal, lengths), flush=True)
    plan = fif.Plan(lengths, 8)
    x = torch.tensor(np.concatenate(sig), dtype=torch.float32).cuda()
    ref = plan.run(x, 1e-4)
    torch.cuda.synchronize()
    ref_imfs, ref_rem = ref.imfs.clone(), ref.remainders.clone()
    ref_info, ref_n = ref.info(), ref.n_imfs.cpu().numpy().copy()
    model = fif.Model(_params(11), max_batch=5) if proposal == "random" else _const_model(proposal)
    plan.set_proposal(model)
    out = plan.run(x, 1e-4)
    torch.cuda.synchronize()
    assert np.array_equal(out.n_imfs.cpu().numpy(), ref_n)
    info = out.info()
    for key in ("k", "L", "m", "sd", "sd_prev"):
        assert np.array_equal(info[key], ref_info[key]), key
    assert np.array_equal(info["flags"] & fif.IMF_CAP, ref_info["flags"] & fif.IMF_CAP)
    assert torch.equal(out.imfs, ref_imfs)
    assert torch.equal(out.remainders, ref_rem)
    plan.set_proposal(None)


def test_trained_network_gains_and_keeps_the_decomposition():
    """The committed network (trained on the GPU by
    `python -m paper_1802_01359_amd.proposal train`) on held-out signals:
    same decomposition, fewer FP32 passes of the search per IMF."""
    from paper_1802_01359_amd import proposal
    path = os.path.join(os.path.dirname(fif.__file__), "data", "proposal_tones3_65536.fifnet")
    model = fif.Model(path=path, max_batch=256)
    print("trained proposal on 256 held-out signals", flush=True)
    r = proposal.evaluate(model, count=256, repeats=1)
    print(r, flush=True)
    assert r["identical"]
    assert r["proposal"]["imfs"] == r["plain"]["imfs"]
    assert r["proposal"]["fp32_passes_per_imf"] <= 0.7 * r["plain"]["fp32_passes_per_imf"]
    assert r["log2_m_abs_err_mean"] < 0.6
