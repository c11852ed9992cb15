"""Pins of the CPU reference of the step-count proposal network.

The reference is checked against finite differences of its own loss (FP64),
against torch's CPU autograd of the same network written with
torch.nn.functional.conv1d (an independent implementation of the
convolution and its gradients), and against closed forms of the features
and of bfloat16 rounding.
"""
import numpy as np
import pytest
import torch

from oracle import proposal_net as pn


def _random_case(B=2, seed=0, scale=0.15):
    rng = np.random.default_rng(seed)
    flat = rng.normal(0.0, scale, pn.n_params())
    P = pn.unpack(flat)
    P["W0"][:, 2:, :] = 0.0       # padded input channels carry no weights
    flat = pn.pack(P)
    x = np.zeros((B, pn.NFEAT, pn.CIN0))
    x[:, :, 0] = rng.normal(-1.0, 0.5, (B, pn.NFEAT))
    x[:, :, 1] = rng.uniform(0.1, 0.8, (B, 1))
    t = rng.uniform(0.0, 1.0, (B, 2))
    return flat, x, t


def test_shapes_and_parameter_count():
    assert [s[2] for s in pn.layer_shapes()] == [512, 256, 128, 64, 32, 16]
    assert pn.n_params() == 7 * 8 * 64 + 64 + 5 * (7 * 64 * 64 + 64) + 2 * 64 + 2 == 147458
    flat = np.arange(pn.n_params(), dtype=np.float64)
    assert np.array_equal(pn.pack(pn.unpack(flat)), flat)


def test_gradient_matches_finite_differences():
    flat, x, t = _random_case()
    loss, g = pn.loss_and_grad(flat, x, t)
    assert loss > 0
    rng = np.random.default_rng(7)
    idx = []
    for name, shape, off in pn.param_layout():
        size = int(np.prod(shape))
        if name == "W0":  # only the two live input channels
            W = np.arange(size).reshape(shape)
            live = W[:, :2, :].reshape(-1)
            idx += list(off + rng.choice(live, 4, replace=False))
        else:
            idx += list(off + rng.choice(size, min(size, 4), replace=False))
    h = 1e-6
    for i in idx:
        fp = flat.copy()
        fm = flat.copy()
        fp[i] += h
        fm[i] -= h
        lp = pn.loss_and_grad(fp, x, t)[0]
        lm = pn.loss_and_grad(fm, x, t)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def _torch_net(flat, x, t):
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in pn.unpack(flat).items()}
    a = torch.tensor(x, dtype=torch.float64).permute(0, 2, 1)  # [B, C, length]
    for l in range(pn.NLAYERS):
        w = P[f"W{l}"].permute(2, 1, 0)                     # [out, in, kernel]
        a = torch.relu(torch.nn.functional.conv1d(a, w, P[f"b{l}"], stride=2, padding=3))
    h = a.mean(dim=2)
    y = h @ P["Wh"].T + P["bh"]
    loss = ((y - torch.tensor(t)) ** 2).sum() / (2 * y.shape[0])
    loss.backward()
    return y.detach().numpy(), float(loss.detach()), pn.pack({k: v.grad.numpy() for k, v in P.items()})


def test_forward_and_gradient_match_torch_autograd():
    flat, x, t = _random_case(B=3, seed=3)
    y_ref, _ = pn.forward(flat, x)
    loss, g = pn.loss_and_grad(flat, x, t)
    y_t, loss_t, g_t = _torch_net(flat, x, t)
    assert np.max(np.abs(y_ref - y_t)) <= 1e-12 * np.max(np.abs(y_t))
    assert abs(loss - loss_t) <= 1e-12 * loss_t
    assert np.linalg.norm(g - g_t) <= 1e-11 * np.linalg.norm(g_t)


def test_bf16_mode_is_close_to_fp64_mode():
    flat, x, t = _random_case(B=2, seed=5)
    l64, g64 = pn.loss_and_grad(flat, x, t)
    l16, g16 = pn.loss_and_grad(flat, x, t, bf16=True)
    assert abs(l16 - l64) <= 0.02 * l64
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


def test_bf16_rounding_closed_forms():
    v = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, -2.5, 0.0, 3.0e38])
    r = pn.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie to even
    assert r[2] == 1 + 2.0 ** -6          # tie to even (upwards)
    assert r[3] == 1 + 2.0 ** -7          # above the tie
    assert r[4] == -2.5 and r[5] == 0.0
    assert abs(r[6] - 3.0e38) <= 3.0e38 * 2.0 ** -8


def test_features_closed_forms():
    H = 4096
    flat = np.ones(H + 1, dtype=complex)   # equal power in every bin
    f = pn.features(flat, 37)
    assert f.shape == (pn.NFEAT, pn.CIN0)
    assert np.allclose(f[:, 0], np.log2(1.0 / H + 2.0 ** -60) / 16.0, rtol=0, atol=1e-15)
    assert np.allclose(f[:, 1], np.log2(37.0) / 16.0)
    assert np.all(f[:, 2:] == 0.0)
    # one line at bin j: only its group holds power (group size H / 1024 = 4)
    R = np.zeros(H + 1, dtype=complex)
    j = 1234
    R[j] = 3.0 + 4.0j
    f = pn.features(R, 5)
    q = (j - 1) // 4
    assert f[q, 0] == pytest.approx(np.log2(0.25 + 2.0 ** -60) / 16.0, abs=1e-15)
    others = np.delete(f[:, 0], q)
    assert np.all(others == -60.0 / 16.0)
    # fewer bins than groups: every group takes one bin
    R = np.arange(1, 302, dtype=float).astype(complex)   # H = 300
    f = pn.features(R, 2)
    pw = np.abs(R[1:]) ** 2
    for q in (0, 511, 1023):
        jj = (q * 300) // 1024
        assert f[q, 0] == pytest.approx(np.log2(pw[jj] / pw.sum() + 2.0 ** -60) / 16.0, abs=1e-14)
