"""The autotuner on the GPU: fif_plan_create_tuned picks a valid choice per
length, never one slower than the built-in choice in its own measurement,
writes the cache file and reuses it, and a tuned plan decomposes like the
built-in one (identical decisions, IMFs equal up to FFT rounding)."""
from __future__ import annotations

import time

import numpy as np
import pytest

import siggen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1802_01359_amd as fif  # noqa: E402


def _signals(lengths, seed0):
    return [siggen.tones3(N=N, freqs=(max(1.0, N / 700.0), max(2.0, N / 90.0), N / 9.0), seed_index=seed0 + i)
            for i, N in enumerate(lengths)]


def _same_decomposition(a, b, B, J):
    ia, ib = a.info(), b.info()
    assert torch.equal(a.n_imfs, b.n_imfs)
    for key in ("k", "L", "m"):
        assert np.array_equal(ia[key], ib[key]), key
    for s in range(B):
        x, y = a.imfs_of(s).double(), b.imfs_of(s).double()
        for j in range(J):
            assert float((x[j] - y[j]).norm()) <= 1e-12 * float(x[j].norm()) + 1e-300


def test_tuned_plan_chooses_caches_and_matches(tmp_path):
    cache = str(tmp_path / "tune.txt")
    lengths = [65536] * 4 + [20736] * 2 + [4096]
    print("tuning lengths %s" % sorted(set(lengths)), flush=True)
    t0 = time.perf_counter()
    tuned = fif.Plan(lengths, 5, tune_cache=cache)
    t_tune = time.perf_counter() - t0
    key = fif.device_tune_key()
    for N in (65536, 20736):
        c = tuned.length_plan(N)
        assert c["N1"] * c["N2"] == N and c["us"] > 0 and c["us_default"] > 0
        assert c["us"] <= c["us_default"]
        assert fif.tune_cache_lookup(cache, key, N) == c
        print("N=%d: %s" % (N, c), flush=True)
    assert fif.tune_cache_lookup(cache, key, 4096) is None       # one LDS pass: not tuned
    # second creation reads the cache: same choices, no timing runs
    t0 = time.perf_counter()
    again = fif.Plan(lengths, 5, tune_cache=cache)
    t_again = time.perf_counter() - t0
    for N in (65536, 20736):
        assert again.length_plan(N) == tuned.length_plan(N)
    print("tuning %.2f s, cached %.2f s" % (t_tune, t_again), flush=True)
    # same decomposition as the built-in plan
    x = torch.tensor(np.concatenate(_signals(lengths, 30)), dtype=torch.float64, device="cuda")
    ref = fif.Plan(lengths, 5).run(x, 1e-3)
    out = tuned.run(x, 1e-3)
    torch.cuda.synchronize()
    _same_decomposition(ref, out, len(lengths), 5)


def test_cache_entry_forces_a_choice(tmp_path):
    """A cache entry with a non-default split, tiles and radix order is used
    as is, and the decomposition is still the built-in plan's."""
    cache = str(tmp_path / "tune.txt")
    key = fif.device_tune_key()
    forced = {"N": 65536, "N1": 128, "N2": 512, "TC": 4, "TR": 16, "rad1": [2, 4, 8, 8], "rad2": [4, 4, 8],
              "us": 1.0, "us_default": 2.0}
    fif.tune_cache_store(cache, key, forced)
    lengths = [65536, 65536, 4096]
    plan = fif.Plan(lengths, 4, tune_cache=cache)
    assert plan.length_plan(65536) == forced
    x = torch.tensor(np.concatenate(_signals(lengths, 50)), dtype=torch.float64, device="cuda")
    ref = fif.Plan(lengths, 4).run(x, 1e-3)
    out = plan.run(x, 1e-3)
    torch.cuda.synchronize()
    _same_decomposition(ref, out, len(lengths), 4)
