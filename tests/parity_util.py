"""Shared checks of the GPU parity tests (not collected by pytest).

Decisions (extrema count k, mask length L, step count m, number of IMFs)
must be identical to the oracle's: there is no tie escape.  When they differ
the failure message says whether the oracle's own margins put the decision
within 1e-10 of its threshold (min |r_{i+1} - r_i| / max|r| for k, |SD/delta
- 1| for m), so a genuine rounding tie can be told from a bug, but it fails
either way.

IMFs: FP64 entry points within ||d|| <= 1e-12 ||IMF|| + 1e-15 ||s||; FP32
entry points within 1e-5 relative L2 per IMF.  Every checked IMF's relative
L2 error is recorded per configuration; the session prints the worst per
configuration and, when FIF_PARITY_LOG names a file, writes them there as
JSON.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TIE = 1e-10

# config -> [worst relative L2 over checked IMFs, IMFs checked, signals checked]
ERRORS: dict = {}


def record(config: str, rel: float, imfs: int = 1, signals: int = 0) -> None:
    e = ERRORS.setdefault(config, [0.0, 0, 0])
    e[0] = max(e[0], float(rel))
    e[1] += imfs
    e[2] += signals


def report() -> str:
    lines = ["worst per-IMF relative L2 error against the FP64 oracle:"]
    for k in sorted(ERRORS):
        w, ni, ns = ERRORS[k]
        lines.append("  %-40s %.3e over %d IMFs of %d signals" % (k, w, ni, ns))
    path = os.environ.get("FIF_PARITY_LOG")
    if path and ERRORS:
        with open(path, "w") as f:
            json.dump({k: {"max_rel_l2": v[0], "imfs": v[1], "signals": v[2]} for k, v in ERRORS.items()}, f,
                      indent=1, sort_keys=True)
    return "\n".join(lines)


def decisions_equal(ref_n, ref_k, ref_L, ref_m, info, n, delta, label="", margin_k=None, sd=None, sd_prev=None):
    """Assert identical IMF count and (k, L, m) for every IMF."""
    got = [(int(info["k"][i]), int(info["L"][i]), int(info["m"][i])) for i in range(n)]
    exp = [(int(a), int(b), int(c)) for a, b, c in zip(ref_k, ref_L, ref_m)]
    if n == ref_n and got == exp:
        return
    j = next((i for i in range(min(n, ref_n)) if got[i] != exp[i]), min(n, ref_n))
    why = "no oracle margin available"
    if j < ref_n and margin_k is not None:
        near = []
        if margin_k[j] < TIE:
            near.append("extrema margin %.2e" % margin_k[j])
        for v in (sd[j], sd_prev[j]) if sd is not None else ():
            if math.isfinite(v) and abs(v / delta - 1.0) < TIE:
                near.append("SD/delta - 1 = %.2e" % (v / delta - 1.0))
        why = ("oracle margin within %.0e: %s" % (TIE, ", ".join(near))) if near else \
            "oracle margins are far from the thresholds (not a tie)"
    raise AssertionError("%s decision mismatch at IMF %d (%s): gpu n=%d %s vs oracle n=%d %s" % (
        label, j, why, n, got, ref_n, exp))


def check(ref, s, imfs, rem, info, n, delta, fp64, lam_abs=None, config=None):
    """Decisions identical to the oracle decomposition `ref`, IMFs and
    remainder within the bar.  lam_abs(m): extra FP64 bound on ||IMF error||
    / ||s|| when both sides' eigenvalues carry independent rounding errors
    (sampled windows)."""
    decisions_equal(ref.n_imfs, ref.k, ref.L, ref.m, info, n, delta, margin_k=ref.margin_k, sd=ref.sd,
                    sd_prev=ref.sd_prev)
    sn = np.linalg.norm(s)
    for j in range(n):
        a, b = ref.imfs[j], imfs[j]
        err = np.linalg.norm(a - b)
        na = np.linalg.norm(a)
        extra = lam_abs(ref.m[j]) * sn if lam_abs is not None else 0.0
        if fp64:
            assert err <= 1e-12 * na + 1e-15 * sn + extra, (j, err, na)
        else:
            assert err <= 1e-5 * na + 1e-30, (j, err / max(na, 1e-300))
        if config is not None and na > 0:
            record(config, err / na)
    if config is not None:
        record(config, 0.0, imfs=0, signals=1)
    err = np.linalg.norm(ref.remainder - rem)
    extra = sum(lam_abs(m) for m in ref.m[:n]) * sn if lam_abs is not None else 0.0
    if fp64:
        assert err <= 1e-12 * np.linalg.norm(ref.remainder) + 1e-15 * sn + extra
    else:
        assert err <= 1e-5 * np.linalg.norm(ref.remainder) + 1e-7 * sn
    assert np.all(imfs[n:] == 0)


def load_golden(name: str) -> dict:
    """Decisions written by tests/golden/make_golden.py: {index: dict(N,
    n_imfs, stop, agree, k, L, m, sd, sd_prev, margin_k, flags)}."""
    out: dict = {}
    with open(os.path.join(HERE, "golden", "decisions_%s.txt" % name)) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "S":
                out[int(p[1])] = dict(N=int(p[2]), n_imfs=int(p[3]), stop=int(p[4]), agree=p[5], k=[], L=[], m=[],
                                      sd=[], sd_prev=[], margin_k=[], flags=[])
            else:
                d = out[int(p[1])]
                assert int(p[2]) == len(d["k"])
                d["k"].append(int(p[3]))
                d["L"].append(int(p[4]))
                d["m"].append(int(p[5]))
                d["sd"].append(float(p[6]))
                d["sd_prev"].append(float(p[7]))
                d["margin_k"].append(float(p[8]))
                d["flags"].append(int(p[9]))
    return out


def golden_equal(g: dict, info, n, delta, label):
    decisions_equal(g["n_imfs"], g["k"], g["L"], g["m"], info, n, delta, label=label, margin_k=g["margin_k"],
                    sd=g["sd"], sd_prev=g["sd_prev"])
