#!/usr/bin/env python3
"""Write the oracle's decisions for the benchmark workloads.

Calls only ``oracle/`` (the FP64 CPU oracles) and ``siggen/`` (the seeded
input generators).  Nothing here runs on or reads from the GPU path.  The
files it writes are the expected decisions the GPU parity tests compare
every signal's (k, L, m) and IMF count with.

Workloads (the FP32 signals the GPU receives, widened exactly to FP64):
  chirps  all 1024 signals of the 1024 x 65536 chirp batch, delta 1e-3,
          12 IMFs: the time-domain iteration of Algorithm 2 (four periodic box
          sums per application of W, pinned to the literal folded taps), and
          the Section 4 direct form with the linear scan N0 = 1, 2, ...
  uneven  64 signals of the 4096-signal uneven batch, stratified by length
          (every 65th in length order, the longest included), delta 1e-4,
          12 IMFs: the direct form with the linear scan; the time-domain
          iteration beside it for the signals of at most 16384 samples (at
          delta 1e-4 m reaches 10^5, and the iteration costs N m)
  long    the single 2^24-sample signal, delta 1e-3, 20 IMFs: the direct form
          with the linear scan only (the time-domain iteration would take
          hours at this length)

Each file holds one line per signal
    S <index> <N> <n_imfs> <stop_reason> <oracles_agree>
followed by one line per IMF
    I <index> <j> <k> <L> <m> <sd> <sd_prev> <margin_k> <flags>
where the decisions are those of the first oracle listed for the workload and
oracles_agree says whether the second one reached the same (k, L, m) for
every IMF and the same IMF count (1), or not (0), or was not run (-).

    python tests/golden/make_golden.py [chirps|uneven|long ...] [--jobs J]
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import siggen  # noqa: E402
from oracle import dif  # noqa: E402
from oracle import fif_spectral  # noqa: E402

UNEVEN_SAMPLE = 64
UNEVEN_TIME_DOMAIN_MAX = 16384


def uneven_picks(lengths) -> list:
    """Indices of a length-stratified sample of the uneven batch: evenly
    spaced positions in length order, the shortest and the longest included."""
    order = np.argsort(np.asarray(lengths), kind="stable")
    B = len(order)
    return [int(order[round(i * (B - 1) / (UNEVEN_SAMPLE - 1))]) for i in range(UNEVEN_SAMPLE)]


def _fp32(x: np.ndarray) -> np.ndarray:
    return x.astype(np.float32).astype(np.float64)


def _job(args):
    name, b, N = args
    if name == "chirps":
        s = _fp32(siggen.chirps(b))
        delta, J, two = 1e-3, 12, True
    elif name == "uneven":
        s = _fp32(siggen.uneven_signal(b, N))
        delta, J, two = 1e-4, 12, False
    else:
        s = _fp32(siggen.long_drift())
        delta, J, two = 1e-3, 20, False
    t0 = time.time()
    if two:
        ref = dif.decompose(s, delta, J)
        other = fif_spectral.decompose(s, delta, J)
        agree = "1" if (other.n_imfs == ref.n_imfs and (other.k, other.L, other.m) == (ref.k, ref.L, ref.m)) else "0"
    else:
        ref = fif_spectral.decompose(s, delta, J)
        agree = "-"
        if name == "uneven" and s.size <= UNEVEN_TIME_DOMAIN_MAX:
            other = dif.decompose(s, delta, J)
            agree = "1" if (other.n_imfs == ref.n_imfs and (other.k, other.L, other.m) == (ref.k, ref.L, ref.m)) \
                else "0"
    lines = ["S %d %d %d %d %s" % (b, s.size, ref.n_imfs, ref.stop_reason, agree)]
    for j in range(ref.n_imfs):
        lines.append("I %d %d %d %d %d %.17g %.17g %.6e %d" % (
            b, j, ref.k[j], ref.L[j], ref.m[j], ref.sd[j], ref.sd_prev[j], ref.margin_k[j], ref.flags[j]))
    return b, lines, time.time() - t0


HEADERS = {
    "chirps": ["chirp batch, 1024 x 65536 FP32 signals, delta 1e-3, 12 IMFs, mask rule 0",
               "decisions: time-domain Algorithm 2 (box-sum form); second oracle: direct form, linear scan"],
    "uneven": ["uneven batch, 64 of 4096 FP32 signals stratified by length, delta 1e-4, 12 IMFs, mask rule 0",
               "decisions: direct form of Section 4, linear scan; second oracle: time-domain Algorithm 2 "
               "(box-sum form) for N <= 16384"],
    "long": ["long signal, 2^24 FP32 samples, delta 1e-3, 20 IMFs, mask rule 0",
             "decisions: direct form of Section 4, linear scan (no second oracle)"],
}


def jobs_for(name: str) -> list:
    if name == "chirps":
        return [("chirps", b, 65536) for b in range(1024)]
    if name == "uneven":
        L = siggen.uneven_lengths(4096)
        return [("uneven", b, int(L[b])) for b in uneven_picks(L)]
    if name == "long":
        return [("long", 0, 1 << 24)]
    raise SystemExit("unknown workload %s" % name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", default=["chirps", "uneven", "long"])
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for name in args.workloads:
        jobs = jobs_for(name)
        # longest first, so the pool does not end on one long signal
        jobs.sort(key=lambda a: -a[2])
        t0 = time.time()
        out = {}
        with mp.get_context("fork").Pool(min(args.jobs, len(jobs))) as pool:
            for b, lines, el in pool.imap_unordered(_job, jobs):
                out[b] = lines
                print("%s signal %d: %.1f s (%d of %d)" % (name, b, el, len(out), len(jobs)), flush=True)
        path = os.path.join(HERE, "decisions_%s.txt" % name)
        with open(path, "w") as f:
            f.write("# Oracle decisions: %s\n" % HEADERS[name][0])
            f.write("# %s\n" % HEADERS[name][1])
            f.write("# written by tests/golden/make_golden.py (oracle/ and siggen/ only)\n")
            f.write("# S index N n_imfs stop_reason oracles_agree | I index j k L m sd sd_prev margin_k flags\n")
            for b in sorted(out):
                f.write("\n".join(out[b]) + "\n")
        print("%s: %d signals in %.0f s -> %s" % (name, len(out), time.time() - t0, path), flush=True)


if __name__ == "__main__":
    main()
