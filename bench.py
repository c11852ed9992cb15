#!/usr/bin/env python3
"""Throughput of batched Fast Iterative Filtering on one MI355X.

One step = one complete decomposition of the whole batch (every outer step:
extrema count, mask length, Parseval scan for m, spectral apply, synthesis of
the IMF and of the new residual), inputs resident in HBM, outputs written to
HBM.  Prints ONE JSON line on stdout; diagnostics go to stderr.

Workloads (synthetic, seeded; see siggen):
  chirps  1024 FP32 signals, N = 65536, 2-6 AM chirps + 30 dB noise,
          delta 1e-3, 12 IMFs (default; the headline configuration)
  uneven  4096 FP32 signals, 7-smooth lengths log-uniform in [1024, 262144],
          three AM tones, delta 1e-4, 12 IMFs
  long    one FP32 signal, N = 2^24, 10 drifting tones + 20 dB pink noise,
          delta 1e-3, 20 IMFs
  tones3  one FP64 signal, N = 4096, three AM tones, delta 1e-3, 8 IMFs
  plain   the chirps batch through the plain single-signal entry point
          (one signal at a time, host loop per outer step)
  learned 4096 FP32 signals, N = 65536, three AM tones at log-uniform
          frequencies + N(0, 0.01^2) noise (held-out members of the family the
          proposal network was trained on), delta 1e-3, 8 IMFs, with the
          trained network proposing m; the same batch without proposals is
          timed after it and reported beside
  window  the chirps batch with a sampled window shape (raised cosine,
          33 samples) instead of the triangle: every outer step tabulates
          the eigenvalues from a forward transform of the folded taps

--variant applies one of the paper's variants of the method to the chosen
workload: gamma (thresholded IMF, gamma = 0.01), abs (absolute stop
criterion), apriori (the a-priori N0 of Theorem 5, no search), rule1 (mask
length 2 floor(1.6 N/k)), peak (spectral-peak mask length, rho = 0.1).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "signal samples decomposed/sec (FP32 batched FIF) vs plain, % HBM peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
MODEL_FILE = os.path.join(ROOT, "paper_1802_01359_amd", "data", "proposal_tones3_65536.fifnet")
TUNE_CACHE = os.path.join(ROOT, "paper_1802_01359_amd", "data", "tune_cache.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


RAISED_COS_33 = [0.5 * (1.0 + float(np.cos(np.pi * i / 32))) for i in range(33)]

# option sets of the library (fif_options) and of the spectral oracle per variant
VARIANTS = {
    "gamma": (dict(gamma=1e-2), dict(gamma=1e-2)),
    "abs": (dict(stop_mode=1), dict(stop="abs")),
    "apriori": (dict(stop_mode=2), dict(stop="apriori")),
    "rule1": (dict(mask_rule=1), dict(mask_rule=1)),
    "peak": (dict(mask_rule=2, peak_rho=0.1), dict(mask_rule=2, peak_rho=0.1)),
}


def workload(name: str):
    import siggen
    if name == "window":
        B, N = 1024, 65536
        return dict(workload="window-raised-cosine-1024x65536", lengths=[N] * B, delta=1e-3, max_imfs=12,
                    io="f32", window=RAISED_COS_33, make=lambda: [siggen.chirps(i) for i in range(B)])
    if name in ("chirps", "plain"):
        B, N = 1024, 65536
        return dict(workload="chirps-1024x65536", lengths=[N] * B, delta=1e-3, max_imfs=12, io="f32",
                    make=lambda: [siggen.chirps(i) for i in range(B)])
    if name == "uneven":
        L = siggen.uneven_lengths(4096)
        return dict(workload="uneven-4096x[1024,262144]", lengths=list(L), delta=1e-4, max_imfs=12, io="f32",
                    make=lambda: [siggen.uneven_signal(i, int(n)) for i, n in enumerate(L)])
    if name == "long":
        return dict(workload="long-1x16777216", lengths=[1 << 24], delta=1e-3, max_imfs=20, io="f32",
                    make=lambda: [siggen.long_drift()])
    if name == "learned":
        B, N, first = 4096, 65536, 10_000_000
        return dict(workload="learned-4096x65536", lengths=[N] * B, delta=1e-3, max_imfs=8, io="f32",
                    make=lambda: [siggen.train_signal(first + i, N) for i in range(B)])
    if name == "tones3":
        return dict(workload="tones3-1x4096", lengths=[4096], delta=1e-3, max_imfs=8, io="f64",
                    make=lambda: [siggen.tones3()])
    raise SystemExit("unknown workload %s" % name)


def src_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1802_01359_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


SINGLE_MAX = 8192          # longest signal handled by one LDS pass
SCAN_REG_BINS = 32768      # most bins the one-workgroup scan keeps resident


def algorithmic_bytes(kind: str, lengths, n_imfs, max_imfs: int, esize: int) -> float:
    """Bytes a kernel kind must move per call of the whole decomposition, by
    the data flow of the path (not by its implementation): half spectra are
    (N/2+1) complex FP64 bins, signals/IMFs/remainders esize bytes/sample.
    Each kind counts only the signals it handles."""
    L = np.asarray(lengths, dtype=np.float64)
    n = np.asarray(n_imfs)
    spec = (np.floor(L / 2) + 1) * 16.0
    single = L <= SINGLE_MAX
    sel = {"single": single, "pass1": ~single, "pass2": ~single,
           "scan": np.floor(L / 2) <= SCAN_REG_BINS, "scan_big": np.floor(L / 2) > SCAN_REG_BINS}
    fam = kind.split("_")[0] if not kind.startswith("scan") else kind
    msk = sel.get(fam, np.ones_like(single))
    Ls, sp, ns = L[msk], spec[msk], n[msk]
    act = sum(float(np.sum(sp[ns > t])) for t in range(max_imfs))
    if kind in ("scan", "scan_big"):
        return act                                          # read the residual spectrum
    if kind == "pass1_step":
        return 2.0 * act                                    # read + write the spectrum
    if kind == "pass2_step":
        return max_imfs * float(np.sum(Ls)) * esize         # IMF rows (zeros once stopped)
    if kind == "single_step":
        return 2.0 * act + max_imfs * float(np.sum(Ls)) * esize
    if kind in ("pass1_fwd", "init_stats"):
        return float(np.sum(Ls)) * esize
    if kind == "pass2_fwd":
        return float(np.sum(sp))
    if kind == "single_fwd":
        return float(np.sum(Ls)) * esize + float(np.sum(sp))
    if kind == "pass1_rem":
        return float(np.sum(sp))
    if kind == "pass2_rem":
        return float(np.sum(Ls)) * esize
    if kind == "single_rem":
        return float(np.sum(sp)) + float(np.sum(Ls)) * esize
    if kind == "window":
        # write the folded taps, transform them (read), write the eigenvalue table
        L_all, sp_all = L, spec
        return sum(float(np.sum(8.0 * L_all[n > t] * 2 + sp_all[n > t] / 2)) for t in range(max_imfs))
    return 0.0                                              # bookkeeping / implementation-only kernels


def host_cores() -> int:
    """Host threads to give the CPU oracle: OMP_NUM_THREADS when the
    environment sets it (a host that shares its cores between jobs states
    this job's share that way), else every core this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sigs, delta, max_imfs, count: int, threads: int, window=None, okw=None, spectral=False):
    """The oracle on the first `count` signals, one signal per host thread
    (the C oracle releases the GIL; numpy's FFT does too) until all are
    done.  Returns (decompositions, samples, wall seconds).  A sampled window
    shape or a variant runs the FP64 spectral oracle (numpy), the
    time-domain one having only the plain method; spectral=True asks for it
    as well."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import dif
    from oracle import fif_spectral

    def one(s):
        s = np.asarray(s, dtype=np.float64)
        if spectral or window is not None or okw:
            return fif_spectral.decompose(s, delta, max_imfs, window=window, **(okw or {}))
        return dif.decompose(s, delta, max_imfs)
    batch = sigs[:count]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        decs = list(ex.map(one, batch))
    el = time.perf_counter() - t0
    return decs, sum(len(s) for s in batch), el


def lane_mismatch(a, b, lengths, J) -> dict:
    """Decision agreement of the FP32 lane's result a with the FP64 path's b
    on the same batch: signals whose decisions all agree, IMFs that agree up
    to a signal's first difference, and the largest relative L2 difference of
    those IMFs."""
    ia, ib = a.info(), b.info()
    na, nb = a.n_imfs.cpu().numpy(), b.n_imfs.cpu().numpy()
    sig_same = imf_same = 0
    worst = 0.0
    for s in range(len(lengths)):
        j = 0
        while j < min(na[s], nb[s]) and all(ia[k][s][j] == ib[k][s][j] for k in ("k", "L", "m")):
            j += 1
        imf_same += j
        sig_same += (j == nb[s] and na[s] == nb[s])
        if j:
            xa, xb = a.imfs_of(s)[:j].double(), b.imfs_of(s)[:j].double()
            e = ((xa - xb).norm(dim=1) / xb.norm(dim=1).clamp_min(1e-300)).max()
            worst = max(worst, float(e))
    ma = np.arange(J)[None, :] < na[:, None]
    return {"signals_with_fp64_decisions": int(sig_same), "signals": len(lengths),
            "imfs_with_fp64_decisions": int(imf_same), "imfs": int(nb.sum()),
            "decision_mismatch_rate_signals": round(float(1.0 - sig_same / len(lengths)), 4),
            "max_imf_rel_l2_where_decisions_agree": worst,
            "imfs_per_signal": round(float(na.mean()), 3), "fp64_imfs_per_signal": round(float(nb.mean()), 3),
            "m_median": int(np.median(ia["m"][ma])), "m_max": int(ia["m"][ma].max())}


def parity_of(decs, sigs, out, J, esize):
    """Decisions and per-IMF relative L2 error of the GPU output `out` for the
    signals the CPU oracle decomposed (signal b = decs[b])."""
    info = out.info()
    n = out.n_imfs.cpu().numpy()
    same = 0
    worst = 0.0
    for b, d in enumerate(decs):
        nb = int(n[b])
        got = [(int(info["k"][b][j]), int(info["L"][b][j]), int(info["m"][b][j])) for j in range(nb)]
        if nb == d.n_imfs and got == list(zip(d.k, d.L, d.m)):
            same += 1
            imfs = out.imfs_of(b).cpu().numpy().astype(np.float64)
            for j in range(nb):
                a = d.imfs[j]
                na = float(np.linalg.norm(a))
                if na > 0:
                    worst = max(worst, float(np.linalg.norm(a - imfs[j])) / na)
    return {"signals": len(decs), "decisions_identical": same, "max_imf_rel_l2": worst}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chirps", choices=["chirps", "uneven", "long", "tones3", "plain", "learned", "window"])
    ap.add_argument("--variant", default=None, choices=sorted(VARIANTS), help="a variant of the method (see above)")
    ap.add_argument("--model", default=MODEL_FILE, help="proposal network file (learned workload)")
    ap.add_argument("--cpu-signals", type=int, default=0,
                    help="signals the CPU oracle decomposes (default: two per host thread)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads for the oracle (default: OMP_NUM_THREADS, else every usable core)")
    ap.add_argument("--plain-signals", type=int, default=64,
                    help="signals of the batch timed through the plain single-signal form (headline workload)")
    ap.add_argument("--no-forms", action="store_true",
                    help="headline workload: skip timing the plain single-signal and learned-proposal forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="time replays of a captured HIP graph (FP32 workloads)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache file (lengths missing from it are timed when the plan is created)")
    ap.add_argument("--no-tune", action="store_true", help="built-in split, tiles and radix order for every length")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 512 MiB device copy first (a known-size kernel to scale HBM counters by)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported (signals are independent, "
              "a multi-GPU run would shard the batch by signal)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1802_01359_amd as fif

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    W = workload(args.workload)
    lib_opt, oracle_opt = VARIANTS[args.variant] if args.variant else ({}, {})
    if args.variant:
        if args.workload in ("plain", "learned", "window"):
            raise SystemExit("--variant applies to the batched workloads chirps, uneven, long, tones3")
        W["workload"] += "+" + args.variant
    lengths = W["lengths"]
    log("generating %s ..." % W["workload"])
    t0 = time.perf_counter()
    sigs = W["make"]()
    log("  %.1f s" % (time.perf_counter() - t0))
    dt = torch.float32 if W["io"] == "f32" else torch.float64
    esize = 4 if W["io"] == "f32" else 8
    packed = torch.tensor(np.concatenate(sigs), dtype=dt, device="cuda")
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (src.numel() * 4, dst.numel() * 4))
        del src, dst
    total = int(packed.numel())
    J = W["max_imfs"]
    delta = W["delta"]

    roofline = None
    extra = {}
    forms = {}
    plans = {}
    if args.workload == "plain":
        # plain single-signal form, one signal after another, host loop per outer step
        N = lengths[0]
        outs = []

        def step():
            for b in range(len(lengths)):
                outs.append(fif.decompose(packed[b * N:(b + 1) * N], delta, J))
                outs.clear()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    else:
        t_plan = time.perf_counter()
        plan = fif.Plan(lengths, J, fif.Options(window=W.get("window"), **lib_opt),
                        tune_cache=None if args.no_tune else args.tune_cache)
        t_plan = time.perf_counter() - t_plan
        plans = {"tuned": not args.no_tune, "create_s": round(t_plan, 2)}
        if not args.no_tune:
            chosen = [plan.length_plan(int(N)) for N in sorted(set(int(v) for v in lengths)) if N > 8192]
            timed = [c for c in chosen if c["us"] > 0 and c["us_default"] > 0]
            plans["lengths_tuned"] = len(timed)
            if timed:
                plans["builtin_over_tuned_time"] = round(float(np.exp(np.mean(
                    [np.log(c["us_default"] / c["us"]) for c in timed]))), 4)
            if len(chosen) <= 4:
                plans["choices"] = [{k: c[k] for k in ("N", "N1", "N2", "TC", "TR", "rad1", "rad2")} for c in chosen]
            log("plans: %s" % plans)
        out = plan.alloc_outputs(dt)
        model = None
        if args.workload == "learned":
            model = fif.Model(path=args.model, max_batch=min(len(lengths), 4096))
            plan.set_proposal(model)
        use_graph = args.graph
        stream = torch.cuda.Stream() if use_graph else torch.cuda.current_stream()
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                plan.run(packed, delta, out=out, graph=use_graph)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                plan.run(packed, delta, out=out, graph=use_graph)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        # per-kernel times from separate profiled runs (events around every
        # launch; profiling issues the whole batch on one stream, so each
        # kernel is timed running alone)
        prof_steps = max(1, min(args.steps, 2))
        plan.profile(True)
        plan.profile_read()
        for _ in range(prof_steps):
            plan.run(packed, delta, out=out)
        torch.cuda.synchronize()
        prof = plan.profile_read()
        plan.profile(False)
        forms = {}
        if args.workload == "chirps" and not args.variant and not args.no_forms:
            # the same batch through the plain single-signal form (a host
            # loop per outer step, one signal after another) on its first
            # signals, and through the batched form with the learned proposal
            N = lengths[0]
            P = min(args.plain_signals, len(lengths))
            fif.decompose(packed[:N], delta, J)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for b in range(P):
                fif.decompose(packed[b * N:(b + 1) * N], delta, J)
            torch.cuda.synchronize()
            el_p = time.perf_counter() - t1
            forms["plain_form"] = {"value": P * N / el_p, "signals": P, "ms_per_signal": 1e3 * el_p / P}
            lmodel = fif.Model(path=args.model, max_batch=len(lengths))
            plan.set_proposal(lmodel)
            lo = plan.alloc_outputs(dt)
            plan.run(packed, delta, out=lo)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                plan.run(packed, delta, out=lo)
            torch.cuda.synchronize()
            el_l = time.perf_counter() - t1
            plan.set_proposal(None)
            li, oi = lo.info(), out.info()
            lm = np.arange(J)[None, :] < lo.n_imfs.cpu().numpy()[:, None]
            forms["learned_form"] = {
                "value": total * args.steps / el_l, "ms_per_step": 1e3 * el_l / args.steps,
                "identical_to_plain_search": bool(torch.equal(lo.imfs, out.imfs) and torch.equal(lo.n_imfs, out.n_imfs)
                                                  and np.array_equal(li["m"], oi["m"])
                                                  and np.array_equal(li["L"], oi["L"])),
                "fp32_passes_per_imf": float((li["evals"][lm] & 0xffff).mean()),
                "model": os.path.basename(args.model)}
            log("plain single-signal form %.3g samples/s, learned proposal %.3g samples/s (identical %s)" % (
                forms["plain_form"]["value"], forms["learned_form"]["value"],
                forms["learned_form"]["identical_to_plain_search"]))
            # the FP32 lane on the same batch: its speed and how often its
            # decisions differ from the FP64 path's (which are the oracle's)
            aplan = fif.Plan(lengths, J, fif.Options(precision=fif.PREC_FP32),
                             tune_cache=None if args.no_tune else args.tune_cache)
            if not args.no_tune:
                plans["fp32_lane_choice"] = {k: aplan.length_plan(lengths[0])[k] for k in ("N1", "N2", "TC", "TR")}
            ao = aplan.alloc_outputs(dt)
            aplan.run(packed, delta, out=ao)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                aplan.run(packed, delta, out=ao)
            torch.cuda.synchronize()
            el_a = time.perf_counter() - t1
            forms["fp32_lane"] = dict(value=total * args.steps / el_a, ms_per_step=1e3 * el_a / args.steps,
                                      **lane_mismatch(ao, out, lengths, J))
            log("FP32 lane %.3g samples/s: %s" % (forms["fp32_lane"]["value"], forms["fp32_lane"]))
            del aplan, ao
        extra = {}
        if model is not None:
            # the same batch with the plain search, for comparison
            ref_info = out.info()
            plan.set_proposal(None)
            ref = plan.alloc_outputs(dt)
            plan.run(packed, delta, out=ref)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                plan.run(packed, delta, out=ref)
            torch.cuda.synchronize()
            el_plain = time.perf_counter() - t1
            pinf = ref.info()
            same = bool(np.array_equal(pinf["m"], ref_info["m"]) and np.array_equal(pinf["L"], ref_info["L"])
                        and torch.equal(ref.imfs, out.imfs))
            pm = np.arange(J)[None, :] < ref.n_imfs.cpu().numpy()[:, None]
            extra = {"plain_search_ms_per_step": 1e3 * el_plain / args.steps,
                     "plain_search_value": total * args.steps / el_plain,
                     "plain_fp32_passes_per_imf": float((pinf["evals"][pm] & 0xffff).mean()),
                     "identical_to_plain": same}
            log("plain search: %.2f ms/step, FP32 passes per IMF %.2f, identical %s" % (
                extra["plain_search_ms_per_step"], extra["plain_fp32_passes_per_imf"], same))
        n_imfs = out.n_imfs.cpu().numpy()
        st = out.sig_status.cpu().numpy()
        assert np.all(st == 0), "non-finite synthetic input"
        log("IMFs per signal: min %d mean %.2f max %d" % (n_imfs.min(), n_imfs.mean(), n_imfs.max()))
        inf = out.info()
        mask = np.arange(J)[None, :] < n_imfs[:, None]
        ev = inf["evals"][mask]
        log("search per IMF: FP32 passes mean %.2f max %d, FP64 evaluations mean %.3f max %d, refined %.2f%%, "
            "m median %d max %d" % ((ev & 0xffff).mean(), (ev & 0xffff).max(), (ev >> 16).mean(), (ev >> 16).max(),
                                    100.0 * np.mean(inf["flags"][mask] & 2 > 0), np.median(inf["m"][mask]),
                                    inf["m"][mask].max()))
        rows = []
        for kind, (launches, ms) in prof.items():
            alg = algorithmic_bytes(kind, lengths, n_imfs, J, esize) * prof_steps
            rows.append((ms, kind, launches, alg))
        rows.sort(reverse=True)
        tot_ms = sum(r[0] for r in rows)
        for ms, kind, launches, alg in rows:
            gbs = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
            log("  %-12s %5d launches %9.3f ms total (%5.1f%%) %8.3f ms/launch  %7.1f GB/s algorithmic" % (
                kind, launches, ms, 100 * ms / tot_ms, ms / launches, gbs))
        ms, kind, launches, alg = rows[0]
        avg_ms = ms / launches
        alg_per_launch = alg / launches
        achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            try:
                tr = json.load(open(TRAFFIC_FILE))
                if tr.get("src_sha") == src_digest() and tr.get("kernel") == kind \
                        and tr.get("workload") == W["workload"]:
                    traffic = float(tr["bytes_per_launch"])
            except (OSError, ValueError, KeyError):
                traffic = None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kind,
                    "algorithmic_bytes_per_launch": alg_per_launch, "avg_launch_ms": round(avg_ms, 4),
                    "kernel_share_of_step": round(ms / tot_ms, 3)}
        if traffic is not None:
            # measured HBM bytes of the same launches over their duration
            tg = traffic / (avg_ms * 1e-3) / 1e9
            roofline["traffic_GBs"] = round(tg, 1)
            roofline["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)

    value = total * args.steps / el
    # I/O floor: read the signals, write max_imfs IMF rows and the remainders
    io_floor = (J + 2) * total * esize * args.steps / el / 1e9
    res = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": W["workload"], "signals": len(lengths), "samples": total, "delta": delta,
                   "max_imfs": J, "io_dtype": W["io"], "io_floor_GBs": round(io_floor, 1),
                   "launch": "hip graph replay" if (args.graph and args.workload != "plain")
                   else "stream",
                   "form": "plain single-signal" if args.workload == "plain" else
                   ("batched, learned proposal of m" if args.workload == "learned" else
                    ("batched, sampled window shape" if args.workload == "window" else "batched"))},
    }
    if args.workload != "plain":
        res["config"]["plans"] = plans
    if args.workload != "plain" and forms:
        res["config"].update(forms)
        res["config"]["vs_plain"] = value / forms["plain_form"]["value"]
    if args.variant:
        res["config"]["variant"] = {"name": args.variant, "options": lib_opt}
    if args.workload not in ("plain",) and extra:
        res["config"].update(extra)
    if roofline is not None:
        res["roofline"] = roofline
    if not args.no_cpu_baseline:
        threads = args.cpu_threads if args.cpu_threads > 0 else host_cores()
        count = args.cpu_signals if args.cpu_signals > 0 else 2 * threads
        count = min(count, len(sigs))
        spectral = bool(W.get("window") or oracle_opt)
        log("CPU oracle: %d signals on %d threads ..." % (count, threads))
        decs, samples, cel = cpu_baseline(sigs, delta, J, count, threads, W.get("window"), oracle_opt)
        res["cpu_baseline"] = {
            "value": samples / cel, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d signals of the same workload, whole decompositions by the FP64 %s oracle, "
                      "one signal per thread, %d threads, %.1f s wall" % (
                          count, len(lengths), "spectral (numpy)" if spectral else "time-domain (C)", threads, cel),
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}
        if args.workload != "plain":
            res["cpu_baseline"]["gpu_parity_on_sample"] = parity_of(decs, sigs, out, J, esize)
        if not spectral and args.workload in ("chirps", "uneven"):
            # context: the FP64 direct form (numpy FFT) on the same signals
            _, s2, c2 = cpu_baseline(sigs, delta, J, count, threads, spectral=True)
            res["cpu_baseline"]["spectral_oracle_value"] = s2 / c2
        log("CPU oracle: %.3g samples/s" % res["cpu_baseline"]["value"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
