#!/usr/bin/env python3
"""PQ fit+encode throughput on one MI355X.

Workload (integer_pq): N = 1,000,000 rows, D = 128, non-negative integer
values in [0, 255] (clipped Gaussian mixture of 1,000 components, sigma 20),
codebooks fitted on a seeded 100,000-row sample with M = 16 subspaces,
Ks = 256 centroids, 25 Lloyd rounds, then all 1M rows encoded with the
reconstruction RMSE of their codes (formed by the encode pass itself).  One
step = fit + encode + RMSE, inputs resident in HBM.  The headline precision
is BF16 on matrix cores; the plain FP32 path runs the same step for
comparison (identical codes).

Other workloads (one JSON line each, same contract, selected with
--workload): batched_uneven (64 uneven problems fitted and encoded together),
ivf_adc (10M-row inverted file with residual PQ, ADC top-100 search) and
diff_codebooks (2M x 256 encode + reconstruction loss + backward).

Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_F32_ADD_T = 256 * 64 * 2.4e9 / 1e12   # unpacked float32 adds per second (T), 39.3
CSRC = os.path.join(ROOT, "paper_2604_21645_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fit_round_bf16_integer_pq_1M_traffic.json")
MFMA_SOURCE = os.path.join(CSRC, "pq_mfma.hip")
ADC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_adc_scan_ivf_adc_10M_traffic.json")
ADC_SOURCE = os.path.join(CSRC, "adc.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash(path: str = MFMA_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_totals(L, names):
    """(launches, summed ms) of each named kernel since the last collection."""
    import ctypes

    from paper_2604_21645_amd import _lib
    out = {}
    for name in names:
        a, b = ctypes.c_int64(0), ctypes.c_double(0)
        L.mipq_profile_collect(_lib.KERNELS[name], ctypes.byref(a), ctypes.byref(b))
        out[name] = (a.value, b.value)
    return out


def batched_roofline(kt, rows, d, m):
    """Roofline of a batched fit's dominant kernel: the fused round
    (assignment + float64 sums, one launch per Lloyd round) when the plan
    runs it, else the batched assignment; algorithmic bytes per launch are
    every row read once (4 d bytes), plus its m codes written by the
    assignment (the fused rounds store no codes: the final encode does)."""
    nl, tot = kt["fit_round_bf16"]
    name = "k_fit_round_bf16_batched"
    alg = rows * 4 * d
    if nl == 0:
        nl, tot = kt["assign_bf16_batched"]
        name = "k_assign_bf16_batched"
        alg = rows * (4 * d + m)
    avg = tot / max(nl, 1)
    achieved = alg / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": None, "alg_bytes_per_launch": alg, "avg_launch_ms": avg,
            "launches": nl}


def drop_profile(L):
    from paper_2604_21645_amd import _lib
    for k in _lib.KERNELS.values():
        L.mipq_profile_collect(k, None, None)


def timed_steps(fn, steps, warmup):
    """Run fn warmup times, then time exactly `steps` calls between two
    device synchronisations; returns ms per step and the last result."""
    import torch
    out = None
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1) * 1e3, out


def base_record(metric, value, unit, steps, warmup, ms, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config}


def measured_traffic(traffic_file: str = TRAFFIC_FILE, source: str = MFMA_SOURCE):
    """HBM bytes per launch of a kernel from committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE counters (copy-calibrated), or None if absent or stale (the
    kernel's source changed since the counters were taken)."""
    try:
        with open(traffic_file) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash(source):
        return None
    return t.get("bytes_per_launch")


COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_fit_round_bf16_integer_pq_1M_counters.json")


def measured_counters(counters_file: str = COUNTERS_FILE, source: str = MFMA_SOURCE):
    """VALU and MFMA busy fractions of a kernel from a committed rocprofv3
    counter record (the step's launch mix), or None if absent or stale."""
    try:
        with open(counters_file) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash(source):
        return None
    return t.get("step_mix")


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


CPU_SHARE = 16   # host threads per GPU on the measurement boxes


def oracle_threads(m: int) -> int:
    return max(1, min(m, CPU_SHARE, os.cpu_count() or 1))


def oracle_fit_encode(train, init, x_enc, m: int, iters: int, threads: int):
    """The oracle's Lloyd fit and float32-rule encode, one subspace per
    thread: the subspaces of a product quantiser are independent problems, so
    running the oracle's functions on each subspace's columns gives its
    results exactly (NumPy releases the GIL inside the array operations).
    Returns (codebook, fit seconds, encode seconds)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from oracle import pq

    ds = train.shape[1] // m

    def fit_one(j):
        return pq.lloyd(np.ascontiguousarray(train[:, j * ds:(j + 1) * ds]), init[j:j + 1], 1, iters,
                        decide="fp32")["codebook"]

    def enc_one(j):
        return pq.encode(np.ascontiguousarray(x_enc[:, j * ds:(j + 1) * ds]), cbs[j], decide="fp32")[0]

    with ThreadPoolExecutor(threads) as ex:
        t0 = time.perf_counter()
        cbs = list(ex.map(fit_one, range(m)))
        t1 = time.perf_counter()
        list(ex.map(enc_one, range(m)))
        t2 = time.perf_counter()
    return np.concatenate(cbs, 0), t1 - t0, t2 - t1


def oracle_row_chunks(k: int, threads: int, fn):
    """Run fn(a, b) on `threads` contiguous row ranges of [0, k) at once (the
    oracle's row-wise work is independent per row; NumPy releases the GIL
    inside the array operations).  Returns (results in row order, seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    bounds = [(k * i // threads, k * (i + 1) // threads) for i in range(threads)]
    with ThreadPoolExecutor(threads) as ex:
        t0 = time.perf_counter()
        out = list(ex.map(lambda ab: fn(*ab), bounds))
        t1 = time.perf_counter()
    return out, t1 - t0


def cpu_baseline(w, frac: float):
    """The oracle, as it stands, on a bounded sample of the same workload:
    fit on frac * n_train training rows (same rounds), encode frac * N rows,
    one subspace per host thread."""
    from synth import workloads as wl

    n_tr = max(w.ks, int(round(frac * len(w.train_rows))))
    n_en = int(round(frac * w.x.shape[0]))
    train = w.x[w.train_rows[:n_tr]]
    init = wl.init_rows_per_subspace(w.meta["seed"], n_tr, w.m, w.ks, key=7)
    threads = oracle_threads(w.m)
    _, tf, te = oracle_fit_encode(train, init, w.x[:n_en], w.m, w.iters, threads)
    return {
        "value": n_en / (tf + te),
        "unit": "vectors/s",
        "cores": threads,
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": "fit on %d training rows x %d rounds, encode %d rows (%.0f%% of the workload); "
                  "float32 decisions, one subspace per thread (%d threads); fit %.1fs, encode %.1fs"
                  % (n_tr, w.iters, n_en, 100 * frac, threads, tf, te),
    }


def oracle_parity(w, codes, cb, rmse, sample: int):
    """Oracle leg, part 2: codes of sampled rows against the float64 oracle
    (and its float32-decision mode) with the GPU's final codebook, and the
    oracle's RMSE of the GPU codes."""
    import numpy as np

    from oracle import pq

    n = w.x.shape[0]
    rs = np.random.default_rng(0).choice(n, min(sample, n), replace=False)
    cbn = cb.astype(np.float64)
    gc = codes[rs].astype(np.int64)
    r64, _, tie = pq.assign(w.x[rs], cbn, "fp64")
    r32, _, _ = pq.assign(w.x[rs], cbn, "fp32")
    _, rmse_o = pq.sse_rmse(w.x, codes.astype(np.int64), cbn)
    return {
        "codes_equal_oracle_pct": 100.0 * float((gc == r64).mean()),
        "codes_equal_oracle_outside_near_ties_pct": 100.0 * float((gc[~tie] == r64[~tie]).mean()),
        "codes_equal_fp32_decision_oracle_pct": 100.0 * float((gc == r32).mean()),
        "oracle_sample_rows": int(len(rs)),
        "oracle_near_ties": int(tie.sum()),
        "rmse_rel_gap_vs_oracle": abs(rmse - rmse_o) / rmse_o if rmse_o else 0.0,
    }


def bench_integer_pq(args) -> dict:
    """Headline workload: fit + encode + decode/RMSE of integer_pq (BF16),
    with the FP32 plain step beside it."""
    import numpy as np
    import torch

    import paper_2604_21645_amd as mipq
    from paper_2604_21645_amd import _lib
    from synth import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating workload")
    w = wl.integer_pq()
    n, d = w.x.shape
    x = torch.from_numpy(w.x).to(dev)
    train_rows = torch.from_numpy(w.train_rows).to(dev)
    init_rows = torch.from_numpy(w.init_rows).to(dev)
    n_train = len(w.train_rows)
    torch.cuda.synchronize()

    def step(prec, ev=None):
        fit = mipq.pq_fit(x, w.m, w.ks, w.iters, init_rows=init_rows, train_rows=train_rows,
                          precision=prec, labels=False, objective=False, deterministic=args.deterministic)
        if ev:
            ev[1].record()
        # the reconstruction error of the codes comes out of the encode itself
        enc = mipq.pq_encode_ex(x, fit["codebook"], prec, sse_rmse=True)
        if ev:
            ev[2].record()
        return fit["codebook"], enc["codes"], enc["sse_rmse"]

    def timed(prec, steps, warmup, profile):
        for i in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        L = _lib.lib()
        if profile:
            L.mipq_profile_enable(1)
            for k in _lib.KERNELS.values():   # drop anything recorded before
                L.mipq_profile_collect(k, None, None)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = None
        for i in range(steps):
            evs[i][0].record()
            out = step(prec, evs[i])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps * 1e3
        if profile:
            L.mipq_profile_enable(0)
        ph = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])] for e in evs]).mean(0)
        return wall, ph, out

    log("bf16: %d warmup + %d timed steps" % (args.warmup, args.steps))
    ms, ph, (cb, codes, sr) = timed("bf16", args.steps, args.warmup, profile=False)
    # per-kernel durations from a separate pass: the event pairs around each
    # launch stall the queue between dependent kernels, so they stay out of
    # the timed steps above
    prof_steps = 2
    log("bf16: %d profiled steps (per-kernel events)" % prof_steps)
    timed("bf16", prof_steps, 0, profile=True)
    L = _lib.lib()
    import ctypes
    kernel_stats = {}
    for name, kid in _lib.KERNELS.items():
        a, b = ctypes.c_int64(0), ctypes.c_double(0)
        L.mipq_profile_collect(kid, ctypes.byref(a), ctypes.byref(b))
        if a.value:
            kernel_stats[name] = (a.value, b.value)
    # the dominant kernel: the fit's fused rounds (assignment + float64 sums),
    # one launch per round over the n_train sampled rows; the encode's
    # assignment of all n rows is reported beside it.  Algorithmic bytes per
    # row: its float32 slice of every subspace read once (4 d); the rounds
    # store no codes (no labels are taken) and the sums and partials are not
    # counted.  The encode also writes its m codes per row.
    nl, tot = kernel_stats.get("fit_round_bf16", (0, 0.0))
    alg_bytes_per_launch = n_train * 4 * d
    avg_launch_ms = tot / max(nl, 1)
    achieved = alg_bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if nl else 0.0
    ne, te = kernel_stats.get("assign_bf16", (0, 0.0))
    enc_alg = n * (4 * d + w.m)
    enc_ms = te / max(ne, 1)
    sse, rmse = sr.cpu().numpy().tolist()

    fp32 = None
    if args.fp32_steps > 0:
        log("fp32 plain: 1 warmup + %d timed steps" % args.fp32_steps)
        ms32, ph32, (cb32, codes32, sr32) = timed("fp32", args.fp32_steps, 1, profile=False)
        fp32 = {
            "vectors_per_s": n / (ms32 * 1e-3),
            "fit_encode_vectors_per_s": n / ((ph32[0] + ph32[1]) * 1e-3),
            "ms_per_step": ms32,
            "codes_identical_to_bf16": bool(torch.equal(codes32, codes)),
            "codebook_identical_to_bf16": bool(torch.equal(cb32, cb)),
            "rmse": float(sr32[1].item()),
        }

    fp8 = None
    if args.fp8_steps > 0:
        log("fp8: 1 warmup + %d timed steps" % args.fp8_steps)
        ms8, ph8, (cb8, codes8, sr8) = timed("fp8", args.fp8_steps, 1, profile=False)
        _, resc8 = mipq.pq_encode(x, cb8, "fp8", rescored=True)
        fp8 = {
            "vectors_per_s": n / (ms8 * 1e-3),
            "fit_encode_vectors_per_s": n / ((ph8[0] + ph8[1]) * 1e-3),
            "ms_per_step": ms8,
            "codes_identical_to_bf16": bool(torch.equal(codes8, codes)),
            "codebook_identical_to_bf16": bool(torch.equal(cb8, cb)),
            "encode_pairs_rescored_pct": 100.0 * float(resc8.item()) / (n * w.m),
            "rmse": float(sr8[1].item()),
        }

    base, parity = None, {}
    if not args.no_cpu_baseline:
        log("oracle leg: parity on %d sampled rows" % args.oracle_sample)
        parity = oracle_parity(w, codes.cpu().numpy(), cb.cpu().numpy(), rmse, args.oracle_sample)
        log("oracle leg: cpu baseline on a %.0f%% sample" % (100 * args.cpu_frac))
        base = cpu_baseline(w, args.cpu_frac)

    traffic = measured_traffic()
    counters = measured_counters()
    res = {
        "metric": "PQ fit+encode vectors/s, BF16-MFMA vs FP32 plain, % codes equal to oracle",
        "value": n / (ms * 1e-3),
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "integer_pq: 1M x 128 rows in [0,255], fit on 100k-row sample, "
                               "M=16, Ks=256, 25 Lloyd rounds, encode 1M with the reconstruction RMSE",
                   "n": n, "d": d, "m": w.m, "ks": w.ks, "iters": w.iters, "n_train": n_train,
                   "precision": "bf16", "parallelism": "single GPU", "deterministic_sums": args.deterministic},
        "phases_ms": {"fit": ph[0], "encode_rmse": ph[1]},
        "fit_encode_vectors_per_s": n / ((ph[0] + ph[1]) * 1e-3),
        "fp32_plain": fp32,
        "fp8": fp8,
        "rmse": rmse,
        "oracle_parity": parity or None,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_fit_round_bf16",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes_per_launch,
            "avg_launch_ms": avg_launch_ms,
            "launches": nl,
            "valu_frac": (counters or {}).get("valu_busy"),
            "mfma_util": (counters or {}).get("mfma_busy"),
            "encode_kernel": {"kernel": "k_assign_bf16", "alg_bytes_per_launch": enc_alg, "avg_launch_ms": enc_ms,
                              "launches": ne,
                              "achieved": enc_alg / (enc_ms * 1e-3) / 1e9 if ne else 0.0,
                              "frac": enc_alg / (enc_ms * 1e-3) / 1e9 / PEAK_HBM_GBS if ne else 0.0},
        },
        "kernels_ms_per_step": {k: v[1] / prof_steps for k, v in kernel_stats.items()},
        "cpu_baseline": base,
    }
    return res


def bench_plain(args) -> dict:
    """plain_pq: 10,000 x 128 rows (64-component mixture), M=8, Ks=256, 20
    Lloyd rounds from seeded rows, encode all rows with the fused error.  The
    step is a few dozen small launches, so it is captured once in a HIP graph
    and replayed; the eager time is reported beside it."""
    import numpy as np
    import torch

    import paper_2604_21645_amd as mipq
    from paper_2604_21645_amd import _lib
    from synth import workloads as wl

    dev = torch.device("cuda:0")
    w = wl.plain_pq()
    n, d = w.x.shape
    x = torch.from_numpy(w.x).to(dev)
    init = torch.from_numpy(w.init_rows).to(dev)
    prec = "bf16"

    def step():
        fit = mipq.pq_fit(x, w.m, w.ks, w.iters, init_rows=init, precision=prec, labels=False, objective=False)
        enc = mipq.pq_encode_ex(x, fit["codebook"], prec, sse_rmse=True)
        return fit["codebook"], enc["codes"], enc["sse_rmse"]

    log("plain_pq eager: %d warmup + %d timed steps" % (args.warmup, args.steps))
    ms_eager, (cb_e, codes_e, sr_e) = timed_steps(step, args.steps, args.warmup)
    # per-kernel durations of one eager step
    L = _lib.lib()
    L.mipq_profile_enable(1)
    drop_profile(L)
    step()
    torch.cuda.synchronize()
    L.mipq_profile_enable(0)
    kt = kernel_totals(L, ["fit_round_bf16", "assign_bf16", "update", "finalize", "pack_bf16"])
    log("plain_pq: capturing one step in a graph")
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step()   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=cs):
        cb_g, codes_g, sr_g = step()
    torch.cuda.synchronize()
    ms, _ = timed_steps(g.replay, args.steps, args.warmup)
    same = bool(torch.equal(cb_g, cb_e) and torch.equal(codes_g, codes_e) and torch.equal(sr_g, sr_e))
    sse, rmse = sr_g.cpu().numpy().tolist()
    # the fit's fused rounds (one launch per round, all n rows) and the
    # encode's assignment: the same n (4 d + m) algorithmic bytes per launch
    nf, tf_ms = kt["fit_round_bf16"]
    ne, te_ms = kt["assign_bf16"]
    na, ta = nf + ne, tf_ms + te_ms
    alg_per_launch = n * (4 * d + w.m)
    avg_ms = ta / max(na, 1)
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9 if na else 0.0
    base = None
    if not args.no_cpu_baseline:
        log("oracle leg: plain_pq fit + encode on the CPU")
        threads = oracle_threads(w.m)
        _, tf, te = oracle_fit_encode(w.x, w.init_rows, w.x, w.m, w.iters, threads)
        base = {"value": n / (tf + te), "unit": "vectors/s", "cores": threads, "kind": "oracle",
                "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
                "sample": "the whole step: 20 Lloyd rounds on all 10,000 rows and their encode, float32 "
                          "decisions, one subspace per thread; fit %.1fs, encode %.1fs" % (tf, te)}
    rec = base_record("PQ fit+encode vectors/s, BF16-MFMA vs FP32 plain, % codes equal to oracle", n / (ms * 1e-3),
                      "vectors/s", args.steps, args.warmup, ms, "bf16",
                      {"workload": "plain_pq: 10,000 x 128 rows, 64-component mixture (sigma 0.05), M=8, Ks=256, "
                                   "20 Lloyd rounds from 256 seeded rows per subspace, encode all, RMSE",
                       "n": n, "d": d, "m": w.m, "ks": w.ks, "iters": w.iters, "precision": prec,
                       "parallelism": "single GPU", "launch": "one HIP graph per step"})
    rec.update({
        "ms_per_step_eager": ms_eager,
        "graph_replay_identical_to_eager": same,
        "rmse": rmse,
        "roofline": {"bound": "hbm", "kernel": "k_fit_round_bf16 + k_assign_bf16", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg_per_launch, "avg_launch_ms": avg_ms, "launches": na,
                     "note": "5 MB per launch: bound by launch and wave start-up latency, not by a roofline"},
        "kernels_ms_per_step_eager": {k: v[1] for k, v in kt.items()},
        "cpu_baseline": base,
    })
    return rec


def bench_batched(args) -> dict:
    """64 uneven problems (N_i log-uniform in [20k, 500k], D=96 unit rows,
    M=12, Ks=256, 20 rounds on all rows of each, then encode + error), fitted
    together: one launch per phase, autotuned plan, HIP graphs."""
    import numpy as np
    import torch

    import paper_2604_21645_amd as mipq
    from paper_2604_21645_amd import _lib
    from synth import workloads as wl

    dev = torch.device("cuda:0")
    log("generating batched_uneven")
    w = wl.batched_uneven()
    sizes = [p.x.shape[0] for p in w.problems]
    total = int(sum(sizes))
    d = w.problems[0].x.shape[1]
    allx = torch.from_numpy(np.concatenate([p.x for p in w.problems])).to(dev)
    xs = list(torch.split(allx, sizes))
    inits = [torch.from_numpy(p.init_rows).to(dev) for p in w.problems]
    torch.cuda.synchronize()
    log("plan: autotune + graph capture")
    t0 = time.perf_counter()
    b = mipq.BatchedFit(xs, inits, w.m, w.ks, w.iters, plan=True, autotune=True, graph=True, objective=False)
    plan_s = time.perf_counter() - t0
    info = b.info()
    log("plan", info, "%.2fs" % plan_s)
    log("%d warmup + %d timed steps" % (args.warmup, args.steps))
    ms, _ = timed_steps(lambda: b.run(), args.steps, args.warmup)
    resc = b.run(rescored=True)
    torch.cuda.synchronize()
    rmse = np.array([r["sse_rmse"][1].item() for r in b.results])

    log("profiled eager run (same kernels, no graphs)")
    L = _lib.lib()
    pe = mipq.BatchedFit(xs, inits, w.m, w.ks, w.iters, plan=True, autotune=True, graph=False, objective=False)
    pe.run()
    torch.cuda.synchronize()
    drop_profile(L)
    L.mipq_profile_enable(1)
    pe.run()
    torch.cuda.synchronize()
    L.mipq_profile_enable(0)
    kt = kernel_totals(L, ["fit_round_bf16", "assign_bf16_batched", "update", "finalize", "pack_bf16", "decode"])
    roof = batched_roofline(kt, total, d, w.m)
    same = all(torch.equal(r0["codes"], r1["codes"]) for r0, r1 in zip(b.results, pe.results))
    pe.close()

    base = None
    if not args.no_cpu_baseline:
        n_s = min(args.batched_cpu_rows, sizes[0])
        xs0 = w.problems[0].x[:n_s]
        init = wl.init_rows_per_subspace(w.meta["seed"], n_s, w.m, w.ks, key=99)
        threads = oracle_threads(w.m)
        log("oracle leg: fit + encode of %d rows of problem 0 (%d threads)" % (n_s, threads))
        _, tf, te = oracle_fit_encode(xs0, init, xs0, w.m, w.iters, threads)
        base = {"value": n_s / (tf + te), "unit": "vectors/s", "cores": threads, "host_cpus": os.cpu_count(),
                "cpu_model": cpu_model(), "kind": "oracle",
                "sample": "%d rows of problem 0 fitted %d rounds and encoded (float32 decisions, one subspace per "
                          "thread; fit %.1fs, encode %.1fs)" % (n_s, w.iters, tf, te)}
    b.close()
    rec = base_record("PQ fit+encode vectors/s, 64 uneven problems batched (BF16-MFMA)", total / (ms * 1e-3),
                      "vectors/s", args.steps, args.warmup, ms, "bf16",
                      {"workload": "batched_uneven: 64 problems, N_i log-uniform in [20k, 500k] (%d rows in total), "
                                   "D=96 unit-norm rows, M=12, Ks=256, 20 Lloyd rounds on all rows of each problem, "
                                   "encode + RMSE per problem" % total,
                       "problems": len(sizes), "rows": total, "d": d, "m": w.m, "ks": w.ks, "iters": w.iters,
                       "precision": "bf16", "parallelism": "single GPU"})
    rec.update({
        "plan": dict(info, seconds=plan_s),
        "rescored_pairs_final_encode": int(resc.item()),
        "graph_and_eager_codes_identical": bool(same),
        "rmse_mean": float(rmse.mean()),
        "roofline": roof,
        "kernels_ms_per_step": {k: v[1] for k, v in kt.items()},
        "cpu_baseline": base,
    })
    return rec


def bench_ivf(args) -> dict:
    """10M x 128 rows, coarse Kc=4096 (20 rounds on a 262,144-row sample),
    residual PQ M=16 Ks=256, stable bucketing; 10k queries, nprobe 32, top-100."""
    import numpy as np
    import torch

    import paper_2604_21645_amd as mipq
    from paper_2604_21645_amd import _lib
    from synth import workloads as wl

    dev = torch.device("cuda:0")
    log("generating ivf_adc")
    w = wl.ivf_adc()
    n, d = w.x.shape
    nq = w.queries.shape[0]
    x = torch.from_numpy(w.x).to(dev)
    q = torch.from_numpy(w.queries).to(dev)
    tr = torch.from_numpy(w.coarse_train).to(dev)
    ci = torch.from_numpy(w.coarse_init).to(dev)
    pi = torch.from_numpy(w.pq_init).to(dev)
    torch.cuda.synchronize()

    def build():
        return mipq.ii_build(x, w.kc, w.coarse_iters, tr, ci, w.m, w.ks, w.pq_iters, pi, labels=False)

    log("index build: 1 warmup + %d timed" % args.build_steps)
    build_ms, idx = timed_steps(build, args.build_steps, 1)
    log("build %.1f ms; search: %d warmup + %d timed" % (build_ms, args.warmup, args.steps))
    ms, (ids, dist) = timed_steps(lambda: mipq.adc_search(q, idx, w.nprobe, w.topk), args.steps, args.warmup)

    log("profiled legs: coarse assignment of all rows, one build, one search")
    L = _lib.lib()
    drop_profile(L)
    L.mipq_profile_enable(1)
    for _ in range(3):
        _, ca_resc = mipq.coarse_assign(x, idx["coarse"], "bf16", rescored=True)
    torch.cuda.synchronize()
    ca = kernel_totals(L, ["coarse_assign"])["coarse_assign"]
    build()
    torch.cuda.synchronize()
    kb = kernel_totals(L, ["coarse_pack", "coarse_assign", "sort", "coarse_update", "fit_round_bf16", "assign_bf16",
                           "update", "finalize", "pack_bf16"])
    mipq.adc_search(q, idx, w.nprobe, w.topk)
    torch.cuda.synchronize()
    ka = kernel_totals(L, ["adc", "adc_scan"])
    L.mipq_profile_enable(0)
    # the work the scans executed (device counters; the exact skips avoid the rest)
    _, _, wk = mipq.adc_search(q, idx, w.nprobe, w.topk, work=True)
    lut_entries, part_rows, full_rows, lists_scanned = [int(v) for v in wk.cpu().numpy()]
    flops = 2.0 * n * d * w.kc
    avg = ca[1] / max(ca[0], 1)
    achieved = flops / (avg * 1e-3) / 1e12
    # candidates scanned: the probed lists of every query, ranked on the CPU in
    # float64 (differs from the GPU's exact-rule probes only at near-ties)
    cc64 = idx["coarse"].cpu().numpy().astype(np.float64)
    sizes = np.diff(idx["offsets"].cpu().numpy())
    cand = 0
    for q0 in range(0, nq, 2000):
        qq = w.queries[q0:q0 + 2000].astype(np.float64)
        dq = (qq * qq).sum(1)[:, None] - 2.0 * qq @ cc64.T + (cc64 * cc64).sum(1)[None, :]
        pr = np.argpartition(dq, w.nprobe - 1, axis=1)[:, :w.nprobe]
        cand += int(sizes[pr].sum())
    scan_bytes = cand * (w.m + 4)
    scan_adds = cand * w.m           # the method's score work: M table entries summed per candidate
    ns, ts = ka["adc_scan"]
    scan_ms = ts / max(ns, 1)
    scan_gbs = scan_bytes / (scan_ms * 1e-3) / 1e9
    # executed: a table entry is ds float32 differences, squares and sums; a
    # partial row sums 4 entries, a full row M; every summed entry is one LDS read
    ds = d // w.m
    pre = 4
    exec_ops = lut_entries * 3 * ds + part_rows * pre + full_rows * w.m
    lds_reads = part_rows * pre + full_rows * w.m
    exec_t = exec_ops / (scan_ms * 1e-3) / 1e12
    lds_peak_t = 256 * 32 * 2.4e9 / 1e12   # 4-byte LDS reads per second: 128 bytes per clock per CU
    lds_t = lds_reads / (scan_ms * 1e-3) / 1e12

    base, parity = None, None
    if not args.no_cpu_baseline:
        from oracle import ivf
        k = min(args.ivf_cpu_queries, nq)
        log("oracle leg: ADC search of %d queries on the GPU-built index" % k)
        cc = idx["coarse"].cpu().numpy()
        pqc = idx["pq_codebook"].cpu().numpy()
        off = idx["offsets"].cpu().numpy()
        idn = idx["ids"].cpu().numpy().astype(np.int64)
        cs = idx["codes_sorted"].cpu().numpy()
        cbi = np.empty_like(cs)
        cbi[idn] = cs
        threads = max(1, min(CPU_SHARE, os.cpu_count() or 1, k))
        parts, tq = oracle_row_chunks(k, threads, lambda a, b: ivf.adc_search(
            w.queries[a:b], cc, pqc, off, idn, cbi, w.nprobe, w.topk, decide="kernel"))
        ri = np.concatenate([p_[0] for p_ in parts])
        rd = np.concatenate([p_[1] for p_ in parts])
        base = {"value": k / tq, "unit": "queries/s", "cores": threads, "host_cpus": os.cpu_count(),
                "cpu_model": cpu_model(), "kind": "oracle",
                "sample": "ADC top-%d of the first %d queries (nprobe %d) on the GPU-built index, float32 table "
                          "arithmetic, queries split over %d threads, %.1fs" % (w.topk, k, w.nprobe, threads, tq)}
        gi = ids.cpu().numpy()[:k].astype(np.int64)
        parity = {"queries": k, "top100_identical_pct": 100.0 * float(np.all(gi == ri, axis=1).mean()),
                  "distances_identical": bool(np.array_equal(dist.cpu().numpy()[:k], rd.astype(np.float32)))}
    rec = base_record("ADC top-100 queries/s on a 10M-row IVF-PQ index (nprobe 32)", nq / (ms * 1e-3), "queries/s",
                      args.steps, args.warmup, ms, "f32",
                      {"workload": "ivf_adc: 10M x 128 rows (4,096-component mixture), coarse Kc=4096 fitted 20 "
                                   "rounds on 262,144 sampled rows, residual PQ M=16 Ks=256 (20 rounds), stable "
                                   "bucketing; 10,000 queries, nprobe 32, top-100",
                       "n": n, "d": d, "kc": w.kc, "m": w.m, "ks": w.ks, "nq": nq, "nprobe": w.nprobe,
                       "topk": w.topk, "precision": "bf16 ranking, exact float32/float64 decisions",
                       "parallelism": "single GPU"})
    rec.update({
        "build_ms": build_ms,
        "build_vectors_per_s": n / (build_ms * 1e-3),
        "oracle_parity": parity,
        "roofline": {"bound": "alu", "kernel": "k_adc_scan", "achieved": exec_t, "peak": PEAK_F32_ADD_T,
                     "unit": "T lane-ops/s", "frac": exec_t / PEAK_F32_ADD_T,
                     "traffic": measured_traffic(ADC_TRAFFIC_FILE, ADC_SOURCE),
                     "executed_ops_per_launch": exec_ops, "avg_launch_ms": scan_ms, "launches": ns,
                     "work_counters": {"table_entries_built": lut_entries, "rows_partial_sum": part_rows,
                                       "rows_full_sum": full_rows, "lists_scanned": lists_scanned,
                                       "pairs": nq * w.nprobe},
                     "lds_view": {"reads_per_launch": lds_reads, "achieved_t_reads_per_s": lds_t,
                                  "peak_t_reads_per_s": lds_peak_t, "frac": lds_t / lds_peak_t},
                     "method_view": {"candidates_per_launch": cand, "table_adds_per_launch": scan_adds,
                                     "alg_bytes_per_launch": scan_bytes, "alg_gbs": scan_gbs},
                     "note": "executed work from device counters in the scan: table entries (3 ds float32 ops "
                             "each) and summed entries (one add and one LDS read each), against unpacked float32 "
                             "issue (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz); the exact list bound and partial "
                             "sums skip the rest of the method's table adds (method_view)"},
        "build_roofline": {"bound": "mfma", "kernel": "k_coarse_assign_mfma + k_coarse_resolve_mfma", "achieved": achieved,
                           "peak": 2500.0,
                           "unit": "TFLOP/s", "frac": achieved / 2500.0, "traffic": None,
                           "alg_flops_per_launch": flops, "avg_launch_ms": avg, "launches": ca[0],
                           "note": "coarse assignment of all 10M rows against Kc=4096 (2*N*D*Kc flops per assignment, "
                                   "timed over both launches: the ranking of every row and the exact decision of the "
                                   "undecided ones)"},
        "coarse_rows_rescored": int(ca_resc.item()),
        "build_kernels_ms": {k2: v[1] for k2, v in kb.items() if v[0]},
        "search_kernels_ms": {k2: v[1] for k2, v in ka.items()},
        "cpu_baseline": base,
    })
    return rec


def bench_diff(args) -> dict:
    """2M x 256 rows, M=32, Ks=256 codebooks (fitted once, 20 rounds on a
    200k sample, BF16): one step = BF16 encode of all rows + reconstruction
    loss + backward to the codebooks and the inputs."""
    import numpy as np
    import torch

    import paper_2604_21645_amd as mipq
    from paper_2604_21645_amd import _lib
    from synth import workloads as wl

    dev = torch.device("cuda:0")
    log("generating diff_codebooks")
    w = wl.diff_codebooks()
    n, d = w.x.shape
    x0 = torch.from_numpy(w.x).to(dev)
    fit = mipq.pq_fit(x0, w.m, w.ks, w.iters, init_rows=torch.from_numpy(w.init_rows).to(dev),
                      train_rows=torch.from_numpy(w.train_rows).to(dev), precision="bf16", labels=False)
    xr = x0.clone().requires_grad_(True)
    cb = fit["codebook"].clone().requires_grad_(True)
    torch.cuda.synchronize()

    def step():
        # the encode's fused error is the loss's forward (no second pass over the rows)
        xr.grad = None
        cb.grad = None
        enc = mipq.pq_encode_ex(xr.detach(), cb.detach(), "bf16", sse_rmse=True)
        loss = mipq.PQReconLoss.apply(xr, cb, enc["codes"], enc["sse_rmse"])
        loss.backward()
        return loss

    log("%d warmup + %d timed steps" % (args.warmup, args.steps))
    ms, loss = timed_steps(step, args.steps, args.warmup)
    L = _lib.lib()
    drop_profile(L)
    L.mipq_profile_enable(1)
    step()
    torch.cuda.synchronize()
    L.mipq_profile_enable(0)
    kt = kernel_totals(L, ["assign_bf16", "pack_bf16", "decode", "backward"])
    nl, tot = kt["backward"]
    alg = n * (8 * d + w.m)
    avg = tot / max(nl, 1)
    achieved = alg / (avg * 1e-3) / 1e9

    base = None
    if not args.no_cpu_baseline:
        from oracle import grad, pq
        k = min(args.diff_cpu_rows, n)
        log("oracle leg: encode + loss + gradients of %d rows" % k)
        cbn = cb.detach().cpu().numpy().astype(np.float64)
        threads = max(1, min(CPU_SHARE, os.cpu_count() or 1))

        def enc_grad(a, b):
            codes_o, _ = pq.encode(w.x[a:b], cbn, decide="fp32")
            return grad.grads(w.x[a:b], codes_o, cbn)

        _, tg = oracle_row_chunks(k, threads, enc_grad)
        base = {"value": k / tg, "unit": "vectors/s", "cores": threads, "host_cpus": os.cpu_count(),
                "cpu_model": cpu_model(), "kind": "oracle",
                "sample": "encode (float32 decisions) + float64 loss and gradients of the first %d rows, rows split "
                          "over %d threads, %.1fs" % (k, threads, tg)}
    rec = base_record("Reconstruction-loss forward+backward vectors/s (BF16 encode, fixed codes)", n / (ms * 1e-3),
                      "vectors/s", args.steps, args.warmup, ms, "bf16",
                      {"workload": "diff_codebooks: 2M x 256 rows (8,192-component mixture), M=32, Ks=256 codebooks "
                                   "fitted once (20 rounds on 200k rows); step = BF16 encode of all rows with its fused "
                                   "float64 error (the loss) + dL/dx and dL/dC",
                       "n": n, "d": d, "m": w.m, "ks": w.ks, "precision": "bf16 encode, float64 loss/sums",
                       "parallelism": "single GPU"})
    rec.update({
        "loss": float(loss.item()),
        "roofline": {"bound": "hbm", "kernel": "k_backward_group<grad_x> (backward)", "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg, "avg_launch_ms": avg, "launches": nl},
        "kernels_ms_per_step": {k2: v[1] for k2, v in kt.items()},
        "cpu_baseline": base,
    })
    return rec


def bench_soil(args) -> dict:
    """The paper's two-level pipeline on a stand-in with its data shape:
    6.7M x 48 rows in 400 chunks of 16,750 rows; per-chunk BF16 fits (M=8,
    Ks=256, 20 rounds) batched in one plan with graphs, the pooled decoded
    centroids (102,400 rows), a global fit on the pool, encode of all rows
    and the RMSE.  A single global fit on all rows is run beside it (untimed)
    for the paper's RMSE comparison."""
    import numpy as np
    import torch

    import paper_2604_21645_amd as mipq
    from paper_2604_21645_amd import _lib
    from synth import workloads as wl

    dev = torch.device("cuda:0")
    log("generating soil_chunks")
    w = wl.soil_chunks()
    n, d = w.x.shape
    ds = d // w.m
    x = torch.from_numpy(w.x).to(dev)
    xs = list(torch.split(x, w.chunk_rows))
    inits = [torch.from_numpy(i).to(dev) for i in w.chunk_inits]
    ginit = torch.from_numpy(w.global_init).to(dev)
    books = torch.empty((len(xs), w.m, w.ks, ds), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = mipq.BatchedFit(xs, inits, w.m, w.ks, w.iters, plan=True, autotune=True, graph=True, objective=False,
                        sse=False, codebooks=books)
    plan_s = time.perf_counter() - t0

    def step():
        b.run()
        pool = mipq.decode_centroids(books)
        g = mipq.pq_fit(pool, w.m, w.ks, w.iters, init_rows=ginit, precision="bf16", labels=False, objective=False)
        codes = mipq.pq_encode(x, g["codebook"], "bf16")
        _, sr = mipq.pq_decode_rmse(codes, g["codebook"], x)
        return g["codebook"], codes, sr

    log("%d warmup + %d timed steps" % (args.warmup, args.steps))
    ms, (cb, codes, sr) = timed_steps(step, args.steps, args.warmup)
    rmse2 = float(sr[1].item())
    log("single global fit for comparison")
    init1 = torch.from_numpy(wl.init_rows_per_subspace(w.meta["seed"], n, w.m, w.ks, key=77)).to(dev)
    one = mipq.pq_fit(x, w.m, w.ks, w.iters, init_rows=init1, precision="bf16", labels=False, objective=False)
    _, sr1 = mipq.pq_decode_rmse(mipq.pq_encode(x, one["codebook"], "bf16"), one["codebook"], x)
    rmse1 = float(sr1[1].item())

    log("profiled eager pass")
    L = _lib.lib()
    pe = mipq.BatchedFit(xs, inits, w.m, w.ks, w.iters, plan=True, autotune=True, graph=False, objective=False,
                         sse=False)
    pe.run()
    torch.cuda.synchronize()
    drop_profile(L)
    L.mipq_profile_enable(1)
    pe.run()
    torch.cuda.synchronize()
    L.mipq_profile_enable(0)
    kt = kernel_totals(L, ["fit_round_bf16", "assign_bf16_batched", "update", "finalize", "decode"])
    pe.close()
    roof = batched_roofline(kt, n, d, w.m)

    base = None
    if not args.no_cpu_baseline:
        k = min(args.soil_cpu_rows, w.chunk_rows)
        xs0 = w.x[:k]
        init = wl.init_rows_per_subspace(w.meta["seed"], k, w.m, w.ks, key=98)
        threads = oracle_threads(w.m)
        log("oracle leg: fit + encode of %d rows of chunk 0 (%d threads)" % (k, threads))
        _, tf, te = oracle_fit_encode(xs0, init, xs0, w.m, w.iters, threads)
        base = {"value": k / (tf + te), "unit": "vectors/s", "cores": threads, "host_cpus": os.cpu_count(),
                "cpu_model": cpu_model(), "kind": "oracle",
                "sample": "%d rows of chunk 0 fitted %d rounds and encoded (float32 decisions, one subspace per "
                          "thread; fit %.1fs, encode %.1fs)" % (k, w.iters, tf, te)}
    info = b.info()
    b.close()
    rec = base_record("Two-level chunked PQ fit+encode vectors/s (the paper's pipeline, BF16-MFMA)",
                      n / (ms * 1e-3), "vectors/s", args.steps, args.warmup, ms, "bf16",
                      {"workload": "soil_chunks: 6.7M x 48 rows (500-component mixture standing in for the paper's "
                                   "SoilGrids sample) in 400 chunks of 16,750 rows; per-chunk fits M=8 (ds=6), "
                                   "Ks=256, 20 rounds; global fit on 102,400 pooled centroids; encode all rows; RMSE",
                       "n": n, "d": d, "chunks": len(xs), "m": w.m, "ks": w.ks, "iters": w.iters,
                       "precision": "bf16", "parallelism": "single GPU"})
    rec.update({
        "plan": dict(info, seconds=plan_s),
        "rmse_two_level": rmse2,
        "rmse_single_global_fit": rmse1,
        "rmse_rel_gap": (rmse2 - rmse1) / rmse1,
        "roofline": roof,
        "kernels_ms_per_local_fit": {k2: v[1] for k2, v in kt.items()},
        "cpu_baseline": base,
    })
    return rec


def bench_opq(args) -> dict:
    """Optimized PQ on the integer-valued 1M x 128 rows: the rotation R and
    the codebooks (M=16, Ks=256) are fitted once on the 100k-row training
    sample (10 alternations of 2 Lloyd rounds and one Procrustes step each;
    timed and reported beside the line), then one step = rotation of all 1M
    rows + BF16 encode + decode/RMSE of the rotated rows."""
    import numpy as np
    import torch

    import paper_2604_21645_amd as mipq
    from paper_2604_21645_amd import _lib
    from synth import workloads as wl

    dev = torch.device("cuda:0")
    log("generating integer_pq rows for opq")
    w = wl.integer_pq()
    n, d = w.x.shape
    x = torch.from_numpy(w.x).to(dev)
    tr = x[torch.from_numpy(w.train_rows).to(dev)].contiguous()
    init = torch.from_numpy(w.init_rows).to(dev)
    outer, inner = 10, 2
    mipq.opq_fit(tr, w.m, w.ks, 1, inner, init)        # warm-up of the fit path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit = mipq.opq_fit(tr, w.m, w.ks, outer, inner, init)
    torch.cuda.synchronize()
    fit_ms = (time.perf_counter() - t0) * 1e3
    r, cb = fit["R"], fit["codebook"]

    def step():
        y = mipq.rotate(x, r)
        codes = mipq.pq_encode(y, cb, "bf16")
        _, sr = mipq.pq_decode_rmse(codes, cb, y)
        return y, codes, sr

    log("%d warmup + %d timed steps" % (args.warmup, args.steps))
    ms, (y, codes, sr) = timed_steps(step, args.steps, args.warmup)
    rmse_opq = float(sr[1].item())
    log("plain PQ on the same sample for comparison")
    pf = mipq.pq_fit(tr, w.m, w.ks, outer * inner, init_rows=init, precision="bf16", labels=False, objective=False)
    _, sp = mipq.pq_decode_rmse(mipq.pq_encode(x, pf["codebook"], "bf16"), pf["codebook"], x)
    rmse_pq = float(sp[1].item())

    L = _lib.lib()
    drop_profile(L)
    L.mipq_profile_enable(1)
    step()
    torch.cuda.synchronize()
    L.mipq_profile_enable(0)
    kt = kernel_totals(L, ["rotate", "assign_bf16", "pack_bf16", "decode"])
    nl, tot = kt["rotate"]
    flops = 2.0 * n * d * d
    avg = tot / max(nl, 1)
    achieved = flops / (avg * 1e-3) / 1e12

    log("oracle parity on 2000 sampled rows")
    from oracle import opq as opq_oracle
    from oracle import pq
    rows = np.random.default_rng(11).choice(n, 2000, replace=False)
    rn = r.cpu().numpy()
    y_ref = opq_oracle.rotate(w.x[rows], rn)
    y_got = y.cpu().numpy()[rows]
    c_ref, _ = pq.encode(y_got, cb.cpu().numpy().astype(np.float64), decide="fp32")
    parity = {"rotated_rows_bit_identical_pct": 100.0 * float(np.mean(np.all(y_got == y_ref, axis=1))),
              "codes_equal_oracle_pct": 100.0 * float(np.mean(codes.cpu().numpy()[rows].astype(np.int64) == c_ref)),
              "sample_rows": len(rows)}

    base = None
    if not args.no_cpu_baseline:
        k = min(n, 1000000)
        log("oracle leg: rotate + encode of %d rows" % k)
        cbn = cb.cpu().numpy().astype(np.float64)
        threads = max(1, min(CPU_SHARE, os.cpu_count() or 1))
        _, tr_s = oracle_row_chunks(k, threads, lambda a, b: pq.encode(opq_oracle.rotate(w.x[a:b], rn), cbn,
                                                                       decide="fp32"))
        base = {"value": k / tr_s, "unit": "vectors/s", "cores": threads, "host_cpus": os.cpu_count(),
                "cpu_model": cpu_model(), "kind": "oracle",
                "sample": "rotation (float64, t ascending) + encode (float32 decisions) of the first %d rows, rows "
                          "split over %d threads, %.1fs" % (k, threads, tr_s)}
    rec = base_record("Optimized-PQ encode vectors/s (float64 rotation + BF16-MFMA encode + RMSE)", n / (ms * 1e-3),
                      "vectors/s", args.steps, args.warmup, ms, "f64 rotation, bf16 encode",
                      {"workload": "opq: 1M x 128 integer-valued rows; R and codebooks (M=16, Ks=256) fitted once on "
                                   "the 100k-row sample (10 x (2 Lloyd rounds + Procrustes)); step = rotate all rows "
                                   "+ encode + decode/RMSE",
                       "n": n, "d": d, "m": w.m, "ks": w.ks, "outer_iters": outer, "lloyd_rounds_per_outer": inner,
                       "precision": "bf16 encode, float64 rotation", "parallelism": "single GPU"})
    rec.update({
        "opq_fit_ms": fit_ms,
        "procrustes_sweeps": [int(s_.item()) for s_ in fit["sweeps"]],
        "rmse_opq": rmse_opq,
        "rmse_pq_same_rounds": rmse_pq,
        "oracle_parity": parity,
        "roofline": {"bound": "alu", "kernel": "k_rotate", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": achieved / 78.6, "traffic": None, "alg_flops_per_launch": flops, "avg_launch_ms": avg,
                     "launches": nl,
                     "note": "float64 vector peak (FMA counted as 2); the rotation's unfused product and sum cap it "
                             "at half of that"},
        "kernels_ms_per_step": {k2: v[1] for k2, v in kt.items()},
        "cpu_baseline": base,
    })
    return rec


PUBLISHED = {   # per-launch rates the roofline fractions are quoted against
    "add_f32": ("T lane-ops/s", 256 * 4 * 16 * 2.4e9 / 1e12),
    "fma_f32": ("T lane-ops/s", 256 * 4 * 16 * 2.4e9 / 1e12),
    "min3_f32": ("T lane-ops/s", 256 * 4 * 16 * 2.4e9 / 1e12),
    "fma_f64": ("T lane-ops/s", 256 * 4 * 16 * 2.4e9 / 1e12),
    "add_vv": ("T lane-ops/s", 256 * 4 * 16 * 2.4e9 / 1e12),
    "min_vv": ("T lane-ops/s", 256 * 4 * 16 * 2.4e9 / 1e12),
    "min3_add": ("T lane-ops/s", 256 * 4 * 16 * 2.4e9 / 1e12),
    "mfma_bf16": ("TFLOP/s", 2500.0),
    "mfma_f8": ("TFLOP/s", 5000.0),
    "copy": ("GB/s", PEAK_HBM_GBS),
}


def bench_peaks(args) -> dict:
    """What one launch of each instruction kind sustains on this device
    (mipq_peak_probe), beside the unit-count or published figure it checks."""
    import torch

    import paper_2604_21645_amd as mipq

    dev = torch.device("cuda:0")
    blocks = 256 * 8   # 8 blocks of 4 waves per CU: 8 waves per SIMD
    buf = torch.empty(blocks * 256 * 8, dtype=torch.uint8, device=dev)
    big = torch.empty(2 << 30, dtype=torch.uint8, device=dev)   # 1 GiB copied within 2 GiB
    rates = {}
    for kind, (unit, pub) in PUBLISHED.items():
        b, t = (big, 256 * 64) if kind == "copy" else (buf, blocks)
        work = mipq.peak_probe(kind, t, b)   # warm-up
        best = float("inf")
        for _ in range(max(args.steps, 3)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mipq.peak_probe(kind, t, b)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        scale = 1e9 if unit == "GB/s" else 1e12
        got = work / (best * 1e-3) / scale
        rates[kind] = {"measured": got, "unit": unit, "derived_or_published": pub, "frac": got / pub,
                       "ms": best}
        log("%-10s %10.2f %s (%.3f of %.1f)" % (kind, got, unit, got / pub, pub))
    rec = base_record("sustained issue rate of unpacked float32 adds (probe)", rates["add_f32"]["measured"],
                      "T lane-ops/s", max(args.steps, 3), 1, rates["add_f32"]["ms"], "f32",
                      {"workload": "peak probes: 2048 blocks x 256 threads, 8 chains x 2048 instructions "
                                   "per lane; MFMA 4 accumulators x 512 per wave; copy 1 GiB"})
    rec["probes"] = rates
    return rec


WORKLOADS = {"integer_pq": bench_integer_pq, "plain_pq": bench_plain, "batched_uneven": bench_batched,
             "ivf_adc": bench_ivf, "diff_codebooks": bench_diff, "soil_chunks": bench_soil, "opq": bench_opq,
             "peaks": bench_peaks}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="integer_pq", choices=sorted(WORKLOADS))
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--fp8-steps", type=int, default=3)
    ap.add_argument("--build-steps", type=int, default=2, help="ivf_adc: timed index builds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frac", type=float, default=0.4)
    ap.add_argument("--batched-cpu-rows", type=int, default=64000)
    ap.add_argument("--ivf-cpu-queries", type=int, default=500)
    ap.add_argument("--diff-cpu-rows", type=int, default=400000)
    ap.add_argument("--soil-cpu-rows", type=int, default=16750)
    ap.add_argument("--oracle-sample", type=int, default=20000)
    ap.add_argument("--deterministic", action="store_true", help="fixed-order centroid sums in the fit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the PQ hot path runs on a single "
              "MI355X); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2
    import torch
    torch.cuda.set_device(0)
    rec = WORKLOADS[args.workload](args)
    if args.copy_calibration:   # a 1 GiB device copy: reference dispatch for the HBM counters
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

