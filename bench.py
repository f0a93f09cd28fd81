#!/usr/bin/env python3
"""PQ fit+encode throughput on one MI355X.

Workload (integer_pq): N = 1,000,000 rows, D = 128, non-negative integer
values in [0, 255] (clipped Gaussian mixture of 1,000 components, sigma 20),
codebooks fitted on a seeded 100,000-row sample with M = 16 subspaces,
Ks = 256 centroids, 25 Lloyd rounds, then all 1M rows encoded, decoded and
the reconstruction RMSE computed.  One step = fit + encode + decode/RMSE,
inputs resident in HBM.  The headline precision is BF16 on matrix cores; the
plain FP32 path runs the same step for comparison (identical codes).

Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_assign_bf16_integer_pq_1M_traffic.json")
MFMA_SOURCE = os.path.join(ROOT, "paper_2604_21645_amd", "csrc", "pq_mfma.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(MFMA_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(per_launch_alg_bytes: float):
    """HBM bytes per launch of the assignment kernel from committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counters, or None if absent or stale."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(w, frac: float):
    """The oracle, as it stands, on a bounded sample of the same workload:
    fit on frac * n_train training rows (same rounds), encode frac * N rows."""
    import numpy as np

    from oracle import pq
    from synth import workloads as wl

    n_tr = max(w.ks, int(round(frac * len(w.train_rows))))
    n_en = int(round(frac * w.x.shape[0]))
    train = w.x[w.train_rows[:n_tr]]
    init = wl.init_rows_per_subspace(w.meta["seed"], n_tr, w.m, w.ks, key=7)
    t0 = time.perf_counter()
    fit = pq.lloyd(train, init, w.m, w.iters, decide="fp32")
    t1 = time.perf_counter()
    pq.encode(w.x[:n_en], fit["codebook"], decide="fp32")
    t2 = time.perf_counter()
    return {
        "value": n_en / (t2 - t0),
        "unit": "vectors/s",
        "cores": 1,
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": "fit on %d training rows x %d rounds, encode %d rows (%.0f%% of the workload); "
                  "float32 decisions, numpy single thread; fit %.1fs, encode %.1fs"
                  % (n_tr, w.iters, n_en, 100 * frac, t1 - t0, t2 - t1),
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frac", type=float, default=0.02)
    ap.add_argument("--oracle-sample", type=int, default=20000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the PQ hot path runs on a single "
              "MI355X); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2

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
                          precision=prec, labels=False, objective=False)
        if ev:
            ev[1].record()
        codes = mipq.pq_encode(x, fit["codebook"], prec)
        if ev:
            ev[2].record()
        _, sr = mipq.pq_decode_rmse(codes, fit["codebook"], x)
        return fit["codebook"], codes, sr

    def timed(prec, steps, warmup, profile):
        for i in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        L = _lib.lib()
        if profile:
            L.mipq_profile_enable(1)
            for k in _lib.KERNELS.values():   # drop anything recorded before
                L.mipq_profile_collect(k, None, None)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = None
        for i in range(steps):
            evs[i][0].record()
            out = step(prec, evs[i])
            evs[i][3].record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps * 1e3
        if profile:
            L.mipq_profile_enable(0)
        ph = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])]
                       for e in evs]).mean(0)
        return wall, ph, out

    log("bf16: %d warmup + %d timed steps" % (args.warmup, args.steps))
    ms, ph, (cb, codes, sr) = timed("bf16", args.steps, args.warmup, profile=True)
    L = _lib.lib()
    import ctypes
    nl, tot = ctypes.c_int64(0), ctypes.c_double(0)
    L.mipq_profile_collect(_lib.KERNELS["assign_bf16"], ctypes.byref(nl), ctypes.byref(tot))
    kernel_stats = {}
    for name, kid in _lib.KERNELS.items():
        if name == "assign_bf16":
            kernel_stats[name] = (nl.value, tot.value)
            continue
        a, b = ctypes.c_int64(0), ctypes.c_double(0)
        L.mipq_profile_collect(kid, ctypes.byref(a), ctypes.byref(b))
        if a.value:
            kernel_stats[name] = (a.value, b.value)
    launches_per_step = w.iters + 1
    rows_per_step = w.iters * n_train + n
    alg_bytes_per_launch = rows_per_step * (4 * d + w.m) / launches_per_step
    avg_launch_ms = tot.value / max(nl.value, 1)
    achieved = alg_bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
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

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    base, parity = None, {}
    if not args.no_cpu_baseline:
        log("oracle leg: parity on %d sampled rows" % args.oracle_sample)
        parity = oracle_parity(w, codes.cpu().numpy(), cb.cpu().numpy(), rmse, args.oracle_sample)
        log("oracle leg: cpu baseline on a %.0f%% sample" % (100 * args.cpu_frac))
        base = cpu_baseline(w, args.cpu_frac)

    traffic = measured_traffic(alg_bytes_per_launch)
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
                               "M=16, Ks=256, 25 Lloyd rounds, encode 1M, decode+RMSE",
                   "n": n, "d": d, "m": w.m, "ks": w.ks, "iters": w.iters, "n_train": n_train,
                   "precision": "bf16", "parallelism": "single GPU"},
        "phases_ms": {"fit": ph[0], "encode": ph[1], "decode_rmse": ph[2]},
        "fit_encode_vectors_per_s": n / ((ph[0] + ph[1]) * 1e-3),
        "fp32_plain": fp32,
        "rmse": rmse,
        "oracle_parity": parity or None,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_assign_bf16",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes_per_launch,
            "avg_launch_ms": avg_launch_ms,
            "launches": nl.value,
        },
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kernel_stats.items()},
        "cpu_baseline": base,
    }
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
