"""Benchmark: banded seed extension (BSW) throughput on one MI355X.

One step = one pass of the whole hot path (validate, bin, DP, results in
caller order) over one batch already resident in HBM: the uneven
4,000,000-pair mix from 100/150/250 bp read sources (query 1-250, target up
to query + 200, 20% of pairs ending by z-drop), default BWA-MEM scoring.

GCUPS = algorithmic band cells / second, where the cells are the ones the
method visits up to each pair's stopping row (the oracle's count; the GPU
reports the same count per pair and the parity tests check it equals the
oracle's).  The batched path (persistent longest-first tile queues) is the
headline value; the plain path (one ordinary launch per bin) is reported
beside it.  The CPU oracle is timed on a bounded sample of the same batch.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K]
[--warmup W] [--pairs N] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# int32 VALU operations per band cell (the recurrence with a staged score
# row): add d+S, gate (compare + select), max3 for H, two subtracts + max3
# for E, two subtracts + max3 for F, shift-or + max for the row maximum and
# its column.
OPS_PER_CELL = 12
# MI355X: 256 CUs x 4 SIMD x 16 lanes = 64 int32 lane-ops per CU per clock,
# 2.4 GHz peak engine clock
PEAK_INT_TOPS = 256 * 64 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=4_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single "
              "MI355X and has no multi-GPU path (pairs are independent; see "
              "DESIGN.md for how batches would shard).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1907_12931_amd import bsw, synth

    workers = min(16, os.cpu_count() or 1)
    t0 = time.time()
    batch = synth.batched_mix(n=args.pairs, workers=workers)
    n = len(batch["h0"])
    log(f"generated {n} pairs in {time.time() - t0:.1f}s")
    dev = bsw.to_device(batch)
    out, diag = bsw.alloc_outputs(n, with_diag=True)
    torch.cuda.synchronize()

    def run_path(path, steps, warmup):
        ctx = bsw.Context(path=path)
        ctx.extend_device(dev, batch["scorings"], out, diag)  # cells + warm
        cells = int(diag.view(torch.int64).view(n, 2)[:, 1].sum().item())
        for _ in range(warmup):
            ctx.extend_device(dev, batch["scorings"], out)
        torch.cuda.synchronize()
        dp_ms, prep_ms, launches = [], [], 0
        per_kernel = {}
        t = time.perf_counter()
        for _ in range(steps):
            ctx.extend_device(dev, batch["scorings"], out)
            tm = ctx.last_timing()
            dp_ms.append(tm[2])
            prep_ms.append(tm[1])
            launches = int(tm[3])
            for name, kc, kms in ctx.last_kernels():
                per_kernel.setdefault(name, []).append((kc, kms))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps
        ctx.close()
        kernels = {name: {"cells": int(np.mean([v[0] for v in vals])),
                          "ms": float(np.mean([v[1] for v in vals]))}
                   for name, vals in per_kernel.items()}
        return {"cells": cells, "ms_per_step": wall * 1e3,
                "dp_ms": float(np.mean(dp_ms)), "prep_ms": float(np.mean(prep_ms)),
                "dp_launches": launches, "kernels": kernels}

    b = run_path(bsw.PATH_BATCHED, args.steps, args.warmup)
    cells = b["cells"]
    gcups = cells / (b["ms_per_step"] / 1e3) / 1e9
    log(f"batched: {b}")
    plain = None
    if not args.no_plain:
        p = run_path(bsw.PATH_PLAIN, args.steps, args.warmup)
        log(f"plain: {p}")
        plain = {"value": round(p["cells"] / (p["ms_per_step"] / 1e3) / 1e9, 2),
                 "unit": "GCUPS", "ms_per_step": round(p["ms_per_step"], 3),
                 "dp_ms": round(p["dp_ms"], 3), "dp_launches": p["dp_launches"]}

    # dominant kernel: the DP launch with the largest device time; its
    # algorithmic work is its settled cells x OPS_PER_CELL int32 operations
    dom, dk = max(b["kernels"].items(), key=lambda kv: kv[1]["ms"])
    achieved = dk["cells"] * OPS_PER_CELL / (dk["ms"] / 1e3) / 1e12
    all_dp = cells * OPS_PER_CELL / (b["dp_ms"] / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": round(PEAK_INT_TOPS, 3), "unit": "TOP/s",
                "frac": round(achieved / PEAK_INT_TOPS, 4), "traffic": None,
                "kernel": f"k_lane8 class {dom}", "kernel_ms": round(dk["ms"], 3),
                "kernel_cells": dk["cells"], "ops_per_cell": OPS_PER_CELL,
                "all_dp_achieved": round(all_dp, 3),
                "all_dp_frac": round(all_dp / PEAK_INT_TOPS, 4),
                "per_kernel_ms": {k: round(v["ms"], 3) for k, v in b["kernels"].items()}}

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        rng = np.random.default_rng(0)
        # calibrate on a small sample, then time a sample sized for about
        # --cpu-seconds of work
        probe = synth.subset(batch, rng.choice(n, size=min(n, 20000), replace=False))
        t = time.perf_counter()
        _, pd = oracle.extend_batch(probe, batch["scorings"], n_threads=threads)
        rate = len(probe["h0"]) / (time.perf_counter() - t)
        m = int(min(n, max(20000, rate * args.cpu_seconds)))
        idx = rng.choice(n, size=m, replace=False)
        sample = synth.subset(batch, idx)
        t = time.perf_counter()
        _, sd = oracle.extend_batch(sample, batch["scorings"], n_threads=threads)
        dt = time.perf_counter() - t
        cpu = {"value": round(int(sd["cells"].sum()) / dt / 1e9, 3), "unit": "GCUPS",
               "cores": threads, "kind": "oracle",
               "sample": f"{m} random pairs of the {n}-pair batch, "
                         f"{int(sd['cells'].sum())} cells, {dt:.1f} s"}
        log(f"cpu: {cpu}")

    res = {
        "metric": "GCUPS (bit-exact vs oracle) batched vs plain; p50/p99 latency under serving",
        "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(b["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": f"batched_mix: {n} pairs, qlen 1-250 from "
                               "100/150/250 bp sources, tlen <= qlen+200, 20% z-drop, "
                               "match 1 mismatch -4 gap 6+k w 100 zdrop 100 bonus 5",
                   "pairs": n, "cells": cells, "path": "batched",
                   "dp_launches": b["dp_launches"], "prep_bin_ms": round(b["prep_ms"], 3)},
        "plain": plain, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
