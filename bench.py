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
# MI355X spec: 256 CUs x 4 SIMD x 16 lanes = 64 int32 lane-ops per CU per
# clock at the 2.4 GHz peak engine clock; packed 16-bit instructions do two
# operations per lane
SPEC_PEAK_I32_TOPS = 256 * 64 * 2.4e9 / 1e12
SPEC_PEAK_PK16_TOPS = 2 * SPEC_PEAK_I32_TOPS


def pack_of(cls):
    """Operations per lane-instruction that a class's arithmetic can reach:
    2 for 8- and 16-bit values (packed 16-bit instructions), 1 for 32-bit
    values."""
    return 2 if cls.startswith(("lane8", "lane16")) else 1


def host_cpu():
    """(CPU model, logical CPUs this process may use)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return model, nproc


def oracle_threads():
    # every host CPU this process may use, at most the 16 of a one-GPU share
    return max(1, min(16, host_cpu()[1]))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the sources an extension kernel is built from (a profile taken on other
# sources no longer describes it): the register-row kernel's own units, or
# the main kernel file for every other one
LANEV_SOURCES = ["bsw_device.h", "bsw_internal.h", "bsw_lanev.h", "bsw_lanev_impl.h",
                 "bsw_lanev_s.hip", "bsw_lanev_m.hip", "bsw_lanev_l.hip", "bsw_lanev_x.hip"]
KERNEL_SOURCES = ["bsw_kernels.hip", "bsw_device.h", "bsw_internal.h"]


def bsw_sources(kernel):
    return LANEV_SOURCES if "k_lanev" in kernel else KERNEL_SOURCES


def traffic_from_profile(kernel, work, profile="bsw"):
    """HBM bytes per launch of a kernel from the committed counter profile
    (FETCH_SIZE + WRITE_SIZE, calibrated on a plain streaming kernel), if
    the profile was taken on the current kernel source and the same work
    per launch (cells for the extension kernels, algorithmic bytes for the
    suffix-array lookup); else None."""
    import hashlib
    import re
    srcs, work_field = {"bsw": (bsw_sources(kernel), "cells_per_launch"),
                        "sal": (["bsw_sal_kernels.hip"], "alg_bytes_per_launch"),
                        "fm": (["bsw_fm_kernels.hip", "bsw_fm_device.h"],
                               "alg_bytes_per_launch")}[profile]
    h = hashlib.sha256()
    for name in srcs:  # the kernel source and the device code it includes
        h.update(open(os.path.join(ROOT, "paper_1907_12931_amd", "csrc", name), "rb").read())
    digest = h.hexdigest()
    prof_dir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(prof_dir):
        return None
    for name in sorted(os.listdir(prof_dir)):
        if not name.endswith(".md"):
            continue
        text = open(os.path.join(prof_dir, name)).read()
        fields = dict(re.findall(r"^- (\w+): `([^`]*)`", text, flags=re.M))
        if (fields.get("kernel") == kernel.split(" (")[0] and fields.get("source_sha256") == digest
                and fields.get(work_field) == str(work)
                and "traffic_bytes_per_launch" in fields):
            return int(fields["traffic_bytes_per_launch"])
    return None


def pinned(a):
    """A copy of a host array in pinned (page-locked) memory, so that the
    library's host-to-device copies run asynchronously at full rate."""
    import numpy as np
    import torch
    a = np.ascontiguousarray(a)
    buf = torch.empty(a.nbytes, dtype=torch.uint8, pin_memory=True)
    out = buf.numpy().view(a.dtype).reshape(a.shape)
    out[...] = a
    return out


def kernel_symbol(cls, scorings):
    """The kernel template instance that runs a class (as profilers name it)."""
    sym = "true" if all(x["o_del"] == x["o_ins"] and x["e_del"] == x["e_ins"]
                        for x in scorings) else "false"
    if cls == "long":
        return "bsw::k_long"
    if cls == "rerun":
        return "bsw::k_wave"
    mode, rest = cls.split("_q")
    cap = int(rest)
    if mode == "wave32":
        return f"bsw::k_wavev<{max(1, (cap + 63) // 64)}>"
    if mode == "lane32":
        return f"bsw::k_lane<2, {cap}, true>"
    if mode == "lane8":
        return f"bsw::k_lanev<{cap}, {sym}>"
    return f"bsw::k_lanec<{cap}, {sym}, 16>"


def rho_key(r):
    return f"load_{r:.1f}"


def serve(bsw, synth, batch, host, capacity, rho, n_requests, seed=3):
    """Serving run: request sizes log-uniform in [1e3, 1e5] pairs, each a
    contiguous slice of the batch's host arrays (in pinned memory), arriving
    as a Poisson process at rho x capacity (pairs/s); rho = None submits
    them all at once (closed loop: the server's sustained capacity, host
    transfers included).  Latency = submit -> results in the caller's
    buffers."""
    import threading
    import numpy as np
    sizes = synth.serving_requests(n_requests=n_requests, seed=seed)
    rng = np.random.default_rng(seed)
    n = len(batch["h0"])
    starts = rng.integers(0, n - sizes + 1)
    arrivals = (np.cumsum(rng.exponential(sizes / (rho * capacity))) if rho
                else np.zeros(n_requests))
    reqs = [{"q": host["q"], "t": host["t"],
             "q_off": host["q_off"][a:a + m + 1], "t_off": host["t_off"][a:a + m + 1],
             "h0": host["h0"][a:a + m], "scorings": batch["scorings"]}
            for a, m in zip(starts.tolist(), sizes.tolist())]
    tickets = [None] * n_requests
    ready = threading.Semaphore(0)
    with bsw.Server(batch["scorings"]) as srv:
        def waiter():
            for k in range(n_requests):
                ready.acquire()
                srv.wait(tickets[k])
        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for k in range(n_requests):
            delay = arrivals[k] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets[k] = srv.submit(reqs[k])
            ready.release()
        th.join()
        st = srv.stats()
    return {"offered_pairs_per_s": round(rho * capacity) if rho else None,
            "delivered_pairs_per_s": round(st["pairs"] / st["window_s"]) if st["window_s"] else None,
            "requests": n_requests,
            "pairs": st["pairs"], "batches": st["batches"],
            "mean_batch_pairs": round(st["mean_batch_pairs"]),
            "p50_ms": round(st["lat_p50_ms"], 3), "p99_ms": round(st["lat_p99_ms"], 3),
            "p999_ms": round(st["lat_p999_ms"], 3), "max_ms": round(st["lat_max_ms"], 3),
            "admit_wait_mean_ms": round(st["admit_wait_mean_ms"], 3),
            "gcups": round(st["gcups"], 2), "window_s": round(st["window_s"], 3)}


def seed_driver(bsw, synth, torch, np, tune_cache, steps, warmup, tune=True):
    """Read-level seed extension (left, end choice, right) over the seed
    benchmark workload, device-resident, reversed reference supplied."""
    t0 = time.time()
    sw = synth.seed_workload(**synth.SEED_BENCH)
    ns, nr = len(sw["seeds"]), len(sw["read_off"]) - 1
    log(f"generated {nr} reads, {ns} seeds in {time.time() - t0:.1f}s")
    dev = bsw.seeds_to_device(sw["reads"], sw["read_off"], sw["ref"], sw["seeds"],
                              with_ref_rev=True)
    out = torch.empty(ns * bsw.SEED_RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    ctx = bsw.Context(tune_cache=tune_cache)
    tuned = None
    if tune:
        # the seed driver's own launch shape (untimed)
        ms, tuned = ctx.tune_seeds(dev, sw["scoring"], out, reps=3)
        tuned["tune_best_ms"] = round(ms, 3)
        log(f"seed driver tuned: {tuned}")
    keep = torch.empty(max(ns, 1), dtype=torch.uint8, device="cuda")
    for _ in range(max(1, warmup)):
        ctx.extend_seeds_device(dev, sw["scoring"], out)
        ctx.filter_seeds_device(dev["seeds"], out, keep)
    cells = ctx.last_cells()
    torch.cuda.synchronize()
    tms = []
    t = time.perf_counter()
    # a step extends every seed, then drops the ones an earlier alignment of
    # the same chain covers (Sec. 5.3.2)
    for _ in range(steps):
        ctx.extend_seeds_device(dev, sw["scoring"], out)
        tms.append(ctx.last_timing())
        ctx.filter_seeds_device(dev["seeds"], out, keep)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    assert ctx.last_cells() == cells
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ctx.filter_seeds_device(dev["seeds"], out, keep, stream=torch.cuda.current_stream())
    e1.record()
    torch.cuda.synchronize()
    filter_ms = e0.elapsed_time(e1) / 5
    kept = int(keep[:ns].sum().item())
    ctx.close()
    tm = np.mean(np.asarray(tms), axis=0)
    leg = {"value": round(ns / wall, 1), "unit": "seeds/s",
           "reads_per_s": round(nr / wall, 1), "gcups": round(cells / wall / 1e9, 2),
           "ms_per_step": round(wall * 1e3, 3), "device_ms": round(float(tm[0]), 3),
           "left_ms": round(float(tm[1]), 3), "right_ms": round(float(tm[2]), 3),
           "dp_launches": int(tm[3]), "filter_ms": round(filter_ms, 3),
           "kept": kept,
           "workload": f"{nr} reads x {synth.SEED_BENCH.get('read_len', 151)} bp from a "
                       f"{len(sw['ref'])}-base random reference, 1-5% substitutions, "
                       f"0.1-1% indels, 1% N; {ns} seeds (exact runs >= 19 bp, <= 3 per "
                       "read); BWA default scoring; reversed reference supplied",
           "seeds": ns, "reads": nr, "cells": int(cells), "tuned": tuned}
    return leg, sw


def seed_cpu_baseline(np, sw, seconds):
    """The reference seed driver on the host cores, on a random sample of the
    seeds sized for about `seconds` of work."""
    from oracle import seeds as oseeds
    threads = oracle_threads()
    rng = np.random.default_rng(0)
    ns = len(sw["seeds"])

    def run(m):
        idx = np.sort(rng.choice(ns, size=m, replace=False))
        t = time.perf_counter()
        oseeds.extend_seeds(sw["reads"], sw["read_off"], sw["ref"], sw["seeds"][idx],
                            sw["scoring"], n_threads=threads)
        return time.perf_counter() - t

    m0 = min(ns, 20000)
    rate = m0 / run(m0)
    m = int(min(ns, max(m0, rate * seconds)))
    dt = run(m)
    return {"value": round(m / dt, 1), "unit": "seeds/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} random seeds of the {ns}, {dt:.1f} s"}


HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def sa_lookup(bsw, synth, torch, np, steps, warmup):
    """Suffix-array lookup (Eq. 1) of the benchmark intervals against the
    resident suffix array of the benchmark text."""
    t0 = time.time()
    w = synth.sa_workload(**synth.SA_BENCH)
    n = len(w["iv"])
    total = int(w["iv"]["s"].astype(np.int64).sum())
    log(f"built a {len(w['sa'])}-entry suffix array and {n} intervals in "
        f"{time.time() - t0:.1f}s")
    sa = torch.from_numpy(w["sa"]).cuda()
    iv = torch.from_numpy(np.ascontiguousarray(w["iv"]).view(np.uint8)).cuda()
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    pos = torch.empty(total, dtype=torch.int64, device="cuda")
    ctx = bsw.Context()
    for _ in range(max(1, warmup)):
        assert ctx.sa_lookup_device(sa, iv, off, pos) == total
    torch.cuda.synchronize()
    tms = []
    t = time.perf_counter()
    for _ in range(steps):
        ctx.sa_lookup_device(sa, iv, off, pos)
        tms.append(ctx.last_timing())
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    ctx.close()
    tm = np.mean(np.asarray(tms), axis=0)
    # the gather's algorithmic bytes: per coordinate an 8-byte entry of S
    # read and an 8-byte coordinate written; per interval its 8-byte start
    # and 8-byte offset read and the offset written back
    alg = 16 * total + 24 * n
    gbs = alg / (tm[2] / 1e3) / 1e9
    kernel = "bsw::k_sal_gather"
    leg = {"value": round(total / wall, 1), "unit": "SA coordinates/s",
           "ms_per_step": round(wall * 1e3, 3), "device_ms": round(float(tm[0]), 3),
           "check_scan_ms": round(float(tm[1]), 3), "gather_ms": round(float(tm[2]), 3),
           "intervals": n, "coordinates": total, "sa_entries": len(w["sa"]),
           "workload": f"suffix array of a {len(w['text'])}-base text (a "
                       f"{len(w['ref'])}-base reference with repeat families, 12% of it, "
                       "2-300 copies at 0-5% divergence, and its reverse complement); "
                       f"{n} intervals of 19-21-base patterns drawn from the reference",
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "traffic": traffic_from_profile(kernel, alg, profile="sal"),
                        "kernel": kernel, "alg_bytes_per_launch": alg}}
    return leg, w


def fm_search(bsw, synth, torch, np, w, steps, warmup):
    """Bi-interval backward search of the benchmark patterns over the FM
    index of the lookup's two-strand text."""
    t0 = time.time()
    entries, meta = bsw.fm_build(w["text"], w["sa"])
    pat, off = synth.fm_patterns(w["text"], synth.FM_BENCH_PATTERNS, seed=44)
    n = len(off) - 1
    log(f"built the FM index ({len(entries)} entries) and {n} patterns in "
        f"{time.time() - t0:.1f}s")
    E = torch.from_numpy(entries.view(np.uint8)).cuda()
    pd = torch.from_numpy(pat).cuda()
    od = torch.from_numpy(off.astype(np.uint64).view(np.int64)).cuda()
    out = torch.empty(n * bsw.BI_INTERVAL_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    ctx = bsw.Context()
    for _ in range(max(1, warmup)):
        ctx.fm_backward_search_device(E, meta, pd, od, out)
    torch.cuda.synchronize()
    ms = []
    t = time.perf_counter()
    for _ in range(steps):
        ctx.fm_backward_search_device(E, meta, pd, od, out)
        ms.append(ctx.last_timing()[0])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    ctx.close()
    res = out.cpu().numpy().view(bsw.BI_INTERVAL_DTYPE)
    L = np.diff(off.astype(np.int64))
    m = res["matched"].astype(np.int64)
    # extension steps run: every matched base, plus the step whose interval
    # came out empty (a pattern stopped by an N takes no step for it)
    stop = m < L
    nxt = np.where(stop, pat[np.minimum(off[1:].astype(np.int64) - m - 1, len(pat) - 1)], 4)
    steps_run = int(m.sum() + np.count_nonzero(stop & (nxt < 4)))
    kms = float(np.mean(ms))
    alg = 2 * 64 * steps_run  # two 64-byte entries read per step
    gbs = alg / (kms / 1e3) / 1e9
    return {"value": round(n / wall, 1), "unit": "patterns/s",
            "extensions_per_s": round(steps_run / wall, 1), "ms_per_step": round(wall * 1e3, 3),
            "kernel_ms": round(kms, 3), "patterns": n, "extension_steps": steps_run,
            "fully_matched": int(np.count_nonzero(~stop)),
            "index_bytes": int(entries.nbytes),
            "workload": f"{n} patterns of 32 bases from the {len(w['ref'])}-base reference "
                        "(2% substitutions, 0.5% N) against the FM index of it and its "
                        f"reverse complement ({len(w['sa'])} rows, 64-byte entries of 32 rows)",
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": traffic_from_profile("bsw::k_fm_search", alg, profile="fm"),
                         "kernel": "bsw::k_fm_search",
                         "alg_bytes_per_launch": alg}}


def smem_reads(synth, w):
    return synth.fm_patterns(w["text"], synth.SMEM_BENCH_READS, seed=54, length=(151, 151),
                             p_sub=0.02, p_n=0.005)


def smem_search(bsw, synth, torch, np, w, steps, warmup):
    """SMEMs of the benchmark reads over the FM index of the lookup's
    two-strand text."""
    entries, meta = bsw.fm_build(w["text"], w["sa"])
    reads, off = smem_reads(synth, w)
    n = len(off) - 1
    E = torch.from_numpy(entries.view(np.uint8)).cuda()
    rd = torch.from_numpy(reads).cuda()
    od = torch.from_numpy(off.astype(np.uint64).view(np.int64)).cuda()
    out = torch.empty(len(reads) * bsw.SMEM_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx = bsw.Context()
    for _ in range(max(1, warmup)):
        ctx.fm_smem_device(E, meta, rd, od, 151, out, counts)
    torch.cuda.synchronize()
    ms = []
    t = time.perf_counter()
    for _ in range(steps):
        ctx.fm_smem_device(E, meta, rd, od, 151, out, counts)
        ms.append(ctx.last_timing()[0])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    ext = ctx.last_cells()
    ctx.close()
    n_smem = int(counts.sum().item())
    kms = float(np.mean(ms))
    alg = 2 * 64 * ext  # two 64-byte entries read per extension step
    gbs = alg / (kms / 1e3) / 1e9
    return {"value": round(n / wall, 1), "unit": "reads/s",
            "smems_per_s": round(n_smem / wall, 1), "extensions_per_s": round(ext / wall, 1),
            "ms_per_step": round(wall * 1e3, 3), "kernel_ms": round(kms, 3), "reads": n,
            "smems": n_smem, "extension_steps": int(ext),
            "workload": f"{n} reads of 151 bases from the {len(w['ref'])}-base reference "
                        "(2% substitutions, 0.5% N) against the FM index of it and its "
                        f"reverse complement ({len(w['sa'])} rows)",
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": traffic_from_profile("bsw::k_fm_smem", alg, profile="fm"),
                         "kernel": "bsw::k_fm_smem",
                         "alg_bytes_per_launch": alg}}


def smem_cpu_baseline(np, synth, w, seconds):
    """The reference SMEMs on the host, on a random sample of the benchmark
    reads sized for about `seconds` of work."""
    from oracle import fm, sal
    reads, off = smem_reads(synth, w)
    txt = sal.to_text(w["text"]) + "$"
    rng = np.random.default_rng(0)
    n = len(off) - 1

    def run(m):
        idx = rng.choice(n, size=m, replace=False)
        t = time.perf_counter()
        for j in idx:
            fm.smems(w["text"], w["sa"], reads[off[j]:off[j + 1]], txt)
        return time.perf_counter() - t

    dt0 = run(50)
    m = int(min(n, max(50, 50 / dt0 * seconds)))
    dt = run(m)
    return {"value": round(m / dt, 1), "unit": "reads/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} random reads of the {n}, {dt:.1f} s"}


def fm_cpu_baseline(np, synth, w, seconds):
    """The reference backward search on the host, on a random sample of the
    benchmark patterns sized for about `seconds` of work."""
    from oracle import fm, sal
    pat, off = synth.fm_patterns(w["text"], synth.FM_BENCH_PATTERNS, seed=44)
    txt = sal.to_text(w["text"]) + "$"
    rng = np.random.default_rng(0)
    n = len(off) - 1

    def run(m):
        idx = rng.choice(n, size=m, replace=False)
        t = time.perf_counter()
        for j in idx:
            fm.backward_search(w["text"], w["sa"], pat[off[j]:off[j + 1]], txt)
        return time.perf_counter() - t

    dt0 = run(200)
    m = int(min(n, max(200, 200 / dt0 * seconds)))
    dt = run(m)
    return {"value": round(m / dt, 1), "unit": "patterns/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} random patterns of the {n}, {dt:.1f} s"}


def sal_cpu_baseline(np, w, seconds):
    """The reference lookup on the host, on a random sample of intervals
    sized for about `seconds` of work."""
    from oracle import sal
    rng = np.random.default_rng(0)
    n = len(w["iv"])

    def run(m):
        idx = np.sort(rng.choice(n, size=m, replace=False))
        t = time.perf_counter()
        _, out = sal.lookup(w["sa"], w["iv"][idx])
        return len(out), time.perf_counter() - t

    c0, dt0 = run(min(n, 20000))
    m = int(min(n, max(20000, 20000 / dt0 * seconds)))
    c, dt = run(m)
    return {"value": round(c / dt, 1), "unit": "SA coordinates/s", "cores": 1,
            "kind": "oracle", "sample": f"{m} random intervals of the {n}, {c} "
                                        f"coordinates, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=4_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-seeds", action="store_true",
                    help="skip the read-level seed driver leg")
    ap.add_argument("--no-sal", action="store_true",
                    help="skip the suffix-array lookup leg")
    ap.add_argument("--sal-only", action="store_true",
                    help="run only the suffix-array lookup leg and print it as the JSON line")
    ap.add_argument("--fm-only", action="store_true",
                    help="run only the FM-index backward search leg and print it as the "
                         "JSON line")
    ap.add_argument("--smem-only", action="store_true",
                    help="run only the SMEM search leg and print it as the JSON line")
    ap.add_argument("--seeds-only", action="store_true",
                    help="run only the seed driver leg and print it as the JSON line "
                         "(for profiling it alone)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the read-scale and wide-band workloads")
    ap.add_argument("--plain-only", action="store_true",
                    help="run only the plain path of the main workload (no tuner) and "
                         "print its timings (for counter profiles of the DP kernels)")
    ap.add_argument("--workload", default="batched_mix",
                    choices=("batched_mix", "read_scale", "wide_band"),
                    help="with --plain-only: the workload to run (default: the main one)")
    ap.add_argument("--peak-only", action="store_true",
                    help="print the measured integer-VALU peaks and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes (skip the autotuner)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one plain streaming kernel over this many MiB "
                         "(read once, written once): the calibration point for "
                         "hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single "
              "MI355X and has no multi-GPU path (pairs are independent, so a "
              "batch would shard into equal-work ranges, one per GPU, with no "
              "collective).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1907_12931_amd import bsw, synth

    if args.copy_mib:
        x = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.bitwise_not(x, out=y)
        torch.cuda.synchronize()
        del x, y
    workers = oracle_threads()
    if args.smem_only:
        w = synth.sa_workload(**synth.SA_BENCH)
        leg = smem_search(bsw, synth, torch, np, w, args.steps, args.warmup)
        if not args.no_cpu:
            leg["cpu_baseline"] = smem_cpu_baseline(np, synth, w, args.cpu_seconds)
        print(json.dumps(leg), flush=True)
        return
    if args.fm_only:
        w = synth.sa_workload(**synth.SA_BENCH)
        leg = fm_search(bsw, synth, torch, np, w, args.steps, args.warmup)
        if not args.no_cpu:
            leg["cpu_baseline"] = fm_cpu_baseline(np, synth, w, args.cpu_seconds)
        print(json.dumps(leg), flush=True)
        return
    if args.sal_only:
        leg, w = sa_lookup(bsw, synth, torch, np, args.steps, args.warmup)
        if not args.no_cpu:
            leg["cpu_baseline"] = sal_cpu_baseline(np, w, args.cpu_seconds)
        print(json.dumps(leg), flush=True)
        return
    if args.seeds_only:
        import tempfile
        tc = os.path.join(tempfile.mkdtemp(prefix="bsw_tune_"), "tune.json")
        leg, sw = seed_driver(bsw, synth, torch, np, tc, args.steps, args.warmup,
                              tune=not args.no_tune)
        if not args.no_cpu:
            leg["cpu_baseline"] = seed_cpu_baseline(np, sw, args.cpu_seconds)
        print(json.dumps(leg), flush=True)
        return
    if args.peak_only:
        print(json.dumps(valu_peaks(bsw)), flush=True)
        return
    t0 = time.time()
    batch = synth.batched_mix(n=args.pairs, workers=workers)
    n = len(batch["h0"])
    log(f"generated {n} pairs in {time.time() - t0:.1f}s")
    import tempfile
    tune_cache = os.path.join(tempfile.mkdtemp(prefix="bsw_tune_"), "tune.json")
    if args.plain_only:
        # one path alone (for counter profiles of the DP kernels)
        if args.workload != "batched_mix":
            batch = {"read_scale": synth.read_scale,
                     "wide_band": synth.wide_band}[args.workload](workers=workers)
        leg = bsw_paths(bsw, torch, np, batch, args.steps, args.warmup, tune_cache,
                        tune=False, batched=False,
                        min_lane_bits=32 if args.workload == "wide_band" else 0)
        print(json.dumps(strip(leg["plain"])), flush=True)
        return
    peaks = valu_peaks(bsw)
    log(f"valu peaks: {peaks}")
    main_leg = bsw_paths(bsw, torch, np, batch, args.steps, args.warmup, tune_cache,
                         tune=not args.no_tune)
    b, p = main_leg["batched"], main_leg["plain"]
    cells = b["cells"]
    gcups = cells / (b["ms_per_step"] / 1e3) / 1e9
    plain = {"value": round(p["cells"] / (p["ms_per_step"] / 1e3) / 1e9, 2),
             "unit": "GCUPS", "ms_per_step": round(p["ms_per_step"], 3),
             "dp_ms": round(p["dp_ms"], 3), "dp_launches": p["dp_launches"]}
    roofline = bsw_roofline(main_leg, peaks, batch["scorings"])
    roofline["traffic"] = traffic_from_profile(roofline["kernel"], roofline["kernel_cells"])

    # the other pair workloads at full size: read-scale reads (1,000,000
    # pairs) and the wide-band stress batch (500,000 pairs, 32-bit values)
    legs = {}
    if not args.no_legs:
        for name, gen, mb in (("read_scale", synth.read_scale, 0),
                              ("wide_band", synth.wide_band, 32)):
            t0 = time.time()
            wb = gen(workers=workers)
            log(f"generated {name}: {len(wb['h0'])} pairs in {time.time() - t0:.1f}s")
            lg = bsw_paths(bsw, torch, np, wb, args.steps, args.warmup, tune_cache,
                           tune=not args.no_tune, min_lane_bits=mb)
            legs[name] = (wb, lg)

    serving = None
    if not args.no_serve:
        resident = n / (b["ms_per_step"] / 1e3)  # pairs/s of the batched path
        # request data in pinned host memory, as a serving front end keeps it
        host = {k: pinned(batch[k]) for k in ("q", "t", "q_off", "t_off", "h0")}
        # the server's own sustained rate (uploads and result copies
        # included): every request submitted at once
        closed = serve(bsw, synth, batch, host, resident, None, args.serve_requests)
        capacity = closed["delivered_pairs_per_s"]
        serving = {"resident_pairs_per_s": round(resident), "capacity": closed}
        serving.update({rho_key(r): serve(bsw, synth, batch, host, capacity, r,
                                          args.serve_requests)
                        for r in (0.5, 0.8)})
        # beside them, the same loads relative to the resident-data rate
        serving.update({"resident_" + rho_key(r): serve(bsw, synth, batch, host, resident, r,
                                                        args.serve_requests)
                        for r in (0.5, 0.8)})
        log(f"serving: {serving}")

    sal_leg = sal_w = None
    if not args.no_sal:
        sal_leg, sal_w = sa_lookup(bsw, synth, torch, np, args.steps, args.warmup)
        log(f"sa lookup: {sal_leg}")
        fm_leg = fm_search(bsw, synth, torch, np, sal_w, args.steps, args.warmup)
        log(f"fm search: {fm_leg}")
        smem_leg = smem_search(bsw, synth, torch, np, sal_w, args.steps, args.warmup)
        log(f"smem search: {smem_leg}")
    else:
        fm_leg = smem_leg = None

    seeds_leg = None
    if not args.no_seeds:
        seeds_leg, sw = seed_driver(bsw, synth, torch, np, tune_cache, args.steps,
                                    args.warmup, tune=not args.no_tune)
        log(f"seed driver: {seeds_leg}")

    # the oracle on the host: timed on a sample of the batch, and its
    # results compared with both GPU paths' results on every pair it ran
    cpu = parity = None
    if not args.no_cpu:
        cpu, parity = cpu_leg(np, synth, batch, main_leg, args.cpu_seconds)
        log(f"cpu: {cpu}; parity: {parity}")
    extra = {}
    for name, (wb, lg) in legs.items():
        extra[name] = leg_summary(lg, peaks, wb)
        if not args.no_cpu:
            c, par = cpu_leg(np, synth, wb, lg, args.cpu_seconds / 3, per_core=False)
            extra[name]["cpu_baseline"] = c
            extra[name]["parity"] = par
        log(f"{name}: {extra[name]}")
    if not args.no_cpu:
        if seeds_leg is not None:
            seeds_leg["cpu_baseline"] = seed_cpu_baseline(np, sw, args.cpu_seconds)
            log(f"cpu seeds: {seeds_leg['cpu_baseline']}")
        if sal_leg is not None:
            sal_leg["cpu_baseline"] = sal_cpu_baseline(np, sal_w, args.cpu_seconds)
            log(f"cpu sa lookup: {sal_leg['cpu_baseline']}")
            fm_leg["cpu_baseline"] = fm_cpu_baseline(np, synth, sal_w, args.cpu_seconds)
            log(f"cpu fm search: {fm_leg['cpu_baseline']}")
            smem_leg["cpu_baseline"] = smem_cpu_baseline(np, synth, sal_w, args.cpu_seconds)
            log(f"cpu smem search: {smem_leg['cpu_baseline']}")

    bad = [k for k, v in [("batched_mix", parity)] +
           [(k, v.get("parity")) for k, v in extra.items()] if v and v["mismatches"]]
    res = {
        "metric": "GCUPS (bit-exact vs oracle) batched vs plain; p50/p99 latency under serving",
        "value": None if bad else round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(b["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i16x2",
        "data": "synthetic",
        "config": {"workload": f"batched_mix: {n} pairs, qlen 1-250 from "
                               "100/150/250 bp sources, tlen <= qlen+200, 20% z-drop, "
                               "match 1 mismatch -4 gap 6+k w 100 zdrop 100 bonus 5",
                   "pairs": n, "cells": cells, "path": "batched",
                   "arithmetic": "8-bit H/E records, packed 16-bit integer cell updates; "
                                 "32-bit values for pairs whose score exceeds 8 bits",
                   "dp_launches": b["dp_launches"], "graph": True, "tuned": main_leg["tuned"],
                   "prep_bin_ms": round(p["prep_ms"], 3),
                   "parity_checked_pairs": parity["checked_pairs"] if parity else 0},
        "plain": plain, "parity": parity, "workloads": extra, "valu_peak": peaks,
        "serving": serving, "seed_driver": seeds_leg, "sa_lookup": sal_leg,
        "fm_search": fm_leg, "smem_search": smem_leg,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    if bad:
        log(f"PARITY FAILURE on {bad}: no value reported")
        sys.exit(1)


def valu_peaks(bsw):
    """Measured integer-VALU rates (TOP/s) of the device beside the spec:
    i32 = the better of v_add_u32 and v_max3_i32 lane-instructions/s, pk16 =
    the better of v_pk_add_u16 and v_pk_max_i16, two operations each."""
    r = {k: round(bsw.valu_peak(k)[1] / 1e12, 3) for k in bsw.PEAK_KINDS}
    return {"i32_tops": max(r["v_add_u32"], r["v_max3_i32"]),
            "pk16_tops": max(r["v_pk_add_u16"], r["v_pk_max_i16"]),
            "kinds_tops": r, "spec_i32_tops": round(SPEC_PEAK_I32_TOPS, 3),
            "spec_pk16_tops": round(SPEC_PEAK_PK16_TOPS, 3)}


def peak_for(cls, peaks):
    return peaks["pk16_tops"] if pack_of(cls) == 2 else peaks["i32_tops"]


def bsw_paths(bsw, torch, np, batch, steps, warmup, tune_cache, tune=True, batched=True,
              min_lane_bits=0):
    """Run a resident batch on the batched path (graph replays, tuned shape)
    and on the plain path, each into its own output buffers.  Returns the
    timings, per-launch cells and work, and both paths' results on the
    host."""
    n = len(batch["h0"])
    dev = bsw.to_device(batch)
    torch.cuda.synchronize()
    tuned = {}

    def run_path(path, graph=True):
        out, diag = bsw.alloc_outputs(n, with_diag=True)
        ctx = bsw.Context(path=path, graph=graph, min_lane_bits=min_lane_bits,
                          tune_cache=tune_cache if path == bsw.PATH_BATCHED else None)
        if path == bsw.PATH_BATCHED and tune:
            # launch shapes from the autotuner, on this batch (untimed)
            ms, shape = ctx.tune(dev, batch["scorings"], out, reps=3)
            tuned.update(shape, tune_best_ms=round(ms, 3))
            log(f"tuned: {tuned}")
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
            # a name can have several launches in a call (the reruns that
            # follow each lane class): summed per call
            step = {}
            for (name, kc, kms), kw in zip(ctx.last_kernels(), ctx.last_work()):
                c0, m0, w0 = step.get(name, (0, 0.0, 0))
                step[name] = (c0 + kc, m0 + kms, w0 + kw)
            for name, v in step.items():
                per_kernel.setdefault(name, []).append(v)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps
        ctx.close()
        kernels = {name: {"cells": int(np.mean([v[0] for v in vals])),
                          "ms": float(np.mean([v[1] for v in vals])),
                          "work": int(np.mean([v[2] for v in vals]))}
                   for name, vals in per_kernel.items()}
        res, dg = bsw.outputs_to_numpy(out, diag)
        del out, diag
        return {"cells": cells, "ms_per_step": wall * 1e3,
                "dp_ms": float(np.mean(dp_ms)), "prep_ms": float(np.mean(prep_ms)),
                "dp_launches": launches, "kernels": kernels, "res": res, "diag": dg}

    leg = {"tuned": tuned}
    if batched:
        leg["batched"] = run_path(bsw.PATH_BATCHED)
        log(f"batched (graph): {strip(leg['batched'])}")
    leg["plain"] = run_path(bsw.PATH_PLAIN)
    log(f"plain: {strip(leg['plain'])}")
    if batched:
        assert leg["plain"]["cells"] == leg["batched"]["cells"]
    del dev
    return leg


def strip(run):
    return {k: v for k, v in run.items() if k not in ("res", "diag")}


def bsw_roofline(leg, peaks, scorings):
    """Roofline of the dominant DP kernel (the plain-path launch with the
    largest device time: there each kernel runs alone on one stream, timed
    by HIP events on that stream) and of the whole batched step.  Work is
    OPS_PER_CELL operations per settled cell; the peak is the measured rate
    of the kernel's arithmetic (packed 16-bit for 8/16-bit values)."""
    b, p = leg["batched"], leg["plain"]
    dom, dk = max(p["kernels"].items(), key=lambda kv: kv[1]["ms"])
    achieved = dk["cells"] * OPS_PER_CELL / (dk["ms"] / 1e3) / 1e12
    peak = peak_for(dom, peaks)
    # the batched step against the cell-weighted peak of its classes
    roof_s = sum(v["cells"] * OPS_PER_CELL / (peak_for(k, peaks) * 1e12)
                 for k, v in b["kernels"].items())
    step = b["cells"] * OPS_PER_CELL / (b["ms_per_step"] / 1e3) / 1e12
    step_peak = b["cells"] * OPS_PER_CELL / roof_s / 1e12 if roof_s else 0.0
    useful = {k: round(v["cells"] / v["work"], 4) for k, v in p["kernels"].items()
              if v["cells"] and v["work"]}
    work = sum(v["work"] for v in p["kernels"].values() if v["work"])
    counted = sum(v["cells"] for v in p["kernels"].values() if v["work"])
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "TOP/s", "frac": round(achieved / peak, 4), "traffic": None,
            "peak_kind": "measured, packed 16-bit" if pack_of(dom) == 2 else "measured, int32",
            "peak_spec": round(SPEC_PEAK_PK16_TOPS if pack_of(dom) == 2 else
                               SPEC_PEAK_I32_TOPS, 3),
            "frac_spec": round(achieved / (SPEC_PEAK_PK16_TOPS if pack_of(dom) == 2 else
                                           SPEC_PEAK_I32_TOPS), 4),
            "kernel": f"{kernel_symbol(dom, scorings)} (class {dom})",
            "kernel_ms": round(dk["ms"], 3),
            "kernel_cells": dk["cells"], "ops_per_cell": OPS_PER_CELL,
            "timed_on": "plain path (each DP kernel alone on one stream)",
            "batched_step_achieved": round(step, 3),
            "batched_step_peak": round(step_peak, 3),
            "batched_step_frac": round(step / step_peak, 4) if step_peak else None,
            "oracle_cells_per_gpu_work": round(counted / work, 4) if work else None,
            "per_kernel_ms": {k: round(v["ms"], 3) for k, v in p["kernels"].items()
                              if v["cells"]},
            "per_kernel_gcups": {k: round(v["cells"] / v["ms"] / 1e6, 1)
                                 for k, v in p["kernels"].items() if v["cells"]},
            "per_kernel_useful": useful}


def leg_summary(leg, peaks, batch):
    b, p = leg["batched"], leg["plain"]
    n = len(batch["h0"])
    r = bsw_roofline(leg, peaks, batch["scorings"])
    return {"value": round(b["cells"] / (b["ms_per_step"] / 1e3) / 1e9, 2), "unit": "GCUPS",
            "pairs": n, "cells": b["cells"], "ms_per_step": round(b["ms_per_step"], 3),
            "plain": round(p["cells"] / (p["ms_per_step"] / 1e3) / 1e9, 2),
            "plain_ms_per_step": round(p["ms_per_step"], 3), "tuned": leg["tuned"],
            "roofline": {k: r[k] for k in ("achieved", "peak", "frac", "kernel", "kernel_ms",
                                           "batched_step_frac", "per_kernel_gcups",
                                           "per_kernel_useful",
                                           "oracle_cells_per_gpu_work")}}


def cpu_leg(np, synth, batch, leg, seconds, per_core=True):
    """The oracle on the host cores: a sample of the batch sized for about
    `seconds` of work (every pair when that fits), three timed runs, the
    median reported; then the GPU results of both paths are compared with
    the oracle's on every sampled pair, all six fields and the diagnostics.
    With per_core, a single-thread run on a length-stratified 1% subsample
    gives the per-core rate."""
    import oracle
    model, nproc = host_cpu()
    threads = oracle_threads()
    n = len(batch["h0"])
    rng = np.random.default_rng(0)
    probe = synth.subset(batch, rng.choice(n, size=min(n, 20000), replace=False))
    t = time.perf_counter()
    oracle.extend_batch(probe, batch["scorings"], n_threads=threads)  # also the warm-up
    rate = len(probe["h0"]) / (time.perf_counter() - t)
    m = int(min(n, max(20000, rate * seconds / 3)))
    idx = np.sort(rng.choice(n, size=m, replace=False)) if m < n else np.arange(n)
    sample = synth.subset(batch, idx)
    times, want = [], None
    for _ in range(3):
        t = time.perf_counter()
        r = oracle.extend_batch(sample, batch["scorings"], n_threads=threads)
        times.append(time.perf_counter() - t)
        if want is None:
            want = r
    dt = float(np.median(times))
    wcells = int(want[1]["cells"].sum())
    cpu = {"value": round(wcells / dt / 1e9, 3), "unit": "GCUPS", "cores": threads,
           "kind": "oracle", "cpu_model": model, "nproc": nproc,
           "sample": f"{m} {'random ' if m < n else ''}pairs of the {n}-pair batch, "
                     f"{wcells} cells, median of 3 runs {dt:.2f} s"}
    if per_core:
        # 1% of the pairs, stratified by query length (every 100th pair in
        # query-length order), on one thread
        ql = np.diff(batch["q_off"].astype(np.int64))
        sub = np.sort(np.argsort(ql, kind="stable")[::100])
        s1 = synth.subset(batch, sub)
        t = time.perf_counter()
        _, d1 = oracle.extend_batch(s1, batch["scorings"], n_threads=1)
        t1 = time.perf_counter() - t
        cpu["per_core_gcups"] = round(int(d1["cells"].sum()) / t1 / 1e9, 3)
        cpu["per_core_sample"] = (f"{len(sub)} pairs (every 100th by query length), "
                                  f"{int(d1['cells'].sum())} cells, 1 thread, {t1:.2f} s")
    mism = 0
    for path in ("batched", "plain"):
        got, gd = leg[path]["res"][idx], leg[path]["diag"][idx]
        for f in want[0].dtype.names:
            mism += int(np.count_nonzero(got[f] != want[0][f]))
        for f in want[1].dtype.names:
            mism += int(np.count_nonzero(gd[f] != want[1][f]))
    parity = {"checked_pairs": m, "paths": ["batched", "plain"],
              "fields": list(want[0].dtype.names) + list(want[1].dtype.names),
              "mismatches": mism}
    return cpu, parity


if __name__ == "__main__":
    main()
