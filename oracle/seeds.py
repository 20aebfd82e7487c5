"""Read-level seed extension (the step around BSW): CPU reference.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

A seed is an exact match of read[qb:qe] at reference position rb, with the
seed score h0.  The read is extended from the seed on both sides with BSW
(Sec. 5.1): first to the left, on the reversed read prefix read[0:qb]
against the reversed reference before the seed, starting from h0; then to
the right, on the read suffix read[qe:] against the reference after the
seed, starting from the score the left side kept (Sec. 2: seeds are
extended on both sides to cover the read).  Every seed is extended; none is
filtered (Sec. 5.3.2 extends all seeds first; the filter afterwards needs
the chains and is not part of this step).

Readings (the paper describes none of this in detail):

N1  After each extension the caller keeps either the local end (the best
    cell: score, qle, tle) or the end of the read (the global-to-end score
    gscore at target end gtle).  It keeps the read end when gscore > 0 and
    gscore > score - end_bonus, i.e. when reaching the end of the read costs
    less than the end bonus; otherwise the local end.  This is the use of
    the end bonus beyond the band cap (R11).
N2  Reference windows: left ref[max(0, rb - qb - w) : rb] (reversed),
    right ref[re : min(len(ref), re + (len(read) - qe) + w)] with
    re = rb + (qe - qb): the read part plus the band half-width w.
N3  A side with nothing to extend (qb = 0, or qe = len(read)) is skipped:
    the seed boundary is kept on that side and the score carries over.
    (The BSW call is still made, on an empty query, and its result ignored.)

Outputs per seed: score; read interval [qbeg, qend); reference interval
[rbeg, rend); how = left choice | right choice << 2 with 0 = local end,
1 = read end, 2 = nothing to extend.

``filter_seeds`` is the step Sec. 5.3.2 puts after extending every seed:
dropping the seeds the sequential mapper would not have extended, because
an alignment it had already produced from the same chain covers them.

F1  A chain is a run of consecutive seeds with the same read, in the order
    given (the mapper's order within a chain, best seed first).
F2  Walking a chain in that order, a seed is dropped when an earlier seed
    of the chain that was kept has an extension whose read interval
    [qbeg, qend) contains the seed's [qb, qe) and whose reference interval
    [rbeg, rend) contains the seed's [rb, rb + qe - qb); otherwise it is
    kept.  The first seed of a chain is always kept.
"""
from __future__ import annotations

import numpy as np

from . import extend_batch

SEED_DTYPE = np.dtype([("read", "<i4"), ("qb", "<i4"), ("qe", "<i4"), ("h0", "<i4"),
                       ("rb", "<i8")])
SEED_RESULT_DTYPE = np.dtype([("score", "<i4"), ("qbeg", "<i4"), ("qend", "<i4"),
                              ("how", "<i4"), ("rbeg", "<i8"), ("rend", "<i8")])
LOCAL, READ_END, NONE = 0, 1, 2


def _offsets(lengths):
    off = np.zeros(len(lengths) + 1, dtype=np.uint64)
    np.cumsum(np.asarray(lengths, dtype=np.uint64), out=off[1:])
    return off


def _keep(res, bonus):
    """(score, query end, target end, choice) kept after one extension (N1)."""
    score, gscore = int(res["score"]), int(res["gscore"])
    if gscore <= 0 or gscore <= score - bonus:
        return score, int(res["qle"]), int(res["tle"]), LOCAL
    return gscore, None, int(res["gtle"]), READ_END


def extend_seeds(reads, read_off, ref, seeds, scoring, n_threads=0):
    """Extend every seed on both sides; returns SEED_RESULT_DTYPE records."""
    reads = np.asarray(reads, dtype=np.uint8)
    ref = np.asarray(ref, dtype=np.uint8)
    read_off = np.asarray(read_off, dtype=np.int64)
    seeds = np.asarray(seeds, dtype=SEED_DTYPE)
    w = int(scoring["w"])
    bonus = int(scoring["end_bonus"])
    n = len(seeds)
    # left batch: reversed prefixes against the reversed reference before the seed
    lq, lt = [], []
    for s in seeds:
        r0 = read_off[s["read"]]
        qb, rb = int(s["qb"]), int(s["rb"])
        lq.append(reads[r0:r0 + qb][::-1])
        lt.append(ref[max(0, rb - qb - w):rb][::-1])
    left = {"q": np.concatenate(lq) if n else np.zeros(0, np.uint8),
            "q_off": _offsets([len(x) for x in lq]),
            "t": np.concatenate(lt) if n else np.zeros(0, np.uint8),
            "t_off": _offsets([len(x) for x in lt]),
            "h0": seeds["h0"].astype(np.int32)}
    lres, _ = extend_batch(left, [scoring], n_threads=n_threads)
    out = np.zeros(n, dtype=SEED_RESULT_DTYPE)
    h1 = np.zeros(n, dtype=np.int32)
    for k, s in enumerate(seeds):
        qb, rb = int(s["qb"]), int(s["rb"])
        if qb == 0:
            sc, qbeg, rbeg, how = int(s["h0"]), 0, rb, NONE
        else:
            sc, qle, tle, how = _keep(lres[k], bonus)
            qbeg = 0 if how == READ_END else qb - qle
            rbeg = rb - tle
        h1[k] = sc
        out[k]["qbeg"], out[k]["rbeg"], out[k]["how"] = qbeg, rbeg, how
    # right batch: the suffix after the seed against the reference after it
    rq, rt = [], []
    for s in seeds:
        r0, r1 = read_off[s["read"]], read_off[s["read"] + 1]
        qe = int(s["qe"])
        re = int(s["rb"]) + qe - int(s["qb"])
        rest = int(r1 - r0) - qe
        rq.append(reads[r0 + qe:r1])
        rt.append(ref[re:min(len(ref), re + rest + w)])
    right = {"q": np.concatenate(rq) if n else np.zeros(0, np.uint8),
             "q_off": _offsets([len(x) for x in rq]),
             "t": np.concatenate(rt) if n else np.zeros(0, np.uint8),
             "t_off": _offsets([len(x) for x in rt]),
             "h0": h1}
    rres, _ = extend_batch(right, [scoring], n_threads=n_threads)
    for k, s in enumerate(seeds):
        lr = int(read_off[s["read"] + 1] - read_off[s["read"]])
        qe = int(s["qe"])
        re = int(s["rb"]) + qe - int(s["qb"])
        if qe == lr:
            sc, qend, rend, how = int(h1[k]), lr, re, NONE
        else:
            sc, qle, tle, how = _keep(rres[k], bonus)
            qend = lr if how == READ_END else qe + qle
            rend = re + tle
        out[k]["score"], out[k]["qend"], out[k]["rend"] = sc, qend, rend
        out[k]["how"] |= how << 2
    return out


def filter_seeds(seeds, results):
    """Keep flags (uint8, 1 = kept) of the seeds after extension (F1, F2)."""
    seeds = np.asarray(seeds, dtype=SEED_DTYPE)
    results = np.asarray(results, dtype=SEED_RESULT_DTYPE)
    keep = np.zeros(len(seeds), dtype=np.uint8)
    start = 0
    while start < len(seeds):
        end = start
        while end < len(seeds) and seeds[end]["read"] == seeds[start]["read"]:
            end += 1
        kept = []
        for k in range(start, end):
            s = seeds[k]
            qb, qe, rb = int(s["qb"]), int(s["qe"]), int(s["rb"])
            re = rb + qe - qb
            covered = False
            for j in kept:
                r = results[j]
                if (int(r["qbeg"]) <= qb and qe <= int(r["qend"]) and
                        int(r["rbeg"]) <= rb and re <= int(r["rend"])):
                    covered = True
                    break
            if not covered:
                kept.append(k)
                keep[k] = 1
        start = end
    return keep
