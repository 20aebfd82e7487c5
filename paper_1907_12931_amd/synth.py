"""Seeded synthetic workloads for banded seed extension.

This module only draws inputs: sequences, seed scores and scoring sets.  It
holds none of the extension's arithmetic and serves the GPU library and the
oracle alike.  The paper's read sets and the pairs it intercepted from
BWA-MEM (Sec. 6.1.2, Table 3; Table 6) are not available, so every workload
is a stand-in with read-shaped statistics:

* a query is the part of a read left of or right of a seed, drawn as
  uniform random ACGT (codes 0..3);
* its target is the query passed through a mutation walk (substitutions,
  and insertions or deletions of geometric length) and followed by random
  reference flank, since the target window reaches past the read end;
* ambiguous bases N (code 4) are sprinkled in where a workload asks for it;
* the seed score h0 is uniform in [19, 50] (a seed of 19-50 matching bases
  at match score 1);
* the RNG is NumPy's PCG64 seeded with the workload index.

A batch is a dict of NumPy arrays: ``q`` (u8 codes), ``q_off`` (u64, n+1),
``t`` (u8), ``t_off`` (u64, n+1), ``h0`` (i32), ``param_id`` (u8, or
absent for a single scoring set) and ``scorings`` (list of dicts).
"""
from __future__ import annotations

import math

import numpy as np


def scoring(match=1, mismatch=-4, n_score=-1, o=6, e=1, w=100, zdrop=100,
            end_bonus=5, o_ins=None, e_ins=None):
    """A scoring set in the library's layout: mat[target][query]."""
    mat = np.full((5, 5), mismatch, dtype=np.int64)
    np.fill_diagonal(mat, match)
    mat[4, :] = n_score
    mat[:, 4] = n_score
    return {"mat": mat.tolist(), "o_del": o, "e_del": e,
            "o_ins": o if o_ins is None else o_ins,
            "e_ins": e if e_ins is None else e_ins,
            "w": w, "zdrop": zdrop, "end_bonus": end_bonus}


BWA_DEFAULT = scoring()  # match 1, mismatch -4, N -1, gap 6+k*1, w 100, z 100, bonus 5
WIDE_A = scoring(1, -4, -1, 6, 1, w=500, zdrop=400, end_bonus=5)
WIDE_B = scoring(2, -3, -1, 5, 2, w=500, zdrop=400, end_bonus=5)


# ---------------------------------------------------------------------------
# vectorised building blocks (all on flat concatenated arrays)

def _offsets(lengths):
    off = np.zeros(len(lengths) + 1, dtype=np.uint64)
    np.cumsum(lengths, out=off[1:])
    return off


def _pair_index(lengths):
    return np.repeat(np.arange(len(lengths), dtype=np.int64), lengths)


def _random_bases(rng, n):
    return rng.integers(0, 4, size=n, dtype=np.uint8)


def _mutate(rng, seq, lengths, p_sub, p_indel, mean_len):
    """Mutation walk over every pair's sequence at once.

    Per position: with probability p_sub (per pair) the base becomes a
    different base chosen uniformly; independently, with probability
    p_indel an indel starts there: a deletion of the next k bases or an
    insertion of k random bases after it (1/2 each), k ~ Geometric(1/mean).
    Returns (mutated flat array, new lengths)."""
    n = len(seq)
    pid = _pair_index(lengths)
    out = seq.copy()
    sub = rng.random(n) < p_sub[pid]
    out[sub] = (out[sub] + rng.integers(1, 4, size=int(sub.sum()),
                                        dtype=np.uint8)) % 4
    ev = np.nonzero(rng.random(n) < p_indel[pid])[0]
    ins = np.zeros(n, dtype=np.int64)
    keep = np.ones(n, dtype=bool)
    if len(ev):
        k = rng.geometric(1.0 / mean_len, size=len(ev)).astype(np.int64)
        is_del = rng.random(len(ev)) < 0.5
        ends = _offsets(lengths).astype(np.int64)[pid[ev] + 1]
        # deletions: mark (ev, ev+k] inside the pair as removed
        de, dk, dend = ev[is_del], k[is_del], ends[is_del]
        diff = np.zeros(n + 1, dtype=np.int64)
        lo = np.minimum(de + 1, dend)
        hi = np.minimum(de + 1 + dk, dend)
        np.add.at(diff, lo, 1)
        np.add.at(diff, hi, -1)
        keep = np.cumsum(diff[:-1]) == 0
        np.add.at(ins, ev[~is_del], k[~is_del])
    slots = keep.astype(np.int64) + ins
    new_len = np.bincount(pid, weights=slots, minlength=len(lengths))
    start = np.cumsum(slots) - slots
    res = _random_bases(rng, int(slots.sum()))
    res[start[keep]] = out[keep]
    return res, new_len.astype(np.int64)


def _join(parts_a, len_a, parts_b, len_b, cap=None):
    """Per pair: a followed by b, truncated to cap (per pair) if given."""
    n = len(len_a)
    tot = len_a + len_b
    if cap is not None:
        tot = np.minimum(tot, cap)
    off_a = _offsets(len_a).astype(np.int64)
    off_b = _offsets(len_b).astype(np.int64)
    out_off = _offsets(tot)
    pid = _pair_index(tot)
    pos = np.arange(int(tot.sum()), dtype=np.int64) - out_off[:-1].astype(np.int64)[pid]
    from_a = pos < len_a[pid]
    out = np.empty(len(pos), dtype=np.uint8)
    out[from_a] = parts_a[off_a[pid[from_a]] + pos[from_a]]
    nb = ~from_a
    out[nb] = parts_b[off_b[pid[nb]] + pos[nb] - len_a[pid[nb]]]
    return out, tot


def _sprinkle_n(rng, seq, p):
    if p > 0:
        seq[rng.random(len(seq)) < p] = 4
    return seq


def _chunk_rngs(seed, nchunks):
    """Independent generators for the chunks of a workload, derived from the
    workload seed (so chunks can be drawn in any order or in parallel)."""
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(nchunks)]


def _map_chunks(fn, args, workers):
    if workers <= 1 or len(args) <= 1:
        return [fn(*a) for a in args]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=min(workers, len(args)),
                                mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(fn, *zip(*args)))


def _assemble(chunks, scorings):
    qs, ts, qls, tls, h0s, pids = zip(*chunks)
    ql = np.concatenate(qls)
    tl = np.concatenate(tls)
    b = {"q": np.concatenate(qs), "q_off": _offsets(ql),
         "t": np.concatenate(ts), "t_off": _offsets(tl),
         "h0": np.concatenate(h0s).astype(np.int32), "scorings": scorings}
    if pids[0] is not None:
        b["param_id"] = np.concatenate(pids).astype(np.uint8)
    return b


def _read_pairs(rng, qlen, p_sub, p_indel, mean_len, flank, cap, p_n, h0_range):
    q = _random_bases(rng, int(qlen.sum()))
    mut, mlen = _mutate(rng, q, qlen, p_sub, p_indel, mean_len)
    fl = _random_bases(rng, int(flank.sum()))
    t, tlen = _join(mut, mlen, fl, flank, cap)
    q = _sprinkle_n(rng, q, p_n)
    t = _sprinkle_n(rng, t, p_n)
    h0 = rng.integers(h0_range[0], h0_range[1] + 1, size=len(qlen))
    return q, t, qlen, tlen, h0


# ---------------------------------------------------------------------------
# workloads

def plain_small(n=1000, seed=0):
    """1,000 pairs: query of 101 uniform ACGT; target = query mutated at 2%
    substitutions and 0.2% indels (geometric, mean 2) + 50 flank bases;
    h0 in [19, 50]; BWA-MEM default scoring, w 100, z-drop 100, bonus 5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    qlen = np.full(n, 101, dtype=np.int64)
    q, t, ql, tl, h0 = _read_pairs(
        rng, qlen, np.full(n, 0.02), np.full(n, 0.002), 2.0,
        np.full(n, 50, dtype=np.int64), None, 0.0, (19, 50))
    return _assemble([(q, t, ql, tl, h0, None)], [BWA_DEFAULT])


def _read_scale_chunk(rng, m):
    qlen = rng.integers(1, 151, size=m).astype(np.int64)
    extra = rng.integers(0, 201, size=m).astype(np.int64)
    p_sub = rng.uniform(0.01, 0.05, size=m)
    p_ind = rng.uniform(0.001, 0.01, size=m)
    # flank long enough that truncation to qlen + extra always applies
    flank = extra + 60
    q, t, ql, tl, h0 = _read_pairs(rng, qlen, p_sub, p_ind, 2.0, flank,
                                   qlen + extra, 0.01, (19, 50))
    return (q, t, ql, tl, h0, None)


def read_scale(n=1_000_000, seed=1, chunk=125_000, workers=1):
    """Extension remainders of simulated 151 bp reads: qlen uniform in
    [1, 150]; per pair substitutions 1-5% and indels 0.1-1%; target = mutated
    query + flank, total qlen + U[0, 200] (2w); 1% of bases N."""
    sizes = [min(chunk, n - s) for s in range(0, n, chunk)] or [0]
    rngs = _chunk_rngs(seed, len(sizes))
    return _assemble(_map_chunks(_read_scale_chunk, list(zip(rngs, sizes)), workers),
                     [BWA_DEFAULT])


def _zdrop_pairs(rng, m):
    """Pairs built to end by the drop-from-best rule (z-drop 100): an exact
    prefix of p bases lifts the score to h0 + p >= ~115, then a tail where
    the target repeats the query with substitutions at 3 of every 8
    positions loses 7/8 of a point per row along the diagonal.  That is
    slower than a deletion run (1 per row), so the diagonal stays the row
    maximum with no drift, and more than 100 below the best after ~115
    rows, before any row empties."""
    qlen = rng.integers(220, 251, size=m).astype(np.int64)
    h0 = rng.integers(19, 51, size=m).astype(np.int64)
    p = np.maximum(115 - h0, 0) + rng.integers(0, 6, size=m)
    p = np.minimum(p, qlen - 125)
    q = _random_bases(rng, int(qlen.sum()))
    pid = _pair_index(qlen)
    pos = np.arange(len(q), dtype=np.int64) - _offsets(qlen).astype(np.int64)[pid]
    tail = pos - p[pid]
    r = tail % 8
    sub = (tail >= 0) & ((r == 1) | (r == 4) | (r == 6))
    tq = q.copy()
    tq[sub] = (tq[sub] + rng.integers(1, 4, size=int(sub.sum()),
                                      dtype=np.uint8)) % 4
    extra = rng.integers(0, 201, size=m).astype(np.int64)
    fl = _random_bases(rng, int(extra.sum()))
    t, tlen = _join(tq, qlen, fl, extra)
    return q, t, qlen, tlen, h0


def _batched_mix_chunk(rng, m, zdrop_frac):
    nz = int(round(m * zdrop_frac))
    nr = m - nz
    src = rng.choice(np.array([100, 150, 250]), size=nr)
    qlen = (rng.random(nr) * src).astype(np.int64) + 1
    d = rng.uniform(0.0, 0.15, size=nr)
    extra = rng.integers(0, 201, size=nr).astype(np.int64)
    q1, t1, ql1, tl1, h01 = _read_pairs(
        rng, qlen, 0.9 * d, 0.1 * d, 2.0, extra + 60, qlen + extra, 0.0,
        (19, 50))
    q2, t2, ql2, tl2, h02 = _zdrop_pairs(rng, nz)
    # interleave the two groups in random order
    order = rng.permutation(m)
    ql = np.concatenate([ql1, ql2])
    tl = np.concatenate([tl1, tl2])
    qo = _offsets(ql).astype(np.int64)
    to = _offsets(tl).astype(np.int64)
    qi = _gather_ranges(qo, order, ql[order])
    ti = _gather_ranges(to, order, tl[order])
    h0 = np.concatenate([h01, h02])[order]
    return (np.concatenate([q1, q2])[qi], np.concatenate([t1, t2])[ti],
            ql[order], tl[order], h0, None)


def batched_mix(n=4_000_000, seed=2, chunk=125_000, zdrop_frac=0.20, workers=1):
    """Uneven pairs from 100/150/250 bp read sources (one third each):
    qlen uniform in [1, L]; divergence d uniform in [0, 15%], 0.9 d as
    substitutions and 0.1 d as indels (geometric, mean 2); target = mutated
    query + flank, total at most qlen + 200.  A fraction zdrop_frac of the
    pairs are built to end by z-drop (see _zdrop_pairs); positions of those
    pairs in the batch are random."""
    sizes = [min(chunk, n - s) for s in range(0, n, chunk)] or [0]
    rngs = _chunk_rngs(seed, len(sizes))
    args = [(r, m, zdrop_frac) for r, m in zip(rngs, sizes)]
    return _assemble(_map_chunks(_batched_mix_chunk, args, workers), [BWA_DEFAULT])


def _gather_ranges(off, order, lens):
    """Flat indices of ranges [off[k], off[k+1]) for k in order."""
    starts = off[order]
    pid = _pair_index(lens)
    base = _offsets(lens).astype(np.int64)
    return starts[pid] + np.arange(int(lens.sum()), dtype=np.int64) - base[:-1][pid]


def _wide_band_chunk(rng, m):
    qlen = np.full(m, 250, dtype=np.int64)
    rich = rng.random(m) < 0.10
    p_sub = np.where(rich, 0.02, rng.uniform(0.0, 0.05, size=m))
    p_ind = np.where(rich, 0.02, rng.uniform(0.001, 0.01, size=m))
    q = _random_bases(rng, int(qlen.sum()))
    # indel-rich pairs: geometric mean 25 (runs mostly within 1..50)
    mut_n, ml_n = _mutate(rng, q, qlen, np.where(rich, 0, p_sub),
                          np.where(rich, 0, p_ind), 2.0)
    mut_r, ml_r = _mutate(rng, q, qlen, np.where(rich, p_sub, 0),
                          np.where(rich, p_ind, 0), 25.0)
    mut, ml = _pick(rich, mut_n, ml_n, mut_r, ml_r)
    flank = rng.integers(0, 501, size=m).astype(np.int64)
    fl = _random_bases(rng, int(flank.sum()))
    t, tlen = _join(mut, ml, fl, flank, np.full(m, 750, dtype=np.int64))
    h0 = rng.integers(19, 51, size=m)
    pid = (rng.random(m) < 0.5).astype(np.uint8)
    return (q, t, qlen, tlen, h0, pid)


def wide_band(n=500_000, seed=4, chunk=50_000, workers=1):
    """250 bp queries against targets of up to 750 bp, w 500, z-drop 400,
    two scoring sets (match 1 / mismatch -4 / gap 6+k; match 2 / mismatch
    -3 / gap 5+2k) chosen per pair with probability 1/2; 10% of pairs are
    indel-rich (runs of 1-50 bp, about one per 50 bp)."""
    sizes = [min(chunk, n - s) for s in range(0, n, chunk)] or [0]
    rngs = _chunk_rngs(seed, len(sizes))
    return _assemble(_map_chunks(_wide_band_chunk, list(zip(rngs, sizes)), workers),
                     [WIDE_A, WIDE_B])


def _pick(mask, a, la, b, lb):
    """Per pair: sequence from b where mask else from a."""
    lens = np.where(mask, lb, la)
    oa = _offsets(la).astype(np.int64)
    ob = _offsets(lb).astype(np.int64)
    pid = _pair_index(lens)
    pos = np.arange(int(lens.sum()), dtype=np.int64) - _offsets(lens).astype(np.int64)[:-1][pid]
    m = mask[pid]
    out = np.empty(len(pos), dtype=np.uint8)
    out[~m] = a[oa[pid[~m]] + pos[~m]]
    out[m] = b[ob[pid[m]] + pos[m]]
    return out, lens


def serving_requests(n_requests=2000, seed=3, lo=1000, hi=100_000):
    """Request sizes log-uniform in [lo, hi] pairs; each request is drawn
    like the uneven batched mix (its own chunk of the same generator)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_requests))
    return sizes.astype(np.int64)


# seeds as the read-level driver takes them (one record per seed)
SEED_FIELDS = np.dtype([("read", "<i4"), ("qb", "<i4"), ("qe", "<i4"), ("h0", "<i4"),
                        ("rb", "<i8")])


def _reads_chunk(rng, ref, m, read_len, min_seed, max_seeds, p_n):
    """m reads drawn from ref by a per-position walk that records where each
    read base came from, and the seeds of each read: its exact runs along
    one reference diagonal of at least min_seed bases (longest first, at
    most max_seeds)."""
    L = read_len
    nref = len(ref)
    p_sub = rng.uniform(0.01, 0.05, size=(m, 1))
    p_ind = rng.uniform(0.001, 0.01, size=(m, 1))
    # insertion runs: positions [i, i + k) of the read come from nowhere
    ins_start = rng.random((m, L)) < p_ind / 2
    ins = np.zeros((m, L + 1), dtype=np.int32)
    r_i, c_i = np.nonzero(ins_start)
    k = rng.geometric(0.5, size=len(r_i))
    np.add.at(ins, (r_i, c_i), 1)
    np.add.at(ins, (r_i, np.minimum(c_i + k, L)), -1)
    inserted = np.cumsum(ins[:, :L], axis=1) > 0
    # deletions: k reference bases skipped before position i
    adv = (~inserted).astype(np.int64)
    del_start = (rng.random((m, L)) < p_ind / 2) & ~inserted
    adv[del_start] += rng.geometric(0.5, size=int(del_start.sum()))
    span = adv.sum(axis=1)
    start = rng.integers(0, max(1, nref - int(span.max()) - 1), size=m)
    src = start[:, None] + np.cumsum(adv, axis=1) - 1
    src = np.minimum(src, nref - 1)
    base = ref[src]
    sub = (rng.random((m, L)) < p_sub) & ~inserted
    base = np.where(sub, (base + rng.integers(1, 4, size=(m, L))) % 4, base)
    base = np.where(inserted, rng.integers(0, 4, size=(m, L)), base).astype(np.uint8)
    if p_n > 0:
        base[rng.random((m, L)) < p_n] = 4
    exact = ~inserted & (base == ref[src]) & (base < 4)
    # a run continues while exact and on the same diagonal
    cont = np.zeros((m, L), dtype=bool)
    cont[:, 1:] = exact[:, 1:] & exact[:, :-1] & (src[:, 1:] == src[:, :-1] + 1)
    begin = exact & ~cont
    end = np.zeros((m, L), dtype=bool)  # last position of a run
    end[:, :-1] = exact[:, :-1] & ~cont[:, 1:]
    end[:, -1] = exact[:, -1]
    br, bc = np.nonzero(begin)
    er, ec = np.nonzero(end)
    qlen = ec + 1 - bc
    keep = qlen >= min_seed
    br, bc, ec, qlen = br[keep], bc[keep], ec[keep], qlen[keep]
    # longest first per read, at most max_seeds
    order = np.lexsort((bc, -qlen, br))
    br, bc, ec, qlen = br[order], bc[order], ec[order], qlen[order]
    first = np.searchsorted(br, br, side="left")
    rank = np.arange(len(br)) - first
    keep = rank < max_seeds
    br, bc, ec, qlen = br[keep], bc[keep], ec[keep], qlen[keep]
    order = np.lexsort((bc, br))  # read order, then position
    br, bc, ec, qlen = br[order], bc[order], ec[order], qlen[order]
    seeds = np.zeros(len(br), dtype=SEED_FIELDS)
    seeds["read"] = br
    seeds["qb"] = bc
    seeds["qe"] = ec + 1
    seeds["h0"] = qlen
    seeds["rb"] = src[br, bc]
    return base.reshape(-1), seeds


def seed_workload(n_reads=2000, seed=5, read_len=151, ref_len=1 << 20, min_seed=19,
                  max_seeds=3, p_n=0.01, p_n_ref=0.0005, chunk=50_000):
    """Reads and seeds for the read-level driver: a uniform random reference
    of ref_len codes (N at rate p_n_ref), reads of read_len bases drawn from
    it with 1-5% substitutions and 0.1-1% indels (geometric length, mean 2)
    per read and N at rate p_n, and up to max_seeds seeds per read (exact
    runs of at least min_seed bases on one diagonal, h0 = their length).
    Reads with no such run have no seed.  Default scoring BWA_DEFAULT."""
    rngs = _chunk_rngs(seed, (n_reads + chunk - 1) // chunk + 1)
    ref = _sprinkle_n(rngs[0], _random_bases(rngs[0], ref_len), p_n_ref)
    reads, seeds = [], []
    done = 0
    for i, rng in enumerate(rngs[1:]):
        m = min(chunk, n_reads - done)
        r, sd = _reads_chunk(rng, ref, m, read_len, min_seed, max_seeds, p_n)
        sd["read"] += done
        reads.append(r)
        seeds.append(sd)
        done += m
    read_off = np.arange(n_reads + 1, dtype=np.uint64) * np.uint64(read_len)
    return {"reads": np.concatenate(reads), "read_off": read_off, "ref": ref,
            "seeds": np.concatenate(seeds), "scoring": BWA_DEFAULT}


# ---------------------------------------------------------------------------
# Suffix-array lookup inputs: a reference with repeat families, the text the
# mapper indexes (the reference and its reverse complement), its suffix
# array, and SA intervals of seed-length patterns.

SA_INTERVAL = np.dtype([("k", "<u8"), ("s", "<u8")])  # rows [k, k + s) of the SA
_KEY_BASES = 21  # bases per 64-bit sort key (3 bits each, 0 = end of text)


def _prefix_keys(t, n):
    """Key of every suffix i of t (codes 0..3) and of the empty suffix n:
    its first 21 bases as 3-bit codes 1..4, 0 past the end."""
    pad = np.concatenate([t.astype(np.uint64) + 1, np.zeros(_KEY_BASES, np.uint64)])
    key = np.zeros(n + 1, dtype=np.uint64)
    for d in range(_KEY_BASES):
        key = (key << np.uint64(3)) | pad[d:d + n + 1]
    return key


def suffix_array(t):
    """Suffix array of t followed by the end marker (smaller than every
    base): n + 1 int64 entries, S[0] = n.  Prefix doubling with group
    refinement: suffixes are sorted by their first 21 bases, then every
    group of still-equal suffixes is split by the rank of the suffix h bases
    further on, h doubling each round, until every group is a singleton."""
    t = np.asarray(t, dtype=np.uint8)
    n = len(t)
    key = _prefix_keys(t, n)
    order = np.argsort(key)
    sk = key[order]
    del key
    new = np.ones(n + 1, dtype=bool)
    new[1:] = sk[1:] != sk[:-1]
    del sk
    head = np.maximum.accumulate(np.where(new, np.arange(n + 1), 0))
    rank = np.empty(n + 1, dtype=np.int64)
    rank[order] = head
    h = _KEY_BASES
    while True:
        starts = np.nonzero(new)[0]
        size = np.diff(np.append(starts, n + 1))
        todo = np.repeat(size, size) > 1
        if not todo.any():
            break
        pos = np.nonzero(todo)[0]
        idx, g = order[pos], head[pos]
        sec = np.where(idx + h <= n, rank[np.minimum(idx + h, n)], -1)
        o = np.lexsort((sec, g))
        idx, g, sec = idx[o], g[o], sec[o]
        order[pos] = idx
        nh = np.ones(len(idx), dtype=bool)
        nh[1:] = (g[1:] != g[:-1]) | (sec[1:] != sec[:-1])
        hh = np.maximum.accumulate(np.where(nh, pos, 0))
        head[pos] = hh
        rank[idx] = hh
        new[pos] = nh
        h *= 2
    return order.astype(np.int64)


def revcomp(t):
    t = np.asarray(t, dtype=np.uint8)
    return (3 - t[::-1]).astype(np.uint8)


def repeat_reference(n, seed, repeat_frac=0.12, copies=(2, 300), length=(100, 400),
                     divergence=(0.0, 0.05)):
    """Uniform random ACGT of length n with repeat families written over
    about repeat_frac of it: each family a random consensus of length U[length]
    copied log-U[copies] times, each copy with its own substitution rate
    U[divergence], at random places."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ref = _random_bases(rng, n)
    covered = 0
    while covered < repeat_frac * n:
        L = int(rng.integers(length[0], length[1] + 1))
        c = int(np.exp(rng.uniform(np.log(copies[0]), np.log(copies[1]))))
        cons = _random_bases(rng, L)
        for _ in range(c):
            p = int(rng.integers(0, n - L))
            cp = cons.copy()
            sub = rng.random(L) < rng.uniform(*divergence)
            cp[sub] = (cp[sub] + rng.integers(1, 4, size=int(sub.sum()), dtype=np.uint8)) % 4
            ref[p:p + L] = cp
        covered += L * c
    return ref


def sa_intervals(text, sa, n_iv, seed, lengths=(19, 21)):
    """SA intervals of n_iv patterns: text[p, p + L) for p uniform over the
    forward half of the text (the reference) and L uniform in lengths, so
    each interval holds every occurrence of the pattern on either strand."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(text)
    allkey = _prefix_keys(np.asarray(text, dtype=np.uint8), n)
    skey = allkey[sa]
    half = n // 2
    L = rng.integers(lengths[0], lengths[1] + 1, size=n_iv)
    p = rng.integers(0, half - lengths[1], size=n_iv)
    iv = np.zeros(n_iv, dtype=SA_INTERVAL)
    pkey = allkey[p]
    del allkey
    for l in range(lengths[0], lengths[1] + 1):
        m = L == l
        sh = np.uint64(3 * (_KEY_BASES - l))
        tk = skey >> sh
        lo = np.searchsorted(tk, pkey[m] >> sh, side="left")
        hi = np.searchsorted(tk, pkey[m] >> sh, side="right")
        iv["k"][m] = lo
        iv["s"][m] = hi - lo
    return iv, p, L


def sa_workload(ref_len=1 << 14, n_iv=2000, seed=6, **kw):
    """Reference with repeats (seed), the indexed text ref + revcomp(ref),
    its suffix array and n_iv SA intervals (seed + 1)."""
    ref = repeat_reference(ref_len, seed, **kw)
    text = np.concatenate([ref, revcomp(ref)])
    sa = suffix_array(text)
    iv, p, L = sa_intervals(text, sa, n_iv, seed + 1)
    return {"ref": ref, "text": text, "sa": sa, "iv": iv, "pattern_pos": p, "pattern_len": L}


def fm_patterns(text, n, seed, length=(32, 32), p_sub=0.02, p_n=0.005):
    """n search patterns from the forward half of a two-strand text: a
    substring of length U[length] at a uniform position, with substitutions
    at rate p_sub and N at rate p_n (a stand-in for read stretches)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = len(text) // 2
    L = rng.integers(length[0], length[1] + 1, size=n)
    off = _offsets(L)
    p = rng.integers(0, max(1, half - length[1]), size=n)
    idx = np.repeat(p, L) + (np.arange(int(L.sum())) - np.repeat(off[:-1].astype(np.int64), L))
    pat = np.asarray(text, dtype=np.uint8)[idx].copy()
    sub = rng.random(len(pat)) < p_sub
    pat[sub] = (pat[sub] + rng.integers(1, 4, size=int(sub.sum()), dtype=np.uint8)) % 4
    return _sprinkle_n(rng, pat, p_n), off


# the lookup's benchmark workload: a 32 Mbase reference (64 Mbase indexed
# text, a 512 MB suffix array) and 4 M intervals
SA_BENCH = dict(ref_len=1 << 25, n_iv=4_000_000, seed=6)
# the backward search's benchmark patterns over the same text: 4 M of 32 bases
FM_BENCH_PATTERNS = 4_000_000
# and the SMEM search's reads: 500,000 of 151 bases
SMEM_BENCH_READS = 500_000


# the read-level driver's benchmark workload: 500,000 reads of 151 bases
# drawn from a 64 Mbase reference (about 1.3 M seeds)
SEED_BENCH = dict(n_reads=500_000, seed=5, ref_len=1 << 26)


WORKLOADS = {
    "plain_small": plain_small,
    "read_scale": read_scale,
    "batched_mix": batched_mix,
    "wide_band": wide_band,
}


def subset(batch, idx):
    """The pairs idx of a batch, as a new batch (same scoring sets)."""
    idx = np.asarray(idx, dtype=np.int64)
    qo = batch["q_off"].astype(np.int64)
    to = batch["t_off"].astype(np.int64)
    ql = qo[idx + 1] - qo[idx]
    tl = to[idx + 1] - to[idx]
    out = {"q": batch["q"][_gather_ranges(qo, idx, ql)] if len(idx) else batch["q"][:0],
           "q_off": _offsets(ql),
           "t": batch["t"][_gather_ranges(to, idx, tl)] if len(idx) else batch["t"][:0],
           "t_off": _offsets(tl),
           "h0": batch["h0"][idx].copy(), "scorings": batch["scorings"]}
    if "param_id" in batch:
        out["param_id"] = batch["param_id"][idx].copy()
    return out


def from_pairs(pairs, scorings, param_id=None):
    """Batch from a list of (q codes, t codes, h0)."""
    ql = np.array([len(p[0]) for p in pairs], dtype=np.int64)
    tl = np.array([len(p[1]) for p in pairs], dtype=np.int64)
    b = {"q": np.array([c for p in pairs for c in p[0]], dtype=np.uint8),
         "q_off": _offsets(ql),
         "t": np.array([c for p in pairs for c in p[1]], dtype=np.uint8),
         "t_off": _offsets(tl),
         "h0": np.array([p[2] for p in pairs], dtype=np.int32),
         "scorings": list(scorings)}
    if param_id is not None:
        b["param_id"] = np.asarray(param_id, dtype=np.uint8)
    return b


def pair(batch, k):
    """(q codes, t codes, h0, scoring) of pair k."""
    qo, to = batch["q_off"], batch["t_off"]
    sc = batch["scorings"][int(batch["param_id"][k]) if "param_id" in batch else 0]
    return (batch["q"][int(qo[k]):int(qo[k + 1])],
            batch["t"][int(to[k]):int(to[k + 1])], int(batch["h0"][k]), sc)
