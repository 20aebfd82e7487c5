"""Pins of the read-level seed extension reference (oracle.seeds).

Each expected value follows from the method's definition by hand: exact
matches grow the score by the match score per base, a mismatch costs 4, a
gap of length k costs 6 + k (default scoring), and the end-of-read choice
keeps the read end only when its score is within the end bonus of the best.
"""
import numpy as np
import pytest

from paper_1907_12931_amd import synth


@pytest.fixture(scope="module")
def seeds_mod(oracle_lib):
    from oracle import seeds
    return seeds


def make(seeds_mod, read_list, ref, seed_rows):
    ql = [len(r) for r in read_list]
    reads = np.concatenate([np.asarray(r, np.uint8) for r in read_list])
    off = np.zeros(len(ql) + 1, np.uint64)
    off[1:] = np.cumsum(ql)
    s = np.zeros(len(seed_rows), dtype=seeds_mod.SEED_DTYPE)
    for k, (read, qb, qe, rb, h0) in enumerate(seed_rows):
        s[k] = (read, qb, qe, h0, rb)
    return reads, off, np.asarray(ref, np.uint8), s


# (read length, reference position, qb, qe); the third clips the left
# reference window at 0, the fourth the right window at the reference end
CASES_EXACT = [(150, 300, 40, 80), (101, 1200, 1, 100), (250, 50, 120, 121),
               (100, 1900, 10, 20)]


def test_exact_read_reaches_both_ends(seeds_mod):
    rng = np.random.default_rng(1)
    ref = rng.integers(0, 4, 2000)
    rows, reads = [], []
    for k, (L, P, qb, qe) in enumerate(CASES_EXACT):
        reads.append(ref[P:P + L])
        rows.append((k, qb, qe, P + qb, qe - qb))
    r, off, rf, s = make(seeds_mod, reads, ref, rows)
    out = seeds_mod.extend_seeds(r, off, rf, s, synth.BWA_DEFAULT)
    for k, (L, P, qb, qe) in enumerate(CASES_EXACT):
        o = out[k]
        assert (o["score"], o["qbeg"], o["qend"], o["rbeg"], o["rend"]) == (L, 0, L, P, P + L)
        assert o["how"] == seeds_mod.READ_END | seeds_mod.READ_END << 2


def test_seed_covering_the_read_is_not_extended(seeds_mod):
    rng = np.random.default_rng(2)
    ref = rng.integers(0, 4, 500)
    r, off, rf, s = make(seeds_mod, [ref[100:160]], ref, [(0, 0, 60, 100, 60)])
    o = seeds_mod.extend_seeds(r, off, rf, s, synth.BWA_DEFAULT)[0]
    assert (o["score"], o["qbeg"], o["qend"], o["rbeg"], o["rend"]) == (60, 0, 60, 100, 160)
    assert o["how"] == seeds_mod.NONE | seeds_mod.NONE << 2


def test_mismatching_prefix_keeps_the_seed_start(seeds_mod):
    # read = 10 x A, then ref[200:260]; the reference before the seed is all
    # C: every path to the read start consumes 10 bases by mismatches or an
    # insertion (at least 6 + 10), so the left end stays at the seed
    ref = np.concatenate([np.full(200, 1), np.random.default_rng(3).integers(0, 4, 300)])
    read = np.concatenate([np.zeros(10, int), ref[200:260]])
    r, off, rf, s = make(seeds_mod, [read], ref, [(0, 10, 40, 200, 30)])
    o = seeds_mod.extend_seeds(r, off, rf, s, synth.BWA_DEFAULT)[0]
    assert (o["qbeg"], o["rbeg"]) == (10, 200)
    assert o["how"] & 3 == seeds_mod.LOCAL
    # the right side is exact: read[40:70] = ref[230:260], 30 more bases on
    # top of the kept left score 30
    assert (o["score"], o["qend"], o["rend"]) == (60, 70, 260)


@pytest.mark.parametrize("bonus,left_read_end", [(5, True), (4, False), (3, False)])
def test_end_bonus_decides_the_left_end(seeds_mod, bonus, left_read_end):
    # read[0] mismatches the reference, read[1:] matches it exactly: the best
    # left cell stops one base short (score h0 + qb - 1); reaching the read
    # start costs the mismatch, 4, so the read end is kept only if 4 < bonus
    rng = np.random.default_rng(4)
    ref = rng.integers(0, 4, 600)
    P, L, qb, qe, h0 = 200, 120, 30, 60, 30
    read = ref[P:P + L].copy()
    read[0] = (read[0] + 1) % 4
    sc = synth.scoring(end_bonus=bonus)
    r, off, rf, s = make(seeds_mod, [read], ref, [(0, qb, qe, P + qb, h0)])
    o = seeds_mod.extend_seeds(r, off, rf, s, sc)[0]
    if left_read_end:
        assert (o["qbeg"], o["rbeg"]) == (0, P) and o["how"] & 3 == seeds_mod.READ_END
        left = h0 + qb - 5
    else:
        assert (o["qbeg"], o["rbeg"]) == (1, P + 1) and o["how"] & 3 == seeds_mod.LOCAL
        left = h0 + qb - 1
    # right side exact to the read end
    assert (o["score"], o["qend"], o["rend"]) == (left + L - qe, L, P + L)


@pytest.mark.parametrize("bonus,right_read_end", [(5, True), (4, False)])
def test_end_bonus_decides_the_right_end(seeds_mod, bonus, right_read_end):
    rng = np.random.default_rng(5)
    ref = rng.integers(0, 4, 600)
    P, L, qb, qe, h0 = 100, 90, 0, 40, 40
    read = ref[P:P + L].copy()
    read[L - 1] = (read[L - 1] + 2) % 4
    sc = synth.scoring(end_bonus=bonus)
    r, off, rf, s = make(seeds_mod, [read], ref, [(0, qb, qe, P + qb, h0)])
    o = seeds_mod.extend_seeds(r, off, rf, s, sc)[0]
    best = h0 + (L - 1 - qe)
    if right_read_end:
        assert (o["score"], o["qend"], o["rend"]) == (best - 4, L, P + L)
    else:
        assert (o["score"], o["qend"], o["rend"]) == (best, L - 1, P + L - 1)


def test_left_extension_is_bsw_on_the_reversed_prefix(seeds_mod, oracle_lib):
    """The left side equals one BSW call written out by hand: reversed read
    prefix, reversed reference window of qb + w bases before the seed."""
    rng = np.random.default_rng(6)
    ref = rng.integers(0, 5, 3000).astype(np.uint8)
    read = np.concatenate([rng.integers(0, 4, 70), ref[1500:1580]]).astype(np.uint8)
    qb, qe, rb, h0 = 90, 110, 1520, 20
    r, off, rf, s = make(seeds_mod, [read], ref, [(0, qb, qe, rb, h0)])
    o = seeds_mod.extend_seeds(r, off, rf, s, synth.BWA_DEFAULT)[0]
    q = read[:qb][::-1].copy()
    t = ref[rb - qb - 100:rb][::-1].copy()
    vals, _ = oracle_lib.extend_one(q, t, h0, synth.BWA_DEFAULT)
    res = dict(zip(oracle_lib.RESULT_DTYPE.names, vals))
    if res["gscore"] > 0 and res["gscore"] > res["score"] - 5:
        assert (o["qbeg"], o["rbeg"]) == (0, rb - res["gtle"])
    else:
        assert (o["qbeg"], o["rbeg"]) == (qb - res["qle"], rb - res["tle"])


def test_synthetic_seeds_are_exact_diagonal_matches():
    """The generator's seeds are what the driver assumes: read[qb, qe)
    equals ref[rb, rb + qe - qb), with no N, and at least 19 bases."""
    w = synth.seed_workload(400, seed=21)
    s = w["seeds"]
    assert len(s) > 400
    for x in s:
        r0 = int(w["read_off"][x["read"]])
        a = w["reads"][r0 + x["qb"]:r0 + x["qe"]]
        b = w["ref"][x["rb"]:x["rb"] + x["qe"] - x["qb"]]
        assert np.array_equal(a, b) and (a < 4).all() and x["qe"] - x["qb"] >= 19
        assert x["h0"] == x["qe"] - x["qb"]


def test_reference_invariants_on_synthetic_reads(seeds_mod):
    """Properties every record has by definition: the extended intervals
    contain the seed; a side with nothing to extend keeps the seed boundary
    and the score; a side that kept the read end reaches it; the reference
    interval stays inside the reference."""
    w = synth.seed_workload(1500, seed=22, ref_len=300_000)
    s, o = w["seeds"], seeds_mod.extend_seeds(w["reads"], w["read_off"], w["ref"],
                                              w["seeds"], synth.BWA_DEFAULT)
    L = (w["read_off"][s["read"] + 1] - w["read_off"][s["read"]]).astype(np.int64)
    re = s["rb"] + s["qe"] - s["qb"]
    assert (o["qbeg"] <= s["qb"]).all() and (o["qend"] >= s["qe"]).all()
    assert (o["rbeg"] <= s["rb"]).all() and (o["rend"] >= re).all()
    assert (o["rbeg"] >= 0).all() and (o["rend"] <= len(w["ref"])).all()
    left, right = o["how"] & 3, o["how"] >> 2
    assert ((left == seeds_mod.NONE) == (s["qb"] == 0)).all()
    assert ((right == seeds_mod.NONE) == (s["qe"] == L)).all()
    assert (o["qbeg"][left == seeds_mod.READ_END] == 0).all()
    assert (o["qend"][right == seeds_mod.READ_END] == L[right == seeds_mod.READ_END]).all()
    both = (left == seeds_mod.NONE) & (right == seeds_mod.NONE)
    assert (o["score"][both] == s["h0"][both]).all()
    # a read-end choice never gives up more than the bonus less one
    # (score, per side, is at least the side's best - (bonus - 1) >= h0 - 4)
    assert (o["score"] >= s["h0"] - 8).all()
    # every choice occurs on read-shaped data
    for side in (left, right):
        assert {0, 1, 2} <= set(np.unique(side).tolist())


# ---------------------------------------------------------------------------
# the filter after extending every seed (Sec. 5.3.2)

def _seed(read, qb, qe, rb, h0=20):
    return (read, qb, qe, h0, rb)


def _res(qbeg, qend, rbeg, rend, score=50):
    return (score, qbeg, qend, 0, rbeg, rend)


def test_filter_hand_cases():
    """Hand-made chains: the first seed of a read is kept; a later seed inside
    a kept extension (read and reference) is dropped; one outside either
    interval, on another read, or only inside a dropped seed's extension is
    kept."""
    from oracle import seeds as osd
    S = np.array([
        _seed(0, 10, 40, 1010),   # kept: first of read 0
        _seed(0, 50, 70, 1050),   # dropped: inside seed 0's extension
        _seed(0, 50, 70, 5050),   # kept: same read interval, other reference place
        _seed(1, 0, 30, 2000),    # kept: first of read 1
        _seed(1, 35, 60, 2035),   # kept: read end 60 past the extension's 50
        _seed(1, 40, 45, 2040),   # dropped: inside the extension of seed 4
        _seed(2, 5, 25, 300),     # kept: first of read 2
    ], dtype=osd.SEED_DTYPE)
    R = np.array([
        _res(0, 151, 1000, 1151),
        _res(0, 151, 1000, 1151),   # (a dropped seed's extension never covers)
        _res(40, 100, 5040, 5100),
        _res(0, 50, 2000, 2050),
        _res(30, 151, 2030, 2151),
        _res(0, 151, 0, 10**9),
        _res(0, 151, 295, 446),
    ], dtype=osd.SEED_RESULT_DTYPE)
    assert osd.filter_seeds(S, R).tolist() == [1, 0, 1, 1, 1, 0, 1]
    # boundaries are inclusive of the extension's ends
    S2 = np.array([_seed(3, 0, 10, 100), _seed(3, 0, 10, 100), _seed(3, 1, 11, 101)],
                  dtype=osd.SEED_DTYPE)
    R2 = np.array([_res(0, 10, 100, 110)] * 3, dtype=osd.SEED_RESULT_DTYPE)
    assert osd.filter_seeds(S2, R2).tolist() == [1, 0, 1]
    assert osd.filter_seeds(S2[:0], R2[:0]).tolist() == []


def test_filter_on_synthetic_reads(oracle_lib):
    """On reads with several seeds: the first seed of every read is kept,
    every later kept seed is outside every earlier kept extension of its
    read, every dropped seed inside one, and some seeds are dropped."""
    from oracle import seeds as osd
    w = synth.seed_workload(n_reads=300, seed=17)
    res = osd.extend_seeds(w["reads"], w["read_off"], w["ref"], w["seeds"], w["scoring"])
    keep = osd.filter_seeds(w["seeds"], res)
    S = w["seeds"]
    assert keep.dtype == np.uint8 and set(np.unique(keep)) <= {0, 1}
    dropped = 0
    for k in range(len(S)):
        earlier = [j for j in range(k) if S[j]["read"] == S[k]["read"] and keep[j]]
        if k == 0 or S[k - 1]["read"] != S[k]["read"]:
            assert keep[k] == 1
        inside = any(res[j]["qbeg"] <= S[k]["qb"] and S[k]["qe"] <= res[j]["qend"] and
                     res[j]["rbeg"] <= S[k]["rb"] and
                     S[k]["rb"] + S[k]["qe"] - S[k]["qb"] <= res[j]["rend"]
                     for j in earlier)
        assert keep[k] == (0 if inside else 1)
        dropped += 1 - int(keep[k])
    assert dropped > 0
