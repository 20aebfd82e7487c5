"""Suffix-array lookup (SAL): CPU reference.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the
smoke check and the benchmark's CPU baseline use it; the library never does.

Sec. 2.2 builds the index of a text R as follows: R is followed by the end
marker $, which sorts before every base ($ < A < C < G < T); all rotations
of R$ sorted lexicographically form the BW matrix, and the suffix array S
gives, for each row, the position in R$ where that row's rotation starts
(the same as sorting the suffixes).  The exact matches of a pattern are the
rows whose rotation begins with it, a contiguous range: its SA interval.
SAL (Sec. 4.5, Eq. (1)) turns a row i into the coordinate j = S[i] in the
text; for an interval of s rows starting at row k it yields S[k], ...,
S[k + s - 1].  Results of several intervals are concatenated in interval
order, interval m's coordinates at out[off[m] : off[m + 1]].

The rotation sort is for small texts (it builds every rotation); larger
suffix arrays come from the input generator and are checked against this
one in the tests.
"""
from __future__ import annotations

import bisect

import numpy as np

BASES = "ACGT"
_LETTERS = np.frombuffer(b"ACGTN", dtype=np.uint8)


def to_text(codes):
    """Codes 0..3 as a string over A, C, G, T (4 as N)."""
    return _LETTERS[np.asarray(codes, dtype=np.uint8)].tobytes().decode()


def suffix_array_by_rotations(codes):
    """S of R$ by sorting the rotations of R$ (Sec. 2.2); '$' sorts before
    'A' in ASCII, so Python's string order is the paper's order."""
    r = to_text(codes) + "$"
    rotations = [r[i:] + r[:i] for i in range(len(r))]
    return np.array(sorted(range(len(r)), key=lambda i: rotations[i]), dtype=np.int64)


def sa_interval(sa, codes, pattern):
    """(k, s): first row and number of rows whose rotation of R$ starts with
    the pattern (rows compared one by one)."""
    r = to_text(codes) + "$"
    p = to_text(pattern)
    rows = [i for i in range(len(sa)) if r[int(sa[i]):].startswith(p)]
    if not rows:
        return 0, 0
    assert rows == list(range(rows[0], rows[0] + len(rows)))  # contiguous
    return rows[0], len(rows)


def sa_interval_sorted(sa, txt, p):
    """The same (k, s) found by bisection over the sorted rows: txt is the
    text followed by '$' (as a string), p the pattern (a string).  Rows in
    suffix order are sorted by their first len(p) characters too, so the
    rows starting with p are those between the two bisection points."""
    L = len(p)
    rows = range(len(sa))
    key = lambda i: txt[sa[i]:sa[i] + L]  # noqa: E731
    lo = bisect.bisect_left(rows, p, key=key)
    hi = bisect.bisect_right(rows, p, key=key)
    return (lo, hi - lo) if hi > lo else (0, 0)


def lookup(sa, intervals):
    """Eq. (1) over every row of every interval: (off, out) with interval
    m's coordinates at out[off[m]:off[m + 1]]."""
    sa = np.asarray(sa)
    k = np.asarray(intervals["k"], dtype=np.int64)
    s = np.asarray(intervals["s"], dtype=np.int64)
    off = np.zeros(len(k) + 1, dtype=np.int64)
    off[1:] = np.cumsum(s)
    out = np.empty(int(off[-1]), dtype=np.int64)
    for m in range(len(k)):
        for r in range(s[m]):
            out[off[m] + r] = sa[k[m] + r]
    return off, out
