"""FM-index quantities and bi-interval backward search: CPU reference.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Definitions (Sec. 2.2; Sec. 4.1-4.2): the index is built over the text
T = R + revcomp(R) (the mapper indexes both strands), followed by the end
marker $.  S is the suffix array of T$; the BWT is B[i] = T[S[i] - 1], or $
where S[i] = 0.  O(c, t) is the number of occurrences of base c in
B[0 .. t] (O(c, -1) = 0).  The bi-interval of a string X is (k, l, s): k the
first row of X's SA interval, s its size, l the first row of the interval
of revcomp(X).  Backward search of a pattern P extends from its last base
to its first, one base at a time; it reports the bi-interval of P when all
of P occurs, and in every case the length of the longest suffix of P that
occurs in T (the bases matched before the interval became empty).

Everything here follows the definitions directly (interval by comparing
every row, counts by counting), for small texts.
"""
from __future__ import annotations

import numpy as np

from . import sal

COMP = np.array([3, 2, 1, 0], dtype=np.uint8)


def bwt(text, sa):
    """B as codes 0..3, with 4 for $ (at the row whose suffix is all of T)."""
    t = np.asarray(text, dtype=np.uint8)
    sa = np.asarray(sa, dtype=np.int64)
    out = np.full(len(sa), 4, dtype=np.uint8)
    m = sa > 0
    out[m] = t[sa[m] - 1]
    return out


def occ(b, c, t):
    """O(c, t): occurrences of c in B[0 .. t]."""
    return int(np.count_nonzero(np.asarray(b[:t + 1]) == c)) if t >= 0 else 0


def revcomp(x):
    return COMP[np.asarray(x, dtype=np.uint8)[::-1]]


def bi_interval(text, sa, x):
    """(k, l, s) of X by definition; (0, 0, 0) when X does not occur."""
    k, s = sal.sa_interval(sa, text, x)
    if s == 0:
        return 0, 0, 0
    l, s2 = sal.sa_interval(sa, text, revcomp(x))
    assert s2 == s  # T holds both strands: X and revcomp(X) occur equally often
    return k, l, s


def backward_search(text, sa, pattern, txt=None):
    """(k, l, s, matched): the bi-interval of the pattern (zeros unless all
    of it occurs) and the length of its longest occurring suffix.  The
    intervals are found by bisection over the sorted rows (txt: the text as
    a string followed by '$', made here when not given)."""
    p = np.asarray(pattern, dtype=np.uint8)
    if txt is None:
        txt = sal.to_text(text) + "$"
    matched = 0
    for m in range(1, len(p) + 1):
        suf = p[len(p) - m:]
        if suf[0] > 3 or sal.sa_interval_sorted(sa, txt, sal.to_text(suf))[1] == 0:
            break
        matched = m
    if matched < len(p):
        return 0, 0, 0, matched
    if len(p) == 0:
        return 0, 0, len(sa), 0
    k, s = sal.sa_interval_sorted(sa, txt, sal.to_text(p))
    l, s2 = sal.sa_interval_sorted(sa, txt, sal.to_text(revcomp(p)))
    assert s2 == s
    return k, l, s, matched


def smems(text, sa, read, txt=None):
    """Super-maximal exact matches of a read (Sec. 2.3, SMEM): with e(a) the
    end of the longest substring starting at a that occurs in T, [a, e(a))
    is a maximal exact match when it is not empty and cannot grow to the
    left (e(a - 1) < e(a)), and it is super-maximal when no match starting
    further left reaches as far (e(a) above every earlier e).  e is
    non-decreasing, so one sweep finds it.  Returns (start, end, k, l, s)
    tuples in order of start."""
    x = np.asarray(read, dtype=np.uint8)
    if txt is None:
        txt = sal.to_text(text) + "$"
    n = len(x)

    def occurs(a, b):
        return (x[a:b] < 4).all() and sal.sa_interval_sorted(sa, txt, sal.to_text(x[a:b]))[1] > 0

    out = []
    best = 0  # largest e so far
    b = 0
    for a in range(n):
        b = max(b, a)
        while b < n and occurs(a, b + 1):
            b += 1
        if b > a and b > best:
            k, l, s = bi_interval_sorted(sa, txt, x[a:b])
            out.append((a, b, k, l, s))
        best = max(best, b)
    return out


def bi_interval_sorted(sa, txt, x):
    k, s = sal.sa_interval_sorted(sa, txt, sal.to_text(x))
    l, s2 = sal.sa_interval_sorted(sa, txt, sal.to_text(revcomp(x)))
    assert s == s2
    return k, l, s
