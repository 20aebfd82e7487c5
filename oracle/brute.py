"""Exhaustive alignment-path enumeration for tiny BSW inputs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Independent pin for the recurrence and boundaries of the seed extension
(paper Sec. 5.1, Eq. (2) and (3), readings R2-R6, R15, R16 in
``bsw_ref.c``).  Nothing here evaluates the recurrence: the score of every
cell is the maximum, over every alignment path from the seed to that cell,
of the path's score, where

* the seed sits before both sequences (row -1, column -1) with score h0,
* an aligned step consumes one target and one query base and adds
  S(target, query),
* an insertion run consumes k >= 1 query bases and costs o_ins + k*e_ins,
* a deletion run consumes k >= 1 target bases and costs o_del + k*e_del,
* a run may only follow the seed or an aligned step (an insertion never
  touches a deletion), and a run is maximal (two runs of the same kind are
  never adjacent).

That is the textbook definition of an affine-gap extension score.  The
method's extra rules (zero floors and the positive-diagonal gate, the band,
the row abort, z-drop and the band shrink) never bind when h0 is large, the
band is wider than both sequences, the end bonus is huge and z-drop is off;
in that regime the outputs follow from the cell scores alone through the
row-scan rules of Sec. 5.4 (a)-(b) and R15:

* per row, m = max over the row and mj = the largest column reaching it,
* the best score moves only on a strict increase (earliest row wins),
* the query-end score is H(i, Lq-1), taking the latest row on ties.

``gated_cell_scores`` / ``extend_gated`` enumerate the same paths under the
one extra rule that gives the method its zero floors and its positive-
diagonal gate (reading R4 of Sec. 5.1 Eq. (2)): a path is only extended
while its running score is positive, i.e. every proper prefix of a path
(the seed, every aligned step and every step of a gap run) scores > 0, and
a cell's score is max(0, best such path).  With a band wider than both
sequences, a huge end bonus and z-drop off, this equals the method as long
as its band shrink never cuts a row short on the right and the first
column (the seed's deletion run) is zero once the band has left column 0;
the method then stops at the first all-zero row, which ``extend_gated``
takes from the cell scores as well.
"""
from __future__ import annotations

import numpy as np


def cell_scores(q, t, h0, sc):
    """Best path score for every cell (i, j); -inf where none exists."""
    Lq, Lt = len(q), len(t)
    S = np.asarray(sc["mat"], dtype=np.int64).reshape(5, 5)
    oD, eD, oI, eI = sc["o_del"], sc["e_del"], sc["o_ins"], sc["e_ins"]
    NEG = -(1 << 60)
    best = np.full((Lt, Lq), NEG, dtype=np.int64)

    # depth-first walk over all paths; state: position, score, whether the
    # last move was a run (then only an aligned step may follow)
    stack = [(-1, -1, h0, False)]
    while stack:
        i, j, s, after_run = stack.pop()
        if i >= 0 and j >= 0 and s > best[i, j]:
            best[i, j] = s
        # aligned step
        if i + 1 < Lt and j + 1 < Lq:
            stack.append((i + 1, j + 1, s + S[t[i + 1], q[j + 1]], False))
        if after_run:
            continue
        # here the position is the seed or a cell reached by an aligned
        # step; insertion runs stay in its row, deletion runs in its column
        for k in range(1, Lq - j):
            stack.append((i, j + k, s - oI - k * eI, True))
        for k in range(1, Lt - i):
            stack.append((i + k, j, s - oD - k * eD, True))
    return best


def extend(q, t, h0, sc):
    """Outputs (score, qle, tle, gtle, gscore, max_off) from the cell scores.

    Only valid in the regime described in the module docstring (checked by
    the caller)."""
    q = list(int(x) for x in q)
    t = list(int(x) for x in t)
    Lq, Lt = len(q), len(t)
    if Lt == 0:
        return (h0, 0, 0, 0, -1, 0)
    if Lq == 0:
        # row 0 has no cell, so the method's all-zero-row rule ends it at
        # once; its query-end value is the first-column value H(0,-1)
        return (h0, 0, 0, 1, max(0, h0 - sc["o_del"] - sc["e_del"]), 0)
    H = cell_scores(q, t, h0, sc)
    best, bi, bj, gbest, gi, moff = h0, -1, -1, -1, -1, 0
    for i in range(Lt):
        row = H[i]
        m = int(row.max())
        mj = int(max(j for j in range(Lq) if row[j] == m))
        if int(row[Lq - 1]) >= gbest:
            gi = i
            gbest = int(row[Lq - 1])
        if m > best:
            best, bi, bj = m, i, mj
            moff = max(moff, abs(mj - i))
    return (best, bj + 1, bi + 1, gi + 1, gbest, moff)


def heuristic_free_scoring(base, qlen, tlen):
    """A copy of ``base`` with the band, end bonus and z-drop opened up so
    that, together with a large h0, no heuristic of the method binds."""
    sc = dict(base)
    sc["w"] = qlen + tlen + 1
    sc["end_bonus"] = 10**6
    sc["zdrop"] = 0
    return sc


def gated_cell_scores(q, t, h0, sc):
    """Cell scores under the positive-prefix rule (see the module
    docstring): max(0, best path whose proper prefixes all score > 0)."""
    Lq, Lt = len(q), len(t)
    S = np.asarray(sc["mat"], dtype=np.int64).reshape(5, 5)
    oD, eD, oI, eI = sc["o_del"], sc["e_del"], sc["o_ins"], sc["e_ins"]
    best = np.zeros((Lt, Lq), dtype=np.int64)
    stack = [(-1, -1, h0, False)]
    while stack:
        i, j, s, after_run = stack.pop()
        if i >= 0 and j >= 0 and s > best[i, j]:
            best[i, j] = s
        if s <= 0:
            continue  # a path is not extended past a non-positive score
        if i + 1 < Lt and j + 1 < Lq:
            stack.append((i + 1, j + 1, s + S[t[i + 1], q[j + 1]], False))
        if after_run:
            continue
        # a run of k steps: each of its first k-1 steps must stay positive
        for k in range(1, Lq - j):
            v = s - oI - k * eI
            stack.append((i, j + k, v, True))
            if v <= 0:
                break
        for k in range(1, Lt - i):
            v = s - oD - k * eD
            stack.append((i + k, j, v, True))
            if v <= 0:
                break
    return best


def extend_gated(q, t, h0, sc):
    """Outputs of the method from ``gated_cell_scores``: rows are scanned up
    to the first all-zero row (the method's all-zero abort), with the row
    rules of Sec. 5.4 (a)-(b) and R15.  Only valid under the conditions in
    the module docstring (checked by the caller)."""
    q = list(int(x) for x in q)
    t = list(int(x) for x in t)
    Lq, Lt = len(q), len(t)
    if Lt == 0:
        return (h0, 0, 0, 0, -1, 0)
    if Lq == 0:
        return (h0, 0, 0, 1, max(0, h0 - sc["o_del"] - sc["e_del"]), 0)
    H = gated_cell_scores(q, t, h0, sc)
    best, bi, bj, gbest, gi, moff = h0, -1, -1, -1, -1, 0
    for i in range(Lt):
        row = H[i]
        m = int(row.max())
        if int(row[Lq - 1]) >= gbest:
            gi = i
            gbest = int(row[Lq - 1])
        if m == 0:
            break
        mj = int(max(j for j in range(Lq) if row[j] == m))
        if m > best:
            best, bi, bj = m, i, mj
            moff = max(moff, abs(mj - i))
    return (best, bj + 1, bi + 1, gi + 1, gbest, moff)
