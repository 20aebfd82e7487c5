"""Full-matrix NumPy re-statement of banded seed extension (BSW).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

This is a second, independent formulation of the rules the C oracle
follows (paper Sec. 5.1, Eq. (2) and (3), readings R1-R16 listed in
``bsw_ref.c``).  Instead of a rolling one-row buffer it keeps

* explicit matrices ``H[i, j]`` and ``E[i + 1, j]`` of every computed cell,
* the left-boundary value ``LB[i]`` of every row, and
* for every buffer index ``j`` the row and kind of its last write
  (initial row, in-band cell, right edge),

and resolves what the one-row buffer of the method would hold at index j
from those.  F along a row is taken from its closed form: with
``u(k) = M(k) - o_ins - e_ins + e_ins * k``, the value entering column j is
``max(0, max_{beg <= k < j} u(k) - e_ins * (j - 1))`` (an exact prefix
maximum; the recurrence F(j+1) = max(F(j) - e, M(j) - o - e, 0) unrolls to
it).  Row maxima and the band shrink are taken with vectorised reductions.
Nothing here is shared with the C oracle; agreement between the two pins
the buffer bookkeeping (stale entries, right-edge write, shrink rules).
"""
from __future__ import annotations

import numpy as np

INIT, CELL, RIGHT = 0, 1, 2


def band_cap(qlen, sc):
    a = max(0, int(np.max(np.asarray(sc["mat"]))))
    caps = []
    for o, e in ((sc["o_ins"], sc["e_ins"]), (sc["o_del"], sc["e_del"])):
        num = qlen * a + sc["end_bonus"] - o
        caps.append(num // e + 1 if num >= 0 else 1)
    return min(sc["w"], *caps)


def extend(q, t, h0, sc, trace=None):
    """Return ((score, qle, tle, gtle, gscore, max_off), (rows, stop, cells)).
    With a list ``trace``, the band [beg, end) of every computed row is
    appended to it."""
    q = np.asarray(q, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    Lq, Lt = len(q), len(t)
    S = np.asarray(sc["mat"], dtype=np.int64).reshape(5, 5)
    oD, eD, oI, eI = sc["o_del"], sc["e_del"], sc["o_ins"], sc["e_ins"]
    Z = sc["zdrop"]
    wb = band_cap(Lq, sc)

    H = np.zeros((max(Lt, 1), Lq), dtype=np.int64)        # H(i, j)
    Enext = np.zeros((max(Lt, 1), Lq + 1), dtype=np.int64)  # E(i+1, j)
    LB = np.zeros(max(Lt, 1), dtype=np.int64)              # H(i, beg_i - 1)
    BEG = np.zeros(max(Lt, 1), dtype=np.int64)
    lw_kind = np.full(Lq + 1, INIT, dtype=np.int64)
    lw_row = np.full(Lq + 1, -1, dtype=np.int64)

    jj = np.arange(Lq + 1, dtype=np.int64)
    first_row = np.maximum(0, h0 - oI - eI * jj)  # H(-1, j-1) for j >= 1
    first_row[0] = h0

    def stored(idx):
        """(H, E) that the one-row buffer would hold at the indices idx."""
        idx = np.asarray(idx, dtype=np.int64)
        kind, r = lw_kind[idx], lw_row[idx]
        rr = np.maximum(r, 0)
        left = np.maximum(idx - 1, 0)
        h_prev = H[rr, np.minimum(left, Lq - 1)] if Lq else np.zeros(len(idx), np.int64)
        first = idx == BEG[rr]
        # before cell j of row r the buffer got H(r, j-1), or the row's left
        # boundary when j was the band's first column; the right-edge write
        # of row r stores H(r, end_r - 1), or the left boundary if the band
        # was empty
        h_cell = np.where(first | (idx < BEG[rr]), LB[rr], h_prev)
        hv = np.where(kind == INIT, first_row[idx], h_cell)
        ev = np.where(kind == CELL, Enext[rr, idx], 0)
        return hv, ev

    best, bi, bj = h0, -1, -1
    gbest, gi, moff = -1, -1, 0
    beg, end = 0, Lq
    rows, stop, cells = 0, 0, 0
    for i in range(Lt):
        rows += 1
        beg = max(beg, i - wb)
        end = min(end, i + wb + 1, Lq)
        BEG[i] = beg
        if trace is not None:
            trace.append((beg, end))
        LB[i] = max(0, h0 - oD - eD * (i + 1)) if beg == 0 else 0
        if end > beg:
            cells += end - beg
            cols = np.arange(beg, end)
            d, e = stored(cols)
            M = np.where(d > 0, d + S[t[i], q[beg:end]], 0)
            # closed-form F (exclusive prefix max of u(k))
            u = M - oI - eI + eI * cols
            pref = np.maximum.accumulate(u)
            excl = np.concatenate(([np.iinfo(np.int64).min // 4], pref[:-1]))
            F = np.maximum(0, excl - eI * (cols - 1))
            h = np.maximum(M, np.maximum(e, F))
            H[i, beg:end] = h
            Enext[i, beg:end] = np.maximum(0, np.maximum(e - eD, M - oD - eD))
            m = int(h.max())
            mj = int(beg + (len(h) - 1 - np.argmax(h[::-1])))
            hl = int(h[-1])
        else:
            m, mj, hl = 0, -1, int(LB[i])
        lw_kind[beg:end] = CELL
        lw_row[beg:end] = i
        lw_kind[end] = RIGHT
        lw_row[end] = i
        if max(beg, end) == Lq:
            if hl >= gbest:
                gi = i
            gbest = max(gbest, hl)
        if m == 0:
            stop = 1
            break
        if m > best:
            best, bi, bj = m, i, mj
            moff = max(moff, abs(mj - i))
        elif Z > 0:
            drift = (i - bi) - (mj - bj)
            drop = best - m - (drift * eD if drift > 0 else -drift * eI)
            if drop > Z:
                stop = 2
                break
        # the row had a positive cell, so its band was not empty
        assert end > beg
        span = np.arange(beg, end + 1)
        hv, ev = stored(span)
        nonempty = (hv != 0) | (ev != 0)
        inside = np.nonzero(nonempty[:-1])[0]      # indices beg .. end-1
        newbeg = beg + int(inside[0]) if len(inside) else end
        tail = np.nonzero(nonempty[newbeg - beg:])[0]  # indices newbeg .. end
        last = newbeg + int(tail[-1]) if len(tail) else newbeg - 1
        beg = newbeg
        end = min(last + 2, Lq)
    return ((best, bj + 1, bi + 1, gi + 1, gbest, moff), (rows, stop, cells))
