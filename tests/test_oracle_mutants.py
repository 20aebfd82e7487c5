"""Planted mistakes in the oracle must be caught by the pins.

Each mutant is a one-line textual change to a private copy of
oracle/bsw_ref.c (a dropped term, a wrong tie rule, a transposed operand
...), compiled into a temporary library.  The pins (hand traces, closed
forms, brute-force path enumeration and the full-matrix model) are run
against it, and at least one must disagree.  This shows that the pins, not
the oracle, fix the semantics.

Not listed: dropping the E = 0 store at the right band edge.  That mutant
is equivalent: E is 0 at every index at or past the band end when a row
starts (true initially; a row only writes E inside its band; the shrink
only pulls the end back over indices whose H and E are both 0; and the
end grows by at most two, onto indices never written since), so the store
never changes a value.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import brute, model2d
from paper_1907_12931_amd import synth

from test_oracle_pins import load_traces, random_scoring

MUTANTS = [
    ("gap open without extend (E)", "ebuf[j] = imax(imax(e - p->e_del, mdiag - p->o_del - p->e_del), 0);",
     "ebuf[j] = imax(imax(e - p->e_del, mdiag - p->o_del), 0);"),
    ("row tie to smaller column", "if (h >= m) mj = j;", "if (h > m) mj = j;"),
    ("no positive-diagonal gate", "mdiag = d > 0 ? d + srow[q[j]] : 0;",
     "mdiag = d + srow[q[j]];"),
    ("insertions open from H", "mdiag - p->o_ins - p->e_ins), 0)",
     "h - p->o_ins - p->e_ins), 0)"),
    ("deletions open from H", "mdiag - p->o_del - p->e_del), 0)",
     "h - p->o_del - p->e_del), 0)"),
    ("band end +1", "end = imin(j + 2, qlen);", "end = imin(j + 1, qlen);"),
    ("right edge H zeroed", "hbuf[end] = hl;", "hbuf[end] = 0;"),
    ("z-drop without drift", "drop = best - m - drift * p->e_del;",
     "drop = best - m;"),
    ("query-end tie to earlier row", "if (hl >= gbest) gi = i;",
     "if (hl > gbest) gi = i;"),
    ("transposed score matrix", "d + srow[q[j]]", "d + p->mat[q[j] * 5 + t[i]]"),
    ("first row uses deletion costs", "h0 - p->o_ins - p->e_ins * j",
     "h0 - p->o_del - p->e_del * j"),
    ("band cap ignores end bonus", "num = qlen * a + p->end_bonus - p->o_ins;",
     "num = qlen * a - p->o_ins;"),
    ("first column off by one", "h0 - p->o_del - p->e_del * (i + 1)",
     "h0 - p->o_del - p->e_del * i"),
    ("max_off on ties too", "moff = imax(moff, abs(mj - i));\n    } else",
     "moff = imax(moff, abs(mj - i));\n    } if (m == best) moff = imax(moff, abs(mj - i)); if (0) {} else"),
]


def build_mutant(tmp_path, old, new):
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "m.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "m.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-D_POSIX_C_SOURCE=200809L",
                    "-I", oracle.HERE, "-shared", "-fPIC", "-o", str(lib),
                    str(path), "-lpthread"], check=True)
    L = ctypes.CDLL(str(lib))
    L.bsw_ref_extend_one.restype = ctypes.c_int
    L.bsw_ref_extend_one.argtypes = [
        ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
        ctypes.c_int32, ctypes.POINTER(oracle.Params), ctypes.c_void_p,
        ctypes.c_void_p]

    def ext(q, t, h0, sc):
        q = np.ascontiguousarray(np.asarray(q, dtype=np.uint8))
        t = np.ascontiguousarray(np.asarray(t, dtype=np.uint8))
        out = np.zeros(1, dtype=oracle.RESULT_DTYPE)
        dg = np.zeros(1, dtype=oracle.DIAG_DTYPE)
        p = oracle.make_params(sc)
        L.bsw_ref_extend_one(len(q), q.ctypes.data if len(q) else None, len(t),
                             t.ctypes.data if len(t) else None, int(h0),
                             ctypes.byref(p), out.ctypes.data, dg.ctypes.data)
        return (tuple(int(out[0][k]) for k in oracle.RESULT_DTYPE.names),
                tuple(int(dg[0][k]) for k in oracle.DIAG_DTYPE.names))
    return ext


def pins_disagree(ext):
    """Name of the first pin the implementation ext fails, or None."""
    for q, t, h0, res, dg in load_traces():
        if ext(q, t, h0, synth.BWA_DEFAULT) != (res, dg):
            return "hand trace"
    rng = np.random.default_rng(0)
    for _ in range(60):
        L = int(rng.integers(1, 60))
        q = rng.integers(0, 4, L)
        t = np.concatenate([q, rng.integers(0, 4, int(rng.integers(0, 30)))])
        h0 = int(rng.integers(1, 60))
        v = h0 + L
        if ext(q, t, h0, dict(synth.BWA_DEFAULT, w=int(rng.integers(0, 70))))[0] \
                != (v, L, L, L, v, 0):
            return "identical sequences"
    for Lq in (3, 40):
        for h0 in range(13, Lq + 11):
            res, (rows, stop, _) = ext([0] * Lq, [1] * (h0 + 5), h0, synth.BWA_DEFAULT)
            if res[:3] != (h0, 0, 0) or stop != 1 or rows != h0 - 9:
                return "all mismatch"
    for _ in range(400):
        lq, lt = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        sc = random_scoring(rng, lq, lt)
        alpha = int(rng.integers(2, 6))
        q, t = rng.integers(0, alpha, lq), rng.integers(0, alpha, lt)
        h0 = int(rng.integers(200, 400))
        if ext(q, t, h0, sc)[0] != brute.extend(q, t, h0, sc):
            return "brute force"
    # cheap gaps and costly mismatches: a deletion next to an insertion
    # would beat a mismatch if the model allowed it
    for _ in range(300):
        lq, lt = int(rng.integers(2, 6)), int(rng.integers(2, 6))
        sc = brute.heuristic_free_scoring(
            synth.scoring(match=int(rng.integers(2, 5)), mismatch=-6, o=0, e=1,
                          o_ins=int(rng.integers(0, 2))), lq, lt)
        q, t = rng.integers(0, 4, lq), rng.integers(0, 4, lt)
        if ext(q, t, 300, sc)[0] != brute.extend(q, t, 300, sc):
            return "brute force (cheap gaps)"
    scs = [synth.scoring(w=3, zdrop=0, end_bonus=0),
           synth.scoring(w=8, zdrop=30, end_bonus=0), synth.BWA_DEFAULT]
    for _ in range(300):
        lq = int(rng.integers(5, 50))
        q = rng.integers(0, 4, lq)
        t = np.concatenate([q[: int(rng.integers(0, lq))],
                            rng.integers(0, 4, int(rng.integers(5, 40)))])
        if rng.random() < 0.5:
            t = np.concatenate([t[:5], t[5 + int(rng.integers(1, 4)):]])
        h0 = int(rng.integers(20, 200))
        sc = scs[int(rng.integers(0, len(scs)))]
        if ext(q, t, h0, sc) != model2d.extend(q, t, h0, sc):
            return "2D model"
    return None


def test_real_oracle_passes_all_pins(oracle_lib, tmp_path):
    assert pins_disagree(build_mutant(tmp_path, "return w;", "return w;")) is None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(oracle_lib, tmp_path, name, old, new):
    assert pins_disagree(build_mutant(tmp_path, old, new)) is not None, name
