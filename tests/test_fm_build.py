"""The library's FM-index builder (bsw_fm_build, host code) against the
definitions of oracle.fm: every O(c, t) read from the 64-byte entries as
Algorithm 1 reads them equals a direct count over the BWT."""
import ctypes

import numpy as np
import pytest

from oracle import fm, sal
from paper_1907_12931_amd import synth


def both_strands(rng, n):
    r = rng.integers(0, 4, n).astype(np.uint8)
    return np.concatenate([r, synth.revcomp(r)])


def occ_from_entries(entries, c, t):
    if t < 0:
        return 0
    e = entries[t // 32]
    return int(e["count"][c]) + int(np.count_nonzero(e["bwt"][:t % 32 + 1] == c))


@pytest.mark.parametrize("n", [1, 15, 31, 32, 33, 100, 257])
def test_entries_give_the_occurrence_counts(n):
    from paper_1907_12931_amd import bsw
    rng = np.random.default_rng(n)
    t = both_strands(rng, n)[:n]
    S = sal.suffix_array_by_rotations(t)
    entries, meta = bsw.fm_build(t, S)
    b = fm.bwt(t, S)
    assert meta.rows == n + 1 and meta.entries == (n + 32) // 32 == len(entries)
    assert list(meta.C) == [1 + int(np.count_nonzero(t < c)) for c in range(4)]
    assert S[meta.primary] == 0 and b[meta.primary] == 4
    for c in range(4):
        for x in range(-1, n + 1):
            assert occ_from_entries(entries, c, x) == fm.occ(b, c, x), (c, x)
    # past the last row the bytes never match a base
    tail = entries[-1]["bwt"][(n + 1) % 32:] if (n + 1) % 32 else []
    assert all(v == 5 for v in tail)


def test_rejects_bad_inputs():
    from paper_1907_12931_amd import bsw
    t = np.array([0, 1, 2, 3], dtype=np.uint8)
    S = sal.suffix_array_by_rotations(t)
    with pytest.raises(bsw.BswError):
        bsw.fm_build(np.array([0, 1, 5, 3], dtype=np.uint8), S)
    bad = S.copy()
    bad[1] = bad[2]
    with pytest.raises(bsw.BswError):
        bsw.fm_build(t, bad)


def test_layout_matches_header():
    from paper_1907_12931_amd import bsw
    assert bsw.FM_ENTRY_DTYPE.itemsize == 64 and bsw.BI_INTERVAL_DTYPE.itemsize == 32
    assert ctypes.sizeof(bsw.FmMeta) == 56
