"""Pins of the FM-index reference (oracle.fm): the paper's index example,
brute-force occurrence counts and ranks, and the identities that backward
extension (Sec. 4.2) rests on, checked on texts of both strands."""
import numpy as np
import pytest

from oracle import fm, sal
from paper_1907_12931_amd import synth


def codes(s):
    return np.array(["ACGT".index(c) for c in s], dtype=np.uint8)


def test_paper_example_bwt_by_hand():
    """R = ATACGAC: S = 7 5 2 0 6 3 4 1, so B = C G T $ A A C A (the base
    before each sorted suffix; $ before the whole text)."""
    r = codes("ATACGAC")
    S = sal.suffix_array_by_rotations(r)
    assert "".join("ACGT$"[c] for c in fm.bwt(r, S)) == "CGT$AACA"
    b = fm.bwt(r, S)
    assert [fm.occ(b, 0, t) for t in range(-1, 8)] == [0, 0, 0, 0, 0, 1, 2, 2, 3]


def both_strands(rng, n, alphabet=4):
    r = rng.integers(0, alphabet, n).astype(np.uint8)
    return np.concatenate([r, fm.revcomp(r)])


@pytest.mark.parametrize("seed", range(4))
def test_interval_counts_and_ranks_by_brute_force(seed):
    """s = occurrences of X in T (direct comparison); k = number of suffixes
    of T$ smaller than X; l = the same for revcomp(X)."""
    rng = np.random.default_rng(seed)
    t = both_strands(rng, int(rng.integers(10, 60)), 4 if seed % 2 else 2)
    S = sal.suffix_array_by_rotations(t)
    txt = sal.to_text(t) + "$"
    for _ in range(25):
        L = int(rng.integers(1, 6))
        p = int(rng.integers(0, len(t) - L + 1))
        x = t[p:p + L]
        k, l, s = fm.bi_interval(t, S, x)
        xs, rs = sal.to_text(x), sal.to_text(fm.revcomp(x))
        assert s == sum(txt.startswith(xs, i) for i in range(len(txt)))
        assert k == sum(txt[i:] < xs for i in range(len(txt)))
        assert l == sum(txt[i:] < rs for i in range(len(txt)))


@pytest.mark.parametrize("seed", range(4))
def test_backward_extension_identities(seed):
    """For every occurring X and base c: k(cX) = C(c) + O(c, k - 1) and
    s(cX) = O(c, k + s - 1) - O(c, k - 1), with C(c) the rows whose suffix
    starts below c; and l(cX) = l(X) + [the row of suffix 0 lies in X's
    interval] + the sizes of dX for every base d after c."""
    rng = np.random.default_rng(10 + seed)
    t = both_strands(rng, int(rng.integers(15, 50)))
    S = sal.suffix_array_by_rotations(t)
    b = fm.bwt(t, S)
    C = [1 + int(np.count_nonzero(t < c)) for c in range(4)]
    for _ in range(20):
        L = int(rng.integers(0, 5))
        p = int(rng.integers(0, len(t) - L + 1))
        x = t[p:p + L]
        k, l, s = fm.bi_interval(t, S, x) if L else (0, 0, len(S))
        prim = int(any(S[i] == 0 for i in range(k, k + s)))
        sizes = {}
        for c in range(4):
            cx = np.concatenate([[c], x]).astype(np.uint8)
            kc, lc, sc = fm.bi_interval(t, S, cx)
            sizes[c] = sc
            assert sc == fm.occ(b, c, k + s - 1) - fm.occ(b, c, k - 1)
            if sc:
                assert kc == C[c] + fm.occ(b, c, k - 1)
        for c in range(4):
            if sizes[c]:
                lc = fm.bi_interval(t, S, np.concatenate([[c], x]).astype(np.uint8))[1]
                assert lc == l + prim + sum(sizes[d] for d in range(c + 1, 4))


def test_backward_search_matched_length():
    rng = np.random.default_rng(20)
    t = both_strands(rng, 80)
    S = sal.suffix_array_by_rotations(t)
    txt = sal.to_text(t)
    for _ in range(40):
        q = rng.integers(0, 4, int(rng.integers(1, 12))).astype(np.uint8)
        if rng.random() < 0.5:
            p = int(rng.integers(0, len(t) - 8))
            q = np.concatenate([q, t[p:p + 8]]).astype(np.uint8)
        k, l, s, m = fm.backward_search(t, S, q)
        want = max(j for j in range(len(q) + 1) if sal.to_text(q[len(q) - j:]) in txt)
        assert m == want
        assert (s > 0) == (m == len(q))


@pytest.mark.parametrize("seed", range(5))
def test_smems_by_brute_force(seed):
    """Every occurring substring of the read is listed; the MEMs are those
    that occur and cannot grow by one base on either side, the SMEMs the
    MEMs no other MEM contains."""
    rng = np.random.default_rng(50 + seed)
    t = both_strands(rng, int(rng.integers(20, 70)), 2 if seed == 0 else 4)
    S = sal.suffix_array_by_rotations(t)
    txt = sal.to_text(t)
    for _ in range(15):
        p = int(rng.integers(0, len(t) - 20))
        x = t[p:p + int(rng.integers(1, 20))].copy()
        for j in rng.integers(0, len(x), int(rng.integers(0, 3))):
            x[j] = int(rng.integers(0, 5))
        xs = sal.to_text(x)
        occ = lambda a, b: a < b and "N" not in xs[a:b] and xs[a:b] in txt  # noqa: E731
        mems = [(a, b) for a in range(len(x)) for b in range(a + 1, len(x) + 1)
                if occ(a, b) and not (a > 0 and occ(a - 1, b))
                and not (b < len(x) and occ(a, b + 1))]
        want = sorted((a, b) for a, b in mems
                      if not any(c <= a and b <= d and (c, d) != (a, b) for c, d in mems))
        got = fm.smems(t, S, x)
        assert [(a, b) for a, b, *_ in got] == want
        for a, b, k, l, s in got:
            assert (k, l, s) == fm.bi_interval(t, S, x[a:b])
