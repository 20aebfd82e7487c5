"""Pins of the suffix-array lookup reference (oracle.sal) and of the suffix
arrays and intervals the input generator builds for it."""
import os

import numpy as np
import pytest

from oracle import sal
from paper_1907_12931_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fm_example.txt")


def codes(s):
    return np.array(["ACGT".index(c) for c in s], dtype=np.uint8)


def golden_rows():
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            ref, pat, a, b = line.split()
            yield ref, pat, int(a), int(b)


def test_paper_example_interval_and_lookup():
    """The paper's example: AC occupies rows [1,2] of ATACGAC$'s BW matrix;
    Eq. (1) over those rows gives the two places AC starts in R."""
    for ref, pat, a, b in golden_rows():
        S = sal.suffix_array_by_rotations(codes(ref))
        k, s = sal.sa_interval(S, codes(ref), codes(pat))
        assert (k, k + s - 1) == (a, b)
        iv = np.zeros(1, dtype=synth.SA_INTERVAL)
        iv[0] = (k, s)
        off, out = sal.lookup(S, iv)
        assert list(off) == [0, 2]
        assert sorted(out.tolist()) == [i for i in range(len(ref)) if ref.startswith(pat, i)]


def test_example_suffix_array_by_hand():
    """Suffixes of ATACGAC$ sorted by hand: $ (7), AC$ (5), ACGAC$ (2),
    ATACGAC$ (0), C$ (6), CGAC$ (3), GAC$ (4), TACGAC$ (1)."""
    assert sal.suffix_array_by_rotations(codes("ATACGAC")).tolist() == [7, 5, 2, 0, 6, 3, 4, 1]


@pytest.mark.parametrize("seed", range(6))
def test_lookup_finds_every_occurrence(seed):
    """Brute force: the interval of a pattern, looked up, lists exactly the
    positions where a direct comparison finds the pattern."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 120))
    r = rng.integers(0, 4 if seed % 2 else 2, n).astype(np.uint8)
    S = sal.suffix_array_by_rotations(r)
    text = sal.to_text(r)
    for _ in range(20):
        L = int(rng.integers(1, 6))
        p = int(rng.integers(0, n - L + 1))
        pat = r[p:p + L]
        k, s = sal.sa_interval(S, r, pat)
        iv = np.zeros(1, dtype=synth.SA_INTERVAL)
        iv[0] = (k, s)
        _, out = sal.lookup(S, iv)
        want = [i for i in range(n) if text.startswith(sal.to_text(pat), i)]
        assert sorted(out.tolist()) == want and s == len(want)


def test_suffix_array_invariants():
    rng = np.random.default_rng(7)
    r = rng.integers(0, 4, 200).astype(np.uint8)
    S = sal.suffix_array_by_rotations(r)
    assert sorted(S.tolist()) == list(range(201)) and S[0] == 200
    t = sal.to_text(r) + "$"
    assert all(t[S[i]:] < t[S[i + 1]:] for i in range(200))


@pytest.mark.parametrize("kind", ["random", "periodic", "repeats", "binary"])
def test_generator_suffix_array_matches_the_definition(kind):
    rng = np.random.default_rng({"random": 1, "periodic": 2, "repeats": 3, "binary": 4}[kind])
    for _ in range(8):
        n = int(rng.integers(1, 400))
        if kind == "random":
            r = rng.integers(0, 4, n)
        elif kind == "periodic":
            r = np.tile(rng.integers(0, 4, int(rng.integers(1, 6))), n)[:n]
        elif kind == "binary":
            r = rng.integers(0, 2, n)
        else:
            r = synth.repeat_reference(max(n, 450), int(rng.integers(1 << 30)),
                                       repeat_frac=0.5, copies=(2, 5), length=(30, 60))
        r = np.asarray(r, dtype=np.uint8)
        assert np.array_equal(synth.suffix_array(r), sal.suffix_array_by_rotations(r))


def test_generator_intervals_match_the_definition():
    w = synth.sa_workload(ref_len=1500, n_iv=60, seed=8)
    assert np.array_equal(w["sa"], sal.suffix_array_by_rotations(w["text"]))
    for m in range(60):
        p, L = int(w["pattern_pos"][m]), int(w["pattern_len"][m])
        k, s = sal.sa_interval(w["sa"], w["text"], w["text"][p:p + L])
        assert (int(w["iv"][m]["k"]), int(w["iv"][m]["s"])) == (k, s)
    # repeats give intervals of more than one row
    assert (w["iv"]["s"] > 1).any()


def test_bisection_interval_equals_row_by_row():
    rng = np.random.default_rng(40)
    for n in (1, 7, 60, 300):
        r = rng.integers(0, 4 if n % 2 else 2, n).astype(np.uint8)
        S = sal.suffix_array_by_rotations(r)
        txt = sal.to_text(r) + "$"
        for _ in range(30):
            L = int(rng.integers(1, 7))
            pat = rng.integers(0, 4, L).astype(np.uint8)
            if rng.random() < 0.6 and n >= L:
                p = int(rng.integers(0, n - L + 1))
                pat = r[p:p + L]
            assert sal.sa_interval_sorted(S, txt, sal.to_text(pat)) == sal.sa_interval(S, r, pat)
