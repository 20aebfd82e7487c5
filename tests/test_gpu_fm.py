"""Parity of the FM-index backward search (bsw_fm_backward_search_device)
with the CPU reference oracle.fm on seeded texts of both strands; edge
cases and error paths."""
import numpy as np
import pytest

from paper_1907_12931_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bsw():
    from paper_1907_12931_amd import bsw as b
    return b


@pytest.fixture(scope="module")
def ctx(bsw):
    with bsw.Context() as c:
        yield c


def upload(bsw, w):
    import torch
    entries, meta = bsw.fm_build(w["text"], w["sa"])
    return torch.from_numpy(entries.view(np.uint8)).cuda(), meta


def search(bsw, ctx, E, meta, pat, off, async_=False):
    import torch
    n = len(off) - 1
    out = torch.full((n * 32,), 0x77, dtype=torch.uint8, device="cuda")
    ctx.fm_backward_search_device(
        E, meta, torch.from_numpy(np.ascontiguousarray(pat, dtype=np.uint8)).cuda(),
        torch.from_numpy(np.asarray(off, dtype=np.uint64).view(np.int64)).cuda(), out,
        async_=async_)
    if async_:
        ctx.wait()
    return out.cpu().numpy().view(bsw.BI_INTERVAL_DTYPE)


def reference(w, pat, off, idx=None):
    from oracle import fm, sal
    txt = sal.to_text(w["text"]) + "$"
    idx = range(len(off) - 1) if idx is None else idx
    return [fm.backward_search(w["text"], w["sa"], pat[off[m]:off[m + 1]], txt) for m in idx]


def assert_same(got, want, idx=None):
    idx = range(len(want)) if idx is None else idx
    for j, m in enumerate(idx):
        g = got[m]
        assert (int(g["k"]), int(g["l"]), int(g["s"]), int(g["matched"])) == want[j], (m, g, want[j])


@pytest.fixture(scope="module")
def small(bsw):
    w = synth.sa_workload(ref_len=30_000, n_iv=10, seed=41)
    return w, upload(bsw, w)


@pytest.mark.parametrize("async_", [False, True])
def test_matches_reference(bsw, ctx, small, async_):
    w, (E, meta) = small
    pat, off = synth.fm_patterns(w["text"], 3000, seed=42, length=(1, 60), p_sub=0.01)
    got = search(bsw, ctx, E, meta, pat, off, async_)
    assert_same(got, reference(w, pat, off))
    full = got["matched"] == np.diff(off.astype(np.int64))
    print("patterns", len(off) - 1, "fully matched", int(full.sum()), flush=True)
    assert 0 < full.sum() < len(full)
    assert ctx.last_timing()[0] > 0


def test_edge_cases(bsw, ctx, small):
    w, (E, meta) = small
    t = w["text"]
    pats = [np.zeros(0, np.uint8),                       # empty: every row
            t[:1], t[-1:],                                # one base
            t[:200], t[len(t) // 2 - 100:len(t) // 2 + 100],  # across the strand junction
            np.array([4], np.uint8), np.concatenate([t[100:140], [4], t[140:160]]),  # N
            np.tile(np.uint8(0), 50)]                     # a run that does not occur
    off = np.zeros(len(pats) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in pats])
    pat = np.concatenate(pats).astype(np.uint8)
    got = search(bsw, ctx, E, meta, pat, off)
    assert_same(got, reference(w, pat, off))
    assert int(got[0]["s"]) == len(w["sa"])


def test_bad_offsets_and_codes(bsw, ctx, small):
    w, (E, meta) = small
    pat, off = synth.fm_patterns(w["text"], 50, seed=43)
    bad = off.copy()
    bad[10], bad[11] = bad[11], bad[10]
    with pytest.raises(bsw.BswError) as ei:
        search(bsw, ctx, E, meta, pat, bad)
    assert ei.value.code == bsw.EINVAL and "pattern 10" in str(ei.value)
    p2 = pat.copy()
    p2[int(off[7]) + 3] = 9
    with pytest.raises(bsw.BswError) as ei:
        search(bsw, ctx, E, meta, p2, off)
    assert "pattern 7" in str(ei.value)
    got = search(bsw, ctx, E, meta, pat, off)
    assert_same(got, reference(w, pat, off))


def test_bench_size_sampled(bsw, ctx):
    """The benchmark's index (the 64 Mbase two-strand text) and its 4 M
    32-base patterns, checked on a seeded sample."""
    w = synth.sa_workload(**synth.SA_BENCH)
    print("built", len(w["sa"]), flush=True)
    E, meta = upload(bsw, w)
    pat, off = synth.fm_patterns(w["text"], synth.FM_BENCH_PATTERNS, seed=44)
    got = search(bsw, ctx, E, meta, pat, off)
    idx = np.sort(np.random.default_rng(45).choice(len(off) - 1, 1500, replace=False))
    assert_same(got, reference(w, pat, off, idx), idx)
