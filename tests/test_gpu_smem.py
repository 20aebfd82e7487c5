"""Parity of the SMEM search (bsw_fm_smem_device) with the CPU reference
oracle.fm.smems (SMEMs from their definition) on seeded reads over texts of
both strands; edge cases and error paths."""
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


def run(bsw, ctx, E, meta, reads, off, max_len=None, async_=False):
    import torch
    off = np.asarray(off, dtype=np.uint64)
    n = len(off) - 1
    L = np.diff(off.astype(np.int64))
    if max_len is None:
        max_len = int(L.max()) if n else 0
    out = torch.full((max(int(off[-1] - off[0]), 0) * 32,), 0x33, dtype=torch.uint8,
                     device="cuda")
    counts = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ctx.fm_smem_device(E, meta, torch.from_numpy(np.ascontiguousarray(reads, np.uint8)).cuda(),
                       torch.from_numpy(off.view(np.int64)).cuda(), max_len, out, counts,
                       async_=async_)
    if async_:
        ctx.wait()
    o = out.cpu().numpy().view(bsw.SMEM_DTYPE)
    c = counts.cpu().numpy()
    return [[tuple(int(v) for v in o[int(off[r] - off[0]) + j]) for j in range(c[r])]
            for r in range(n)]


def reference(w, reads, off, idx):
    from oracle import fm, sal
    txt = sal.to_text(w["text"]) + "$"
    return [[tuple(x) for x in fm.smems(w["text"], w["sa"], reads[off[r]:off[r + 1]], txt)]
            for r in idx]


@pytest.fixture(scope="module")
def small(bsw):
    import torch
    w = synth.sa_workload(ref_len=40_000, n_iv=10, seed=51)
    entries, meta = bsw.fm_build(w["text"], w["sa"])
    return w, torch.from_numpy(entries.view(np.uint8)).cuda(), meta


@pytest.mark.parametrize("async_", [False, True])
def test_matches_reference(bsw, ctx, small, async_):
    w, E, meta = small
    reads, off = synth.fm_patterns(w["text"], 600, seed=52, length=(60, 151), p_sub=0.03,
                                   p_n=0.005)
    got = run(bsw, ctx, E, meta, reads, off, async_=async_)
    want = reference(w, reads, off, range(600))
    assert got == want
    print("reads", 600, "smems", sum(len(x) for x in got), flush=True)
    assert ctx.last_cells() > 0


def test_edge_cases(bsw, ctx, small):
    w, E, meta = small
    t = w["text"]
    rs = [np.zeros(0, np.uint8), np.full(30, 4, np.uint8), t[1000:1151],
          t[len(t) // 2 - 70:len(t) // 2 + 70],                     # across the strand junction
          np.concatenate([t[5:40], [4], t[40:90]]).astype(np.uint8),
          np.tile(np.uint8(3), 40), t[:1], np.array([4, 0, 4], np.uint8)]
    off = np.zeros(len(rs) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rs])
    reads = np.concatenate(rs).astype(np.uint8)
    got = run(bsw, ctx, E, meta, reads, off)
    assert got == reference(w, reads, off, range(len(rs)))
    assert got[0] == [] and got[1] == [] and got[2] == [(0, 151) + got[2][0][2:]]


def test_errors_write_nothing(bsw, ctx, small):
    w, E, meta = small
    reads, off = synth.fm_patterns(w["text"], 40, seed=53, length=(100, 100))
    with pytest.raises(bsw.BswError) as ei:
        run(bsw, ctx, E, meta, reads, off, max_len=99)
    assert "read 0" in str(ei.value)
    r2 = reads.copy()
    r2[int(off[5]) + 7] = 8
    with pytest.raises(bsw.BswError) as ei:
        run(bsw, ctx, E, meta, r2, off)
    assert "read 5" in str(ei.value)
    assert run(bsw, ctx, E, meta, reads, off) == reference(w, reads, off, range(40))


def test_bench_size_sampled(bsw, ctx):
    """The benchmark's reads (500,000 of 151 bases) over the 64 Mbase
    two-strand text, checked on a seeded sample of reads."""
    import torch
    w = synth.sa_workload(**synth.SA_BENCH)
    print("built", len(w["sa"]), flush=True)
    entries, meta = bsw.fm_build(w["text"], w["sa"])
    E = torch.from_numpy(entries.view(np.uint8)).cuda()
    reads, off = synth.fm_patterns(w["text"], synth.SMEM_BENCH_READS, seed=54,
                                   length=(151, 151), p_sub=0.02, p_n=0.005)
    got = run(bsw, ctx, E, meta, reads, off)
    idx = np.sort(np.random.default_rng(55).choice(len(off) - 1, 300, replace=False))
    assert [got[r] for r in idx] == reference(w, reads, off, idx)
