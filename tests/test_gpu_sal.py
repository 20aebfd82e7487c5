"""Parity of the suffix-array lookup (bsw_sa_lookup_device) with the CPU
reference oracle.sal on seeded synthetic suffix arrays and intervals, plus
edge cases and error paths."""
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


def reference(sa, iv):
    from oracle import sal
    return sal.lookup(sa, iv)


def run(bsw, ctx, sa_dev, iv, cap=None, async_=False, sentinel=-5):
    import torch
    ivd = torch.from_numpy(np.ascontiguousarray(iv).view(np.uint8)).cuda()
    n = len(iv)
    if cap is None:
        cap = int(np.asarray(iv["s"], dtype=np.int64).sum())
    off = torch.full((n + 1,), sentinel, dtype=torch.int64, device="cuda")
    pos = torch.full((max(cap, 0),), sentinel, dtype=torch.int64, device="cuda")
    total = ctx.sa_lookup_device(sa_dev, ivd, off, pos, async_=async_)
    if async_:
        ctx.wait()
        total = int(off[-1].item())
    return total, off.cpu().numpy(), pos.cpu().numpy()


@pytest.fixture(scope="module")
def small(bsw):
    import torch
    w = synth.sa_workload(ref_len=20_000, n_iv=20_000, seed=31)
    return w, torch.from_numpy(w["sa"]).cuda()


def test_matches_reference(bsw, ctx, small):
    w, sa = small
    want_off, want = reference(w["sa"], w["iv"])
    total, off, pos = run(bsw, ctx, sa, w["iv"])
    print("intervals", len(w["iv"]), "coordinates", total, flush=True)
    assert total == len(want)
    assert np.array_equal(off, want_off) and np.array_equal(pos, want)
    t = ctx.last_timing()
    assert t[0] > 0 and t[2] > 0


@pytest.mark.parametrize("case", ["one", "tile", "empties", "whole", "none", "random_big",
                                  "sparse", "async"])
def test_edge_cases(bsw, ctx, small, case):
    w, sa = small
    rng = np.random.default_rng(32)
    iv = w["iv"]
    if case == "one":
        iv = iv[5:6].copy()
    elif case == "tile":
        iv = iv[:2048].copy()          # exactly one scan tile
    elif case == "empties":
        iv = iv[:4097].copy()          # two tiles and one more, with empty intervals
        iv["s"][::3] = 0
    elif case == "whole":
        iv = np.zeros(3, dtype=synth.SA_INTERVAL)
        iv[1] = (0, len(w["sa"]))
    elif case == "none":
        iv = np.zeros(9, dtype=synth.SA_INTERVAL)
    elif case == "random_big":
        iv = np.zeros(500, dtype=synth.SA_INTERVAL)
        iv["s"] = rng.integers(0, 3000, 500)
        iv["k"] = rng.integers(0, len(w["sa"]) - 3000, 500)
    elif case == "sparse":
        # tiles that span more intervals than the gather stages in LDS
        iv = w["iv"][:6000].copy()
        iv["s"][rng.random(6000) < 0.97] = 0
    want_off, want = reference(w["sa"], iv)
    total, off, pos = run(bsw, ctx, sa, iv, async_=case == "async")
    assert total == len(want)
    assert np.array_equal(off, want_off) and np.array_equal(pos[:total], want)


def test_errors_write_nothing(bsw, ctx, small):
    w, sa = small
    iv = w["iv"][:100].copy()
    iv[37] = (len(w["sa"]) - 1, 2)     # leaves the suffix array
    with pytest.raises(bsw.BswError) as ei:
        run(bsw, ctx, sa, iv, cap=10_000)
    assert ei.value.code == bsw.EINVAL and "interval 37" in str(ei.value)
    iv = w["iv"][:100].copy()
    need = int(iv["s"].astype(np.int64).sum())
    import torch
    ivd = torch.from_numpy(iv.view(np.uint8)).cuda()
    off = torch.full((101,), -5, dtype=torch.int64, device="cuda")
    pos = torch.full((need - 1,), -5, dtype=torch.int64, device="cuda")
    with pytest.raises(bsw.BswError) as ei:
        ctx.sa_lookup_device(sa, ivd, off, pos)
    assert ei.value.code == bsw.ETOOBIG and str(need) in str(ei.value)
    assert bool((off == -5).all()) and bool((pos == -5).all())
    # the context still works
    total, o, p = run(bsw, ctx, sa, iv)
    assert total == need


def test_bench_size_sampled(bsw, ctx):
    """The workload the benchmark times (a 64 Mbase indexed text, 4 M
    intervals), checked on a seeded sample of intervals."""
    import torch
    w = synth.sa_workload(**synth.SA_BENCH)
    print("built", len(w["sa"]), flush=True)
    sa = torch.from_numpy(w["sa"]).cuda()
    total, off, pos = run(bsw, ctx, sa, w["iv"])
    idx = np.sort(np.random.default_rng(33).choice(len(w["iv"]), 3000, replace=False))
    _, want = reference(w["sa"], w["iv"][idx])
    got = np.concatenate([pos[off[m]:off[m + 1]] for m in idx])
    assert np.array_equal(got, want)
    assert total == int(w["iv"]["s"].astype(np.int64).sum())
