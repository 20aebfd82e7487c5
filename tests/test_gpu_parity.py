"""GPU parity: every output field (and the diagnostics) of the HIP path
must equal the CPU oracle's, bit for bit, on the same seeded inputs.

All calls go through the C ABI (libbsw.so) via the ctypes binding.
"""
import numpy as np
import pytest

from paper_1907_12931_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ("score", "qle", "tle", "gtle", "gscore", "max_off")


@pytest.fixture(scope="module")
def bsw():
    from paper_1907_12931_amd import bsw as m
    return m


@pytest.fixture(scope="module")
def ctx(bsw):
    c = bsw.Context()
    yield c
    c.close()


def oracle_run(oracle_lib, batch):
    return oracle_lib.extend_batch(batch, batch["scorings"])


def assert_same(got, want, gdiag=None, wdiag=None, label=""):
    for f in FIELDS:
        bad = np.nonzero(got[f] != want[f])[0]
        assert len(bad) == 0, (
            f"{label}: field {f} differs at {len(bad)} pairs, first {bad[:5]}: "
            f"got {got[bad[:5]]} want {want[bad[:5]]}")
    if gdiag is not None:
        for f in ("rows", "stop", "cells"):
            bad = np.nonzero(gdiag[f] != wdiag[f])[0]
            assert len(bad) == 0, f"{label}: diag {f} differs at {bad[:5]}"


def edge_batch():
    """Degenerate and boundary pairs: empty query/target, single bases,
    identical, all-mismatch, N-rich, high h0 (wide values), long queries."""
    rng = np.random.default_rng(123)
    pairs = [([], [], 5), ([0, 1, 2], [], 9), ([], [0, 1], 10), ([0], [0], 1),
             ([0], [1], 1), ([4] * 10, [4] * 10, 20), ([0] * 40, [1] * 60, 25)]
    for L in (1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 1000):
        q = rng.integers(0, 4, L)
        pairs.append((q, np.concatenate([q, rng.integers(0, 4, 30)]), 30))
        pairs.append((q, rng.integers(0, 5, L + 17), 40))
    # values beyond 8 bits (h0 > 255) and beyond 16 bits (h0 > 65535)
    for h0 in (200, 250, 256, 300, 5000, 65000, 65600, 70000, 1 << 24):
        q = rng.integers(0, 4, 90)
        pairs.append((q, np.concatenate([q[:50], rng.integers(0, 4, 60)]), h0))
    return synth.from_pairs(pairs, [synth.BWA_DEFAULT])


def test_edge_cases(oracle_lib, ctx):
    b = edge_batch()
    want, wdiag = oracle_run(oracle_lib, b)
    got, gdiag = ctx.extend(b, with_diag=True)
    assert_same(got, want, gdiag, wdiag, "edge")


def test_hand_traces_on_gpu(ctx):
    from test_oracle_pins import load_traces
    cases = load_traces()
    b = synth.from_pairs([(q, t, h0) for q, t, h0, _, _ in cases], [synth.BWA_DEFAULT])
    got, gdiag = ctx.extend(b, with_diag=True)
    for k, (_, _, _, res, dg) in enumerate(cases):
        assert tuple(int(got[k][f]) for f in FIELDS) == res
        assert (int(gdiag[k]["rows"]), int(gdiag[k]["stop"]), int(gdiag[k]["cells"])) == dg


@pytest.mark.parametrize("min_bits", [0, 16, 32])
def test_plain_small_full(oracle_lib, bsw, min_bits):
    """1,000-pair workload, every pair, at every forced minimum width."""
    b = synth.plain_small()
    want, wdiag = oracle_run(oracle_lib, b)
    with bsw.Context(min_lane_bits=min_bits) as c:
        got, gdiag = c.extend(b, with_diag=True)
    assert_same(got, want, gdiag, wdiag, f"plain_small/{min_bits}")


@pytest.mark.parametrize("path", [0, 1])
def test_read_scale(oracle_lib, bsw, path):
    b = synth.read_scale(n=200_000)
    want, wdiag = oracle_run(oracle_lib, b)
    with bsw.Context(path=path) as c:
        got, gdiag = c.extend(b, with_diag=True)
    assert_same(got, want, gdiag, wdiag, f"read_scale/path{path}")


def test_batched_mix(oracle_lib, ctx):
    b = synth.batched_mix(n=300_000)
    want, wdiag = oracle_run(oracle_lib, b)
    got, gdiag = ctx.extend(b, with_diag=True)
    assert_same(got, want, gdiag, wdiag, "batched_mix")


def test_wide_band(oracle_lib, bsw):
    b = synth.wide_band(n=20_000)
    want, wdiag = oracle_run(oracle_lib, b)
    with bsw.Context(min_lane_bits=32) as c:
        got, gdiag = c.extend(b, with_diag=True)
    assert_same(got, want, gdiag, wdiag, "wide_band")


def test_order_and_path_invariance(ctx, bsw):
    """Results do not depend on batch order or on the execution path."""
    b = synth.batched_mix(n=50_000, seed=77)
    base = ctx.extend(b)
    perm = np.random.default_rng(1).permutation(len(b["h0"]))
    shuffled = ctx.extend(synth.subset(b, perm))
    assert np.array_equal(shuffled, base[perm])
    with bsw.Context(path=bsw.PATH_PLAIN) as c:
        assert np.array_equal(c.extend(b), base)
    with bsw.Context(min_lane_bits=32) as c:
        assert np.array_equal(c.extend(b), base)


def test_device_api_matches_host_api(ctx, bsw):
    import torch
    b = synth.read_scale(n=30_000, seed=9)
    host = ctx.extend(b)
    dev = bsw.to_device(b)
    out, diag = bsw.alloc_outputs(len(b["h0"]), with_diag=True)
    ctx.extend_device(dev, b["scorings"], out, diag)
    got = bsw.outputs_to_numpy(out)
    assert np.array_equal(got, host)
    # asynchronous form on a torch stream
    s = torch.cuda.Stream()
    out2, _ = bsw.alloc_outputs(len(b["h0"]))
    ctx.extend_device(dev, b["scorings"], out2, stream=s, async_=True)
    ctx.wait()
    assert np.array_equal(bsw.outputs_to_numpy(out2), host)


def test_invalid_pairs_rejected(ctx, bsw):
    b = synth.plain_small(n=100)
    bad = dict(b)
    bad["h0"] = b["h0"].copy()
    bad["h0"][37] = 0
    with pytest.raises(bsw.BswError) as ei:
        ctx.extend(bad)
    assert ei.value.code == bsw.EINVAL and "37" in str(ei.value)
    # device path: a bad code is found on the device; nothing is written
    bad = dict(b)
    bad["q"] = b["q"].copy()
    bad["q"][int(b["q_off"][55]) + 3] = 9
    dev = bsw.to_device(bad)
    out, _ = bsw.alloc_outputs(100)
    out.fill_(0xAB)
    with pytest.raises(bsw.BswError) as ei:
        ctx.extend_device(dev, b["scorings"], out)
    assert ei.value.code == bsw.EINVAL and "55" in str(ei.value)
    assert bool((out == 0xAB).all())


def test_empty_batch(ctx):
    b = synth.from_pairs([], [synth.BWA_DEFAULT])
    assert len(ctx.extend(b)) == 0


def test_eight_bit_speculation_boundaries(oracle_lib, ctx):
    """Pairs whose score bound exceeds 8 bits start in 8-bit records and are
    rerun with 16-bit records when their best score shows a stored value may
    have overflowed.  Scores straddling 255, seeds near 255, and a scoring
    whose match exceeds the gap-open cost (so E can exceed the best score)
    must all come out exact."""
    rng = np.random.default_rng(31)
    scs = [synth.BWA_DEFAULT, synth.scoring(match=5, mismatch=-2, o=0, e=1),
           synth.scoring(match=3, mismatch=-1, o=1, e=1, w=40)]
    pairs, pids = [], []
    for _ in range(6000):
        L = int(rng.integers(1, 257))
        q = rng.integers(0, 4, L)
        keep = int(rng.integers(0, L + 1))
        t = np.concatenate([q[:keep], rng.integers(0, 5, int(rng.integers(0, 80)))])
        h0 = int(rng.choice([int(rng.integers(1, 60)), int(rng.integers(150, 300))]))
        pairs.append((q, t, h0))
        pids.append(int(rng.integers(0, len(scs))))
    b = synth.from_pairs(pairs, scs, param_id=pids)
    want, wdiag = oracle_run(oracle_lib, b)
    got, gdiag = ctx.extend(b, with_diag=True)
    assert_same(got, want, gdiag, wdiag, "speculation")
    assert (want["score"] > 255).sum() > 500  # the rerun path is exercised


@pytest.mark.parametrize("w,zdrop,asym", [(3, 0, False), (20, 30, False), (40, 60, True),
                                           (7, 0, True)])
def test_narrow_bands_long_queries(oracle_lib, ctx, w, zdrop, asym):
    """Long queries with narrow bands: the 8-bit kernels keep the row buffer
    in a ring sized from w; the ring must never alias a live column, for
    symmetric and asymmetric gap costs."""
    b = synth.batched_mix(n=30_000, seed=40 + w)
    ql = np.diff(b["q_off"].astype(np.int64))
    b = synth.subset(b, np.nonzero(ql > 96)[0])
    sc = (synth.scoring(match=2, mismatch=-3, o=4, e=2, o_ins=7, e_ins=1, w=w, zdrop=zdrop)
          if asym else synth.scoring(w=w, zdrop=zdrop))
    b["scorings"] = [sc]
    want, wdiag = oracle_run(oracle_lib, b)
    got, gdiag = ctx.extend(b, with_diag=True)
    assert_same(got, want, gdiag, wdiag, f"narrow w={w}")
