"""The allocation-free entry point (bsw_extend_batch_device_noalloc) gives
the same results as the ordinary device entry point, call after call, with
its workspace in the library's fixed device array."""
import numpy as np
import pytest

from paper_1907_12931_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ("score", "qle", "tle", "gtle", "gscore", "max_off")


def test_noalloc_matches_device_entry_twice():
    import torch
    from paper_1907_12931_amd import bsw
    big = synth.batched_mix(n=bsw.NOALLOC_MAX_PAIRS, seed=91, workers=8)
    # the second call is smaller, with long and 16-bit pairs mixed in
    small = synth.read_scale(n=20_000, seed=92)
    rng = np.random.default_rng(93)
    extra = []
    for L in (300, 700, 257):
        qq = rng.integers(0, 4, L)
        extra.append((qq, np.concatenate([qq[:200], rng.integers(0, 4, 100)]), 40))
    for h0 in (300, 5000, 70000):
        qq = rng.integers(0, 4, 120)
        extra.append((qq, qq.copy(), h0))
    pairs = [synth.pair(small, k)[:3] for k in range(len(small["h0"]))] + extra
    small = synth.from_pairs(pairs, small["scorings"])
    with bsw.Context() as ref, bsw.Context() as na:
        for k, b in enumerate((big, small)):
            n = len(b["h0"])
            print(f"noalloc call {k}: {n} pairs", flush=True)
            dev = bsw.to_device(b)
            o1, d1 = bsw.alloc_outputs(n, with_diag=True)
            o2, d2 = bsw.alloc_outputs(n, with_diag=True)
            o2.fill_(0x77)
            torch.cuda.synchronize()
            ref.extend_device(dev, b["scorings"], o1, d1)
            na.extend_device_noalloc(dev, b["scorings"], o2, d2)
            r1, g1 = bsw.outputs_to_numpy(o1, d1)
            r2, g2 = bsw.outputs_to_numpy(o2, d2)
            for f in FIELDS:
                assert np.array_equal(r1[f], r2[f]), (k, f)
            for f in ("rows", "stop", "cells"):
                assert np.array_equal(g1[f], g2[f]), (k, f)
        # past the limit: refused before anything is enqueued
        b = synth.read_scale(n=bsw.NOALLOC_MAX_PAIRS + 1, seed=94, workers=8)
        dev = bsw.to_device(b)
        o, _ = bsw.alloc_outputs(len(b["h0"]))
        with pytest.raises(bsw.BswError) as ei:
            na.extend_device_noalloc(dev, b["scorings"], o)
        assert ei.value.code == bsw.ETOOBIG
