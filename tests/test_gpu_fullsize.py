"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (batched path, graph replay, autotuned shape): every pair of
the 4,000,000-pair uneven mix, the 1,000,000-pair read-scale batch and the
500,000-pair wide-band batch (32-bit values, two scoring sets), all six
result fields and the diagnostics compared with the oracle element by
element.  At these sizes every persistent workgroup of the busy classes
takes many tiles.  All calls go through the C ABI."""
import numpy as np
import pytest

from paper_1907_12931_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ("score", "qle", "tle", "gtle", "gscore", "max_off")


@pytest.fixture(scope="module")
def bsw():
    from paper_1907_12931_amd import bsw as m
    return m


def _check(bsw, oracle_lib, b, min_bits, label, tmp_path):
    import torch
    n = len(b["h0"])
    print(f"{label}: {n} pairs", flush=True)
    want, wdiag = oracle_lib.extend_batch(b, b["scorings"])
    dev = bsw.to_device(b)
    out, diag = bsw.alloc_outputs(n, with_diag=True)
    with bsw.Context(min_lane_bits=min_bits, tune_cache=str(tmp_path / "t.json")) as c:
        c.tune(dev, b["scorings"], out, reps=1)
        out.fill_(0x5A)
        diag.fill_(0x5A)
        torch.cuda.synchronize()
        for _ in range(2):  # capture, then replay
            c.extend_device(dev, b["scorings"], out, diag)
        got, gd = bsw.outputs_to_numpy(out, diag)
    for f in FIELDS:
        bad = np.nonzero(got[f] != want[f])[0]
        assert len(bad) == 0, f"{label}: {f} differs at {len(bad)} pairs, first {bad[:5]}"
    for f in ("rows", "stop", "cells"):
        bad = np.nonzero(gd[f] != wdiag[f])[0]
        assert len(bad) == 0, f"{label}: diag {f} differs at {len(bad)} pairs"


def test_batched_mix_full(bsw, oracle_lib, tmp_path):
    _check(bsw, oracle_lib, synth.batched_mix(workers=8), 0, "batched_mix 4M", tmp_path)


def test_read_scale_full(bsw, oracle_lib, tmp_path):
    _check(bsw, oracle_lib, synth.read_scale(workers=8), 0, "read_scale 1M", tmp_path)


def test_wide_band_full(bsw, oracle_lib, tmp_path):
    _check(bsw, oracle_lib, synth.wide_band(workers=8), 32, "wide_band 500k", tmp_path)
