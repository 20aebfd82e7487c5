"""Address- and undefined-behaviour-sanitizer builds of the host code.

* The CPU oracle (oracle/bsw_ref.c) built with -fsanitize=address,undefined
  into tests/sanitize/ref_driver.c runs a batch of synthetic pairs (every
  length class, empty sequences, several scoring sets, 8- and 16-bit lane
  forms); any sanitizer report fails the run, and its results must equal
  those of the ordinary oracle build.
* The host-only parts of the runtime (the serving arena, the input
  validation of the host-memory entry points and the tune cache format, in
  paper_1907_12931_amd/csrc/bsw_hostutil.h) run their checks in
  tests/sanitize/host_checks.cpp under the same sanitizers.
No GPU is involved."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1907_12931_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")


def compile_or_skip(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "asan" in r.stderr.lower() or "ubsan" in r.stderr.lower():
            pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
        raise AssertionError(r.stderr)


def run_checked(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=600)
    if "LeakSanitizer has encountered a fatal error" in r.stderr:
        # leak checking needs ptrace, which some containers forbid
        env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:exitcode=23")
        r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-3000:]
    return r


@pytest.fixture(scope="module")
def ref_driver(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path_factory.mktemp("san") / "ref_driver")
    compile_or_skip(["gcc", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-pthread", *SAN,
                     "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "bsw_ref.c"),
                     os.path.join(ROOT, "tests", "sanitize", "ref_driver.c"), "-o", exe])
    return exe


def write_batch(path, b, scorings):
    from oracle import Params, make_params
    n = len(b["h0"])
    params = (Params * len(scorings))(*[make_params(s) for s in scorings])
    pid = np.asarray(b.get("param_id", np.zeros(n, np.uint8)), np.uint8)
    with open(path, "wb") as f:
        f.write(np.int64(n).tobytes())
        f.write(np.int32(len(scorings)).tobytes())
        f.write(bytes(params))
        for a, dt in ((b["q_off"], np.uint64), (b["t_off"], np.uint64), (b["h0"], np.int32),
                      (pid, np.uint8)):
            f.write(np.ascontiguousarray(a, dtype=dt).tobytes())
        for s in (b["q"], b["t"]):
            s = np.ascontiguousarray(s, dtype=np.uint8)
            f.write(np.uint64(len(s)).tobytes())
            f.write(s.tobytes())


def read_out(path, n):
    import oracle
    raw = open(path, "rb").read()
    rc = int(np.frombuffer(raw[:4], np.int32)[0])
    bad = int(np.frombuffer(raw[4:12], np.int64)[0])
    o = 12
    res = np.frombuffer(raw[o:o + 24 * n], oracle.RESULT_DTYPE)
    o += 24 * n
    dg = np.frombuffer(raw[o:o + 16 * n], oracle.DIAG_DTYPE)
    o += 16 * n
    lanes = np.dtype([("rc", "<i4"), ("r", oracle.RESULT_DTYPE)])
    ln = np.frombuffer(raw[o:], lanes).reshape(-1, 2) if rc == 0 else None
    return rc, bad, res, dg, ln


def mixed_batch():
    """Pairs of every length class, empty query or target, two scoring sets
    (the second with unequal gaps, a narrow band and z-drop)."""
    rng = np.random.default_rng(31)
    parts = [synth.plain_small(400, seed=32), synth.batched_mix(600, seed=33)]
    qs, ts, h0 = [], [], []
    for p in parts:
        for k in range(len(p["h0"])):
            qs.append(p["q"][p["q_off"][k]:p["q_off"][k + 1]])
            ts.append(p["t"][p["t_off"][k]:p["t_off"][k + 1]])
            h0.append(int(p["h0"][k]))
    for lq, lt in ((0, 0), (0, 30), (30, 0), (1, 1), (300, 350)):
        qs.append(rng.integers(0, 5, lq).astype(np.uint8))
        ts.append(rng.integers(0, 5, lt).astype(np.uint8))
        h0.append(int(rng.integers(1, 60)))
    q_off = np.zeros(len(qs) + 1, np.uint64)
    t_off = np.zeros(len(ts) + 1, np.uint64)
    q_off[1:] = np.cumsum([len(x) for x in qs])
    t_off[1:] = np.cumsum([len(x) for x in ts])
    n = len(h0)
    return {"q": np.concatenate(qs), "q_off": q_off, "t": np.concatenate(ts), "t_off": t_off,
            "h0": np.asarray(h0, np.int32), "param_id": rng.integers(0, 2, n).astype(np.uint8)}


def test_oracle_under_sanitizers(ref_driver, tmp_path, oracle_lib):
    import oracle
    b = mixed_batch()
    scorings = [synth.BWA_DEFAULT, synth.scoring(2, -5, -2, 4, 2, w=30, zdrop=25, end_bonus=8)]
    scorings[1]["o_ins"], scorings[1]["e_ins"] = 3, 1
    write_batch(tmp_path / "in.bin", b, scorings)
    run_checked([ref_driver, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), "4"])
    n = len(b["h0"])
    rc, bad, res, dg, ln = read_out(tmp_path / "out.bin", n)
    assert rc == 0 and bad == -1
    want, wdg = oracle.extend_batch(b, scorings)
    assert np.array_equal(res, want) and np.array_equal(dg, wdg)
    # the lane forms against the ordinary build, on every pair whose h0 fits
    for k in range(0, n, 7):
        q = b["q"][b["q_off"][k]:b["q_off"][k + 1]]
        t = b["t"][b["t_off"][k]:b["t_off"][k + 1]]
        sc = scorings[b["param_id"][k]]
        for j, bits in enumerate((16, 8)):
            if b["h0"][k] > (1 << bits) - 1:
                assert ln[k, j]["rc"] == -100
                continue
            r, _ = oracle.extend_one(q, t, int(b["h0"][k]), sc, bits=bits)
            assert ln[k, j]["rc"] == 0
            assert tuple(int(x) for x in ln[k, j]["r"]) == r, (k, bits)


def test_oracle_rejects_bad_codes_under_sanitizers(ref_driver, tmp_path):
    b = mixed_batch()
    k = 777
    b["t"][b["t_off"][k + 1] - 1] = 7  # last target byte of pair k
    write_batch(tmp_path / "in.bin", b, [synth.BWA_DEFAULT, synth.BWA_DEFAULT])
    run_checked([ref_driver, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), "3"])
    rc, bad, *_ = read_out(tmp_path / "out.bin", len(b["h0"]))
    assert rc == -1 and bad == k


def test_host_runtime_parts_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not found")
    exe = str(tmp_path / "host_checks")
    compile_or_skip(["g++", "-std=c++17", *SAN, "-Wall",
                     os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"), "-o", exe])
    r = run_checked([exe, str(tmp_path)])
    assert r.stdout.strip() == "OK"
