"""Serving loop (bsw_server_*): per-request results must equal the oracle
and the same pairs run alone, whatever else is in flight; admission under
the device budget, oversize requests, a full queue, timeouts and a request
with a bad code must behave as documented.  All calls go through the C ABI.
"""
import threading

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
def pool(oracle_lib):
    """A batched-mix pool, its oracle results and request slices of it."""
    b = synth.batched_mix(n=150_000, seed=51)
    want, wdiag = oracle_lib.extend_batch(b, b["scorings"])
    return b, want, wdiag


def slices(batch, sizes):
    """Consecutive requests over a batch.  Each keeps the caller's offsets
    (not rebased to zero) into the shared sequence arrays."""
    out, a = [], 0
    n = len(batch["h0"])
    for s in sizes:
        s = int(min(s, n - a))
        if s <= 0:
            break
        r = {"q": batch["q"], "t": batch["t"],
             "q_off": batch["q_off"][a:a + s + 1], "t_off": batch["t_off"][a:a + s + 1],
             "h0": batch["h0"][a:a + s], "scorings": batch["scorings"]}
        out.append((a, s, r))
        a += s
    return out


def _same(got, want, label):
    for f in FIELDS:
        bad = np.nonzero(got[f] != want[f])[0]
        assert len(bad) == 0, f"{label}: {f} differs at {bad[:5]}"


def test_requests_equal_oracle_and_run_alone(bsw, pool):
    b, want, wdiag = pool
    sizes = synth.serving_requests(n_requests=40, seed=52, lo=500, hi=12_000)
    reqs = slices(b, sizes)
    with bsw.Server(b["scorings"], max_inflight=2) as srv:
        tickets = [(a, s, srv.submit(r, with_diag=True)) for a, s, r in reqs]
        for a, s, tk in tickets:
            got, gd = srv.wait(tk)
            _same(got, want[a:a + s], f"request at {a}")
            assert np.array_equal(gd["cells"], wdiag["cells"][a:a + s])
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["pairs"] == sum(s for _, s, _ in reqs)
    assert st["cells"] == int(sum(wdiag["cells"][a:a + s].sum() for a, s, _ in reqs))
    assert st["lat_p50_ms"] > 0 and st["lat_p99_ms"] >= st["lat_p50_ms"]
    # the same requests run alone through an ordinary context
    ctx = bsw.Context()
    for a, s, r in reqs[:6]:
        alone = ctx.extend(synth.subset(b, np.arange(a, a + s)))
        _same(alone, want[a:a + s], f"alone {a}")
    ctx.close()


def test_concurrent_submitters(bsw, pool):
    b, want, _ = pool
    reqs = slices(b, [3000] * 24)
    errors = []
    with bsw.Server(b["scorings"], max_inflight=3) as srv:
        def client(part):
            try:
                tks = [(a, s, srv.submit(r)) for a, s, r in part]
                for a, s, tk in tks:
                    _same(srv.wait(tk), want[a:a + s], f"client request {a}")
            except Exception as e:  # reported below
                errors.append(e)
        th = [threading.Thread(target=client, args=(reqs[i::4],)) for i in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
    assert not errors, errors[0]


def test_admission_under_small_budget(bsw, pool):
    b, want, _ = pool
    reqs = slices(b, [4000] * 12)
    # about two requests' data fit at a time; the rest wait in order
    with bsw.Server(b["scorings"], hbm_budget=3 << 20) as srv:
        tks = [(a, s, srv.submit(r)) for a, s, r in reqs]
        for a, s, tk in tks:
            _same(srv.wait(tk), want[a:a + s], f"request {a}")
        st = srv.stats(reset=True)
        assert st["completed"] == 12 and st["batches"] >= 3
        assert srv.stats()["completed"] == 0  # window reset


def test_oversize_request_and_full_queue(bsw, pool):
    b, want, _ = pool
    with bsw.Server(b["scorings"], hbm_budget=1 << 20, max_queued=1) as srv:
        big = slices(b, [20_000])[0][2]
        with pytest.raises(bsw.BswError) as ei:
            srv.submit(big)
        assert ei.value.code == bsw.ETOOBIG
        # each request fills the arena alone, so submissions outrun admission
        reqs = slices(b, [2500] * 40)
        accepted, busy = [], 0
        for a, s, r in reqs:
            try:
                accepted.append((a, s, srv.submit(r)))
            except bsw.BswError as e:
                assert e.code == bsw.EBUSY
                busy += 1
        assert busy > 0
        for a, s, tk in accepted:
            _same(srv.wait(tk), want[a:a + s], f"request {a}")


def test_wait_timeout_and_unknown_ticket(bsw, pool):
    b, want, _ = pool
    with bsw.Server(b["scorings"]) as srv:
        a, s, r = slices(b, [100_000])[0]
        tk = srv.submit(r)
        with pytest.raises(bsw.BswError) as ei:
            srv.wait(tk, timeout_ms=0)
        assert ei.value.code == bsw.ETIMEOUT
        _same(srv.wait(tk), want[a:a + s], "after timeout")
        with pytest.raises(bsw.BswError) as ei:
            srv.wait(tk)
        assert ei.value.code == bsw.EINVAL


def test_bad_request_fails_alone(bsw, pool):
    b, want, _ = pool
    reqs = slices(b, [2000] * 6)
    a3, s3, r3 = reqs[3]
    bad = dict(r3)
    bad["t"] = b["t"].copy()
    bad["t"][int(b["t_off"][a3 + 17]) + 2] = 6
    reqs[3] = (a3, s3, bad)
    # host-side checks reject h0 and offsets at submit
    hb = dict(reqs[0][2])
    hb["h0"] = reqs[0][2]["h0"].copy()
    hb["h0"][5] = 0
    with bsw.Server(b["scorings"]) as srv:
        with pytest.raises(bsw.BswError) as ei:
            srv.submit(hb)
        assert ei.value.code == bsw.EINVAL
        tks = [(a, s, srv.submit(r)) for a, s, r in reqs]
        for k, (a, s, tk) in enumerate(tks):
            if k == 3:
                with pytest.raises(bsw.BswError) as ei:
                    srv.wait(tk)
                assert ei.value.code == bsw.EINVAL and "17" in str(ei.value)
            else:
                _same(srv.wait(tk), want[a:a + s], f"request {k}")
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 5


def _pinned(a):
    """A copy of a host array in pinned (page-locked) memory."""
    import torch
    a = np.ascontiguousarray(a)
    buf = torch.empty(max(a.nbytes, 1), dtype=torch.uint8, pin_memory=True)
    out = buf.numpy()[:a.nbytes].view(a.dtype).reshape(a.shape)
    out[...] = a
    return out, buf


def test_pinned_requests_read_by_the_device(bsw, pool):
    # requests whose arrays are in pinned memory are gathered by the device
    # itself; mixed in one batch with requests in pageable memory, and one
    # pinned request with a bad code, which fails alone
    b, want, wdiag = pool
    keep = []
    pq, bq = _pinned(b["q"])
    pt, bt = _pinned(b["t"])
    pqo, bqo = _pinned(b["q_off"])
    pto, bto = _pinned(b["t_off"])
    ph0, bh0 = _pinned(b["h0"])
    keep += [bq, bt, bqo, bto, bh0]
    bad_t, bbt = _pinned(b["t"])
    keep.append(bbt)
    reqs = slices(b, synth.serving_requests(n_requests=30, seed=53, lo=300, hi=9_000))
    sent = []
    for k, (a, s, r) in enumerate(reqs):
        if k % 3 != 2:  # two of three requests in pinned memory
            r = {"q": pq, "t": pt, "q_off": pqo[a:a + s + 1], "t_off": pto[a:a + s + 1],
                 "h0": ph0[a:a + s], "scorings": b["scorings"]}
        sent.append((a, s, r))
    a7, s7, r7 = sent[7]
    bad_t[int(b["t_off"][a7 + 5]) + 1] = 9
    sent[7] = (a7, s7, dict(r7, t=bad_t))
    with bsw.Server(b["scorings"], max_inflight=2) as srv:
        tks = [(a, s, srv.submit(r, with_diag=True)) for a, s, r in sent]
        for k, (a, s, tk) in enumerate(tks):
            if k == 7:
                with pytest.raises(bsw.BswError) as ei:
                    srv.wait(tk)
                assert ei.value.code == bsw.EINVAL and "5" in str(ei.value)
                continue
            got, gd = srv.wait(tk)
            _same(got, want[a:a + s], f"request {k} at {a}")
            assert np.array_equal(gd["cells"], wdiag["cells"][a:a + s])
        st = srv.stats()
    assert st["failed"] == 1 and st["completed"] == len(sent) - 1
    del keep
