"""Parity of the read-level seed driver (bsw_extend_seeds, and the device
form bsw_extend_seeds_device) with the CPU reference oracle.seeds, field by
field, on seeded synthetic reads and seeds; edge cases and error paths."""
import numpy as np
import pytest

from paper_1907_12931_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = ("score", "qbeg", "qend", "how", "rbeg", "rend")


@pytest.fixture(scope="module")
def bsw():
    from paper_1907_12931_amd import bsw as b
    return b


@pytest.fixture(scope="module")
def ctx(bsw):
    with bsw.Context() as c:
        yield c


def reference(w, seeds=None, scoring=None):
    from oracle import seeds as oseeds
    sd = w["seeds"] if seeds is None else seeds
    return oseeds.extend_seeds(w["reads"], w["read_off"], w["ref"],
                               np.asarray(sd, dtype=oseeds.SEED_DTYPE),
                               scoring or w["scoring"])


def assert_same(got, want, what=""):
    assert len(got) == len(want)
    for f in FIELDS:
        bad = np.nonzero(got[f] != want[f])[0]
        assert len(bad) == 0, (f"{what} field {f}: {len(bad)} of {len(got)} differ; first "
                               f"seed {bad[0]}: got {got[bad[0]]}, want {want[bad[0]]}")


def run_device(bsw, ctx, w, with_rev=False, async_=False, scoring=None):
    import torch
    dev = bsw.seeds_to_device(w["reads"], w["read_off"], w["ref"], w["seeds"],
                              with_ref_rev=with_rev)
    n = len(w["seeds"])
    out = torch.full((n * bsw.SEED_RESULT_DTYPE.itemsize,), 0x5a, dtype=torch.uint8,
                     device="cuda")
    ctx.extend_seeds_device(dev, scoring or w["scoring"], out, async_=async_)
    if async_:
        ctx.wait()
    return out.cpu().numpy().view(bsw.SEED_RESULT_DTYPE)


def test_host_form_matches_reference(bsw, ctx, oracle_lib):
    w = synth.seed_workload(2000, seed=11)
    print("seeds", len(w["seeds"]), flush=True)
    got = ctx.extend_seeds(w["reads"], w["read_off"], w["ref"], w["seeds"], w["scoring"])
    assert_same(got, reference(w))
    t = ctx.last_timing()
    assert t[0] > 0 and t[0] >= t[1] and t[3] >= 2
    assert ctx.last_cells() > 0


@pytest.mark.parametrize("with_rev,async_", [(False, False), (True, False), (True, True)])
def test_device_form_matches_reference(bsw, ctx, oracle_lib, with_rev, async_):
    w = synth.seed_workload(3000, seed=12, ref_len=200_000)
    got = run_device(bsw, ctx, w, with_rev=with_rev, async_=async_)
    assert_same(got, reference(w))


def test_plain_path_matches_reference(bsw, oracle_lib):
    w = synth.seed_workload(1500, seed=13)
    with bsw.Context(path=bsw.PATH_PLAIN) as c:
        got = c.extend_seeds(w["reads"], w["read_off"], w["ref"], w["seeds"], w["scoring"])
    assert_same(got, reference(w))


@pytest.mark.parametrize("sc", [synth.WIDE_B, synth.scoring(end_bonus=40),
                                synth.scoring(end_bonus=0, zdrop=30),
                                synth.scoring(2, -5, -2, 4, 2, w=30, zdrop=0, end_bonus=8)])
def test_other_scorings(bsw, ctx, oracle_lib, sc):
    w = synth.seed_workload(1200, seed=14)
    # seed scores in the scoring's match units
    w["seeds"]["h0"] *= int(np.asarray(sc["mat"]).reshape(25)[0])
    got = ctx.extend_seeds(w["reads"], w["read_off"], w["ref"], w["seeds"], sc)
    assert_same(got, reference(w, scoring=sc), str(sc))


def edge_workload():
    """Hand-made reads at the ends of a short reference, an empty read, a
    read that is all N but for its seed, zero-length and whole-read seeds."""
    rng = np.random.default_rng(15)
    ref = rng.integers(0, 4, 700).astype(np.uint8)
    ref[350:353] = 4
    reads, seeds = [], []

    def add(read, qb, qe, rb, h0):
        seeds.append((len(reads), qb, qe, h0, rb))
        reads.append(np.asarray(read, dtype=np.uint8))

    add(ref[0:120], 30, 60, 30, 30)              # left window clipped at 0
    add(ref[580:700], 40, 90, 620, 50)           # right window clipped at the end
    add(ref[600:700], 0, 100, 600, 100)          # whole read, at the end
    add(ref[0:90], 0, 25, 0, 25)                 # qb = 0 at the reference start
    add(ref[200:320], 95, 120, 295, 25)          # qe = read length
    add(np.zeros(0, np.uint8), 0, 0, 10, 7)      # empty read
    add(ref[100:220], 50, 50, 150, 3)            # zero-length seed
    r = ref[300:450].copy()                      # N in reference and read
    r[:40] = 4
    add(r, 60, 90, 360, 30)
    r = ref[400:551].copy()
    r[::7] = (r[::7] + 1) % 4                    # dense substitutions
    add(r, 71, 76, 471, 5)
    add(ref[0:151], 0, 0, 0, 1)                  # zero-length seed at 0
    add(ref[549:700], 151, 151, 700, 1)          # zero-length seed at the end
    ql = [len(x) for x in reads]
    off = np.zeros(len(ql) + 1, np.uint64)
    off[1:] = np.cumsum(ql)
    sd = np.zeros(len(seeds), dtype=synth.SEED_FIELDS)
    for k, s in enumerate(seeds):
        sd[k] = s
    return {"reads": np.concatenate(reads), "read_off": off, "ref": ref, "seeds": sd,
            "scoring": synth.BWA_DEFAULT}


def test_edge_cases(bsw, ctx, oracle_lib):
    w = edge_workload()
    want = reference(w)
    assert_same(ctx.extend_seeds(w["reads"], w["read_off"], w["ref"], w["seeds"],
                                 w["scoring"]), want, "host form")
    assert_same(run_device(bsw, ctx, w, with_rev=False), want, "device form")
    assert_same(run_device(bsw, ctx, w, with_rev=True), want, "device form, ref_rev")


def test_bad_seed_is_rejected_and_nothing_written(bsw, ctx):
    import torch
    w = synth.seed_workload(300, seed=16)
    bad = w["seeds"].copy()
    bad[7]["qe"] = 152                             # past the read end
    with pytest.raises(bsw.BswError) as ei:
        ctx.extend_seeds(w["reads"], w["read_off"], w["ref"], bad, w["scoring"])
    assert ei.value.code == bsw.EINVAL and "seed 7" in str(ei.value)
    # device form: the check runs on the device and out keeps its bytes
    for k, field, val in ((5, "rb", len(w["ref"])), (3, "h0", 0), (9, "read", 10**6)):
        b = w["seeds"].copy()
        b[k][field] = val
        dev = bsw.seeds_to_device(w["reads"], w["read_off"], w["ref"], b)
        out = torch.full((len(b) * 32,), 0x5a, dtype=torch.uint8, device="cuda")
        with pytest.raises(bsw.BswError) as ei:
            ctx.extend_seeds_device(dev, w["scoring"], out)
        assert ei.value.code == bsw.EINVAL and f"seed {k}" in str(ei.value), str(ei.value)
        assert bool((out == 0x5a).all())
    # a code > 4 in the reads
    reads = w["reads"].copy()
    reads[1000] = 9
    dev = bsw.seeds_to_device(reads, w["read_off"], w["ref"], w["seeds"])
    out = torch.full((len(w["seeds"]) * 32,), 0x5a, dtype=torch.uint8, device="cuda")
    with pytest.raises(bsw.BswError) as ei:
        ctx.extend_seeds_device(dev, w["scoring"], out)
    assert "read byte" in str(ei.value)
    assert bool((out == 0x5a).all())
    # the context still works afterwards
    got = ctx.extend_seeds(w["reads"], w["read_off"], w["ref"], w["seeds"], w["scoring"])
    assert len(got) == len(w["seeds"])


def test_bench_size_sampled(bsw, ctx, oracle_lib):
    """The workload the benchmark times, in its launch configuration (device
    form with a reversed reference), checked on a seeded sample of seeds."""
    w = synth.seed_workload(**synth.SEED_BENCH)
    got = run_device(bsw, ctx, w, with_rev=True)
    idx = np.sort(np.random.default_rng(17).choice(len(w["seeds"]), 3000, replace=False))
    assert_same(got[idx], reference(w, seeds=w["seeds"][idx]), "sample")


def test_seed_tuner_keeps_results_and_caches_its_own_entry(bsw, oracle_lib, tmp_path):
    import json
    import torch
    w = synth.seed_workload(4000, seed=18)
    want = reference(w)
    dev = bsw.seeds_to_device(w["reads"], w["read_off"], w["ref"], w["seeds"],
                              with_ref_rev=True)
    out = torch.zeros(len(w["seeds"]) * 32, dtype=torch.uint8, device="cuda")
    cache = str(tmp_path / "tune.json")
    with bsw.Context(tune_cache=cache) as c:
        ms, shape = c.tune_seeds(dev, w["scoring"], out, reps=1)
        assert ms > 0 and shape["side_streams"] in (1, 2, 4)
        assert_same(out.cpu().numpy().view(bsw.SEED_RESULT_DTYPE), want, "tuner call")
        pairs_shape = c.tune_info()
    entries = json.load(open(cache))
    (key, val), = entries.items()
    assert key.endswith(":seeds") and val["nside"] == shape["side_streams"]
    # a new context takes it for seed calls only
    with bsw.Context(tune_cache=cache) as c2:
        out.zero_()
        c2.extend_seeds_device(dev, w["scoring"], out)
        assert_same(out.cpu().numpy().view(bsw.SEED_RESULT_DTYPE), want, "cached shape")
        assert c2.tune_info() == pairs_shape


def filter_device(bsw, ctx, seeds, res, async_=False):
    import torch
    n = len(seeds)
    sd = torch.from_numpy(np.ascontiguousarray(seeds).view(np.uint8).copy()).cuda()
    rs = torch.from_numpy(np.ascontiguousarray(res).view(np.uint8).copy()).cuda()
    keep = torch.full((max(n, 1),), 0x5a, dtype=torch.uint8, device="cuda")
    ctx.filter_seeds_device(sd, rs, keep, async_=async_)
    if async_:
        ctx.wait()
    return keep[:n].cpu().numpy()


@pytest.mark.parametrize("max_seeds,async_", [(3, False), (12, True)])
def test_filter_matches_reference(bsw, ctx, oracle_lib, max_seeds, async_):
    from oracle import seeds as oseeds
    w = synth.seed_workload(4000, seed=17, ref_len=300_000, max_seeds=max_seeds)
    res = reference(w)
    want = oseeds.filter_seeds(w["seeds"], res)
    got = filter_device(bsw, ctx, w["seeds"], res, async_=async_)
    print("seeds", len(want), "dropped", int((want == 0).sum()), flush=True)
    assert (want == 0).sum() > 0 and want.sum() > 0
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{len(bad)} keep flags differ; first seed {bad[0]}"


def test_filter_after_device_extension(bsw, ctx, oracle_lib):
    # the flags of the whole device path (extend, then filter) on its own
    # results equal the reference's flags on the reference's results
    from oracle import seeds as oseeds
    w = synth.seed_workload(2500, seed=18, max_seeds=8)
    got_res = run_device(bsw, ctx, w, with_rev=True)
    want = oseeds.filter_seeds(w["seeds"], reference(w))
    assert np.array_equal(filter_device(bsw, ctx, w["seeds"], got_res), want)


def test_filter_hand_cases(bsw, ctx):
    from oracle import seeds as oseeds
    sd = np.zeros(9, dtype=synth.SEED_FIELDS)
    res = np.zeros(9, dtype=bsw.SEED_RESULT_DTYPE)
    rows = [  # read, qb, qe, rb | qbeg, qend, rbeg, rend
        (0, 10, 40, 110, 0, 100, 100, 200),
        (0, 20, 30, 120, 0, 0, 0, 0),      # inside seed 0's extension: dropped
        (0, 20, 30, 500, 5, 50, 490, 540),  # same read interval, other place: kept
        (0, 60, 99, 160, 0, 0, 0, 0),       # inside 0 (ends at qend, rend): dropped
        (0, 60, 101, 160, 0, 0, 0, 0),      # one past qend: kept
        (1, 20, 30, 120, 0, 0, 0, 0),       # new chain: first seed kept
        (1, 20, 30, 120, 0, 0, 0, 0),       # empty extension covers nothing: kept
        (2, 0, 0, 7, 0, 1, 7, 8),           # zero-length seed: kept (first)
        (2, 0, 0, 7, 0, 0, 0, 0),           # empty seed inside [0,1) x [7,8): dropped
    ]
    for k, (rd, qb, qe, rb, a, b, c, d) in enumerate(rows):
        sd[k]["read"], sd[k]["qb"], sd[k]["qe"], sd[k]["rb"], sd[k]["h0"] = rd, qb, qe, rb, 1
        res[k]["qbeg"], res[k]["qend"], res[k]["rbeg"], res[k]["rend"] = a, b, c, d
    want = oseeds.filter_seeds(sd, res)
    assert list(want) == [1, 0, 1, 0, 1, 1, 1, 1, 0]
    assert list(filter_device(bsw, ctx, sd, res)) == list(want)
    assert len(filter_device(bsw, ctx, sd[:0], res[:0])) == 0
