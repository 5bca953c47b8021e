"""Batched / served queries: every query's answer equals the single-query
path's (and the oracle's where it is small), whatever it shares launches
with, however its attempts are cut into shares, whatever the walk budget."""
import numpy as np
import pytest

from oracle import cpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

COUNTERS = ("attempts", "hits", "dead_ends", "cycles", "steps", "evaluations", "walk_ids",
            "covered", "spread_est", "suspension_est", "suspension_nodes_est")


def say(*a):
    print("[batch]", *a, flush=True)


@pytest.fixture(scope="module")
def sia():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05854_amd import sia as _sia
    _sia.lib()
    return _sia


@pytest.fixture(scope="module")
def er1k(sia):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    host = wl.host()
    g = sia.Graph(*host)
    yield wl, g, cpu.Graph(*host)
    g.close()


@pytest.fixture(scope="module")
def rmat16(sia):
    from paper_1702_05854_amd import workloads
    say("generating rmat16")
    wl = workloads.load("rmat22", device="cuda", scale=16)
    g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
    yield wl, g
    g.close()


@pytest.fixture(scope="module")
def rmat16_general(sia):
    """R-MAT s16 with random normalised weights: stored with 32-byte records."""
    from paper_1702_05854_amd import workloads
    wl = workloads.load("rmat22", device="cuda", scale=16, weights="normalized")
    g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
    assert g.arc_bytes == 32
    yield wl, g
    g.close()


def mix(n, count, seed, **kw):
    from paper_1702_05854_amd import workloads
    return workloads.query_mix(n, count, seed, **kw)


def solo(sia, g, q):
    return sia.solve(g, q["sources"], q["mode"], q["k"], q["n_attempts"], q.get("offset", 0),
                     q["seed"], cycle_steps=q.get("cycle_steps", True))


def assert_same(got, ref, what):
    assert np.array_equal(got["selected"], ref["selected"]), what
    assert np.array_equal(got["gains"], ref["gains"]), what
    for c in COUNTERS:
        assert got["stats"][c] == ref["stats"][c], (what, c)


def done(b, t, limit_ms=100_000):
    """The ticket's result; fails (with the batch's counters) instead of hanging."""
    r = b.wait(t, limit_ms)
    if r is None:
        pytest.fail(f"ticket {t} not finished after {limit_ms} ms: {b.stats()}")
    return r


def serve(sia, g, queries, **kw):
    with sia.Batch(g, **kw) as b:
        tickets = [b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], q.get("offset", 0),
                            q["seed"], q.get("cycle_steps", True)) for q in queries]
        out = [done(b, t) for t in tickets]
        return out, b.stats()


def test_mix_matches_solo_and_oracle_er1k(sia, er1k):
    wl, g, og = er1k
    qs = mix(wl.n, 12, 11, max_sources=100, k_range=(1, 50), attempts_range=(1000, 200_000))
    qs[3]["offset"] = 123_456
    got, st = serve(sia, g, qs, wave_attempts=1 << 16, min_share=4096)
    say("served", st["completed"], "queries in", st["waves"], "waves")
    assert st["completed"] == len(qs) and st["failed"] == 0
    for i, q in enumerate(qs):
        assert_same(got[i], solo(sia, g, q), i)
        if q["n_attempts"] <= 50_000:
            om = cpu.MODE_EDGES if q["mode"] == "edges" else cpu.MODE_NODES
            ref = cpu.solve(og, q["sources"], om, q["k"], q["n_attempts"], q.get("offset", 0), q["seed"])
            assert np.array_equal(got[i]["selected"], ref["selected"]), i
            assert np.array_equal(got[i]["gains"], ref["gains"]), i
            assert got[i]["stats"]["hits"] == ref["walks"].hits


@pytest.mark.parametrize("greedy", [(0, 0, 8), (0, 0, 1), (1, 0, 0), (1, 32, 0)])
def test_mix_matches_solo_rmat16_more_queries_than_slots(sia, rmat16, greedy):
    wl, g = rmat16
    mode, cus, batch = greedy
    qs = mix(wl.n, 40, 12, max_sources=1000, k_range=(10, 200), attempts_range=(10_000, 1_000_000))
    got, st = serve(sia, g, qs, greedy_mode=mode, greedy_cus=cus, greedy_batch=batch)
    assert st["config"]["greedy_mode"] == mode and st["config"]["greedy_cus"] == cus
    say("served", st["completed"], "in", st["waves"], "waves,", st["greedy_launches"], "greedy launches")
    assert st["completed"] == 40 and st["greedy_jobs"] == 40
    assert st["greedy_launches"] < 40  # greedies shared launches
    for i, q in enumerate(qs):
        assert_same(got[i], solo(sia, g, q), i)
        info = got[i]["info"]
        assert info["t_submit"] <= info["t_admit"] <= info["t_sampled"] <= info["t_done"]


def test_mix_matches_solo_general_records(sia, rmat16_general):
    """Batches on a graph with 32-byte records (per-slot tag bits in them)."""
    wl, g = rmat16_general
    qs = mix(wl.n, 20, 21, max_sources=1000, k_range=(10, 200), attempts_range=(10_000, 500_000))
    got, st = serve(sia, g, qs, max_slots=8)
    assert st["completed"] == len(qs) and st["failed"] == 0
    for i, q in enumerate(qs):
        assert_same(got[i], solo(sia, g, q), i)


def test_mix_with_cycles_stopped_at_detection(sia, rmat16):
    """Queries that skip the cycle-entry search share launches with queries
    that do not; each equals its own single-query call with the same flag."""
    wl, g = rmat16
    qs = mix(wl.n, 16, 22, max_sources=1000, k_range=(10, 200), attempts_range=(10_000, 500_000))
    for i, q in enumerate(qs):
        q["cycle_steps"] = i % 2 == 0
    got, st = serve(sia, g, qs, max_slots=8)
    assert st["completed"] == len(qs) and st["failed"] == 0
    for i, q in enumerate(qs):
        assert_same(got[i], solo(sia, g, q), i)


def test_graph_replays_match_eager(sia, rmat16):
    wl, g = rmat16
    qs = mix(wl.n, 10, 13, max_sources=300, k_range=(5, 100), attempts_range=(20_000, 400_000))
    eager, st0 = serve(sia, g, qs, wave_attempts=1 << 18)
    assert st0["graph_replays"] == 0
    for rep in range(2):  # replays across two batches, with other device work between
        solo(sia, g, qs[0])
        replay, st1 = serve(sia, g, qs, wave_attempts=1 << 18, use_graph=1)
        assert st1["graph_replays"] == st1["waves"] > 1
        for i in range(len(qs)):
            assert_same(replay[i], eager[i], (rep, i))


def test_many_small_shares(sia, rmat16):
    wl, g = rmat16
    qs = mix(wl.n, 6, 14, max_sources=100, k_range=(5, 50), attempts_range=(50_000, 200_000))
    got, st = serve(sia, g, qs, wave_attempts=8192, min_share=1024)
    assert all(r["info"]["waves"] > 5 for r in got)
    for i, q in enumerate(qs):
        assert_same(got[i], solo(sia, g, q), i)


def test_tiny_budget_waits_reruns_and_evicts(sia, er1k):
    wl, g, og = er1k
    from paper_1702_05854_amd import workloads
    qs = [dict(sources=workloads.pick_sources(wl.n, 10, 200 + i), mode="edges" if i % 2 else "nodes",
               k=20, n_attempts=20_000 + 5000 * i, seed=3000 + i) for i in range(8)]
    budget = 2 << 20
    got, st = serve(sia, g, qs, walk_budget_bytes=budget, wave_attempts=1 << 15, min_share=2048)
    say("tiny budget:", {k: st[k] for k in ("waves", "reruns", "evictions", "walk_bytes_peak")})
    assert st["walk_bytes_peak"] <= budget
    assert st["reruns"] + st["evictions"] > 0
    for i, q in enumerate(qs):
        assert_same(got[i], solo(sia, g, q), i)


def test_query_larger_than_budget_fails_alone(sia, er1k):
    wl, g, og = er1k
    with sia.Batch(g, walk_budget_bytes=1 << 20) as b:
        big = b.submit(wl.sources, "edges", 10, 100_000, 0, 1)
        with pytest.raises(sia.SiaError) as e:
            done(b, big)
        assert e.value.status == -3  # SIA_ENOMEM
        small = dict(sources=wl.sources, mode="edges", k=5, n_attempts=2000, seed=5)
        t = b.submit(small["sources"], "edges", 5, 2000, 0, 5)
        assert_same(done(b, t), solo(sia, g, small), "after ENOMEM")
        assert b.stats()["failed"] == 1


def test_cancel_and_invalid(sia, rmat16):
    wl, g = rmat16
    qs = mix(wl.n, 6, 15, max_sources=200, k_range=(5, 50), attempts_range=(200_000, 800_000))
    with sia.Batch(g, max_slots=2) as b:
        ts = [b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"]) for q in qs]
        b.cancel(ts[5])  # still queued behind two slots
        b.cancel(ts[0])  # sampling, or already further
        for bad in (dict(sources=[1, 1]), dict(k=0), dict(sources=[wl.n]), dict(n_attempts=0)):
            args = dict(sources=[3, 4], mode="edges", k=5, n_attempts=1000, offset=0, seed=1)
            args.update(bad)
            with pytest.raises(sia.SiaError) as e:
                b.submit(args["sources"], args["mode"], args["k"], args["n_attempts"], 0, 1)
            assert e.value.status == -1
        with pytest.raises(sia.SiaError) as e:
            done(b, ts[5])
        assert e.value.status == -6  # SIA_ECANCELLED
        try:
            r0 = done(b, ts[0])  # it may have finished before the cancel arrived
        except sia.SiaError as err:
            assert err.status == -6
            r0 = None
        if r0 is not None:
            assert_same(r0, solo(sia, g, qs[0]), 0)
        for i in (1, 2, 3, 4):
            assert_same(done(b, ts[i]), solo(sia, g, qs[i]), i)
        with pytest.raises(sia.SiaError) as e:
            b.cancel(ts[1])  # released
        assert e.value.status == -1
        with pytest.raises(sia.SiaError):
            b.poll(987654321)
        st = b.stats()
        assert st["cancelled"] >= 1 and st["busy_slots"] == 0 and st["pending"] == 0


def test_poll_until_done(sia, rmat16):
    wl, g = rmat16
    q = mix(wl.n, 1, 16, max_sources=50, k_range=(20, 20), attempts_range=(300_000, 300_001))[0]
    with sia.Batch(g) as b:
        t = b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"])
        r = None
        import time
        t0 = time.time()
        while r is None and time.time() - t0 < 60:
            r = b.poll(t)
            time.sleep(0.001)
        assert r is not None
        assert_same(r, solo(sia, g, q), "poll")


def test_tune_then_serve(sia, rmat16):
    wl, g = rmat16
    from paper_1702_05854_amd import sia as S
    with S.Batch(g) as b:
        cfg = b.tune(wl.sources[:100], "edges", 1_000_000, target_ms=10.0)
        say("tuned", cfg)
        assert cfg["sampler_blocks_per_cu"] >= 1 and cfg["refill_chunk"] in (64, 128, 256, 512)
        assert cfg["wave_attempts"] >= 1 << 20
        assert cfg["hist_blocks"] >= 1
        assert b.stats()["config"] == cfg
        qs = mix(wl.n, 8, 17, max_sources=300, k_range=(5, 100), attempts_range=(20_000, 500_000))
        ts = [b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"]) for q in qs]
        with pytest.raises(sia.SiaError) as e:  # not idle
            b.tune(wl.sources[:100], "edges", 100_000)
        assert e.value.status == -7
        for i, t in enumerate(ts):
            assert_same(done(b, t), solo(sia, g, qs[i]), i)


def test_tune_with_the_served_flags(sia, rmat16):
    """Tuning on a probe whose cyclic walks stop at detection (as the queries
    served after it), then fast-mode queries equal to single calls; unknown
    probe flag bits are rejected."""
    import ctypes
    wl, g = rmat16
    from paper_1702_05854_amd import sia as S
    with S.Batch(g) as b:
        cfg = b.tune(wl.sources[:100], "edges", 1_000_000, target_ms=10.0, cycle_steps=False)
        assert cfg["sampler_blocks_per_cu"] >= 1 and cfg["wave_attempts"] >= 1 << 20
        q, keep = S._query(wl.sources[:100], "edges", 0, 100_000, 0, 7)
        q.flags = 4
        assert S.lib().sia_batch_tune(b._h, ctypes.byref(q), 10.0, None) == -1
        qs = mix(wl.n, 8, 23, max_sources=300, k_range=(5, 100), attempts_range=(20_000, 500_000))
        for q in qs:
            q["cycle_steps"] = False
        ts = [b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"], False) for q in qs]
        for i, t in enumerate(ts):
            assert_same(done(b, t), solo(sia, g, qs[i]), i)


def test_batch_and_solo_calls_share_a_graph(sia, rmat16):
    wl, g = rmat16
    qs = mix(wl.n, 12, 18, max_sources=500, k_range=(10, 100), attempts_range=(100_000, 1_000_000))
    refs = [solo(sia, g, q) for q in qs]
    with sia.Batch(g, max_slots=8) as b:
        ts = [b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"]) for q in qs]
        for i in range(4):  # single-query calls while the batch runs (tag bit 31 vs 0..7)
            assert_same(solo(sia, g, qs[i]), refs[i], ("solo", i))
        for i, t in enumerate(ts):
            assert_same(done(b, t), refs[i], ("batch", i))


def test_tag_bits_are_shared_out(sia, er1k):
    wl, g, og = er1k
    a = sia.Batch(g, max_slots=30)
    b2 = sia.Batch(g, max_slots=1)
    with pytest.raises(sia.SiaError) as e:
        sia.Batch(g, max_slots=1)
    assert e.value.status == -7  # SIA_EBUSY
    b2.close()
    c = sia.Batch(g, max_slots=1)
    q = dict(sources=wl.sources, mode="nodes", k=7, n_attempts=5000, seed=9)
    t = c.submit(q["sources"], "nodes", 7, 5000, 0, 9)
    assert_same(done(c, t), solo(sia, g, q), "bits")
    c.close()
    a.close()
    with pytest.raises(sia.SiaError):
        sia.Batch(g, max_slots=32)
