"""GPU parity at full workload sizes.

* cl1m (Chung-Lu, n=10^6, m=1.6*10^7, 1000 sources, N=10^7): the whole path,
  edges and nodes, compared with the oracle run on all N attempts.
* rmat24 (R-MAT scale 24, 2.6*10^8 edges, 10^4 sources, N=10^8 -- the bench
  workload, in the same launch configuration): the sampler's kept walks for
  sampled attempt ids (kept and not kept) against the oracle walking those
  attempts one by one; counters against invariants; the greedy on a prefix
  of the kept walks against the oracle; and properties of the full solve
  that hold at any size; and the whole query against the oracle's digest
  (every counter, the kept walks in attempt order, the counts, all k picks
  and gains).
* rmat26 (R-MAT scale 26, edge factor 24, 1.6*10^9 edges, 10^5 sources,
  N=2*10^8): the whole query against the oracle's digest as for rmat24; the
  full solve's invariants, a window of kept walks against the oracle
  attempt by attempt, and the greedy on a prefix of them.
* rmat22 (R-MAT scale 22) with mixed queries: batched answers equal the
  single-query path's, the eight smallest also the oracle's.
"""
import numpy as np
import pytest


def say(*a):
    print("[fullsize]", *a, flush=True)

from oracle import cpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sia():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05854_amd import sia as _sia
    _sia.lib()
    return _sia


@pytest.fixture(scope="module")
def cl1m(sia):
    from paper_1702_05854_amd import workloads
    say("generating cl1m")
    wl = workloads.load("cl1m")
    say("ingest")
    g = sia.Graph(wl.col_off.cuda(), wl.row_idx.cuda(), wl.w.cuda())
    og = cpu.Graph(*wl.host())
    yield wl, g, og
    g.close()


@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_cl1m_solve_matches_oracle(sia, cl1m, mode):
    wl, g, og = cl1m
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    got = sia.solve(g, wl.sources, mode, wl.k, wl.n_attempts, 0, wl.seed)
    say("oracle solve", mode)
    ref = cpu.solve(og, wl.sources, om, wl.k, wl.n_attempts, 0, wl.seed)
    st = got["stats"]
    assert (st["hits"], st["dead_ends"], st["cycles"], st["steps"]) == (
        ref["walks"].hits, ref["walks"].dead_ends, ref["walks"].cycles, ref["walks"].steps)
    assert st["walk_ids"] == ref["walks"].ids.shape[0]
    assert np.array_equal(got["selected"], ref["selected"])
    assert np.array_equal(got["gains"], ref["gains"])
    assert st["suspension_est"] == ref["suspension"]
    assert st["suspension_nodes_est"] == ref["suspension_nodes"]


def test_cl1m_walks_match_oracle(sia, cl1m):
    wl, g, og = cl1m
    got = sia.sample(g, wl.sources, "edges", 1_000_003, 5_000_000, wl.seed)
    ref = og.sample(wl.sources, cpu.MODE_EDGES, 1_000_003, 5_000_000, wl.seed)
    assert np.array_equal(got.attempt, ref.attempt)
    assert np.array_equal(got.off, ref.off)
    assert np.array_equal(got.ids, ref.ids)


@pytest.fixture(scope="module")
def rmat24(sia):
    from paper_1702_05854_amd import workloads
    say("generating rmat24")
    wl = workloads.load("rmat24", device="cuda")
    g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
    host = wl.host()
    say("oracle thresholds")
    og = cpu.Graph(*host)
    yield wl, g, og, host
    g.close()


def test_rmat24_sampled_walks_match_oracle(sia, rmat24):
    wl, g, og, (col_off, row_idx, w) = rmat24
    N = wl.n_attempts
    say("gpu sample")
    got = sia.sample(g, wl.sources, "edges", N, 0, wl.seed)
    say("walks on host")
    st = got.stats
    assert st["hits"] + st["dead_ends"] + st["cycles"] == N
    assert got.n_walks == st["hits"] and got.ids.shape[0] == st["walk_ids"]
    assert st["evaluations"] >= st["steps"]
    rng = np.random.default_rng(24)
    kept = got.attempt[rng.choice(got.n_walks, 1000, replace=False)]
    anyid = rng.choice(N, 2000, replace=False).astype(np.uint64)
    probe = np.unique(np.concatenate([kept, anyid, np.array([0, N - 1], np.uint64)]))
    say("oracle on", probe.shape[0], "attempts")
    ref = og.sample_list(wl.sources, cpu.MODE_EDGES, probe, wl.seed)
    # the oracle's kept walks among the probed attempts are exactly the GPU's
    pos = np.minimum(np.searchsorted(got.attempt, probe), got.n_walks - 1)
    gpu_kept = probe[got.attempt[pos] == probe]
    assert np.array_equal(ref.attempt, gpu_kept)
    for i, a in enumerate(ref.attempt):
        j = int(np.searchsorted(got.attempt, a))
        assert np.array_equal(got.walk(j), ref.walk(i)), int(a)
    # walks chain backwards: the tail of edge j_i is the head (column) of j_{i+1}
    for i in range(min(got.n_walks, 2000)):
        e = got.walk(i).astype(np.int64)
        heads = np.searchsorted(col_off, e, side="right") - 1
        assert np.all(row_idx[e[:-1]] == heads[1:]), i
    # greedy on a prefix of the kept walks: identical to the oracle's
    nw = 20_000
    off = got.off[: nw + 1].copy()
    ids = got.ids[: int(off[-1])]
    a = sia.greedy(g.m, off, ids, 200)
    say("oracle greedy")
    b = cpu.greedy_csr(g.m, off, ids, 200)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_rmat24_solve_properties(sia, rmat24):
    wl, g, og, host = rmat24
    res = sia.solve(g, wl.sources, "edges", wl.k, wl.n_attempts, 0, wl.seed)
    sel, gains, st = res["selected"], res["gains"], res["stats"]
    assert len(set(sel.tolist())) == wl.k
    assert np.all(np.diff(gains.astype(np.int64)) <= 0)      # submodular: gains never grow
    assert st["covered"] == int(gains.sum()) <= st["hits"]
    walks = sia.sample(g, wl.sources, "edges", wl.n_attempts, 0, wl.seed)
    cnt = np.bincount(walks.ids, minlength=g.m)
    assert int(gains[0]) == int(cnt.max())
    assert int(sel[0]) == int(np.flatnonzero(cnt == cnt.max())[0])  # lowest id on ties
    # coverage of the selected set, recomputed from the walks
    chosen = np.zeros(g.m, bool)
    chosen[sel] = True
    hit = np.add.reduceat(chosen[walks.ids].astype(np.int64), walks.off[:-1].astype(np.int64)) > 0
    assert int(hit.sum()) == st["covered"]


def test_rmat24_nodes_greedy_equals_oracle_greedy(sia, rmat24):
    """Node removal on the same query (10^8 attempts, k = 1000): every kept
    walk holds its terminal source, so the first picks cover nearly all
    walks (the counts are recomputed instead of decremented) and the picks'
    walk lists run to 10^5 entries.  The library's picks and gains equal the
    oracle's greedy (Algorithm 7) over the same kept walks."""
    wl, g, og, host = rmat24
    say("gpu sample (nodes)")
    walks = sia.sample(g, wl.sources, "nodes", wl.n_attempts, 0, wl.seed)
    say("gpu solve (nodes)")
    r = sia.solve(g, wl.sources, "nodes", wl.k, wl.n_attempts, 0, wl.seed, cycle_steps=False)
    assert r["stats"]["hits"] == walks.n_walks and r["stats"]["walk_ids"] == walks.ids.shape[0]
    say("oracle greedy over", walks.n_walks, "walks,", walks.ids.shape[0], "ids")
    sel, gains = cpu.greedy_csr(g.n, walks.off, walks.ids, wl.k)
    say("compare")
    assert np.array_equal(r["selected"], sel) and np.array_equal(r["gains"], gains)
    assert r["stats"]["covered"] == int(gains.sum())


def _digest(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_digest.json")
    with open(path) as f:
        return json.load(f)


def _sha(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def compare_with_digest(sia, g, wl, D):
    """The whole query against the oracle's digest (tests/golden/*_digest.json,
    written by tests/golden/make_fullsize_digest.py from the oracle alone, run
    over disjoint attempt ranges in several processes and merged in attempt
    order): the graph, the counters, the attempt-ordered kept walks, the
    coverage counts, and the k picks and gains of the full solve, with
    cyclic walks searched for their entry and stopped at detection."""
    assert (g.n, g.m, wl.seed) == (D["n"], D["m"], D["seed"])
    assert _sha(np.asarray(wl.sources, np.int32)) == D["sources_sha256"]
    col_off, row_idx, w = wl.host()
    assert _sha(col_off.astype("<i8")) == D["sha256"]["col_off"]
    assert _sha(row_idx.astype("<i4")) == D["sha256"]["row_idx"]
    assert _sha(w.astype("<f4")) == D["sha256"]["w"]
    N, k = D["n_attempts"], D["k"]
    say("gpu sample", N)
    got = sia.sample(g, wl.sources, D["mode"], N, D["attempt_offset"], wl.seed)
    st = got.stats
    C = D["counters"]
    assert (st["attempts"], st["hits"], st["dead_ends"], st["cycles"], st["steps"], st["walk_ids"]) == (
        C["attempts"], C["hits"], C["dead_ends"], C["cycles"], C["steps"], C["walk_ids"])
    say("stream digests")
    assert _sha(got.attempt.astype("<u8")) == D["sha256"]["attempt"]
    assert _sha(got.off.astype("<u8")) == D["sha256"]["off"]
    assert _sha(got.ids.astype("<u4")) == D["sha256"]["ids"]
    space = g.m if D["mode"] == "edges" else g.n
    cnt = np.bincount(got.ids, minlength=space).astype("<u4")
    assert _sha(cnt) == D["sha256"]["counts"]
    del got, cnt
    say("gpu solve k =", k)
    res = sia.solve(g, wl.sources, D["mode"], k, N, D["attempt_offset"], wl.seed)
    assert res["selected"].tolist() == D["selected"]
    assert res["gains"].tolist() == D["gains"]
    assert res["stats"]["covered"] == D["covered"]
    assert res["stats"]["hits"] == C["hits"] and res["stats"]["steps"] == C["steps"]
    # the launch the benchmark times: cyclic walks stopped at detection
    say("gpu solve k =", k, "(cyclic walks stopped at detection)")
    res = sia.solve(g, wl.sources, D["mode"], k, N, D["attempt_offset"], wl.seed, cycle_steps=False)
    st = res["stats"]
    assert res["selected"].tolist() == D["selected"] and res["gains"].tolist() == D["gains"]
    assert (st["covered"], st["hits"], st["dead_ends"], st["cycles"], st["walk_ids"]) == (
        D["covered"], C["hits"], C["dead_ends"], C["cycles"], C["walk_ids"])
    assert st["steps"] <= C["steps"] - C["cycles"]


def test_rmat24_whole_query_matches_oracle_digest(sia, rmat24):
    """The bench's query (R-MAT scale 24, 10^4 sources, N = 10^8, k = 1000)
    equal to the oracle as a whole: every counter, the digest of every kept
    walk in attempt order, the counts, all 1000 picks and gains."""
    wl, g, og, host = rmat24
    compare_with_digest(sia, g, wl, _digest("rmat24"))


# ---------------------------------------------------------------- billion-edge graph
@pytest.fixture(scope="module")
def rmat26(sia):
    from paper_1702_05854_amd import workloads
    say("generating rmat26 (R-MAT scale 26, edge factor 24)")
    wl = workloads.load("rmat26", device="cuda")
    say("ingest", wl.m, "edges")
    g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
    torch.cuda.synchronize()
    yield wl, g
    g.close()


def test_rmat26_whole_query_matches_oracle_digest(sia, rmat26):
    """The billion-edge query (R-MAT scale 26, edge factor 24, 1.6*10^9
    edges with 32-byte records, 10^5 sources, N = 2*10^8, k = 1000) equal to
    the oracle as a whole: counters, the attempt-ordered kept walks, the
    counts, all 1000 picks and gains."""
    wl, g = rmat26
    compare_with_digest(sia, g, wl, _digest("rmat26"))


def test_rmat26_billion_edges(sia, rmat26):
    """1.6*10^9 edges, 10^5 sources, 2*10^8 attempts, k = 1000 (the launch the
    bench uses).  The whole solve's invariants; the kept walks of a window of
    2*10^6 attempts against the oracle walking sampled attempts one by one;
    the greedy on a prefix of those walks against the oracle's."""
    wl, g = rmat26
    N = wl.n_attempts
    say("gpu solve", N, "attempts")
    res = sia.solve(g, wl.sources, "edges", wl.k, N, 0, wl.seed)
    sel, gains, st = res["selected"], res["gains"], res["stats"]
    assert st["hits"] + st["dead_ends"] + st["cycles"] == N
    assert st["evaluations"] >= st["steps"]
    assert len(set(sel.tolist())) == wl.k and sel.min() >= 0 and sel.max() < g.m
    assert np.all(np.diff(gains.astype(np.int64)) <= 0)
    assert st["covered"] == int(gains.sum()) <= st["hits"]
    say("solve:", {k: st[k] for k in ("hits", "dead_ends", "cycles", "steps", "walk_ids", "covered")})

    W, W0 = 2_000_000, N - 2_000_000
    say("gpu sample of attempts", W0, "..", N)
    got = sia.sample(g, wl.sources, "edges", W, W0, wl.seed)
    say("host copy")
    col_off, row_idx, w = wl.host()
    say("oracle thresholds")
    og = cpu.Graph(col_off, row_idx, w)
    rng = np.random.default_rng(26)
    kept = got.attempt[rng.choice(got.n_walks, min(1000, got.n_walks), replace=False)]
    anyid = (W0 + rng.choice(W, 2000, replace=False)).astype(np.uint64)
    probe = np.unique(np.concatenate([kept, anyid, np.array([W0, N - 1], np.uint64)]))
    say("oracle on", probe.shape[0], "attempts")
    ref = og.sample_list(wl.sources, cpu.MODE_EDGES, probe, wl.seed)
    pos = np.minimum(np.searchsorted(got.attempt, probe), got.n_walks - 1)
    assert np.array_equal(ref.attempt, probe[got.attempt[pos] == probe])
    for i, a in enumerate(ref.attempt):
        j = int(np.searchsorted(got.attempt, a))
        assert np.array_equal(got.walk(j), ref.walk(i)), int(a)
    for i in range(min(got.n_walks, 2000)):  # walks chain backwards through the graph
        e = got.walk(i).astype(np.int64)
        heads = np.searchsorted(col_off, e, side="right") - 1
        assert np.all(row_idx[e[:-1]] == heads[1:]), i
    nw = min(20_000, got.n_walks)
    off = got.off[: nw + 1].copy()
    ids = got.ids[: int(off[-1])]
    say("greedy on", nw, "walks")
    a = sia.greedy(g.m, off, ids, 200)
    b = cpu.greedy_csr(g.m, off, ids, 200)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------- mixed queries, full graph
def test_rmat22_mix_batched_equals_plain(sia):
    """R-MAT scale 22 with queries drawn as for serving (|X| log-uniform in
    1..10^4, k in 10..1000, N log-uniform in 10^5..10^7, both modes): every
    batched answer equals the single-query path's; the eight smallest
    queries also equal the oracle's (picks, gains, every counter)."""
    from paper_1702_05854_amd import workloads
    say("generating rmat22")
    wl = workloads.load("rmat22", device="cuda")
    g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
    qs = workloads.query_mix(wl.n, 32, seed=22)
    with sia.Batch(g, use_graph=1) as b:
        ts = [b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"]) for q in qs]
        got = []
        for t in ts:
            r = b.wait(t, 120_000)
            assert r is not None, b.stats()
            got.append(r)
        say("batched:", {k: b.stats()[k] for k in ("waves", "greedy_launches", "reruns")})
    for i, q in enumerate(qs):
        ref = sia.solve(g, q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"])
        assert np.array_equal(got[i]["selected"], ref["selected"]), i
        assert np.array_equal(got[i]["gains"], ref["gains"]), i
        for c in ("hits", "dead_ends", "cycles", "steps", "walk_ids", "covered"):
            assert got[i]["stats"][c] == ref["stats"][c], (i, c)
    # the eight smallest queries (a quarter of the mix, both modes) against the
    # oracle, each solved whole in a worker process of its own
    from oracle import shards
    small = sorted(range(len(qs)), key=lambda i: qs[i]["n_attempts"])[:8]
    say("oracle on the 8 smallest queries:", [qs[i]["n_attempts"] for i in small], "attempts")
    og = cpu.Graph(*wl.host())
    refs = shards.solve_many(og, [qs[i] for i in small], procs=8, log=say)
    for i, ref in zip(small, refs):
        assert np.array_equal(got[i]["selected"], ref["selected"]), i
        assert np.array_equal(got[i]["gains"], ref["gains"]), i
        for c in ("hits", "dead_ends", "cycles", "steps", "walk_ids", "covered"):
            assert got[i]["stats"][c] == ref[c], (i, c)
    g.close()
