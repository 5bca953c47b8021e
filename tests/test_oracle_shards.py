"""The oracle's sampler over disjoint attempt ranges in worker processes,
merged in attempt order, equals one run over the whole range (attempt ids
key the random stream): the merge the full-size digests and the multi-core
CPU baseline rely on."""
import numpy as np

from oracle import cpu, shards


def test_sharded_sampling_equals_one_run():
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    g = cpu.Graph(*wl.host())
    for mode in (cpu.MODE_EDGES, cpu.MODE_NODES):
        m = shards.sample(g, wl.sources, mode, 60_000, 7, wl.seed, procs=3, shards=5)
        w = g.sample(wl.sources, mode, 60_000, 7, wl.seed)
        assert np.array_equal(m.attempt, w.attempt) and np.array_equal(m.off, w.off)
        assert np.array_equal(m.ids, w.ids)
        assert (m.attempts, m.hits, m.steps, m.dead_ends, m.cycles) == (
            w.attempts, w.hits, w.steps, w.dead_ends, w.cycles)


def test_solve_many_equals_one_by_one():
    """Queries solved in worker processes equal cpu.solve in this process."""
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    g = cpu.Graph(*wl.host())
    qs = workloads.query_mix(wl.n, 5, seed=3, max_sources=50, k_range=(1, 20), attempts_range=(1000, 20_000))
    got = shards.solve_many(g, qs, procs=3)
    for q, r in zip(qs, got):
        mode = cpu.MODE_EDGES if q["mode"] == "edges" else cpu.MODE_NODES
        ref = cpu.solve(g, q["sources"], mode, q["k"], q["n_attempts"], 0, q["seed"])
        assert np.array_equal(r["selected"], ref["selected"]) and np.array_equal(r["gains"], ref["gains"])
        assert (r["hits"], r["dead_ends"], r["cycles"], r["steps"], r["covered"]) == (
            ref["walks"].hits, ref["walks"].dead_ends, ref["walks"].cycles, ref["walks"].steps, ref["covered"])
