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
