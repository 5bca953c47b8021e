"""The oracle's range sampler over disjoint attempt ranges in worker
processes, merged in attempt order.

TEST INFRASTRUCTURE ONLY (the full-size digest script, the benchmark's
multi-core CPU-baseline leg, and the full-size tests that solve several
queries with the oracle at once).

Attempt ids key the random stream (Philox keyed by (seed, attempt id)), so
the walks of a range do not depend on which process samples it, and the
concatenation of the ranges' kept walks in range order is exactly the
single-process run over the whole range; the counters add.  The graph's
arrays and the oracle's threshold table are shared with the workers as
read-only memory maps of files in a temporary directory (under /dev/shm
when it exists); workers are started fresh (spawn), so they share nothing
else with the parent process.
"""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor, as_completed
import tempfile
import time

import numpy as np

from . import cpu


class MergedWalks:
    """Kept walks of a merged run (the fields of cpu.Walks)."""

    def __init__(self, attempt, off, ids, counters):
        self.attempt, self.off, self.ids = attempt, off, ids
        self.attempts, self.hits, self.dead_ends, self.cycles, self.steps = (int(x) for x in counters)

    @property
    def n_walks(self):
        return self.attempt.shape[0]


def _worker(job):
    d, src, mode, a0, a1, seed, out = job
    g = cpu.Graph.from_tables(np.load(os.path.join(d, "col_off.npy"), mmap_mode="r"),
                              np.load(os.path.join(d, "row_idx.npy"), mmap_mode="r"),
                              np.load(os.path.join(d, "thr.npy"), mmap_mode="r"))
    t0 = time.perf_counter()
    w = g.sample(src, mode, a1 - a0, a0, seed)
    np.savez(out, attempt=w.attempt, off=w.off, ids=w.ids,
             counters=np.array([w.attempts, w.hits, w.dead_ends, w.cycles, w.steps], np.uint64))
    return out, time.perf_counter() - t0


def sample(graph, sources, mode, n_attempts, offset=0, seed=0, procs=None, shards=None, log=None):
    """Attempts [offset, offset + n_attempts) of `graph` (a cpu.Graph) in
    `procs` worker processes over `shards` contiguous ranges (default 4 per
    process).  Returns MergedWalks."""
    procs = max(1, procs or os.cpu_count() or 1)
    shards = max(1, shards or 4 * procs)
    bounds = [offset + n_attempts * i // shards for i in range(shards + 1)]
    base_dir = "/dev/shm" if os.path.isdir("/dev/shm") else None
    src = np.ascontiguousarray(sources, dtype=np.int32)
    with tempfile.TemporaryDirectory(prefix="sia_oracle_", dir=base_dir) as d:
        np.save(os.path.join(d, "col_off.npy"), graph.col_off)
        np.save(os.path.join(d, "row_idx.npy"), graph.row_idx)
        np.save(os.path.join(d, "thr.npy"), graph.thr)
        jobs = [(d, src, mode, bounds[i], bounds[i + 1], seed, os.path.join(d, f"shard{i:04d}.npz"))
                for i in range(shards)]
        # (a worker that dies raises BrokenProcessPool here instead of hanging)
        with ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn")) as pool:
            futs = [pool.submit(_worker, job) for job in jobs]
            for done, f in enumerate(as_completed(futs), 1):
                _, dt = f.result()
                if log:
                    log(f"oracle shard {done}/{shards} done ({dt:.0f} s)")
        att, offs, idss = [], [], []
        counters = np.zeros(5, np.uint64)
        base = 0
        for job in jobs:
            z = np.load(job[-1])
            att.append(z["attempt"])
            o = z["off"].astype(np.uint64)
            offs.append(o[:-1] + np.uint64(base))
            idss.append(z["ids"])
            base += int(o[-1])
            counters += z["counters"]
    attempt = np.concatenate(att)
    off = np.concatenate(offs + [np.array([base], np.uint64)])
    ids = np.concatenate(idss)
    return MergedWalks(attempt, off, ids, counters)


def _solve_worker(job):
    d, q = job
    g = cpu.Graph.from_tables(np.load(os.path.join(d, "col_off.npy"), mmap_mode="r"),
                              np.load(os.path.join(d, "row_idx.npy"), mmap_mode="r"),
                              np.load(os.path.join(d, "thr.npy"), mmap_mode="r"))
    mode = cpu.MODE_EDGES if q["mode"] == "edges" else cpu.MODE_NODES
    r = cpu.solve(g, np.asarray(q["sources"], np.int32), mode, q["k"], q["n_attempts"], q.get("offset", 0),
                  q["seed"])
    w = r["walks"]
    return dict(selected=r["selected"], gains=r["gains"], covered=r["covered"], hits=w.hits,
                dead_ends=w.dead_ends, cycles=w.cycles, steps=w.steps, walk_ids=int(w.ids.shape[0]))


def solve_many(graph, queries, procs=None, log=None):
    """cpu.solve of every query (dicts with sources, mode 'edges'/'nodes', k,
    n_attempts, seed and optional offset) on `graph`, one query per worker
    process at a time; returns, in query order, dicts with the picks, gains,
    covered count and the walk counters."""
    procs = max(1, procs or os.cpu_count() or 1)
    base_dir = "/dev/shm" if os.path.isdir("/dev/shm") else None
    with tempfile.TemporaryDirectory(prefix="sia_oracle_", dir=base_dir) as d:
        np.save(os.path.join(d, "col_off.npy"), graph.col_off)
        np.save(os.path.join(d, "row_idx.npy"), graph.row_idx)
        np.save(os.path.join(d, "thr.npy"), graph.thr)
        out = [None] * len(queries)
        with ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn")) as pool:
            futs = {pool.submit(_solve_worker, (d, q)): i for i, q in enumerate(queries)}
            for done, f in enumerate(as_completed(futs), 1):
                out[futs[f]] = f.result()
                if log:
                    log(f"oracle query {done}/{len(queries)} done")
    return out
