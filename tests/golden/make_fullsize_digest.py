"""Writes tests/golden/<workload>_digest.json: the oracle's answer to a
full-size query, computed on the host by the plain C oracle alone.

The workload's graph is generated on the CPU (the generators are
device-independent, so the GPU tests generate the same graph on the device).
Attempts [0, N) are cut into P contiguous ranges sampled by P forked
processes with the oracle's range sampler (attempt ids are the Philox keys,
so a range gives the same walks whichever process samples it); the ranges'
walks are concatenated in attempt order and their counters summed.  The
oracle's count and greedy (Algorithm 4, k rounds, lowest id on ties) then
run once over the merged walks.

Stored: the counters (attempts, hits, dead ends, cycles, steps, walk ids),
sha256 digests of the attempt-ordered walk stream (attempt ids as uint64,
offsets as uint64, ids as uint32, little-endian) and of the count array
(uint32 per id), the k picks and gains, P, the host and the phase times.

This script calls only oracle/ and the input generators.
Run:  python tests/golden/make_fullsize_digest.py rmat24 [--attempts N] [--procs P]
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import platform
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cpu  # noqa: E402
from paper_1702_05854_amd import workloads  # noqa: E402

_G = {}  # the graph and query, inherited by the forked workers


def say(*a):
    print("[digest]", *a, flush=True)


def _shard(args):
    i, a0, a1, tmp = args
    g, src, mode, seed = _G["g"], _G["src"], _G["mode"], _G["seed"]
    t0 = time.time()
    w = g.sample(src, mode, a1 - a0, a0, seed)
    path = os.path.join(tmp, f"shard{i:03d}.npz")
    np.savez(path, attempt=w.attempt, off=w.off, ids=w.ids,
             counters=np.array([w.attempts, w.hits, w.dead_ends, w.cycles, w.steps], np.uint64))
    return i, path, time.time() - t0


def host_cpu():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--attempts", type=int, default=0, help="N (default: the workload's)")
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    ap.add_argument("--shards", type=int, default=0, help="attempt ranges (default 4 per process)")
    ap.add_argument("--k", type=int, default=0)
    ap.add_argument("--mode", default="edges")
    ap.add_argument("--out", default="")
    args = ap.parse_args()

    t0 = time.time()
    wl = workloads.load(args.workload)
    n_attempts = args.attempts or wl.n_attempts
    k = args.k or wl.k
    mode = cpu.MODE_EDGES if args.mode == "edges" else cpu.MODE_NODES
    t_gen = time.time() - t0
    say(f"{args.workload}: n={wl.n} m={wl.m} generated in {t_gen:.0f} s")
    g = cpu.Graph(*wl.host())
    w_sha = sha(g.w.astype("<f4"))
    g.w = None  # the sampler reads the threshold table only
    wl.w = None
    _G.update(g=g, src=wl.sources, mode=mode, seed=wl.seed)
    id_space = g.m if mode == cpu.MODE_EDGES else g.n

    P = max(1, args.procs)
    S = args.shards or 4 * P
    bounds = [n_attempts * i // S for i in range(S + 1)]
    t1 = time.time()
    with tempfile.TemporaryDirectory(prefix="sia_digest_") as tmp:
        jobs = [(i, bounds[i], bounds[i + 1], tmp) for i in range(S)]
        paths = [None] * S
        with mp.get_context("fork").Pool(P) as pool:
            for i, path, dt in pool.imap_unordered(_shard, jobs):
                paths[i] = path
                say(f"shard {i + 1}/{S} attempts [{bounds[i]}, {bounds[i + 1]}) in {dt:.0f} s")
        t_sample = time.time() - t1
        att, offs, ids = [], [], []
        counters = np.zeros(5, np.uint64)
        base = 0
        for p in paths:
            z = np.load(p)
            att.append(z["attempt"])
            o = z["off"].astype(np.uint64)
            offs.append(o[:-1] + np.uint64(base))
            ids.append(z["ids"])
            base += int(o[-1])
            counters += z["counters"]
        attempt = np.concatenate(att)
        off = np.concatenate(offs + [np.array([base], np.uint64)])
        ids = np.concatenate(ids)
    del att, offs
    assert np.all(np.diff(attempt.astype(np.int64)) > 0)
    attempts, hits, dead, cycles, steps = (int(x) for x in counters)
    assert attempts == n_attempts and hits == attempt.shape[0] and hits + dead + cycles == attempts
    say(f"sampled in {t_sample:.0f} s: hits {hits} dead ends {dead} cycles {cycles} steps {steps}")

    t2 = time.time()
    walks_stub = type("W", (), {})()
    walks_stub.off, walks_stub.ids, walks_stub.n_walks = off, ids, attempt.shape[0]
    cnt = cpu.count(id_space, walks_stub)
    t_count = time.time() - t2
    t3 = time.time()
    sel, gains = cpu.greedy_csr(id_space, off, ids, k)
    t_greedy = time.time() - t3
    say(f"count {t_count:.0f} s, greedy k={k} {t_greedy:.0f} s, covered {int(gains.sum())}")

    out = dict(
        workload=args.workload, n=g.n, m=g.m, mode=args.mode, sources=int(len(wl.sources)),
        sources_sha256=sha(np.asarray(wl.sources, np.int32)), seed=wl.seed, attempt_offset=0,
        n_attempts=n_attempts, k=k,
        counters=dict(attempts=attempts, hits=hits, dead_ends=dead, cycles=cycles, steps=steps,
                      walk_ids=int(ids.shape[0])),
        sha256=dict(attempt=sha(attempt.astype("<u8")), off=sha(off.astype("<u8")), ids=sha(ids.astype("<u4")),
                    counts=sha(cnt.astype("<u4")),
                    col_off=sha(g.col_off.astype("<i8")), row_idx=sha(g.row_idx.astype("<i4")),
                    w=w_sha),
        selected=[int(x) for x in sel], gains=[int(x) for x in gains], covered=int(gains.sum()),
        oracle=dict(processes=P, shards=S, host_cpu=host_cpu(), host_threads=os.cpu_count(),
                    seconds=dict(generate=round(t_gen, 1), sample=round(t_sample, 1), count=round(t_count, 1),
                                 greedy=round(t_greedy, 1))),
        generator="tests/golden/make_fullsize_digest.py (oracle/ and the input generators only)",
    )
    path = args.out or os.path.join(HERE, f"{args.workload}_digest.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    say("wrote", path)


if __name__ == "__main__":
    main()
