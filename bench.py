"""Benchmark: HSAW attempts/s of the whole hot path on one MI355X.

One step = one eSIA query through the C ABI on a device-resident graph:
sample N HSAW attempts, count coverage, build the inverted index, run k
greedy rounds (sia_solve).  Graph ingest (weights -> threshold tables) runs
once before the timed region and is reported as ``ingest_ms``.

Default workload: R-MAT scale 24, edge factor 16 (a,b,c,d = .57,.19,.19,.05,
self-loops and duplicates dropped), w = 1/d_in, 10^4 random sources, 10^8
attempts, k = 1000, edges.  Inputs are synthetic (seeded) and generated on
the GPU; they stand in for the paper's Twitter-scale graph.

The JSON line carries ``roofline`` for the sampling kernel (algorithmic bytes
/ its HIP-event time) and ``cpu_baseline`` (the single-threaded oracle on a
bounded prefix of the same attempts).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_sample_rmat24.json")
KERNEL_SOURCES = ["paper_1702_05854_amd/csrc/sample.hip", "paper_1702_05854_amd/csrc/philox.hpp",
                  "paper_1702_05854_amd/csrc/common.hpp"]


def kernel_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(st):
    """Bytes the method itself must move in one sampling launch.

    Per live-edge draw of the plain walk (Algorithm 1): the 16-byte node record
    (offset, degree, last threshold) and one byte of source membership; a
    draw that finds a live edge also reads the two thresholds bracketing r and
    the tail node (12 bytes).  Per kept walk: its ids (4 bytes each) and a
    20-byte record.  Extra evaluations of the cycle-detection and re-walk
    passes are not counted."""
    s, d = st["steps"], st["dead_ends"]
    return 17 * s + 12 * (s - d) + 4 * st["walk_ids"] + 20 * st["hits"]


def load_traffic():
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("traffic_bytes_per_launch")


def cpu_baseline(wl, mode, k, budget_s):
    """The oracle as it stands, single-threaded, on attempts [0, n_s)."""
    import numpy as np
    from oracle import cpu
    col_off, row_idx, w = wl.host()
    og = cpu.Graph(col_off, row_idx, w)
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    # size the sample from a short probe so the timed run takes ~budget_s
    probe = 20_000
    t0 = time.perf_counter()
    og.sample(wl.sources, om, probe, 0, wl.seed)
    per = (time.perf_counter() - t0) / probe
    n_s = int(max(probe, min(wl.n_attempts, budget_s * 0.7 / max(per, 1e-9))))
    t0 = time.perf_counter()
    res = cpu.solve(og, wl.sources, om, k, n_s, 0, wl.seed)
    dt = time.perf_counter() - t0
    return {"value": n_s / dt, "unit": "HSAW attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"attempts [0, {n_s}) of the same query (sample + count + greedy k={k}), "
                      f"{dt:.1f} s on one host core",
            "hsaw_per_s": res["walks"].hits / dt, "steps_per_s": res["walks"].steps / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--mode", default=None)
    ap.add_argument("--attempts", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(this build runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1702_05854_amd import sia, workloads

    torch.cuda.set_device(0)
    dev = "cuda"
    print(f"[bench] generating {args.workload} on the GPU", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    wl = workloads.load(args.workload, device=dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    mode = args.mode or wl.modes[0]
    n_att = args.attempts or wl.n_attempts
    k = wl.k
    print(f"[bench] n={wl.n} m={wl.m} gen {gen_s:.1f}s; ingest", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
    torch.cuda.synchronize()
    ingest_ms = (time.perf_counter() - t0) * 1e3

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for i in range(args.warmup):
        sia.solve(g, wl.sources, mode, k, n_att, 0, wl.seed, timing=True)
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(sia.solve(g, wl.sources, mode, k, n_att, 0, wl.seed, timing=True))
        print(f"[bench] step {i + 1}/{args.steps}: {runs[-1]['stats']['ms_total']:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = runs[-1]["stats"]
    for r in runs[1:]:
        assert (r["selected"] == runs[0]["selected"]).all(), "non-deterministic selection"
    ms_sample = sum(r["stats"]["ms_sample"] for r in runs) / len(runs)
    ms_count = sum(r["stats"]["ms_count"] for r in runs) / len(runs)
    ms_greedy = sum(r["stats"]["ms_greedy"] for r in runs) / len(runs)
    ms_step = elapsed * 1e3 / args.steps
    b_alg = algorithmic_bytes(st)
    achieved = b_alg / (ms_sample * 1e-3) / 1e9

    out = {
        "metric": "HSAW attempts/s (whole eSIA hot path: sample + count + greedy)",
        "value": n_att * args.steps / elapsed,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: R-MAT s{wl.desc.get('scale')} ef{wl.desc.get('ef')}"
                   if wl.desc.get("kind") == "rmat" else args.workload,
                   "n": wl.n, "m": wl.m, "sources": int(len(wl.sources)), "n_attempts": n_att,
                   "k": k, "mode": mode, "weights": wl.desc.get("weights"), "seed": wl.seed},
        "hsaw_per_s": st["hits"] * args.steps / elapsed,
        "steps_per_s": st["steps"] * args.steps / elapsed,
        "evaluations_per_s": st["evaluations"] * args.steps / elapsed,
        "sampler_attempts_per_s": n_att / (ms_sample * 1e-3),
        "ms_sample": ms_sample, "ms_count_index": ms_count, "ms_greedy": ms_greedy,
        "ingest_ms": ingest_ms,
        "counts": {key: st[key] for key in ("hits", "dead_ends", "cycles", "steps", "evaluations",
                                            "walk_ids", "covered")},
        "suspension_est": st["suspension_est"],
        "roofline": {"bound": "hbm", "kernel": "k_sample", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": b_alg, "traffic": load_traffic()},
        "cpu_baseline": None,
    }
    g.close()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, mode, k, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
