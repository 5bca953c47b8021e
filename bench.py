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
/ its HIP-event time), ``serve`` (the other half of the metric: 512 mixed
queries on R-MAT scale 22, batched closed-loop queries/s against one query
per call with every plain answer checked equal to the batched one, and
p50/p99 latency at an open-loop load of the batched rate) and
``cpu_baseline`` (the oracle on bounded prefixes of the same attempts: one
host core, and P processes on disjoint attempt ranges merged exactly, with
the host's CPU model and core counts).
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
                  "paper_1702_05854_amd/csrc/layout.hpp"]


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


def per_step_bytes(st, n_attempts, step_bytes):
    """The flat reading of the same launch: step_bytes per plain step (node
    record, the two bracketing thresholds, the tail id, membership), 4 bytes per
    attempt for its start, and 4 bytes per id plus 16 per kept walk written.
    29 bytes per step prices the two column offsets as 64-bit words, 21 as the
    32-bit words the node records actually hold."""
    return step_bytes * st["steps"] + 4 * n_attempts + 4 * st["walk_ids"] + 16 * st["hits"]


def load_traffic(workload, mode, n_attempts, cycle_steps):
    """Counter figures of the sampler launch of this query (the traffic file's
    fields), if they were taken on the same workload, mode, attempt count and
    cycle handling and on the current kernel sources; else {}."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("kernel_sha") != kernel_sha() or t.get("workload") != workload:
        return {}
    if (t.get("mode"), t.get("n_attempts"), t.get("cycle_steps")) != (mode, n_attempts, bool(cycle_steps)):
        return {}
    return t


def host_cpu():
    """CPU model, logical CPUs this process may use, physical cores."""
    model, cores = "", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and not model:
                    model = val
                elif key == "physical id":
                    phys = val
                elif key == "core id":
                    core = val
                elif not key and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    if phys is not None:
        cores.add((phys, core))
    try:
        logical = len(os.sched_getaffinity(0))
    except AttributeError:
        logical = os.cpu_count() or 1
    return model, logical, len(cores) or logical


def cpu_baseline(wl, mode, k, budget_s, max_procs=16):
    """The oracle as it stands: single-threaded on attempts [0, n_s), then P
    oracle processes on disjoint attempt ranges of a larger prefix, merged in
    attempt order (exact), counted and greedily solved by one process -- the
    one-core and multi-core columns of the paper's CPU/GPU comparison."""
    import numpy as np
    from oracle import cpu, shards
    col_off, row_idx, w = wl.host()
    og = cpu.Graph(col_off, row_idx, w)
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    model, logical, physical = host_cpu()
    # size the sample from a short probe so the timed run takes ~budget_s
    probe = 20_000
    t0 = time.perf_counter()
    og.sample(wl.sources, om, probe, 0, wl.seed)
    per = (time.perf_counter() - t0) / probe
    n_s = int(max(probe, min(wl.n_attempts, budget_s * 0.7 / max(per, 1e-9))))
    t0 = time.perf_counter()
    res = cpu.solve(og, wl.sources, om, k, n_s, 0, wl.seed)
    dt = time.perf_counter() - t0
    out = {"value": n_s / dt, "unit": "HSAW attempts/s", "cores": 1, "kind": "oracle",
           "sample": f"attempts [0, {n_s}) of the same query (sample + count + greedy k={k}), "
                     f"{dt:.1f} s on one host core",
           "hsaw_per_s": res["walks"].hits / dt, "steps_per_s": res["walks"].steps / dt,
           "host_cpu": model, "host_logical_cpus": logical, "host_physical_cores": physical}
    # multi-process: P workers on disjoint ranges of P times the sample
    P = max(1, min(max_procs, logical, physical))
    n_p = int(min(wl.n_attempts, n_s * P))
    print(f"[bench] cpu baseline: {P} oracle processes on {n_p} attempts", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    walks = shards.sample(og, wl.sources, om, n_p, 0, wl.seed, procs=P)
    t_sample = time.perf_counter() - t0
    id_space = og.m if om == cpu.MODE_EDGES else og.n
    t1 = time.perf_counter()
    sel, gains = cpu.greedy_csr(id_space, walks.off, walks.ids, k)
    t_greedy = time.perf_counter() - t1
    dt_p = time.perf_counter() - t0
    out["multi"] = {"value": n_p / dt_p, "unit": "HSAW attempts/s", "cores": P, "processes": P,
                    "sample": f"attempts [0, {n_p}) of the same query: {P} processes on disjoint "
                              f"ranges merged in attempt order, then one count + greedy k={k}",
                    "seconds": {"sample": t_sample, "count_greedy": t_greedy, "total": dt_p},
                    "hsaw_per_s": walks.hits / dt_p, "steps_per_s": walks.steps / dt_p,
                    "speedup_vs_one_core": (n_p / dt_p) / (n_s / dt)}
    return out


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def serve_measure(args, name, n_queries, loads, skip_plain=False):
    """Batched / served queries vs the plain path (one query per call, FIFO).

    Closed loop: every query of the mix is submitted at t=0; queries/s =
    count / makespan.  Open loop: Poisson arrivals at fractions of the
    batched closed-loop rate; the batch is fed in real time and per-query
    latency (done - arrival) is recorded.  The plain path serves one query at
    a time, so its open-loop latencies follow from its measured service times
    by the FIFO recurrence finish_i = max(arrival_i, finish_{i-1}) + service_i
    on the same arrival trace."""
    import numpy as np
    import torch
    from paper_1702_05854_amd import sia, workloads

    torch.cuda.set_device(0)
    print(f"[serve] generating {name}", file=sys.stderr, flush=True)
    wl = workloads.load(name, device="cuda")
    g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
    torch.cuda.synchronize()
    qs = workloads.query_mix(wl.n, n_queries, seed=5)
    total_att = sum(q["n_attempts"] for q in qs)
    print(f"[serve] n={wl.n} m={wl.m}: {len(qs)} queries, {total_att} attempts", file=sys.stderr,
          flush=True)

    cs = bool(getattr(args, "cycle_steps", False))  # cyclic walks stop at detection unless asked

    def submit_all(b, qlist):
        return [b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"], cs) for q in qlist]

    with sia.Batch(g, walk_budget_bytes=args.walk_budget << 20, use_graph=1,
                   greedy_mode=args.greedy_mode, greedy_cus=args.greedy_cus,
                   greedy_batch=args.greedy_batch) as b:
        # the tuner samples the largest query's sources for 1.6*10^7 attempts per candidate
        # shape, cyclic walks handled as they will be served: shorter probes let launch tails
        # decide the choice, and the exact-steps rate sized launches at 40% of the target
        probe = qs[int(np.argmax([q["n_attempts"] for q in qs]))]
        cfg = b.tune(probe["sources"], probe["mode"], 16_000_000,
                     seed=probe["seed"], target_ms=args.wave_ms, cycle_steps=cs)
        print(f"[serve] tuned {cfg}", file=sys.stderr, flush=True)
        # warm-up: a few queries through every path
        for t in submit_all(b, qs[:8]):
            b.wait(t)
        t0 = time.perf_counter()
        tickets = submit_all(b, qs)
        batched = []
        for i, t in enumerate(tickets):
            batched.append(b.wait(t))
            if (i + 1) % 64 == 0:
                print(f"[serve] batched {i + 1}/{len(qs)} done", file=sys.stderr, flush=True)
        makespan = time.perf_counter() - t0
        bstats = b.stats()
        closed_lat = [r["info"]["t_done"] - r["info"]["t_submit"] for r in batched]
        rate_b = len(qs) / makespan
        print(f"[serve] batched closed loop: {rate_b:.1f} q/s ({makespan:.2f} s)", file=sys.stderr,
              flush=True)

        # plain: one query per call, in order; the answers must agree
        service = []
        for i, q in enumerate(qs if not skip_plain else []):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = sia.solve(g, q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"], cycle_steps=cs)
            service.append(time.perf_counter() - t1)
            assert (r["selected"] == batched[i]["selected"]).all(), f"query {i}: batched != plain"
            assert (r["gains"] == batched[i]["gains"]).all(), f"query {i}: batched != plain"
            if (i + 1) % 64 == 0:
                print(f"[serve] plain {i + 1}/{len(qs)} done", file=sys.stderr, flush=True)
        rate_p = len(qs) / sum(service) if service else None
        if rate_p:
            print(f"[serve] plain: {rate_p:.1f} q/s", file=sys.stderr, flush=True)

        open_loop = []
        rng = np.random.default_rng(6)
        for frac in loads:
            lam = frac * rate_b
            arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(qs)))
            ts, lat = [], []
            base = time.perf_counter()
            for i, q in enumerate(qs):
                delay = arrivals[i] - (time.perf_counter() - base)
                if delay > 0:
                    time.sleep(delay)
                ts.append(b.submit(q["sources"], q["mode"], q["k"], q["n_attempts"], 0, q["seed"], cs))
            for t in ts:
                r = b.wait(t)
                lat.append(r["info"]["t_done"] - r["info"]["t_submit"])
            fin, plain_lat = 0.0, []
            for i in range(len(service)):
                fin = max(arrivals[i], fin) + service[i]
                plain_lat.append(fin - arrivals[i])
            open_loop.append({"load": frac, "arrivals_per_s": lam,
                              "batched_p50_s": percentile(lat, 50), "batched_p99_s": percentile(lat, 99),
                              "plain_p50_s": percentile(plain_lat, 50),
                              "plain_p99_s": percentile(plain_lat, 99)})
            print(f"[serve] open loop {frac}: {open_loop[-1]}", file=sys.stderr, flush=True)
    g.close()
    return {
        "workload": f"{name}: R-MAT s{wl.desc.get('scale')} ef{wl.desc.get('ef')}, {len(qs)} mixed queries",
        "n": wl.n, "m": wl.m, "queries": len(qs), "attempts_total": total_att,
        "batched_queries_per_s": rate_b, "makespan_s": makespan,
        "plain_queries_per_s": rate_p, "speedup_vs_plain": rate_b / rate_p if rate_p else None,
        "plain_answers_checked": len(service),
        "closed_loop_p50_s": percentile(closed_lat, 50), "closed_loop_p99_s": percentile(closed_lat, 99),
        "attempts_per_s_batched": total_att / makespan, "cycle_steps": cs,
        "open_loop": open_loop, "batch_stats": bstats,
    }


def serve_bench(args):
    name = args.workload if args.workload != "rmat24" else "rmat22"
    r = serve_measure(args, name, args.queries, args.loads, args.skip_plain)
    out = {
        "metric": "queries/s (mixed interdiction queries, batched and served)",
        "value": r["batched_queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": r["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": r["workload"], "n": r["n"], "m": r["m"], "queries": r["queries"],
                   "attempts_total": r["attempts_total"]},
        **{k: v for k, v in r.items() if k not in ("workload", "n", "m", "queries", "attempts_total")},
    }
    print(json.dumps(out), flush=True)


def sas_bench(args, sia, wl, g, mode, k, ingest_ms):
    """Stop-and-Stare driver (eSIA Algorithm 6 / nSIA Algorithm 9): wall time of
    whole runs with eps = args.eps and delta = 1/n; the sample count is the
    driver's own."""
    runs = []
    for i in range(args.warmup + args.steps):
        t0 = time.perf_counter()
        r = sia.sas_solve(g, wl.sources, mode, k, args.eps, None, wl.seed)
        dt = time.perf_counter() - t0
        print(f"[bench] sas run {i + 1}/{args.warmup + args.steps}: {dt * 1e3:.1f} ms", file=sys.stderr,
              flush=True)
        if i >= args.warmup:
            runs.append((dt, r))
    ms = sum(d for d, _ in runs) / len(runs) * 1e3
    info = runs[-1][1]["info"]
    out = {"metric": "Stop-and-Stare runs/s (eSIA/nSIA to (1-1/e-eps) with delta = 1/n)",
           "value": 1e3 / ms, "unit": "runs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"{wl.name}: {wl.desc['kind']} n={wl.n} m={wl.m}", "mode": mode, "k": k,
                      "eps": args.eps, "delta": 1.0 / wl.n, "sources": len(wl.sources), "seed": wl.seed},
           "ingest_ms": ingest_ms, "info": info,
           "attempts_per_s": info["attempts_sampled"] / (ms * 1e-3)}
    print(json.dumps(out), flush=True)


def sweep_bench(args):
    """Scalability sweep, as the paper's scalability test runs it (Section
    6.3, "Scalability Test"): nSIA end to end -- the Stop-and-Stare driver
    over the sampler, counts and greedy -- on uniform random graphs with n
    from 10^4 to --sweep-max nodes and m/n in {5, 10, 15}; w = 1/d_in, 1000
    random suspects with probabilities uniform in (0, 1), k = 100 nodes,
    eps = 0.1, delta = 1/n (the experiments' settings, Section 6.1).  One
    untimed run per point, then one timed run (wall time of the call).  At
    n <= --sweep-check the oracle's driver runs the same point and its
    iteration, sample sizes, picks and gains must be equal."""
    import numpy as np
    import torch
    from paper_1702_05854_amd import sia, workloads

    torch.cuda.set_device(0)
    rows = []
    n = 10_000
    while n <= args.sweep_max:
        for ratio in (5, 10, 15):
            t0 = time.perf_counter()
            wl = workloads.load("er1k", device="cuda", n=n, m=n * ratio, n_src=10, k=100, gseed=11 + ratio,
                                sseed=211)
            torch.cuda.synchronize()
            gen_s = time.perf_counter() - t0
            g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
            rng = np.random.default_rng(1000 + ratio)
            sus = np.sort(rng.choice(n, 1000, replace=False)).astype(np.int32)
            p = rng.uniform(0, 1, 1000).astype(np.float32)
            sia.sas_solve_suspects(g, sus, p, "nodes", 100, 0.1, None, wl.seed)  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = sia.sas_solve_suspects(g, sus, p, "nodes", 100, 0.1, None, wl.seed)
            dt = time.perf_counter() - t1
            I = r["info"]
            row = {"n": n, "m": wl.m, "m_over_n": ratio, "seconds": dt, "status": I["status"], "t": I["t"],
                   "n_t": I["n_t"], "attempts_sampled": I["attempts_sampled"], "eps_t": I["eps_t"],
                   "gen_seconds": gen_s, "oracle_equal": None}
            if n <= args.sweep_check:
                from oracle import cpu, sas
                og = cpu.Graph(*wl.host())
                ref = sas.stop_and_stare(og, sus, cpu.MODE_NODES, 100, 0.1, None, wl.seed, p=p)
                row["oracle_equal"] = bool(
                    ref["status"] == "passed" and I["status"] == 1 and (I["t"], I["n_t"]) == (ref["t"], ref["n_t"])
                    and np.array_equal(r["selected"], ref["selected"]) and np.array_equal(r["gains"], ref["gains"])
                    and (I["cov_r"], I["cov_rp"]) == (ref["cov_r"], ref["cov_rp"]))
                assert row["oracle_equal"], (n, ratio)
            rows.append(row)
            print(f"[bench] sweep n={n} m={wl.m}: nSIA {dt:.3f} s (t={I['t']}, N_t={I['n_t']}, "
                  f"{I['attempts_sampled']} attempts; oracle equal: {row['oracle_equal']})", file=sys.stderr,
                  flush=True)
            g.close()
            del wl, g
            torch.cuda.empty_cache()
        n *= 10
    out = {"metric": "nSIA running time across graph sizes (scalability sweep, Stop-and-Stare end to end)",
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "uniform random graphs, w = 1/d_in, 1000 suspects with p ~ U(0,1), "
                                  "nSIA k = 100, eps = 0.1, delta = 1/n"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def sweep_fixed_bench(args):
    """The sweep's graphs with a fixed sample count: eSIA, n/1000 sources, k =
    100 edges, 10^7 attempts per point (fewer where the kept walks would hold
    more than 2^30 ids); whole-path attempts/s."""
    import torch
    from paper_1702_05854_amd import sia, workloads

    torch.cuda.set_device(0)
    rows = []
    n = 10_000
    while n <= args.sweep_max:
        for ratio in (5, 10, 15):
            wl = workloads.load("er1k", device="cuda", n=n, m=n * ratio, n_src=max(10, n // 1000), k=100,
                                gseed=11 + ratio, sseed=211)
            g = sia.Graph(wl.col_off, wl.row_idx, wl.w)
            # pilot (also the warm-up): walks on these graphs can be long, so the
            # attempts are capped to keep the kept walks' ids within 2^30
            pilot = sia.solve(g, wl.sources, "edges", 100, 100_000, 0, wl.seed)["stats"]
            ids_per_attempt = max(pilot["walk_ids"], 1) / 100_000
            N = int(min(10_000_000, max(100_000, (1 << 30) / ids_per_attempt)))
            sia.solve(g, wl.sources, "edges", 100, N, 0, wl.seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sia.solve(g, wl.sources, "edges", 100, N, 0, wl.seed, timing=True)
            dt = time.perf_counter() - t0
            st = r["stats"]
            rows.append({"n": n, "m": wl.m, "m_over_n": ratio, "attempts": N, "ms": dt * 1e3,
                         "attempts_per_s": N / dt, "hits": st["hits"], "steps": st["steps"],
                         "ms_sample": st["ms_sample"], "ms_count": st["ms_count"], "ms_greedy": st["ms_greedy"]})
            print(f"[bench] sweep n={n} m={wl.m}: {N / dt / 1e6:.1f}M attempts/s", file=sys.stderr, flush=True)
            g.close()
            del wl, g
            torch.cuda.empty_cache()
        n *= 10
    out = {"metric": "HSAW attempts/s across graph sizes (fixed-sample sweep, whole path, edges)",
           "unit": "attempts/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "uniform random graphs, w = 1/d_in, up to 10^7 attempts, k = 100"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--mode", default=None)
    ap.add_argument("--attempts", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cycle-steps", action="store_true",
                    help="timed runs also search cyclic walks for their entry (exact step counts)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the batched-vs-plain block (mixed queries on R-MAT s22) of the default run")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="batched/served queries vs plain on the mixed-query workload (rmat22)")
    ap.add_argument("--queries", type=int, default=512)
    ap.add_argument("--walk-budget", type=int, default=16384, help="MiB of walk buffers (--serve)")
    ap.add_argument("--wave-ms", type=float, default=50.0, help="target sampling launch (--serve)")
    ap.add_argument("--loads", type=float, nargs="*", default=[0.5, 0.8, 1.0])
    ap.add_argument("--greedy-mode", type=int, default=0,
                    help="0: greedy between sampling launches, 1: on a second stream (--serve)")
    ap.add_argument("--greedy-cus", type=int, default=0, help="CUs reserved for the greedy (--serve)")
    ap.add_argument("--greedy-batch", type=int, default=0, help="queries per greedy launch (--serve)")
    ap.add_argument("--skip-plain", action="store_true", help="batched side only (--serve, profiling)")
    ap.add_argument("--sas", action="store_true",
                    help="time the Stop-and-Stare driver (eSIA / nSIA) on the workload instead")
    ap.add_argument("--eps", type=float, default=0.1, help="epsilon of the Stop-and-Stare driver (--sas)")
    ap.add_argument("--sweep", action="store_true",
                    help="scalability sweep: nSIA (Stop-and-Stare) time on random graphs, n = 10^4 .. --sweep-max, "
                         "m/n = 5, 10, 15")
    ap.add_argument("--sweep-fixed", action="store_true",
                    help="the same graphs with a fixed sample count (eSIA attempts/s)")
    ap.add_argument("--sweep-max", type=int, default=100_000_000)
    ap.add_argument("--sweep-check", type=int, default=100_000,
                    help="largest n whose sweep point is also run by the oracle and compared")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the benchmark runs on one MI355X)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.sweep:
        sweep_bench(args)
        return
    if args.sweep_fixed:
        sweep_fixed_bench(args)
        return

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

    if args.sas:
        sas_bench(args, sia, wl, g, mode, k, ingest_ms)
        return

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # The first warm-up run (untimed) counts every walk's steps exactly,
    # cyclic walks included: its counters give the algorithmic bytes.  The
    # timed runs stop cyclic walks at detection unless --cycle-steps asks
    # otherwise (the walk is discarded either way; picks and gains are
    # checked equal to the exact run's).
    exact = None
    for i in range(max(args.warmup, 1)):
        r = sia.solve(g, wl.sources, mode, k, n_att, 0, wl.seed, timing=True,
                      cycle_steps=args.cycle_steps or i == 0)
        exact = exact or r
        print(f"[bench] warmup {i + 1}/{max(args.warmup, 1)} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(sia.solve(g, wl.sources, mode, k, n_att, 0, wl.seed, timing=True,
                              cycle_steps=args.cycle_steps))
        print(f"[bench] step {i + 1}/{args.steps}: {runs[-1]['stats']['ms_total']:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = dict(exact["stats"])  # exact counters (same walks, same picks)
    st_timed = runs[-1]["stats"]
    for r in runs:
        assert (r["selected"] == exact["selected"]).all() and (r["gains"] == exact["gains"]).all(), \
            "timed runs must select what the exact run selects"
        for key in ("hits", "dead_ends", "cycles", "walk_ids", "covered"):
            assert r["stats"][key] == st[key], key
    ms_sample = sum(r["stats"]["ms_sample"] for r in runs) / len(runs)
    ms_count = sum(r["stats"]["ms_count"] for r in runs) / len(runs)
    ms_greedy = sum(r["stats"]["ms_greedy"] for r in runs) / len(runs)
    ms_step = elapsed * 1e3 / args.steps
    b_alg = algorithmic_bytes(st)
    achieved = b_alg / (ms_sample * 1e-3) / 1e9
    counters = load_traffic(args.workload, mode, n_att, args.cycle_steps)
    traffic, fetched = counters.get("traffic_bytes_per_launch"), counters.get("fetch_bytes_per_launch")

    out = {
        "metric": f"HSAW attempts/s (whole {'eSIA' if mode == 'edges' else 'nSIA'} hot path: sample + count + greedy)",
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
        "evaluations_per_s": st_timed["evaluations"] * args.steps / elapsed,
        "cycle_steps_in_timed_runs": bool(args.cycle_steps),
        "ms_sample_exact_cycle_steps": exact["stats"]["ms_sample"],
        "evaluations_exact_cycle_steps": exact["stats"]["evaluations"],
        "sampler_attempts_per_s": n_att / (ms_sample * 1e-3),
        "ms_sample": ms_sample, "ms_count": ms_count, "ms_greedy": ms_greedy,
        "ms_sample_median": sorted(r["stats"]["ms_sample"] for r in runs)[len(runs) // 2],
        "ingest_ms": ingest_ms,
        "arc_record_bytes": g.arc_bytes,
        "counts": {**{key: st[key] for key in ("hits", "dead_ends", "cycles", "steps", "walk_ids", "covered")},
                   "evaluations": st_timed["evaluations"]},
        "suspension_est": st["suspension_est"],
        "roofline": {"bound": "hbm", "kernel": "k_sample", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": b_alg, "traffic": traffic,
                     "gather_efficiency": b_alg / fetched if fetched else None,
                     "l2_hit_rate": counters.get("l2_hit_rate"),
                     "frac_other_readings": {
                         **{f"{sb} B/step flat": per_step_bytes(st, n_att, sb) / (ms_sample * 1e-3) / 1e9
                            / HBM_PEAK_GBS for sb in (29, 21)},
                         "cycle entries searched (untimed exact run)":
                             b_alg / (exact["stats"]["ms_sample"] * 1e-3) / 1e9 / HBM_PEAK_GBS}},
        "cpu_baseline": None,
    }
    g.close()
    # random-gather ceiling of the device: the sampler's line rate against it
    ceil_ind, _ = sia.probe_gather(2 << 30, 512, dependent=False)
    ceil_dep, _ = sia.probe_gather(2 << 30, 512, dependent=True)
    traffic = out["roofline"]["traffic"]
    samp_lines = traffic / 128.0 / (ms_sample * 1e-3) if traffic else None
    out["gather_ceiling"] = {
        "probe": "4-byte loads at uniformly random positions of a 2 GiB array, full occupancy",
        "independent_lines_per_s": ceil_ind, "dependent_lines_per_s": ceil_dep,
        "sampler_lines_per_s": samp_lines,
        "sampler_frac_of_independent": samp_lines / ceil_ind if samp_lines else None,
        "sampler_frac_of_dependent": samp_lines / ceil_dep if samp_lines else None}
    del g
    torch.cuda.empty_cache()
    if not args.no_serve:
        # the other half of the metric: batched vs plain queries/s on the mixed workload
        out["serve"] = serve_measure(args, "rmat22", args.queries, [1.0])
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, mode, k, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
