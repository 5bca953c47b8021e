"""Seeded synthetic workloads (input generators only).

This module builds graphs, LT weights, source sets and query mixes.  It holds
none of the method's arithmetic (no thresholds, no random walks, no counting,
no greedy); both the oracle-based tests and the HIP path draw their inputs
from here, and it imports neither.

The paper evaluates on public social/Internet graphs (its dataset table:
DBLP, Pokec, Skitter, LiveJournal, Twitter).  Those files are not available;
seeded synthetic graphs of the same shapes stand in for them:

* ``er``:        directed G(n, m) -- ordered pairs u != v, first m distinct;
* ``chung_lu``:  power-law digraph, endpoint probabilities ~ i^(-1/(gamma-1))
                 under independent random id permutations for tails and heads;
* ``rmat``:      R-MAT (a, b, c, d) with a random relabelling of vertex ids,
                 self-loops and duplicate edges dropped.

Weights follow the paper's experimental setting w(u,v) = 1/d_in(v), or random
weights normalised per column (the normalisation of the GreedyCutting
comparison), or random weights with a random column sum.

All generators use torch so they run on the CPU (small cases) or on the GPU
(hundreds of millions of edges); results depend on (seed, device type).
"""
from dataclasses import dataclass, field
import math

import numpy as np
import torch

WALK_SEED = 2017


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _first_distinct(draw, n, m, device):
    """Draw (u, v) batches until m distinct non-loop pairs exist; keep the first
    m distinct pairs in draw order.  Returns int64 tensors (u, v)."""
    keys = torch.empty(0, dtype=torch.int64, device=device)
    distinct = 0
    while True:
        u, v = draw(int((m - distinct) * 1.25) + 4096)
        ok = u != v
        keys = torch.cat([keys, (u[ok] * n + v[ok])])
        uniq, inv = torch.unique(keys, return_inverse=True)
        distinct = uniq.numel()
        if distinct >= m:
            pos = torch.arange(keys.numel(), device=device)
            first = torch.full((uniq.numel(),), keys.numel(), dtype=torch.int64, device=device)
            first.scatter_reduce_(0, inv, pos, reduce="amin")
            order = torch.argsort(first)[:m]
            sel = uniq[order]
            return sel // n, sel % n


def er(n, m, seed, device="cpu"):
    g = _gen(seed, device)

    def draw(b):
        u = torch.randint(0, n, (b,), generator=g, device=device)
        v = torch.randint(0, n, (b,), generator=g, device=device)
        return u, v

    return _first_distinct(draw, n, m, device)


def chung_lu(n, m, gamma, seed, device="cpu"):
    g = _gen(seed, device)
    i = torch.arange(1, n + 1, dtype=torch.float64, device=device)
    p = i.pow(-1.0 / (gamma - 1.0))
    cdf = torch.cumsum(p, 0)
    cdf = cdf / cdf[-1]
    perm_out = torch.randperm(n, generator=g, device=device)
    perm_in = torch.randperm(n, generator=g, device=device)

    def pick(b, perm):
        x = torch.rand(b, generator=g, dtype=torch.float64, device=device)
        k = torch.searchsorted(cdf, x).clamp_(max=n - 1)
        return perm[k]

    def draw(b):
        return pick(b, perm_out), pick(b, perm_in)

    return _first_distinct(draw, n, m, device)


def rmat(scale, edge_factor, abcd, seed, device="cpu"):
    """R-MAT with Graph500-style vertex relabelling; loops and duplicates dropped."""
    a, b, c, _ = abcd
    g = _gen(seed, device)
    n = 1 << scale
    e = edge_factor * n
    u = torch.zeros(e, dtype=torch.int64, device=device)
    v = torch.zeros(e, dtype=torch.int64, device=device)
    for level in range(scale):
        r = torch.rand(e, generator=g, device=device)
        bit = 1 << (scale - 1 - level)
        row = r >= (a + b)                       # quadrants c, d
        col = ((r >= a) & (r < a + b)) | (r >= (a + b + c))  # quadrants b, d
        u += row.to(torch.int64) * bit
        v += col.to(torch.int64) * bit
        del r, row, col
    perm = torch.randperm(n, generator=g, device=device)
    u = perm[u]
    v = perm[v]
    ok = u != v
    key = torch.unique(v[ok] * n + u[ok])  # sorted, (head, tail) order
    del u, v, ok
    return key % n, key // n


def to_csc(n, tail, head):
    """In-edge CSC sorted by (head, tail): col_off int64[n+1], row_idx int32[m]."""
    key = torch.unique(head.to(torch.int64) * n + tail.to(torch.int64))
    col = key // n
    row = (key % n).to(torch.int32)
    deg = torch.bincount(col, minlength=n)
    col_off = torch.zeros(n + 1, dtype=torch.int64, device=key.device)
    col_off[1:] = torch.cumsum(deg, 0)
    return col_off, row


def _edge_cols(col_off):
    n = col_off.numel() - 1
    deg = (col_off[1:] - col_off[:-1])
    return torch.repeat_interleave(torch.arange(n, device=col_off.device), deg), deg


def weights_inv_indeg(col_off):
    """w(u,v) = 1/d_in(v) in fp32 (the paper's parameter setting)."""
    cols, deg = _edge_cols(col_off)
    return (1.0 / deg.to(torch.float32))[cols]


def _col_sums(col_off, x, cols_per_call=1 << 22):
    """Per-column sums of x: a segmented sum (differences of one prefix sum over
    every edge lose the small columns once the total is large), taken over
    ranges of columns so each call stays within the reduction's launch limits."""
    n = col_off.numel() - 1
    deg = col_off[1:] - col_off[:-1]
    out = torch.empty(n, dtype=x.dtype, device=x.device)
    for c0 in range(0, n, cols_per_call):
        c1 = min(n, c0 + cols_per_call)
        e0, e1 = int(col_off[c0]), int(col_off[c1])
        out[c0:c1] = torch.segment_reduce(x[e0:e1], "sum", lengths=deg[c0:c1], unsafe=True,
                                          initial=0.0)
    return out


def weights_random_colsum(col_off, lo, hi, seed):
    """x ~ U(0,1) per edge, column sum s_v ~ U(lo, hi): w = fp32(x * s_v / sum x)."""
    g = _gen(seed, col_off.device)
    m = int(col_off[-1])
    n = col_off.numel() - 1
    x = torch.rand(m, generator=g, dtype=torch.float64, device=col_off.device)
    s = lo + (hi - lo) * torch.rand(n, generator=g, dtype=torch.float64, device=col_off.device)
    cols, _ = _edge_cols(col_off)
    tot = _col_sums(col_off, x)
    return (x * s[cols] / tot[cols]).to(torch.float32)


def weights_normalized(col_off, seed):
    """x ~ U(0,1) per edge normalised to column sum 1 (GreedyCutting setting)."""
    g = _gen(seed, col_off.device)
    m = int(col_off[-1])
    x = torch.rand(m, generator=g, dtype=torch.float64, device=col_off.device)
    cols, _ = _edge_cols(col_off)
    tot = _col_sums(col_off, x)
    return (x / tot[cols]).to(torch.float32)


def pick_sources(n, count, seed):
    """count distinct nodes uniformly at random, ascending (int32 numpy)."""
    g = _gen(seed, "cpu")
    return np.sort(torch.randperm(n, generator=g)[:count].numpy().astype(np.int32))


@dataclass
class Workload:
    name: str
    n: int
    col_off: torch.Tensor
    row_idx: torch.Tensor
    w: torch.Tensor
    sources: np.ndarray
    n_attempts: int
    k: int
    modes: tuple
    seed: int = WALK_SEED
    desc: dict = field(default_factory=dict)

    @property
    def m(self):
        return int(self.row_idx.numel())

    def host(self):
        return (self.col_off.cpu().numpy(), self.row_idx.cpu().numpy(), self.w.cpu().numpy())


RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)

WORKLOAD_SPECS = {
    # name: (generator description, sources, attempts, k, modes)
    "er1k": dict(kind="er", n=1000, m=8000, gseed=1, weights="inv_indeg", n_src=10, sseed=101,
                 n_attempts=100_000, k=10, modes=("edges",)),
    "cl1m": dict(kind="chung_lu", n=1_000_000, m=16_000_000, gamma=2.1, gseed=2,
                 weights="colsum", lo=0.5, hi=1.0, n_src=1000, sseed=102,
                 n_attempts=10_000_000, k=100, modes=("edges", "nodes")),
    "rmat24": dict(kind="rmat", scale=24, ef=16, gseed=3, weights="inv_indeg", n_src=10_000,
                   sseed=103, n_attempts=100_000_000, k=1000, modes=("edges",)),
    "rmat26": dict(kind="rmat", scale=26, ef=24, gseed=4, weights="normalized", n_src=100_000,
                   sseed=104, n_attempts=200_000_000, k=1000, modes=("edges",)),
    "rmat22": dict(kind="rmat", scale=22, ef=16, gseed=5, weights="inv_indeg", n_src=10_000,
                   sseed=105, n_attempts=1_000_000, k=100, modes=("edges", "nodes")),
}


def build_graph(spec, device="cpu"):
    kind = spec["kind"]
    if kind == "er":
        n = spec["n"]
        t, h = er(n, spec["m"], spec["gseed"], device)
    elif kind == "chung_lu":
        n = spec["n"]
        t, h = chung_lu(n, spec["m"], spec["gamma"], spec["gseed"], device)
    elif kind == "rmat":
        n = 1 << spec["scale"]
        t, h = rmat(spec["scale"], spec["ef"], spec.get("abcd", RMAT_ABCD), spec["gseed"], device)
    else:
        raise ValueError(kind)
    col_off, row_idx = to_csc(n, t, h)
    del t, h
    wk = spec["weights"]
    if wk == "inv_indeg":
        w = weights_inv_indeg(col_off)
    elif wk == "colsum":
        w = weights_random_colsum(col_off, spec["lo"], spec["hi"], spec["gseed"] + 1000)
    elif wk == "normalized":
        w = weights_normalized(col_off, spec["gseed"] + 1000)
    else:
        raise ValueError(wk)
    return n, col_off, row_idx, w


def load(name, device="cpu", **override):
    spec = dict(WORKLOAD_SPECS[name])
    spec.update(override)
    n, col_off, row_idx, w = build_graph(spec, device)
    sources = pick_sources(n, spec["n_src"], spec["sseed"])
    return Workload(name=name, n=n, col_off=col_off, row_idx=row_idx, w=w, sources=sources,
                    n_attempts=spec["n_attempts"], k=spec["k"], modes=tuple(spec["modes"]),
                    desc=spec)


def query_mix(n, count, seed, max_sources=10_000, k_range=(10, 1000),
              attempts_range=(100_000, 10_000_000)):
    """Mixed interdiction queries: |X| log-uniform in [1, max_sources], k uniform
    in k_range, attempts log-uniform in attempts_range, mode edges/nodes 1/2 each."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        ns = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_sources + 1)))))
        ns = min(max(ns, 1), max_sources)
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        na = int(math.floor(math.exp(rng.uniform(math.log(attempts_range[0]),
                                                 math.log(attempts_range[1])))))
        mode = "edges" if rng.uniform() < 0.5 else "nodes"
        src = np.sort(rng.choice(n, size=ns, replace=False).astype(np.int32))
        out.append(dict(sources=src, k=k, n_attempts=na, mode=mode, seed=WALK_SEED + q))
    return out
