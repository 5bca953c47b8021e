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

Every random draw comes from a counter-based integer hash (the SplitMix64
finaliser of Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) of (seed, stream, index), evaluated with wrapping
int64 tensor arithmetic, and every later step is integer work, sorting of
distinct keys, or correctly rounded float64 division: a graph is the same bit
for bit whether it is generated on the CPU or on the GPU.
"""
from dataclasses import dataclass, field
import math

import numpy as np
import torch

WALK_SEED = 2017


def _i64(x):
    """Python int in [0, 2^64) -> the int64 value with the same bits."""
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


_GAMMA = _i64(0x9E3779B97F4A7C15)
_MIX1 = _i64(0xBF58476D1CE4E5B9)
_MIX2 = _i64(0x94D049BB133111EB)
_LO32 = (1 << 32) - 1


def _shr(x, s):
    """Logical right shift of an int64 tensor."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def mix64(z):
    """SplitMix64 finaliser on an int64 tensor (wrapping arithmetic)."""
    z = (z ^ _shr(z, 30)) * _MIX1
    z = (z ^ _shr(z, 27)) * _MIX2
    return z ^ _shr(z, 31)


def _mix64_int(z):
    """The same finaliser on a Python int (for keys)."""
    M = (1 << 64) - 1
    z &= M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def hash64(seed, stream, idx):
    """64 random bits for every index of the int64 tensor idx, keyed by
    (seed, stream): mix64(idx * gamma + key)."""
    key = _i64(_mix64_int(_mix64_int(int(seed) * 0x9E3779B97F4A7C15 + 1) + int(stream)))
    return mix64(idx * _GAMMA + key)


def _unit53(h):
    """Uniform double in [0, 1) from the high 53 bits (exact)."""
    return _shr(h, 11).to(torch.float64) * (2.0 ** -53)


def _below(r32, n):
    """floor(r32 * n / 2^32) for 32-bit draws r32 and n < 2^31."""
    return _shr(r32 * n, 32)


def random_permutation(n, seed, stream, device):
    """A permutation of 0..n-1: the ids sorted by (hash, id) keys, which are
    distinct, so any sort gives the same order."""
    bits = max(1, (n - 1).bit_length())
    i = torch.arange(n, dtype=torch.int64, device=device)
    key = (_shr(hash64(seed, stream, i), bits + 1) << bits) | i
    return torch.argsort(key)


def _first_distinct(draw, n, m, device):
    """Draw (u, v) batches until m distinct non-loop pairs exist; keep the first
    m distinct pairs in draw order.  draw(start, count) returns the pairs of
    draws start .. start+count-1.  Returns int64 tensors (u, v)."""
    keys = torch.empty(0, dtype=torch.int64, device=device)
    distinct = 0
    drawn = 0
    while True:
        b = int((m - distinct) * 1.25) + 4096
        u, v = draw(drawn, b)
        drawn += b
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
    """Directed G(n, m): ordered pairs (u, v), u != v, the first m distinct in
    draw order; draw i takes u and v from the two halves of hash(seed, 0, i)."""
    def draw(start, count):
        h = hash64(seed, 0, torch.arange(start, start + count, dtype=torch.int64, device=device))
        return _below(_shr(h, 32), n), _below(h & _LO32, n)

    return _first_distinct(draw, n, m, device)


def chung_lu(n, m, gamma, seed, device="cpu"):
    """Chung-Lu digraph: tail and head of each draw picked with probability
    proportional to i^(-1/(gamma-1)) (i = 1..n) under independent random id
    permutations.  The cumulative table is summed on the CPU in ascending
    order, so both devices search the same table."""
    i = np.arange(1, n + 1, dtype=np.float64)
    cdf = np.cumsum(i ** (-1.0 / (gamma - 1.0)))
    cdf = torch.from_numpy(cdf / cdf[-1]).to(device)
    perm_out = random_permutation(n, seed, 1, device)
    perm_in = random_permutation(n, seed, 2, device)

    def pick(x, perm):
        k = torch.searchsorted(cdf, x).clamp_(max=n - 1)
        return perm[k]

    def draw(start, count):
        idx = torch.arange(start, start + count, dtype=torch.int64, device=device)
        return (pick(_unit53(hash64(seed, 3, idx)), perm_out), pick(_unit53(hash64(seed, 4, idx)), perm_in))

    return _first_distinct(draw, n, m, device)


def rmat_keys(scale, edge_factor, abcd, seed, device="cpu", chunk=1 << 25):
    """R-MAT edge keys head * n + tail after the Graph500-style random vertex
    relabelling, self-loops removed, duplicates kept, in generation order.
    Edge e at level l (l = 0 is the top bit) takes a 32-bit draw from
    hash(seed, 16 + l // 2, e) (high half for even l, low half for odd) and
    picks quadrant a, b, c or d by integer thresholds round(a 2^32),
    round((a+b) 2^32), round((a+b+c) 2^32)."""
    a, b, c, _ = abcd
    TA = int(round(a * 2 ** 32))
    TAB = int(round((a + b) * 2 ** 32))
    TABC = int(round((a + b + c) * 2 ** 32))
    n = 1 << scale
    total = edge_factor * n
    perm = random_permutation(n, seed, 1, device)
    out = torch.empty(total, dtype=torch.int64, device=device)
    filled = 0
    for e0 in range(0, total, chunk):
        idx = torch.arange(e0, min(total, e0 + chunk), dtype=torch.int64, device=device)
        u = torch.zeros_like(idx)
        v = torch.zeros_like(idx)
        for level in range(scale):
            if level % 2 == 0:
                h = hash64(seed, 16 + level // 2, idx)
                r = _shr(h, 32)
            else:
                r = h & _LO32
            bit = 1 << (scale - 1 - level)
            row = r >= TAB                                   # quadrants c, d
            col = ((r >= TA) & (r < TAB)) | (r >= TABC)      # quadrants b, d
            u += row.to(torch.int64) * bit
            v += col.to(torch.int64) * bit
        u = perm[u]
        v = perm[v]
        ok = u != v
        kept = v[ok] * n + u[ok]
        out[filled:filled + kept.numel()] = kept
        filled += kept.numel()
        del idx, u, v, ok, h, r, kept
    return out[:filled]


def unique_sorted(keys):
    """The distinct values of an int64 tensor, ascending.  On the CPU the
    tensor's own memory is sorted in place and compacted (billion-edge graphs
    fit in host memory that way); on the GPU torch.unique."""
    if keys.device.type != "cpu":
        return torch.unique(keys)
    a = keys.numpy()
    a.sort()  # in place (equal keys are identical, so the order among them cannot matter)
    w = 0
    step = 1 << 26
    prev = None
    for i0 in range(0, a.shape[0], step):
        blk = a[i0:i0 + step]
        keep = np.empty(blk.shape[0], dtype=bool)
        keep[1:] = blk[1:] != blk[:-1]
        keep[0] = prev is None or blk[0] != prev
        prev = blk[-1]
        kept = blk[keep]            # a copy, so the forward write below is safe
        a[w:w + kept.shape[0]] = kept
        w += kept.shape[0]
    return keys[:w]


def csc_from_keys(n, key, step=1 << 26):
    """In-edge CSC from sorted distinct keys head * n + tail: col_off
    int64[n+1] (where each head's keys start), row_idx int32[m]."""
    bounds = torch.arange(n + 1, dtype=torch.int64, device=key.device) * n
    col_off = torch.searchsorted(key, bounds)
    row = torch.empty(key.numel(), dtype=torch.int32, device=key.device)
    for i0 in range(0, key.numel(), step):
        row[i0:i0 + step] = (key[i0:i0 + step] % n).to(torch.int32)
    return col_off, row


def rmat(scale, edge_factor, abcd, seed, device="cpu"):
    """R-MAT with Graph500-style vertex relabelling; loops and duplicates
    dropped.  Returns the in-edge CSC (col_off, row_idx)."""
    n = 1 << scale
    key = unique_sorted(rmat_keys(scale, edge_factor, abcd, seed, device))  # sorted (head, tail)
    return csc_from_keys(n, key)


def to_csc(n, tail, head):
    """In-edge CSC sorted by (head, tail): col_off int64[n+1], row_idx int32[m]."""
    key = unique_sorted(head.to(torch.int64) * n + tail.to(torch.int64))
    return csc_from_keys(n, key)


def _column_chunks(col_off, max_edges=1 << 25):
    """(c0, c1, e0, e1): ranges of whole columns holding about max_edges
    in-edges each (a longer column is a range of its own)."""
    co = col_off.cpu().numpy()
    n, m = co.shape[0] - 1, int(co[-1])
    c0 = 0
    while c0 < n:
        c1 = int(np.searchsorted(co, co[c0] + max_edges, side="right")) - 1
        c1 = min(n, max(c1, c0 + 1))
        yield c0, c1, int(co[c0]), int(co[c1])
        c0 = c1
    if n == 0 or m == 0:
        return


def _per_column(col_off, fn):
    """fp32 weights built column range by column range: fn(c0, c1, e0, e1,
    local column of each edge, local in-degrees) -> fp32 weights of edges
    e0..e1-1."""
    m = int(col_off[-1])
    w = torch.empty(m, dtype=torch.float32, device=col_off.device)
    for c0, c1, e0, e1 in _column_chunks(col_off):
        deg = col_off[c0 + 1:c1 + 1] - col_off[c0:c1]
        cols = torch.repeat_interleave(torch.arange(c1 - c0, device=col_off.device), deg)
        w[e0:e1] = fn(c0, c1, e0, e1, cols, deg)
    return w


def weights_inv_indeg(col_off):
    """w(u,v) = 1/d_in(v) in fp32 (the paper's parameter setting), rounded
    once from the float64 quotient (d_in < 2^28 makes that the correctly
    rounded fp32 quotient)."""
    def fn(c0, c1, e0, e1, cols, deg):
        return (1.0 / deg.clamp(min=1).to(torch.float64)).to(torch.float32)[cols]
    return _per_column(col_off, fn)


def _edge_draws(seed, stream, e0, e1, device):
    """An integer in [1, 2^24] for every edge e0..e1-1, keyed by its CSC
    position."""
    j = torch.arange(e0, e1, dtype=torch.int64, device=device)
    return _shr(hash64(seed, stream, j), 40) + 1


def _local_sums(x, cols, ncols):
    """Exact per-column sums of int64 values (integer, so order-free)."""
    return torch.zeros(ncols, dtype=torch.int64, device=x.device).index_add_(0, cols, x)


def weights_random_colsum(col_off, lo, hi, seed):
    """x ~ U{1..2^24} per edge, column sum s_v ~ U(lo, hi) (53-bit fixed
    point): w = fp32(x * s_v / sum x), the product and quotient in float64."""
    dev = col_off.device

    def fn(c0, c1, e0, e1, cols, deg):
        x = _edge_draws(seed, 5, e0, e1, dev)
        s = lo + (hi - lo) * _unit53(hash64(seed, 6, torch.arange(c0, c1, dtype=torch.int64, device=dev)))
        tot = _local_sums(x, cols, c1 - c0).to(torch.float64)
        return (x.to(torch.float64) * s[cols] / tot[cols]).to(torch.float32)
    return _per_column(col_off, fn)


def weights_normalized(col_off, seed):
    """x ~ U{1..2^24} per edge normalised to column sum 1 (the GreedyCutting
    setting): w = fp32(x / sum x), the quotient in float64."""
    dev = col_off.device

    def fn(c0, c1, e0, e1, cols, deg):
        x = _edge_draws(seed, 7, e0, e1, dev)
        tot = _local_sums(x, cols, c1 - c0).to(torch.float64)
        return (x.to(torch.float64) / tot[cols]).to(torch.float32)
    return _per_column(col_off, fn)


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


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
        t = h = None
        col_off, row_idx = rmat(spec["scale"], spec["ef"], spec.get("abcd", RMAT_ABCD), spec["gseed"], device)
    else:
        raise ValueError(kind)
    if t is not None:
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
