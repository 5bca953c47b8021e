"""Exact rational enumeration on tiny graphs (TEST INFRASTRUCTURE ONLY).

Three independent routes to the quantities the sampler estimates, all in
``fractions.Fraction`` arithmetic:

* route 1, ``hsaw_paths``: the sum over simple backward paths (HSAWs) of the
  product of their edge probabilities -- the walk-probability formula of
  Section 3.1 (equation "compute_path_inf" with p == 1) together with the
  walk-uniqueness property;
* route 2, ``live_edge_spread``: the product over every live-edge graph
  (each node keeps at most one in-edge, Section 2.1) of its probability
  times the number of nodes reachable from the seeds, in the original and in
  the residual network -- the definition of influence suspension (equation
  "sus_nod");
* route 3, ``walk_tree``: the full tree of the sampling process of
  Algorithm 1 (start uniform over the non-sources, live in-edge each step,
  stop at a source, a repeated node or no live edge), giving the exact
  probabilities of every outcome and the expected number of draws.

Theorem "lem:rr_edge" / "lem:rr_node" say routes 1 and 2 give the same
suspension; the tests check that they agree exactly.

Probabilistic suspects (Section 2.2: V_I = (V_I, p), seed sets X drawn with
the probability of equation "prob_src_set") have their own three routes:
``hsaw_paths_p`` (equation "compute_path_inf" with its factor p(v_l) times
(1 - p(u)) over the other suspects on the walk), ``live_edge_spread_p``
(every live-edge graph times every seed set X within V_I, the definitions
"def:eis" and "sus_nod" written out) and ``walk_tree_p`` (the sampling
process with a coin per suspect, start uniform over V).

Edge probabilities come in two flavours:

* ``exact_edge_probs``: the real-valued LT weights, as exact rationals;
* ``quantized_edge_probs``: the discretised model the sampler realises
  (weight -> round-half-even(w * 2^32), running sums clamped to 2^32 - 1),
  derived here with Python integers, independently of the C oracle.
"""
from fractions import Fraction
from itertools import product

import numpy as np

TWO32 = 1 << 32


class TinyGraph:
    """In-edge CSC graph with one probability per edge and a 'none' probability per node."""

    def __init__(self, col_off, row_idx, p_edge, p_none):
        self.col_off = [int(x) for x in col_off]
        self.row_idx = [int(x) for x in row_idx]
        self.n = len(self.col_off) - 1
        self.m = len(self.row_idx)
        self.p_edge = list(p_edge)
        self.p_none = list(p_none)

    def in_edges(self, v):
        return range(self.col_off[v], self.col_off[v + 1])


def exact_edge_probs(col_off, row_idx, w):
    """Real LT weights as exact rationals; 'no edge' takes the rest (Section 2.1).
    A column whose fp32 weights sum above 1 by rounding (at most 2^-20) is
    scaled to sum exactly 1, so every column is a probability law."""
    p_edge = [Fraction(float(x)) for x in np.asarray(w, dtype=np.float32)]
    p_none = []
    for v in range(len(col_off) - 1):
        js = range(int(col_off[v]), int(col_off[v + 1]))
        s = sum((p_edge[j] for j in js), Fraction(0))
        if s > 1 + Fraction(1, 1 << 20):
            raise ValueError("column weight sum above 1")
        if s > 1:
            for j in js:
                p_edge[j] /= s
            s = Fraction(1)
        p_none.append(1 - s)
    return TinyGraph(col_off, row_idx, p_edge, p_none)


def quantize_exact(x: float) -> int:
    """round-half-even(x * 2^32) via Fraction (Python's round() on a Fraction is half-even)."""
    return round(Fraction(float(np.float32(x))) * TWO32)


def quantized_thresholds(col_off, w):
    thr = []
    for v in range(len(col_off) - 1):
        run = 0
        for j in range(int(col_off[v]), int(col_off[v + 1])):
            run += quantize_exact(w[j])
            thr.append(min(run, TWO32 - 1))
    return thr


def quantized_edge_probs(col_off, row_idx, w):
    """Probabilities of the discretised live-edge rule: edge j is live with
    probability (thr_j - thr_{j-1}) / 2^32 and no edge with (2^32 - thr_last) / 2^32."""
    thr = quantized_thresholds(col_off, w)
    p_edge = [Fraction(0)] * len(thr)
    p_none = []
    for v in range(len(col_off) - 1):
        lo, hi = int(col_off[v]), int(col_off[v + 1])
        prev = 0
        for j in range(lo, hi):
            p_edge[j] = Fraction(thr[j] - prev, TWO32)
            prev = thr[j]
        p_none.append(Fraction(TWO32 - prev, TWO32))
    return TinyGraph(col_off, row_idx, p_edge, p_none)


# ---------------------------------------------------------------- route 1
def hsaw_paths(g: TinyGraph, sources, starts=None):
    """All HSAWs h = <v_1..v_l> with v_1 not a source (and in ``starts`` when
    given), as (start, nodes, edges, probability); distinct nodes, only v_l a
    source."""
    X = set(int(s) for s in sources)
    out = []

    def dfs(start, nodes, edges, prob):
        x = nodes[-1]
        for j in g.in_edges(x):
            pj = g.p_edge[j]
            if pj == 0:
                continue
            u = g.row_idx[j]
            if u in nodes:
                continue
            if u in X:
                out.append((start, tuple(nodes + [u]), tuple(edges + [j]), prob * pj))
            else:
                dfs(start, nodes + [u], edges + [j], prob * pj)

    for v in (range(g.n) if starts is None else starts):
        if v not in X:
            dfs(v, [v], [], Fraction(1))
    return out


def spread_from_paths(g: TinyGraph, sources):
    """I(X) = |X| + sum over non-sources of Pr[its backward trace hits X]."""
    return len(set(sources)) + sum((p for (_, _, _, p) in hsaw_paths(g, sources)), Fraction(0))


def suspension_from_paths(g: TinyGraph, sources, removed, mode, starts=None):
    """D(T) = sum of Pr[h] over HSAWs that T interdicts (+|T & X| for nodes).
    With ``starts`` only the suspension of those nodes is counted."""
    removed = set(int(x) for x in removed)
    total = Fraction(0)
    for (_, nodes, edges, p) in hsaw_paths(g, sources, starts):
        ids = edges if mode == "edges" else nodes
        if removed.intersection(ids):
            total += p
    if mode == "nodes":
        counted = set(int(s) for s in sources)
        if starts is not None:
            counted &= set(starts)
        total += len(removed & counted)
    return total


# ---------------------------------------------------------------- route 2
def live_edge_spread(g: TinyGraph, sources, removed=(), mode="edges", count_only=None):
    """Expected number of nodes reachable from X over all live-edge graphs,
    after removing the edge set (mode 'edges') or node set (mode 'nodes').
    With ``count_only`` only those nodes are counted."""
    X = set(int(s) for s in sources)
    removed = set(int(x) for x in removed)
    choices = []
    for v in range(g.n):
        opts = [(None, g.p_none[v])] if g.p_none[v] > 0 else []
        opts += [(j, g.p_edge[j]) for j in g.in_edges(v) if g.p_edge[j] > 0]
        choices.append(opts)
    total = Fraction(0)
    for combo in product(*choices):
        prob = Fraction(1)
        parent = [None] * g.n
        for v, (j, pj) in enumerate(combo):
            prob *= pj
            if j is None:
                continue
            u = g.row_idx[j]
            if mode == "edges" and j in removed:
                continue
            if mode == "nodes" and (u in removed or v in removed):
                continue
            parent[v] = u
        infected = 0
        for v in (range(g.n) if count_only is None else count_only):
            if mode == "nodes" and v in removed:
                continue
            seen = set()
            x = v
            while x is not None and x not in seen:
                if x in X:
                    infected += 1
                    break
                seen.add(x)
                x = parent[x]
        total += prob * infected
    return total


def live_edge_suspension(g: TinyGraph, sources, removed, mode, count_only=None):
    return (live_edge_spread(g, sources, count_only=count_only)
            - live_edge_spread(g, sources, removed, mode, count_only=count_only))


# ---------------------------------------------------------------- route 3
def walk_tree(g: TinyGraph, sources):
    """Exact law of one sampler attempt: start uniform over V \\ X, then the
    live in-edge of the current node each draw, stopping at a source (hit),
    a node already on the walk (cycle) or no live edge (dead end).

    Returns dict with Fractions: hit, dead_end, cycle, steps (expected draws),
    and walks: {(nodes, edges): probability} of the accepted walks."""
    X = set(int(s) for s in sources)
    starts = [v for v in range(g.n) if v not in X]
    n_ns = len(starts)
    res = dict(hit=Fraction(0), dead_end=Fraction(0), cycle=Fraction(0), steps=Fraction(0))
    walks = {}

    def rec(nodes, edges, prob):
        x = nodes[-1]
        # every draw is one step, whatever it yields
        res["steps"] += prob
        if g.p_none[x] > 0:
            res["dead_end"] += prob * g.p_none[x]
        for j in g.in_edges(x):
            pj = g.p_edge[j]
            if pj == 0:
                continue
            u = g.row_idx[j]
            q = prob * pj
            if u in nodes:
                res["cycle"] += q
            elif u in X:
                res["hit"] += q
                key = (tuple(nodes + [u]), tuple(edges + [j]))
                walks[key] = walks.get(key, Fraction(0)) + q
            else:
                rec(nodes + [u], edges + [j], q)

    for v in starts:
        rec([v], [], Fraction(1, n_ns))
    res["walks"] = walks
    return res


def id_frequencies(g: TinyGraph, sources, mode):
    """Exact Pr[id lies on the accepted walk of one attempt] for every id."""
    size = g.m if mode == "edges" else g.n
    freq = [Fraction(0)] * size
    for (nodes, edges), p in walk_tree(g, sources)["walks"].items():
        for i in (edges if mode == "edges" else nodes):
            freq[i] += p
    return freq


def subdivide(col_off, row_idx, w):
    """Edge -> node subdivision of the hardness reduction (appendix, proof of
    Theorem "theo:hard"): every edge (u,v) becomes a node e_uv on the path
    u -> e_uv -> v, so that removing e_uv has the effect of removing (u,v).

    The paper gives w(u,e_uv) = w(u,v) and w(e_uv,v) = 1, which breaks the LT
    constraint (sum of in-weights <= 1) as soon as v has two in-edges.  The
    assignment that keeps the live-edge law of every original walk is the
    swapped one: w(u,e_uv) = 1 and w(e_uv,v) = w(u,v); that is what is built.

    Node ids: originals keep theirs, edge j becomes node n + j.  Returns a
    TinyGraph with exact probabilities."""
    n = len(col_off) - 1
    m = len(row_idx)
    base = exact_edge_probs(col_off, row_idx, w)
    new_off = [0]
    new_row = []
    p_edge = []
    for v in range(n):
        for j in range(int(col_off[v]), int(col_off[v + 1])):
            new_row.append(n + j)
            p_edge.append(base.p_edge[j])
        new_off.append(len(new_row))
    for j in range(m):
        new_row.append(int(row_idx[j]))
        p_edge.append(Fraction(1))
        new_off.append(len(new_row))
    p_none = []
    for v in range(n + m):
        s = sum((p_edge[j] for j in range(new_off[v], new_off[v + 1])), Fraction(0))
        if s > 1:
            raise ValueError("column weight sum above 1")
        p_none.append(1 - s)
    return TinyGraph(new_off, new_row, p_edge, p_none)


# ---------------------------------------------------------------- probabilistic suspects
def coin_probs_exact(p):
    """Suspect probabilities as exact rationals of their fp32 values."""
    return [Fraction(float(np.float32(x))) for x in p]


def coin_probs_quantized(p):
    """The discretised coin the sampler realises: x is a seed when a 32-bit
    draw is below pq = min(round-half-even(p * 2^32), 2^32 - 1)."""
    return [Fraction(min(round(Fraction(float(np.float32(x))) * TWO32), TWO32 - 1), TWO32) for x in p]


def hsaw_paths_p(g: TinyGraph, suspects, probs):
    """Route 1 with probabilistic suspects: every HSAW h = <v_1 .. v_l> (any
    start v_1, distinct nodes, v_l a suspect; l = 1 when v_1 itself is one)
    with Pr[h] = p(v_l) * prod over the other suspects u on h of (1 - p(u))
    * prod of its edge probabilities (equation "compute_path_inf").  Returns
    (start, nodes, edges, probability)."""
    P = {int(v): q for v, q in zip(suspects, probs)}
    out = []

    def dfs(start, nodes, edges, prob):
        x = nodes[-1]
        if x in P:
            if P[x] > 0:
                out.append((start, tuple(nodes), tuple(edges), prob * P[x]))
            prob = prob * (1 - P[x])  # x is not a seed: the walk goes on
            if prob == 0:
                return
        for j in g.in_edges(x):
            pj = g.p_edge[j]
            if pj == 0:
                continue
            u = g.row_idx[j]
            if u in nodes:
                continue
            dfs(start, nodes + [u], edges + [j], prob * pj)

    for v in range(g.n):
        dfs(v, [v], [], Fraction(1))
    return out


def spread_p_from_paths(g: TinyGraph, suspects, probs):
    """I(V_I) = sum over nodes of Pr[the node is infected] = sum of Pr[h]
    over all HSAWs (walk uniqueness: the HSAWs from one start are disjoint
    events)."""
    return sum((p for (_, _, _, p) in hsaw_paths_p(g, suspects, probs)), Fraction(0))


def suspension_p_from_paths(g: TinyGraph, suspects, probs, removed, mode):
    """D(T) = sum of Pr[h] over the HSAWs T interdicts (Theorems "lem:rr_edge"
    / "lem:rr_node"); for nodes a walk holds its start and its end."""
    removed = set(int(x) for x in removed)
    total = Fraction(0)
    for (_, nodes, edges, p) in hsaw_paths_p(g, suspects, probs):
        if removed.intersection(edges if mode == "edges" else nodes):
            total += p
    return total


def live_edge_spread_p(g: TinyGraph, suspects, probs, removed=(), mode="edges"):
    """Route 2: I(V_I) in the network after removing the edge set (mode
    'edges') or node set ('nodes'), by summing over every live-edge graph
    and every seed set X within V_I (probability of equation
    "prob_src_set"; a removed node is neither a seed nor counted)."""
    sus = [int(v) for v in suspects]
    removed = set(int(x) for x in removed)
    choices = []
    for v in range(g.n):
        opts = [(None, g.p_none[v])] if g.p_none[v] > 0 else []
        opts += [(j, g.p_edge[j]) for j in g.in_edges(v) if g.p_edge[j] > 0]
        choices.append(opts)
    seed_sets = []
    for bits in product((0, 1), repeat=len(sus)):
        pr = Fraction(1)
        X = set()
        for v, b, q in zip(sus, bits, probs):
            pr *= q if b else 1 - q
            if b:
                X.add(v)
        if pr:
            seed_sets.append((X, pr))
    total = Fraction(0)
    for combo in product(*choices):
        prob = Fraction(1)
        parent = [None] * g.n
        for v, (j, pj) in enumerate(combo):
            prob *= pj
            if j is None:
                continue
            u = g.row_idx[j]
            if mode == "edges" and j in removed:
                continue
            if mode == "nodes" and (u in removed or v in removed):
                continue
            parent[v] = u
        # the nodes on each node's backward trace (at most one in-edge each)
        traces = []
        for v in range(g.n):
            if mode == "nodes" and v in removed:
                continue
            seen, x, tr = set(), v, []
            while x is not None and x not in seen:
                seen.add(x)
                tr.append(x)
                x = parent[x]
            traces.append(tr)
        for X, px in seed_sets:
            Xr = X - removed if mode == "nodes" else X
            infected = sum(1 for tr in traces if any(x in Xr for x in tr))
            total += prob * px * infected
    return total


def walk_tree_p(g: TinyGraph, suspects, probs):
    """Route 3: the exact law of one sampler attempt with probabilistic
    suspects -- start uniform over V; on arriving at a node: a node already
    on the walk ends it (cycle), a suspect is a seed with its probability
    (hit), else the live in-edge is drawn (no edge: dead end).  Returns the
    outcome probabilities, expected draws, and the kept walks' law
    {(nodes, edges): probability}."""
    P = {int(v): q for v, q in zip(suspects, probs)}
    res = dict(hit=Fraction(0), dead_end=Fraction(0), cycle=Fraction(0), steps=Fraction(0))
    walks = {}

    def arrive(nodes, edges, prob):
        x = nodes[-1]
        if x in P and P[x] > 0:
            q = prob * P[x]
            res["hit"] += q
            key = (tuple(nodes), tuple(edges))
            walks[key] = walks.get(key, Fraction(0)) + q
            prob = prob * (1 - P[x])
            if prob == 0:
                return
        res["steps"] += prob  # one draw
        if g.p_none[x] > 0:
            res["dead_end"] += prob * g.p_none[x]
        for j in g.in_edges(x):
            pj = g.p_edge[j]
            if pj == 0:
                continue
            u = g.row_idx[j]
            if u in nodes:
                res["cycle"] += prob * pj
            else:
                arrive(nodes + [u], edges + [j], prob * pj)

    for v in range(g.n):
        arrive([v], [], Fraction(1, g.n))
    res["walks"] = walks
    return res


def id_frequencies_p(g: TinyGraph, suspects, probs, mode):
    """Exact Pr[id lies on the kept walk of one attempt], suspect coins."""
    size = g.m if mode == "edges" else g.n
    freq = [Fraction(0)] * size
    for (nodes, edges), p in walk_tree_p(g, suspects, probs)["walks"].items():
        for i in (edges if mode == "edges" else nodes):
            freq[i] += p
    return freq
