"""Pins of the oracle with probabilistic suspects (Section 2.2: V_I = (V_I, p),
seed sets drawn with the probability of equation "prob_src_set"; Algorithm 1's
suspect test, which makes a suspect the walk meets a seed with probability p(u)).

* The exact routes agree in rationals: HSAW path sums with the factor
  p(v_l) prod (1 - p(u)) of equation "compute_path_inf" against every
  live-edge graph times every seed set (definitions "def:eis", "sus_nod").
* The sampling process's exact law (start uniform over V) gives
  n Pr[hit] = I(V_I) and n Pr[id on the kept walk] = D({id}) (Theorems
  "lem:rr_edge" / "lem:rr_node" as the estimators use them).
* The C oracle's outcome rates, id frequencies and walk frequencies follow
  that law (Bernstein / chi-square), and a brute-force tracer built from
  numpy's Philox and Fraction-derived tables reproduces it walk by walk.
* Closed forms: a two-node chain worked by hand, an isolated suspect, p = 0.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chi2

from oracle import cpu, exact
from test_oracle_rng import numpy_block
from tiny import catalogue, count_tolerance, csc_from_edges, random_tiny

SEED = 2017
N = 200_000


def suspect_cases():
    """(name, n, edges, suspects, p) on the tiny catalogue and random graphs."""
    out = []
    rng = np.random.default_rng(5)
    for name, n, edges, src in catalogue():
        k = min(n, len(src) + 2)
        sus = sorted(rng.choice(n, size=k, replace=False).tolist())
        p = rng.choice([0.0, 0.125, 0.3, 0.5, 0.9, 1.0], size=k).astype(np.float32)
        out.append((name, n, edges, sus, p))
    for seed in range(4):
        n = 5 + seed % 2
        edges = random_tiny(n, 0.5, 40 + seed, "rand" if seed % 2 else "inv")
        sus = sorted(rng.choice(n, size=2 + seed % 2, replace=False).tolist())
        out.append((f"prand{seed}", n, edges, sus, rng.uniform(0, 1, len(sus)).astype(np.float32)))
    return out


CASES = suspect_cases()


def graphs(n, edges):
    col, row, w = csc_from_edges(n, edges)
    return col, row, w, exact.exact_edge_probs(col, row, w), exact.quantized_edge_probs(col, row, w)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_routes_agree_exactly(case):
    """Route 1 (HSAW path sums) == route 2 (live-edge graphs x seed sets)
    for the expected spread and for the suspension of single ids and of a
    random set, edges and nodes."""
    name, n, edges, sus, p = case
    col, row, w, tg, _ = graphs(n, edges)
    probs = exact.coin_probs_exact(p)
    assert exact.spread_p_from_paths(tg, sus, probs) == exact.live_edge_spread_p(tg, sus, probs)
    rng = np.random.default_rng(len(name))
    for mode, size in (("edges", len(row)), ("nodes", n)):
        sets = [[i] for i in range(size)] + [sorted(rng.choice(size, size=min(2, size), replace=False).tolist())] \
            if size else []
        for T in sets:
            r1 = exact.suspension_p_from_paths(tg, sus, probs, T, mode)
            r2 = exact.live_edge_spread_p(tg, sus, probs) - exact.live_edge_spread_p(tg, sus, probs, T, mode)
            assert r1 == r2, (name, mode, T)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_sampling_law_is_the_estimator(case):
    """The exact law of one attempt (start uniform over V): n Pr[hit] is the
    expected spread I(V_I), and n Pr[id on the kept walk] is D({id})."""
    name, n, edges, sus, p = case
    _, row, _, tg, _ = graphs(n, edges)
    probs = exact.coin_probs_exact(p)
    law = exact.walk_tree_p(tg, sus, probs)
    assert law["hit"] + law["dead_end"] + law["cycle"] == 1
    assert n * law["hit"] == exact.spread_p_from_paths(tg, sus, probs)
    for mode, size in (("edges", len(row)), ("nodes", n)):
        freq = exact.id_frequencies_p(tg, sus, probs, mode)
        for i in range(size):
            assert n * freq[i] == exact.suspension_p_from_paths(tg, sus, probs, [i], mode), (name, mode, i)


def test_two_node_chain_by_hand():
    """a -> b with w(a,b) = 1, both suspects with p = 1/2 (every node a
    suspect, as in the appendix's reduction from influence maximisation).
    By hand: a is infected w.p. 1/2, b w.p. 3/4, so I(V_I) = 5/4; removing b
    leaves a alone, I = 1/2, so D({b}) = 3/4; removing a leaves b, I = 1/2,
    D({a}) = 3/4.  The influence of {b} as a seed set is 1 (b has no
    out-edge), so D({b}) is not I({b})/2 = 1/2: the appendix's identity
    D(S, V_I) = I(S)/2 is not used as a pin."""
    col, row, w = csc_from_edges(2, [(0, 1, 1.0)])
    tg = exact.exact_edge_probs(col, row, w)
    half = [Fraction(1, 2), Fraction(1, 2)]
    assert exact.spread_p_from_paths(tg, [0, 1], half) == Fraction(5, 4)
    assert exact.live_edge_spread_p(tg, [0, 1], half) == Fraction(5, 4)
    for T in ([0], [1]):
        assert exact.suspension_p_from_paths(tg, [0, 1], half, T, "nodes") == Fraction(3, 4)
        assert exact.live_edge_spread_p(tg, [0, 1], half) - exact.live_edge_spread_p(tg, [0, 1], half, T, "nodes") \
            == Fraction(3, 4)
    # the edge (a, b) carries b's infection from a: D({(a,b)}) = Pr[a seed, b not] = 1/4
    assert exact.suspension_p_from_paths(tg, [0, 1], half, [0], "edges") == Fraction(1, 4)


def test_coin_thresholds():
    """pq = min(round-half-even(p 2^32), 2^32 - 1): hand cases and a Fraction
    derivation on random fp32 values."""
    got = cpu.coin_thresholds(np.array([0.0, 0.5, 1.0, 0.25, 2.0 ** -33, 3 * 2.0 ** -33], np.float32))
    assert got.tolist() == [0, 1 << 31, (1 << 32) - 1, 1 << 30, 0, 2]  # 0.5 and 1.5 round to even
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, 20000).astype(np.float32)
    want = [min(round(Fraction(float(x)) * (1 << 32)), (1 << 32) - 1) for x in p]
    assert cpu.coin_thresholds(p).tolist() == want
    with pytest.raises(ValueError):
        cpu.coin_thresholds(np.array([1.5], np.float32))


def test_coin_is_the_low_half_of_the_node_word():
    """The coin is the low 32 bits of word 0 of counter (x,0,0,0), the word
    whose high half is the live-edge draw (checked against numpy's Philox)."""
    for a, x in ((0, 0), (5, 17), (123456789, 99)):
        word = numpy_block((x, 0, 0, 0), (SEED, a))[0]
        assert cpu.draw_node_word(SEED, a, x) == word
        assert cpu.draw_node(SEED, a, x) == word >> 32


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_outcome_rates_and_frequencies(case):
    name, n, edges, sus, p = case
    col, row, w, _, tq = graphs(n, edges)
    law = exact.walk_tree_p(tq, sus, exact.coin_probs_quantized(p))
    g = cpu.Graph(col, row, w)
    for mode, label, size in ((cpu.MODE_EDGES, "edges", len(row)), (cpu.MODE_NODES, "nodes", n)):
        walks = g.sample_suspects(np.array(sus, np.int32), p, mode, N, 0, SEED)
        assert walks.hits + walks.dead_ends + walks.cycles == N
        for key, got in (("hit", walks.hits), ("dead_end", walks.dead_ends), ("cycle", walks.cycles)):
            q = float(law[key])
            assert abs(got - N * q) <= count_tolerance(N, q), (name, key, got, N * q)
        es = float(law["steps"])
        assert abs(walks.steps - N * es) <= n * math.sqrt(math.log(2 / 1e-12) / (2 * N)) * N
        cnt = cpu.count(max(size, 1), walks)
        freq = exact.id_frequencies_p(tq, sus, exact.coin_probs_quantized(p), label)
        for i in range(size):
            q = float(freq[i])
            assert abs(int(cnt[i]) - N * q) <= count_tolerance(N, q), (name, label, i)


@pytest.mark.parametrize("case", [c for c in CASES if c[0] in ("intree", "loopmulti", "prand1", "prand2")],
                         ids=lambda c: c[0])
def test_walk_frequencies_chi2(case):
    name, n, edges, sus, p = case
    col, row, w, _, tq = graphs(n, edges)
    law = exact.walk_tree_p(tq, sus, exact.coin_probs_quantized(p))["walks"]
    walks = cpu.Graph(col, row, w).sample_suspects(np.array(sus, np.int32), p, cpu.MODE_NODES, N, 0, SEED)
    obs = {}
    for i in range(walks.n_walks):
        key = tuple(int(x) for x in walks.walk(i))
        obs[key] = obs.get(key, 0) + 1
    expected = {}
    for (nodes, _), q in law.items():  # walks with the same nodes (multi-edges) add up
        expected[nodes] = expected.get(nodes, 0.0) + float(q) * N
    assert set(obs) <= set(expected), name
    big = [k for k, e in expected.items() if e >= 5]
    stat = sum((obs.get(k, 0) - expected[k]) ** 2 / expected[k] for k in big)
    rest_e = N - sum(expected[k] for k in big)
    rest_o = N - sum(obs.get(k, 0) for k in big)
    dof = len(big)
    if rest_e >= 5:
        stat += (rest_o - rest_e) ** 2 / rest_e
    assert stat < chi2.ppf(1 - 1e-9, max(dof, 1)), (name, stat, dof)


def brute_walk_p(col, row, thr, pq, n, seed, a):
    """One attempt from numpy's Philox and the Fraction-derived tables:
    start floor(x0 n / 2^64); on arrival a node already on the walk is a
    cycle, a suspect whose coin (low half of its word) is below pq a hit,
    else the first in-edge with threshold above the draw (high half)."""
    x0 = numpy_block((0, 1, 0, 0), (seed, a))[0]
    v = (x0 * n) >> 64
    nodes, edges, steps = [v], [], 0
    while True:
        word = numpy_block((v, 0, 0, 0), (seed, a))[0]
        if v in pq and (word & 0xFFFFFFFF) < pq[v]:
            return "hit", steps, nodes, edges
        r = word >> 32
        steps += 1
        lo, hi = col[v], col[v + 1]
        js = [j for j in range(lo, hi) if thr[j] > r]
        if not js:
            return "dead", steps, nodes, edges
        j = js[0]
        u = row[j]
        edges.append(j)
        if u in nodes:
            return "cycle", steps, nodes, edges
        nodes.append(u)
        v = u


@pytest.mark.parametrize("case", [c for c in CASES if c[0] in ("chain", "twocycle", "loopmulti", "thirds",
                                                                "prand0", "prand3")], ids=lambda c: c[0])
def test_walks_match_brute_force_tracer(case):
    name, n, edges_, sus, p = case
    col, row, w = csc_from_edges(n, edges_)
    thr = exact.quantized_thresholds(col, w)
    pq = {int(v): min(round(Fraction(float(x)) * (1 << 32)), (1 << 32) - 1) for v, x in zip(sus, p)}
    offset, count = 911, 300
    g = cpu.Graph(col, row, w)
    we = g.sample_suspects(np.array(sus, np.int32), p, cpu.MODE_EDGES, count, offset, SEED)
    wn = g.sample_suspects(np.array(sus, np.int32), p, cpu.MODE_NODES, count, offset, SEED)
    kept_e = {int(a): we.walk(i).tolist() for i, a in enumerate(we.attempt)}
    kept_n = {int(a): wn.walk(i).tolist() for i, a in enumerate(wn.attempt)}
    tot = dict(hit=0, dead=0, cycle=0, steps=0)
    for a in range(offset, offset + count):
        out, steps, nodes, edges = brute_walk_p([int(c) for c in col], [int(r) for r in row], thr, pq, n, SEED, a)
        tot[out] += 1
        tot["steps"] += steps
        if out == "hit":
            assert kept_e[a] == edges and kept_n[a] == nodes, (name, a)
        else:
            assert a not in kept_e and a not in kept_n
    assert (tot["hit"], tot["dead"], tot["cycle"], tot["steps"]) == (we.hits, we.dead_ends, we.cycles, we.steps)
    # the attempt list gives the same walks as the range
    wl = g.sample_suspects_list(np.array(sus, np.int32), p, cpu.MODE_NODES,
                                np.arange(offset, offset + count, dtype=np.uint64), SEED)
    assert np.array_equal(wl.attempt, wn.attempt) and np.array_equal(wl.ids, wn.ids)


def test_special_cases():
    """p = 0 everywhere: no kept walk.  An isolated suspect (no in-edge) with
    p: its own zero-edge walk w.p. pq/2^32 per start on it.  Every node a
    suspect with p = 1 on a graph without edges: every attempt is a kept
    zero-edge walk except with probability 2^-32 (the clamped coin)."""
    col, row, w = csc_from_edges(4, [(1, 0, 0.5), (2, 1, 1.0)])
    g = cpu.Graph(col, row, w)
    none = g.sample_suspects(np.array([0, 2], np.int32), np.zeros(2, np.float32), cpu.MODE_EDGES, 50_000, 0, SEED)
    assert none.hits == 0 and none.n_walks == 0
    iso = g.sample_suspects(np.array([3], np.int32), np.array([0.3], np.float32), cpu.MODE_NODES, N, 0, SEED)
    q = float(exact.coin_probs_quantized([0.3])[0]) / 4
    assert abs(iso.hits - N * q) <= count_tolerance(N, q)
    assert all(iso.walk(i).tolist() == [3] for i in range(iso.n_walks))
    col, row, w = csc_from_edges(3, [])
    g = cpu.Graph(col, row, w)
    allw = g.sample_suspects(np.arange(3, dtype=np.int32), np.ones(3, np.float32), cpu.MODE_EDGES, 30_000, 0, SEED)
    assert allw.hits == 30_000 and allw.steps == 0 and allw.ids.shape[0] == 0
    assert np.all(np.diff(allw.off.astype(np.int64)) == 0)


def test_coin_boundary_is_strict():
    """A suspect is a seed when its coin is strictly below pq: on a
    one-node graph (every start is node 0), attempts whose coin c is a
    multiple of 2^8 (so c / 2^32 is an exact fp32) are kept with p = (c + 256)
    / 2^32 and not with p = c / 2^32."""
    col, row, w = csc_from_edges(1, [])
    g = cpu.Graph(col, row, w)
    found = 0
    for a in range(200_000):
        c = cpu.draw_node_word(SEED, a, 0) & 0xFFFFFFFF
        if c % 256 or c + 256 >= 1 << 32:
            continue
        at = np.array([a], np.uint64)
        for p, kept in ((c / 2.0 ** 32, 0), ((c + 256) / 2.0 ** 32, 1)):
            assert float(np.float32(p)) == p
            wk = g.sample_suspects_list(np.array([0], np.int32), np.array([p], np.float32), cpu.MODE_NODES, at, SEED)
            assert wk.hits == kept, (a, c, p)
        found += 1
        if found == 5:
            break
    assert found == 5
