"""Pins of the oracle's sampler: exact laws from the enumerator (route 3, the
sampling process of Algorithm 1 in rationals), the HSAW invariants of
Definition "self_walk", and a brute-force walk-by-walk tracer built from
numpy's Philox and the Fraction-derived thresholds."""
import numpy as np
import pytest
from scipy.stats import chi2

from oracle import cpu, exact
from test_oracle_rng import numpy_block
from tiny import catalogue, count_tolerance, csc_from_edges

CAT = catalogue()
N = 200_000
SEED = 2017


def run(name, n, edges, src, mode, n_attempts=N, offset=0):
    col, row, w = csc_from_edges(n, edges)
    g = cpu.Graph(col, row, w)
    return g, g.sample(np.array(src, np.int32), mode, n_attempts, offset, SEED)


@pytest.mark.parametrize("case", CAT, ids=[c[0] for c in CAT])
def test_outcome_rates_match_exact_law(case):
    name, n, edges, src = case
    col, row, w = csc_from_edges(n, edges)
    law = exact.walk_tree(exact.quantized_edge_probs(col, row, w), src)
    _, walks = run(name, n, edges, src, cpu.MODE_EDGES)
    assert walks.attempts == N
    assert walks.hits + walks.dead_ends + walks.cycles == N
    for key, got in (("hit", walks.hits), ("dead_end", walks.dead_ends), ("cycle", walks.cycles)):
        p = float(law[key])
        assert abs(got - N * p) <= count_tolerance(N, p), (name, key, got, N * p)
    # steps: mean of a bounded variable (at most n draws per attempt)
    es = float(law["steps"])
    tol = n * np.sqrt(np.log(2 / 1e-12) / (2 * N)) * N
    assert abs(walks.steps - N * es) <= tol, (name, walks.steps, N * es)


@pytest.mark.parametrize("case", CAT, ids=[c[0] for c in CAT])
def test_id_frequencies_match_exact(case):
    name, n, edges, src = case
    col, row, w = csc_from_edges(n, edges)
    tg = exact.quantized_edge_probs(col, row, w)
    for mode, label, size in ((cpu.MODE_EDGES, "edges", len(row)), (cpu.MODE_NODES, "nodes", n)):
        _, walks = run(name, n, edges, src, mode)
        cnt = cpu.count(max(size, 1), walks)
        freq = exact.id_frequencies(tg, src, label)
        for i in range(size):
            p = float(freq[i])
            assert abs(int(cnt[i]) - N * p) <= count_tolerance(N, p), (name, label, i)


@pytest.mark.parametrize("case", [c for c in CAT if c[0].startswith("rand") or c[0] in
                                  ("intree", "loopmulti", "thirds", "zeros")],
                         ids=lambda c: c[0])
def test_path_frequencies_chi2(case):
    """Kept walks follow the walk-probability formula (equation
    "compute_path_inf", p == 1) divided by |V\\X|."""
    name, n, edges, src = case
    col, row, w = csc_from_edges(n, edges)
    law = exact.walk_tree(exact.quantized_edge_probs(col, row, w), src)["walks"]
    _, walks = run(name, n, edges, src, cpu.MODE_EDGES)
    obs = {}
    for i in range(walks.n_walks):
        key = tuple(int(x) for x in walks.walk(i))
        obs[key] = obs.get(key, 0) + 1
    expected = {edges_: float(p) * N for (nodes_, edges_), p in law.items()}
    assert set(obs) <= set(expected), name      # no walk outside the support
    big = [k for k, e in expected.items() if e >= 5]
    if len(big) < 2:
        return
    stat = sum((obs.get(k, 0) - expected[k]) ** 2 / expected[k] for k in big)
    rest_e = N * float(sum(law.values())) - sum(expected[k] for k in big)
    rest_o = walks.n_walks - sum(obs.get(k, 0) for k in big)
    dof = len(big) - 1
    if rest_e >= 5:
        stat += (rest_o - rest_e) ** 2 / rest_e
        dof += 1
    assert stat < chi2.ppf(1 - 1e-9, dof), (name, stat, dof)


def check_invariants(col, row, src, walks, mode):
    X = set(int(s) for s in src)
    col = [int(x) for x in col]
    for i in range(walks.n_walks):
        ids = [int(x) for x in walks.walk(i)]
        if mode == cpu.MODE_EDGES:
            assert len(ids) >= 1
            # edge j_i lies in the column of v_i and its tail is v_{i+1}
            nodes = []
            for j in ids:
                v = next(c for c in range(len(col) - 1) if col[c] <= j < col[c + 1])
                if nodes:
                    assert nodes[-1] == v
                else:
                    nodes.append(v)
                nodes.append(int(row[j]))
        else:
            nodes = ids
            assert len(nodes) >= 2
        assert nodes[0] not in X                       # start is not a source
        assert nodes[-1] in X                          # ends at a source
        assert not (set(nodes[:-1]) & X)               # h & X = {v_l}
        assert len(set(nodes)) == len(nodes)           # self-avoiding


def test_invariants_and_counter_identities():
    for name, n, edges, src in CAT:
        col, row, w = csc_from_edges(n, edges)
        for mode in (cpu.MODE_EDGES, cpu.MODE_NODES):
            g, walks = run(name, n, edges, src, mode, n_attempts=20_000, offset=12345)
            check_invariants(col, row, src, walks, mode)
            assert walks.hits == walks.n_walks
            assert walks.hits + walks.dead_ends + walks.cycles == 20_000
            size = len(row) if mode == cpu.MODE_EDGES else n
            cnt = cpu.count(max(size, 1), walks)
            assert int(cnt.sum()) == walks.ids.shape[0]
            assert np.all(np.diff(walks.attempt.astype(np.int64)) > 0)


def test_special_cases():
    # in-degree 0 everywhere but the source's out-edge target: dead end after one draw
    g, walks = run("indeg0", 4, [(1, 3, 0.5)], [3], cpu.MODE_EDGES, n_attempts=10_000)
    assert walks.steps == walks.attempts == walks.dead_ends == 10_000
    # no source reachable: nothing kept
    g, walks = run("twocycle", 3, [(0, 1, 1.0), (1, 0, 1.0)], [2], cpu.MODE_EDGES, 10_000)
    assert walks.hits == 0 and walks.cycles + walks.dead_ends == 10_000
    # chain with w = 1: every walk is the full path to the source
    chain = [(i + 1, i, 1.0) for i in range(5)]
    g, walks = run("chain1", 6, chain, [5], cpu.MODE_NODES, 5_000)
    for i in range(walks.n_walks):
        v = int(walks.walk(i)[0])
        assert walks.walk(i).tolist() == list(range(v, 6))


def brute_walk(col, row, thr, X, nonsrc, seed, a):
    """Walk of attempt a from first principles: numpy's Philox for the draws,
    the Fraction-derived thresholds, an explicit visited list."""
    x0 = numpy_block((0, 1, 0, 0), (seed, a))[0]
    v = nonsrc[(x0 * len(nonsrc)) >> 64]
    nodes, edges, steps = [v], [], 0
    while True:
        r = numpy_block((v, 0, 0, 0), (seed, a))[0] >> 32
        steps += 1
        lo, hi = col[v], col[v + 1]
        live = [j for j in range(lo, hi) if thr[j] > r]
        if not live:
            return "dead", steps, nodes, edges
        j = live[0]
        u = row[j]
        edges.append(j)
        if u in nodes:
            return "cycle", steps, nodes, edges
        nodes.append(u)
        if u in X:
            return "hit", steps, nodes, edges
        v = u


@pytest.mark.parametrize("case", CAT[:8] + CAT[-2:], ids=lambda c: c[0])
def test_walks_match_brute_force_tracer(case):
    name, n, edges_, src = case
    col, row, w = csc_from_edges(n, edges_)
    thr = exact.quantized_thresholds(col, w)
    X = set(src)
    nonsrc = [v for v in range(n) if v not in X]
    offset, count = 777, 300
    g = cpu.Graph(col, row, w)
    we = g.sample(np.array(src, np.int32), cpu.MODE_EDGES, count, offset, SEED)
    wn = g.sample(np.array(src, np.int32), cpu.MODE_NODES, count, offset, SEED)
    kept_e = {int(a): we.walk(i).tolist() for i, a in enumerate(we.attempt)}
    kept_n = {int(a): wn.walk(i).tolist() for i, a in enumerate(wn.attempt)}
    tot = dict(hit=0, dead=0, cycle=0, steps=0)
    for a in range(offset, offset + count):
        out, steps, nodes, edges = brute_walk([int(c) for c in col], [int(r) for r in row], thr,
                                              X, nonsrc, SEED, a)
        tot[out] += 1
        tot["steps"] += steps
        if out == "hit":
            assert kept_e[a] == edges and kept_n[a] == nodes, (name, a)
        else:
            assert a not in kept_e and a not in kept_n
    assert (tot["hit"], tot["dead"], tot["cycle"], tot["steps"]) == \
        (we.hits, we.dead_ends, we.cycles, we.steps)
