"""Pins of the oracle's greedy max-coverage (Algorithm 4 / Algorithm 7) and of
the estimates (Theorem "lem:rr_edge" / "lem:rr_node")."""
from itertools import combinations
import math

import numpy as np
import pytest

from oracle import cpu, exact
from tiny import catalogue, count_tolerance, csc_from_edges


def random_walk_sets(seed, n_walks, id_space, max_len):
    rng = np.random.default_rng(seed)
    walks = []
    for _ in range(n_walks):
        L = int(rng.integers(1, max_len + 1))
        walks.append(sorted(rng.choice(id_space, size=min(L, id_space), replace=False).tolist()))
    off = np.zeros(len(walks) + 1, np.uint64)
    off[1:] = np.cumsum([len(w) for w in walks])
    ids = np.array([i for w in walks for i in w], np.uint32)
    return walks, off, ids


def naive_greedy(walks, id_space, k):
    """Recompute every marginal gain from scratch each round (a different
    algorithm from the oracle's decrement-maintained counts)."""
    covered = [False] * len(walks)
    chosen = []
    gains = []
    for _ in range(k):
        best, best_gain = None, -1
        for c in range(id_space):
            if c in chosen:
                continue
            g = sum(1 for i, w in enumerate(walks) if not covered[i] and c in w)
            if g > best_gain:
                best, best_gain = c, g
        chosen.append(best)
        gains.append(best_gain)
        for i, w in enumerate(walks):
            if best in w:
                covered[i] = True
    return chosen, gains


@pytest.mark.parametrize("seed", range(12))
def test_greedy_matches_naive_recompute(seed):
    id_space = [5, 12, 40, 200][seed % 4]
    walks, off, ids = random_walk_sets(seed, 30 + 10 * seed, id_space, 6)
    k = min(id_space, 3 + seed)
    sel, gains = cpu.greedy_csr(id_space, off, ids, k)
    ns, ng = naive_greedy(walks, id_space, k)
    assert sel.tolist() == ns and gains.tolist() == ng


def coverage(walks, T):
    T = set(T)
    return sum(1 for w in walks if T & set(w))


@pytest.mark.parametrize("seed", range(8))
def test_greedy_vs_brute_force_opt(seed):
    id_space = 9
    walks, off, ids = random_walk_sets(100 + seed, 25, id_space, 4)
    for k in (1, 2, 3):
        sel, gains = cpu.greedy_csr(id_space, off, ids, k)
        opt = max(coverage(walks, T) for T in combinations(range(id_space), k))
        got = coverage(walks, sel.tolist())
        assert got == int(gains.sum())
        assert opt >= got >= (1 - (1 - 1 / k) ** k) * opt - 1e-9
        assert got >= (1 - 1 / math.e) * opt - 1e-9


def test_k1_is_argmax_lowest_id_and_gains_nonincreasing():
    walks, off, ids = random_walk_sets(7, 500, 60, 8)
    cnt = np.zeros(60, np.int64)
    for w in walks:
        cnt[w] += 1
    sel, gains = cpu.greedy_csr(60, off, ids, 1)
    assert sel[0] == int(np.flatnonzero(cnt == cnt.max())[0]) and gains[0] == cnt.max()
    sel, gains = cpu.greedy_csr(60, off, ids, 60)
    assert np.all(np.diff(gains.astype(np.int64)) <= 0)     # submodularity (Corollary "lem:mon_sub")
    assert sorted(sel.tolist()) == list(range(60))


def test_ties_and_zero_gain_rounds():
    # walks {1,2}, {3}: round 1 tie between 1 and 2 (gain 1) and 3 (gain 1) -> 1
    off = np.array([0, 2, 3], np.uint64)
    ids = np.array([1, 2, 3], np.uint32)
    sel, gains = cpu.greedy_csr(6, off, ids, 5)
    assert sel.tolist() == [1, 3, 0, 2, 4]
    assert gains.tolist() == [1, 1, 0, 0, 0]
    sel, gains = cpu.greedy_csr(4, np.zeros(1, np.uint64), np.zeros(0, np.uint32), 4)
    assert sel.tolist() == [0, 1, 2, 3] and gains.tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("case", [c for c in catalogue() if c[0] not in ("twocycle", "indeg0")],
                         ids=lambda c: c[0])
def test_estimates_converge_to_exact_suspension(case):
    """|V\\X| * Cov(T)/N estimates D(T) (Theorem "lem:rr_edge"); the nodes
    version adds the removed sources themselves (Theorem "lem:rr_node")."""
    name, n, edges, src = case
    col, row, w = csc_from_edges(n, edges)
    g = cpu.Graph(col, row, w)
    tg = exact.quantized_edge_probs(col, row, w)
    N = 200_000
    n_ns = n - len(src)
    for mode, label in ((cpu.MODE_EDGES, "edges"), (cpu.MODE_NODES, "nodes")):
        size = g.m if mode == cpu.MODE_EDGES else n
        k = min(2, size)
        res = cpu.solve(g, np.array(src, np.int32), mode, k, N, 0, 2017)
        T = res["selected"].tolist()
        d_exact = exact.suspension_from_paths(tg, src, T, label)
        # Cov(T)/N estimates Pr[T interdicts the walk of one attempt]
        p = float(d_exact - (len(set(T) & set(src)) if label == "nodes" else 0)) / n_ns
        assert abs(res["covered"] - N * p) <= count_tolerance(N, p), (name, label)
        est = res["suspension_nodes"] if label == "nodes" else res["suspension"]
        assert abs(est - float(d_exact)) <= n_ns * count_tolerance(N, p) / N + 1e-12
        spread = float(exact.spread_from_paths(tg, src))
        p_hit = (spread - len(src)) / n_ns
        assert abs(res["spread"] - spread) <= n_ns * count_tolerance(N, p_hit) / N + 1e-12
