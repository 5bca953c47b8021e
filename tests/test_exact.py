"""Self-consistency of the exact enumerator: its independent routes must agree
exactly (in rationals), which also checks Theorems "lem:rr_edge" and
"lem:rr_node" (suspension = probability mass of interdicted HSAWs) and
Corollary "lem:mon_sub" on each instance."""
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

from oracle import exact
from tiny import catalogue, csc_from_edges

CAT = catalogue()


def graphs(quantized):
    for name, n, edges, src in CAT:
        col, row, w = csc_from_edges(n, edges)
        f = exact.quantized_edge_probs if quantized else exact.exact_edge_probs
        yield name, f(col, row, w), src, (col, row, w)


@pytest.mark.parametrize("quantized", [False, True])
def test_spread_paths_equal_live_edge(quantized):
    for name, g, src, _ in graphs(quantized):
        assert exact.spread_from_paths(g, src) == exact.live_edge_spread(g, src), name


@pytest.mark.parametrize("quantized", [False, True])
def test_suspension_routes_agree(quantized):
    rng = np.random.default_rng(1)
    for name, g, src, _ in graphs(quantized):
        for mode, size in (("edges", g.m), ("nodes", g.n)):
            if size == 0:
                continue
            for _ in range(4):
                k = int(rng.integers(1, min(3, size) + 1))
                T = sorted(rng.choice(size, size=k, replace=False).tolist())
                a = exact.suspension_from_paths(g, src, T, mode)
                b = exact.live_edge_suspension(g, src, T, mode)
                assert a == b, (name, mode, T)


def test_walk_tree_is_a_distribution_and_matches_paths():
    for name, g, src, _ in graphs(True):
        t = exact.walk_tree(g, src)
        assert t["hit"] + t["dead_end"] + t["cycle"] == 1, name
        n_ns = g.n - len(set(src))
        spread = exact.spread_from_paths(g, src)
        assert t["hit"] == (spread - len(set(src))) / n_ns, name
        assert sum(t["walks"].values()) == t["hit"]
        assert t["steps"] >= 1


def test_chain_closed_form():
    # 0 <- 1 <- 2 <- 3 <- 4 with w = 1/2 each, source 4: Pr[hit from v] = 2^-(4-v)
    name, n, edges, src = CAT[0]
    col, row, w = csc_from_edges(n, edges)
    g = exact.exact_edge_probs(col, row, w)
    expect = sum(Fraction(1, 2 ** (4 - v)) for v in range(4))
    assert exact.spread_from_paths(g, src) == 1 + expect
    # removing the edge 3 -> 2 cuts the walks from 2, 1 and 0
    j = [k for k in range(g.m) if g.row_idx[k] == 3][0]
    cut = Fraction(1, 4) + Fraction(1, 8) + Fraction(1, 16)
    assert exact.suspension_from_paths(g, src, [j], "edges") == cut


def test_single_in_edge_from_source():
    col, row, w = csc_from_edges(2, [(1, 0, 0.375)])
    g = exact.quantized_edge_probs(col, row, w)
    t = exact.walk_tree(g, [1])
    assert t["hit"] == Fraction(exact.quantize_exact(0.375), 1 << 32) == Fraction(3, 8)
    assert t["dead_end"] == Fraction(5, 8) and t["cycle"] == 0 and t["steps"] == 1


def test_monotone_submodular():
    for name, g, src, _ in graphs(False):
        for mode, size in (("edges", g.m), ("nodes", g.n)):
            ids = list(range(size))[:6]
            D = {}
            for r in range(0, 4):
                for T in combinations(ids, r):
                    D[T] = exact.suspension_from_paths(g, src, T, mode)
            for T, d in D.items():
                for e in ids:
                    if e in T:
                        continue
                    T2 = tuple(sorted(T + (e,)))
                    if T2 not in D:
                        continue
                    assert D[T2] >= d, (name, T, e)          # monotone
                    for f in ids:
                        if f in T2 or f == e:
                            continue
                        T3 = tuple(sorted(T + (f,)))
                        T4 = tuple(sorted(T2 + (f,)))
                        if T4 in D:
                            # gain of f shrinks once e is present
                            assert D[T3] - d >= D[T4] - D[T2], (name, T, e, f)


def test_edge_node_subdivision_identity():
    """Edge interdiction on G equals node interdiction of the subdivision
    nodes on the subdivided graph, counting the original nodes (appendix,
    proof of Theorem "theo:hard", with the LT-valid weight placement)."""
    rng = np.random.default_rng(3)
    for name, n, edges, src in CAT[:10]:
        col, row, w = csc_from_edges(n, edges)
        g = exact.exact_edge_probs(col, row, w)
        gs = exact.subdivide(col, row, w)
        for _ in range(3):
            if g.m == 0:
                break
            T = sorted(rng.choice(g.m, size=min(2, g.m), replace=False).tolist())
            d_edge = exact.suspension_from_paths(g, src, T, "edges")
            S = [n + j for j in T]
            d_node = exact.suspension_from_paths(gs, src, S, "nodes", starts=range(n))
            assert d_edge == d_node, (name, T)
            d_node_le = exact.live_edge_suspension(gs, src, S, "nodes", count_only=range(n))
            assert d_edge == d_node_le, (name, T)
