"""Catalogue of tiny graphs and statistical tolerances shared by the tests.

Graphs are given as edge lists (u, v, w): a directed edge u -> v whose LT
weight w(u,v) sits in column v of the in-edge CSC.  Within a column, edges
keep the listed order (that order is the threshold order).
"""
import math

import numpy as np


def csc_from_edges(n, edges):
    cols = [[] for _ in range(n)]
    for (u, v, w) in edges:
        cols[v].append((u, w))
    col_off = [0]
    row_idx, ws = [], []
    for v in range(n):
        for (u, w) in cols[v]:
            row_idx.append(u)
            ws.append(w)
        col_off.append(len(row_idx))
    return (np.array(col_off, dtype=np.int64), np.array(row_idx, dtype=np.int32),
            np.array(ws, dtype=np.float32))


def random_tiny(n, p_edge, seed, wmode="inv", max_deg=3):
    rng = np.random.default_rng(seed)
    edges = []
    for v in range(n):
        tails = [u for u in range(n) if u != v and rng.uniform() < p_edge][:max_deg]
        if not tails:
            continue
        if wmode == "inv":
            ws = [np.float32(1.0) / np.float32(len(tails))] * len(tails)
        else:
            x = rng.uniform(0.05, 1.0, len(tails))
            s = rng.uniform(0.3, 1.0)
            ws = list((x * s / x.sum()).astype(np.float32))
        edges += [(u, v, w) for u, w in zip(tails, ws)]
    return edges


def catalogue():
    """(name, n, edges, sources) of tiny instances with distinct behaviours."""
    out = []
    # chain 0 <- 1 <- 2 <- 3 <- 4 (edges point towards lower ids), source 4
    out.append(("chain", 5, [(i + 1, i, 0.5) for i in range(4)], [4]))
    # in-tree: every node's single in-edge comes from its parent; root 0 is a source
    tree = [(0, 1, 0.9), (0, 2, 0.6), (1, 3, 1.0), (1, 4, 0.25), (2, 5, 0.75)]
    out.append(("intree", 6, tree, [0]))
    # 2-cycle with sum w = 1 and no reachable source
    out.append(("twocycle", 3, [(0, 1, 1.0), (1, 0, 1.0)], [2]))
    # in-degree 0 everywhere except into the source
    out.append(("indeg0", 4, [(1, 3, 0.5)], [3]))
    # zero-weight edges and an isolated node
    out.append(("zeros", 5, [(1, 0, 0.0), (2, 0, 0.5), (3, 1, 0.0), (4, 1, 1.0), (0, 2, 0.3)], [4]))
    # all but one node are sources
    out.append(("allsrc", 4, [(1, 0, 0.3), (2, 0, 0.3), (3, 0, 0.4)], [1, 2, 3]))
    # self-loop (picking it is a cycle) and a multi-edge
    out.append(("loopmulti", 4, [(0, 0, 0.25), (1, 0, 0.25), (1, 0, 0.25), (2, 1, 0.5),
                                 (3, 2, 1.0)], [3]))
    # 1/3 weights: fp32(1/3) * 3 exceeds 1 after quantisation and is clamped
    third = float(np.float32(1.0) / np.float32(3.0))
    out.append(("thirds", 5, [(1, 0, third), (2, 0, third), (3, 0, third), (4, 1, 1.0),
                              (0, 2, 0.5), (4, 3, 0.5)], [4]))
    # seeded random instances
    for seed in range(6):
        n = 6 + seed % 2
        edges = random_tiny(n, 0.45, seed, "inv" if seed % 2 == 0 else "rand")
        rng = np.random.default_rng(100 + seed)
        src = sorted(rng.choice(n, size=1 + seed % 2, replace=False).tolist())
        out.append((f"rand{seed}", n, edges, src))
    return out


LN_DELTA = math.log(2.0 / 1e-12)


def count_tolerance(n_trials, p):
    """Two-sided Bernstein bound on |count - n p| failing with probability
    below 1e-12 (per assertion) -- the concentration the paper's Chernoff
    lemma ("lem:chernoff") gives for sums of independent Bernoullis."""
    return math.sqrt(2.0 * n_trials * p * (1.0 - p) * LN_DELTA) + (2.0 / 3.0) * LN_DELTA + 1e-9
