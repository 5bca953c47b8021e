"""Hand-derived golden law (tests/golden/three_node_cycle.json, with its
derivation and citation): the exact enumerator must reproduce it exactly, the
oracle sampler's frequencies must match it within sampling error, and the
oracle greedy must pick the edge every kept walk holds."""
import json
import os
from fractions import Fraction

import numpy as np

from oracle import cpu, exact
from tiny import csc_from_edges

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    with open(os.path.join(HERE, "golden", "three_node_cycle.json")) as f:
        fx = json.load(f)
    law = {}
    for flavour in ("exact", "quantized"):
        d = fx[flavour]
        law[flavour] = {k: Fraction(v) for k, v in d.items() if k != "walks"}
        law[flavour]["walks"] = {k: Fraction(v) for k, v in d["walks"].items()}
    edges = [(int(u), int(v), float(w)) for u, v, w in fx["graph"]["edges_u_v_w"]]
    return fx, law, csc_from_edges(fx["graph"]["n"], edges)


def key(nodes, edges):
    return ",".join(str(int(x)) for x in nodes) + "|" + ",".join(str(int(j)) for j in edges)


def test_enumerator_reproduces_hand_law():
    fx, law, (col, row, w) = load()
    for flavour, probs in (("exact", exact.exact_edge_probs), ("quantized", exact.quantized_edge_probs)):
        t = exact.walk_tree(probs(col, row, w), fx["sources"])
        for k in ("hit", "dead_end", "cycle", "steps"):
            assert t[k] == law[flavour][k], (flavour, k)
        got = {key(n, e): p for (n, e), p in t["walks"].items()}
        assert got == law[flavour]["walks"], flavour


def test_oracle_sampler_frequencies():
    fx, law, (col, row, w) = load()
    q = law["quantized"]
    N = 400_000
    og = cpu.Graph(col, row, w)
    walks = og.sample(np.array(fx["sources"], np.int32), cpu.MODE_EDGES, N, 0, 2017)
    for k, got in (("hit", walks.hits), ("dead_end", walks.dead_ends), ("cycle", walks.cycles)):
        p = float(q[k])
        assert abs(got - N * p) < 5 * np.sqrt(N * p * (1 - p)) + 1, k
    mean_steps = walks.steps / N
    assert abs(mean_steps - float(q["steps"])) < 0.01
    # every kept walk is one of the two walks of the law, with its frequency
    off = [int(x) for x in walks.off] + [len(walks.ids)]
    assert walks.hits == len(walks.attempt)
    seen = {}
    for i in range(len(walks.attempt)):
        ids = tuple(int(x) for x in walks.ids[off[i]:off[i + 1]])
        seen[ids] = seen.get(ids, 0) + 1
    assert set(seen) <= {(1,), (2, 1)}
    for ids, p in (((1,), q["walks"]["0,2|1"]), ((2, 1), q["walks"]["1,0,2|2,1"])):
        p = float(p)
        assert abs(seen.get(ids, 0) - N * p) < 5 * np.sqrt(N * p * (1 - p)) + 1, ids


def test_oracle_greedy_takes_the_shared_edge():
    fx, law, (col, row, w) = load()
    og = cpu.Graph(col, row, w)
    r = cpu.solve(og, np.array(fx["sources"], np.int32), cpu.MODE_EDGES, 2, 100_000, 0, 7)
    hits = r["walks"].hits
    # edge 1 (2->0) lies on every kept walk; then edge 2 (0->1) has nothing left
    assert r["selected"].tolist() == [1, 0] and r["gains"].tolist() == [hits, 0]
