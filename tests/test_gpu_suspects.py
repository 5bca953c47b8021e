"""GPU parity with probabilistic suspects (Section 2.2, equation
"prob_src_set"; Algorithm 1's suspect test): the HIP sampler's kept walks,
counters, picks, gains and estimates against the oracle's, walk for walk, on
the tiny catalogue, the 1000-node random graph (every node a suspect, and a
random tenth), the Chung-Lu graph with 1000 suspects of random probability
(the paper's experimental setting) and a scale-16 R-MAT graph."""
import numpy as np
import pytest

from oracle import cpu
from test_oracle_suspects import CASES
from tiny import csc_from_edges

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 2017


@pytest.fixture(scope="module")
def sia():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05854_amd import sia as _sia
    _sia.lib()
    return _sia


def omode(mode):
    return cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES


def assert_walks_equal(got, ref, label):
    assert (got.stats["hits"], got.stats["dead_ends"], got.stats["cycles"], got.stats["steps"]) == (
        ref.hits, ref.dead_ends, ref.cycles, ref.steps), label
    assert np.array_equal(got.attempt, ref.attempt), label
    assert np.array_equal(got.off, ref.off), label
    assert np.array_equal(got.ids, ref.ids), label


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tiny_walks_match_oracle(sia, case):
    name, n, edges, sus, p = case
    if n < 2:
        pytest.skip("the library needs n >= 2")
    col, row, w = csc_from_edges(n, edges)
    g = sia.Graph(col, row, w)
    og = cpu.Graph(col, row, w)
    for mode in ("edges", "nodes"):
        got = sia.sample_suspects(g, sus, p, mode, 30_000, 5_000, SEED)
        ref = og.sample_suspects(np.array(sus, np.int32), p, omode(mode), 30_000, 5_000, SEED)
        assert_walks_equal(got, ref, (name, mode))
    g.close()


def er1k_graphs(sia):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    col, row, w = wl.host()
    return wl, sia.Graph(col, row, w), cpu.Graph(col, row, w)


@pytest.mark.parametrize("layout", ["all_half", "tenth_random", "all_zero_but_one"])
def test_er1k_solve_matches_oracle(sia, layout):
    """1000 nodes, 8000 edges (w = 1/d_in): every node a suspect with p = 1/2
    (the setting of the appendix's reduction), a random tenth with random p,
    and every node a suspect with p = 0 except one with p = 1."""
    wl, g, og = er1k_graphs(sia)
    rng = np.random.default_rng(11)
    if layout == "all_half":
        sus, p = np.arange(1000), np.full(1000, 0.5)
    elif layout == "tenth_random":
        sus = np.sort(rng.choice(1000, 100, replace=False))
        p = rng.uniform(0, 1, 100)
    else:
        sus, p = np.arange(1000), np.zeros(1000)
        p[417] = 1.0
    sus, p = sus.astype(np.int32), p.astype(np.float32)
    for mode, k in (("edges", 10), ("nodes", 10)):
        got = sia.sample_suspects(g, sus, p, mode, 60_000, 0, SEED)
        ref = og.sample_suspects(sus, p, omode(mode), 60_000, 0, SEED)
        assert_walks_equal(got, ref, (layout, mode))
        r = sia.solve_suspects(g, sus, p, mode, k, 60_000, 0, SEED)
        o = cpu.solve_suspects(og, sus, p, omode(mode), k, 60_000, 0, SEED)
        assert np.array_equal(r["selected"], o["selected"]), (layout, mode)
        assert np.array_equal(r["gains"], o["gains"]), (layout, mode)
        st = r["stats"]
        assert st["hits"] == o["walks"].hits and st["covered"] == o["covered"]
        assert st["spread_est"] == o["spread"] and st["suspension_est"] == o["suspension"]
        assert st["suspension_nodes_est"] == st["suspension_est"]
    g.close()


def test_suspect_arguments_rejected(sia):
    wl, g, og = er1k_graphs(sia)
    for sus, p in (([1, 1], [0.5, 0.5]), ([1, 1000], [0.5, 0.5]), ([-1], [0.5]), ([3], [1.5]),
                   ([3], [float("nan")]), ([3], [-0.1]), ([], [])):
        with pytest.raises(sia.SiaError) as e:
            sia.sample_suspects(g, np.array(sus, np.int32), np.array(p, np.float32), "edges", 1000)
        assert e.value.status == -1, (sus, p)
    g.close()


def test_cl1m_solve_matches_oracle(sia):
    """Chung-Lu, 10^6 nodes, 1.6*10^7 edges, random column sums; 1000 random
    suspects with random probabilities; 2*10^6 attempts; k = 100, both modes."""
    from paper_1702_05854_amd import workloads
    print("[suspects] generating cl1m", flush=True)
    wl = workloads.load("cl1m")
    col, row, w = wl.host()
    g = sia.Graph(wl.col_off.cuda(), wl.row_idx.cuda(), wl.w.cuda())
    og = cpu.Graph(col, row, w)
    rng = np.random.default_rng(12)
    sus = np.sort(rng.choice(wl.n, 1000, replace=False)).astype(np.int32)
    p = rng.uniform(0, 1, 1000).astype(np.float32)
    N = 2_000_000
    for mode in ("edges", "nodes"):
        print("[suspects] cl1m", mode, flush=True)
        r = sia.solve_suspects(g, sus, p, mode, 100, N, 0, SEED)
        o = cpu.solve_suspects(og, sus, p, omode(mode), 100, N, 0, SEED)
        st = r["stats"]
        assert (st["hits"], st["dead_ends"], st["cycles"], st["steps"], st["walk_ids"]) == (
            o["walks"].hits, o["walks"].dead_ends, o["walks"].cycles, o["walks"].steps, o["walks"].ids.shape[0])
        assert np.array_equal(r["selected"], o["selected"]), mode
        assert np.array_equal(r["gains"], o["gains"]), mode
    g.close()


def test_rmat16_walks_match_oracle(sia):
    """R-MAT scale 16 (w = 1/d_in: 16-byte records) and the same graph with
    normalised random weights (32-byte records), 3000 suspects."""
    from paper_1702_05854_amd import workloads
    rng = np.random.default_rng(13)
    for weights in ("inv_indeg", "normalized"):
        wl = workloads.load("rmat22", scale=16, weights=weights)
        col, row, w = wl.host()
        g = sia.Graph(col, row, w)
        assert g.arc_bytes == (16 if weights == "inv_indeg" else 32)
        og = cpu.Graph(col, row, w)
        sus = np.sort(rng.choice(wl.n, 3000, replace=False)).astype(np.int32)
        p = rng.uniform(0, 1, 3000).astype(np.float32)
        for mode in ("edges", "nodes"):
            got = sia.sample_suspects(g, sus, p, mode, 300_000, 123, SEED)
            ref = og.sample_suspects(sus, p, omode(mode), 300_000, 123, SEED)
            assert_walks_equal(got, ref, (weights, mode))
        g.close()
