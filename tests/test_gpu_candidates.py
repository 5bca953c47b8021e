"""GPU parity of the candidate-set path (sia_solve_candidates: the greedy
draws its k ids from C within E or V) against the oracle's."""
import numpy as np
import pytest

from oracle import candidates, cpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sia():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05854_amd import sia as _sia
    _sia.lib()
    return _sia


@pytest.fixture(scope="module")
def er20k(sia):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k", n=20_000, m=160_000, n_src=100, k=50, n_attempts=400_000)
    g = sia.Graph(*wl.host())
    yield wl, g, cpu.Graph(*wl.host())
    g.close()


@pytest.mark.parametrize("mode,frac,k", [("edges", 0.3, 50), ("nodes", 0.5, 50), ("edges", 0.001, 160),
                                         ("nodes", 0.02, 300)])
def test_candidates_match_oracle(sia, er20k, mode, frac, k):
    """Random candidate sets from 0.1% to 50% of the ids; the last two take
    k = |C| or close to it, so zero-gain picks come from C too."""
    wl, g, og = er20k
    S = g.m if mode == "edges" else g.n
    rng = np.random.default_rng(int(frac * 1000) + k)
    cand = rng.choice(S, max(k, int(frac * S)), replace=False)
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    got = sia.solve(g, wl.sources, mode, k, wl.n_attempts, 0, wl.seed, candidates=cand)
    ref = candidates.solve_candidates(og, wl.sources, om, k, wl.n_attempts, 0, wl.seed, cand)
    assert np.array_equal(got["selected"], ref["selected"])
    assert np.array_equal(got["gains"], ref["gains"])
    assert got["stats"]["covered"] == ref["covered"]
    assert got["stats"]["hits"] == ref["walks"].hits
    assert np.isin(got["selected"], cand).all()


def test_candidates_nodes_with_every_source(sia, er20k):
    """Node removal with every source and half the other nodes as candidates:
    the first picks (sources) cover most walks, so the counts are recomputed
    from the walks left, whose ids outside C must keep their mark."""
    wl, g, og = er20k
    rng = np.random.default_rng(77)
    others = np.setdiff1d(np.arange(g.n), wl.sources)
    cand = np.concatenate([wl.sources, rng.choice(others, others.shape[0] // 2, replace=False)])
    got = sia.solve(g, wl.sources, "nodes", 150, wl.n_attempts, 0, wl.seed, candidates=cand)
    ref = candidates.solve_candidates(og, wl.sources, cpu.MODE_NODES, 150, wl.n_attempts, 0, wl.seed, cand)
    assert np.array_equal(got["selected"], ref["selected"])
    assert np.array_equal(got["gains"], ref["gains"])
    assert got["stats"]["covered"] == ref["covered"]
    assert np.isin(got["selected"], cand).all()


def test_candidates_every_id_equals_plain_solve(sia, er20k):
    wl, g, og = er20k
    a = sia.solve(g, wl.sources, "edges", 50, wl.n_attempts, 0, wl.seed)
    b = sia.solve(g, wl.sources, "edges", 50, wl.n_attempts, 0, wl.seed,
                  candidates=np.random.default_rng(1).permutation(g.m))
    assert np.array_equal(a["selected"], b["selected"]) and np.array_equal(a["gains"], b["gains"])


def test_candidates_rejected(sia, er20k):
    wl, g, og = er20k
    for cand, k in (([1, 2, 3], 4), ([5, 5, 6], 2), ([g.m], 1), ([-1, 2], 1), ([], 1)):
        with pytest.raises(sia.SiaError) as e:
            sia.solve(g, wl.sources, "edges", k, 1000, 0, wl.seed, candidates=np.array(cand, np.int64))
        assert e.value.status == -1
