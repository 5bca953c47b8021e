"""GPU parity of the out-of-sample evaluation (sia_evaluate) against the
oracle's: exact counters and coverage on a second seed."""
import numpy as np
import pytest

from oracle import cpu, evaluate

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sia():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05854_amd import sia as _sia
    _sia.lib()
    return _sia


@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_evaluate_matches_oracle(sia, mode):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k", n=20_000, m=160_000, n_src=100, k=50, n_attempts=300_000)
    g = sia.Graph(*wl.host())
    og = cpu.Graph(*wl.host())
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    sol = sia.solve(g, wl.sources, mode, wl.k, wl.n_attempts, 0, wl.seed)
    same = sia.evaluate(g, wl.sources, mode, sol["selected"], wl.n_attempts, 0, wl.seed)
    assert same["covered"] == int(sol["gains"].sum())
    got = sia.evaluate(g, wl.sources, mode, sol["selected"], 400_000, 7, wl.seed + 1)
    ref = evaluate.evaluate(og, wl.sources, om, sol["selected"], 400_000, 7, wl.seed + 1)
    assert got["covered"] == ref["covered"] and got["hits"] == ref["walks"].hits
    assert (got["dead_ends"], got["cycles"], got["steps"]) == (ref["walks"].dead_ends, ref["walks"].cycles,
                                                              ref["walks"].steps)
    for a, b in (("spread_est", "spread"), ("suspension_est", "suspension"),
                 ("suspension_nodes_est", "suspension_nodes")):
        assert got[a] == pytest.approx(ref[b], rel=1e-12), a
    with pytest.raises(sia.SiaError):
        sia.evaluate(g, wl.sources, mode, np.array([-1], np.int64), 1000, 0, wl.seed)
    g.close()
