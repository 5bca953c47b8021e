"""GPU parity of the Stop-and-Stare driver (sia_sas_solve: eSIA Algorithm 6 /
nSIA Algorithm 9 with Check) against the oracle's driver, on the same seeded
graphs: the same iteration, sample sizes, attempt bounds, picks, gains and
coverages, and Check's bound to rounding."""
import math

import numpy as np
import pytest

from oracle import cpu, sas

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STATUS = {"passed": 1, "n_max": 0, "attempts": -1}


def say(*a):
    print("[sas]", *a, flush=True)


@pytest.fixture(scope="module")
def sia():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05854_amd import sia as _sia
    _sia.lib()
    return _sia


def graphs(sia, name, **override):
    from paper_1702_05854_amd import workloads
    wl = workloads.load(name, **override)
    return wl, sia.Graph(*wl.host()), cpu.Graph(*wl.host())


@pytest.fixture(scope="module")
def er1k(sia):
    wl, g, og = graphs(sia, "er1k")
    yield wl, g, og
    g.close()


@pytest.fixture(scope="module")
def er20k(sia):
    wl, g, og = graphs(sia, "er1k", n=20_000, m=160_000, n_src=100, k=50)
    yield wl, g, og
    g.close()


def compare(got, ref):
    I = got["info"]
    assert I["status"] == STATUS[ref["status"]]
    assert (I["t"], I["n_t"]) == (ref["t"], ref["n_t"])
    P = ref["params"]
    assert I["t_max"] == P["t_max"]
    for a, b in (("lambda_", "lam"), ("lambda1", "lam1"), ("n_max", "n_max")):
        assert I[a] == pytest.approx(P[b], rel=1e-12), a
    if ref["status"] == "attempts":
        return
    assert (I["attempts_r"], I["attempts_rp"], I["cov_r"], I["cov_rp"]) == (
        ref["attempts_r"], ref["attempts_rp"], ref["cov_r"], ref["cov_rp"])
    assert np.array_equal(got["selected"], ref["selected"])
    assert np.array_equal(got["gains"], ref["gains"])
    if ref["eps_t"] is None:
        assert math.isnan(I["eps_t"])
    else:
        assert I["eps_t"] == pytest.approx(ref["eps_t"], rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("eps", [0.1, 0.3])
@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_sas_matches_oracle_er1k(sia, er1k, mode, eps):
    wl, g, og = er1k
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    say("er1k", mode, eps)
    got = sia.sas_solve(g, wl.sources, mode, wl.k, eps, None, wl.seed)
    ref = sas.stop_and_stare(og, wl.sources, om, wl.k, eps, None, wl.seed)
    compare(got, ref)
    I = got["info"]
    n_ns = wl.n - len(wl.sources)
    assert I["suspension_est"] == pytest.approx(n_ns * ref["cov_r"] / ref["attempts_r"], rel=1e-12)
    assert I["spread_est"] == pytest.approx(len(wl.sources) + n_ns * ref["n_t"] / ref["attempts_r"], rel=1e-12)


@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_sas_matches_oracle_er20k(sia, er20k, mode):
    """20000 nodes, 160000 edges, 100 sources, k = 50: five doublings (edges)."""
    wl, g, og = er20k
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    say("er20k", mode)
    got = sia.sas_solve(g, wl.sources, mode, wl.k, 0.1, None, wl.seed)
    ref = sas.stop_and_stare(og, wl.sources, om, wl.k, 0.1, None, wl.seed)
    compare(got, ref)


def test_sas_attempt_cap_and_arguments(sia, er1k):
    """A stream capped below 2 N_1 walks stops with status -1 at t = 1 (as
    the oracle); eps outside (0, 1 - 1/e) and delta outside (0, 1) are
    rejected."""
    wl, g, og = er1k
    got = sia.sas_solve(g, wl.sources, "edges", wl.k, 0.1, None, wl.seed, max_attempts=10_000)
    ref = sas.stop_and_stare(og, wl.sources, cpu.MODE_EDGES, wl.k, 0.1, None, wl.seed, max_attempts=10_000)
    compare(got, ref)
    assert got["info"]["status"] == -1 and got["info"]["attempts_sampled"] == 10_000
    for kw in (dict(eps=0.0), dict(eps=0.7), dict(delta=0.0), dict(delta=1.0)):
        with pytest.raises(sia.SiaError):
            sia.sas_solve(g, wl.sources, "edges", wl.k, **{**dict(eps=0.1, delta=1e-3), **kw})


@pytest.mark.parametrize("mode,eps,name", [("nodes", 0.5, "er1k_nodes"), ("edges", 0.1, "er1k_edges")])
def test_sas_driver_parameters_match_hand_derivation(sia, er1k, mode, eps, name):
    """The driver's Lambda, Lambda_1, N_max and t_max on the 1000-node graph
    (delta = 1/n, k = 10) equal the hand-derived values of
    tests/golden/sas_check.json (equations "lambda", "lambda_1", "nguard" /
    "guard", iteration lemma), and its N_t is ceil(Lambda 2^(t-1))."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sas_check.json")) as f:
        P = {p["name"]: p for p in json.load(f)["params"]}[name]
    wl, g, og = er1k
    assert (P["S"], P["k"]) == ((g.n if mode == "nodes" else g.m), 10) and wl.k == 10
    say("golden params", name)
    I = sia.sas_solve(g, wl.sources, mode, 10, eps, None, wl.seed)["info"]
    assert I["t_max"] == P["t_max"]
    assert I["n_max"] == pytest.approx(float(P["n_max"]), rel=1e-9)
    assert I["lambda_"] == pytest.approx(float(P["lam"]), rel=1e-13)
    assert I["lambda1"] == pytest.approx(float(P["lam1"]), rel=1e-13)
    assert I["n_t"] == math.ceil(float(P["lam"]) * 2 ** (I["t"] - 1))


@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_sas_suspects_matches_oracle(sia, er20k, mode):
    """Stop-and-Stare over the probabilistic-suspect sampler (500 suspects
    with random probabilities on the 20000-node graph): the same iteration,
    sample sizes, bounds, picks, gains and coverages as the oracle's driver."""
    wl, g, og = er20k
    rng = np.random.default_rng(21)
    sus = np.sort(rng.choice(wl.n, 500, replace=False)).astype(np.int32)
    p = rng.uniform(0, 1, 500).astype(np.float32)
    om = cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES
    say("er20k suspects", mode)
    got = sia.sas_solve_suspects(g, sus, p, mode, wl.k, 0.1, None, wl.seed)
    ref = sas.stop_and_stare(og, sus, om, wl.k, 0.1, None, wl.seed, p=p)
    compare(got, ref)
    I = got["info"]
    assert I["suspension_est"] == pytest.approx(wl.n * ref["cov_r"] / ref["attempts_r"], rel=1e-12)
    assert I["spread_est"] == pytest.approx(wl.n * ref["n_t"] / ref["attempts_r"], rel=1e-12)
    assert I["suspension_nodes_est"] == I["suspension_est"]
