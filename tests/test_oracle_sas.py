"""Pins of the oracle's Stop-and-Stare driver (eSIA Algorithm 6 / nSIA
Algorithm 9, Check Algorithm 5 / 8), against what the mathematics fixes."""
import math

import numpy as np
import pytest

from oracle import cpu, sas


def test_ln_binom_matches_exact_binomials():
    for a in (1, 2, 10, 57, 300, 1000):
        for b in sorted({0, 1, a // 3, a // 2, a - 1, a}):
            exact = math.log(math.comb(a, b))
            assert abs(sas.ln_binom(a, b) - exact) <= 1e-9 * max(1.0, exact), (a, b)


@pytest.mark.parametrize("S,k,delta", [(8000, 10, 1e-3), (1000, 100, 1e-3), (263_430_593, 1000, 1 / 16_777_216)])
def test_t_max_is_the_lemma_bound_and_free_of_eps(S, k, delta):
    """The iteration bound's lemma simplifies log2(2 N_max / Upsilon) to
    log2(2 (2-1/e)^2 S (ln(6/delta) + ln C(S,k)) / (k ln(3/delta))): eps
    cancels, so t_max is the same for every eps."""
    lnc = math.lgamma(S + 1) - math.lgamma(k + 1) - math.lgamma(S - k + 1)
    bound = math.log2(2 * (2 - 1 / math.e) ** 2 * S * (math.log(6 / delta) + lnc) / (k * math.log(3 / delta)))
    for eps in (0.02, 0.1, 0.3, 0.9):
        P = sas.params(S, k, eps, delta)
        assert P["t_max"] == math.ceil(bound - 1e-9) or P["t_max"] == math.ceil(bound + 1e-9)
        # Lambda and Lambda_1 share the factor (2 + 2eps/3) ln(3 t_max / delta) / eps^2
        assert P["lam1"] - 1 == pytest.approx((1 + eps) * P["lam"], rel=1e-12)
        # N_max / Upsilon does not depend on eps either
        assert P["n_max"] / P["upsilon"] == pytest.approx(2 ** bound / 2, rel=1e-9)


def test_check_thresholds_and_monotonicity():
    eps, lam1 = 0.1, 500.0
    assert sas.check(10_000, 499, 5000, 1, eps, lam1) == (False, None)
    # more coverage on the verification set (same ratio) -> smaller error bound
    et = [sas.check(c, c, 20_000, 3, eps, lam1)[1] for c in (500, 1000, 4000, 16_000)]
    assert all(a > b for a, b in zip(et, et[1:]))
    # a candidate that covers more of R_t than of R'_t (overfit) -> larger bound
    e_fit = [sas.check(c, 2000, 20_000, 3, eps, lam1)[1] for c in (2000, 2500, 4000)]
    assert all(a < b for a, b in zip(e_fit, e_fit[1:]))
    # equal coverage, eps_1 = 0: with the whole verification set covered and
    # R'_t tiny relative to 2^(t-1) the bound vanishes and Check passes
    ok, e = sas.check(10 ** 6, 10 ** 6, 10 ** 6, 40, eps, lam1)
    assert ok and e < 1e-6


def test_coverage_matches_set_intersection():
    rng = np.random.default_rng(5)
    lens = rng.integers(1, 7, 300)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    ids = rng.integers(0, 200, int(lens.sum())).astype(np.uint32)
    chosen = rng.choice(200, 9, replace=False)
    want = sum(1 for i in range(300) if set(ids[off[i]:off[i + 1]].tolist()) & set(chosen.tolist()))
    assert sas.coverage(off, ids, chosen, 200) == want
    assert sas.coverage(np.zeros(1, np.uint64), np.zeros(0, np.uint32), chosen, 200) == 0


@pytest.fixture(scope="module")
def er1k():
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    return wl, cpu.Graph(*wl.host())


@pytest.mark.parametrize("mode", [cpu.MODE_EDGES, cpu.MODE_NODES])
def test_driver_follows_the_stream(er1k, mode):
    """R_t / R'_t are the first 2 N_t accepted walks of one sampling run over
    attempts [0, attempts_rp) in attempt order; the answer is the greedy on
    R_t; Check fails at every earlier iteration and passes (or N_max is
    reached) at the returned one."""
    wl, g = er1k
    S = g.m if mode == cpu.MODE_EDGES else g.n
    r = sas.stop_and_stare(g, wl.sources, mode, wl.k, 0.1, None, wl.seed, chunk=1 << 12)
    P = r["params"]
    assert r["status"] in ("passed", "n_max")
    assert r["n_t"] == math.ceil(P["lam"] * 2 ** (r["t"] - 1))
    whole = g.sample(wl.sources, mode, r["attempts_rp"], 0, wl.seed)
    assert whole.n_walks == 2 * r["n_t"] and np.all(np.diff(whole.attempt.astype(np.int64)) > 0)
    assert int(whole.attempt[r["n_t"] - 1]) + 1 == r["attempts_r"]

    def first(a, b):
        o = whole.off[a:b + 1].astype(np.int64)
        return (o - o[0]).astype(np.uint64), whole.ids[o[0]:o[-1]]

    for t in range(1, r["t"] + 1):
        n_t = math.ceil(P["lam"] * 2 ** (t - 1))
        off, ids = first(0, n_t)
        sel, gains = cpu.greedy_csr(S, off, ids, wl.k)
        offp, idsp = first(n_t, 2 * n_t)
        covp = sum(1 for i in range(n_t) if set(idsp[int(offp[i]):int(offp[i + 1])].tolist()) & set(sel.tolist()))
        ok, _ = sas.check(int(gains.sum()), covp, n_t, t, 0.1, P["lam1"])
        if t < r["t"]:
            assert not ok, t
        else:
            assert ok == (r["status"] == "passed")
            assert np.array_equal(sel, r["selected"]) and np.array_equal(gains, r["gains"])
            assert covp == r["cov_rp"] and int(gains.sum()) == r["cov_r"]


@pytest.mark.parametrize("mode", [cpu.MODE_EDGES, cpu.MODE_NODES])
def test_evaluation_on_the_greedy_sample_is_its_coverage(er1k, mode):
    """Evaluated on the very sample the greedy chose from, a set covers
    exactly the sum of its marginal gains (Algorithm 4 / 7); on a second seed
    the estimate agrees with the first within sampling error."""
    from oracle import evaluate
    wl, g = er1k
    r = cpu.solve(g, wl.sources, mode, wl.k, 50_000, 0, wl.seed)
    same = evaluate.evaluate(g, wl.sources, mode, r["selected"], 50_000, 0, wl.seed)
    assert same["covered"] == int(r["gains"].sum()) and same["walks"].hits == r["walks"].hits
    other = evaluate.evaluate(g, wl.sources, mode, r["selected"], 200_000, 0, wl.seed + 1)
    p = other["covered"] / 200_000
    sd = math.sqrt(p * (1 - p) / 200_000) + math.sqrt(p * (1 - p) / 50_000)
    assert abs(same["covered"] / 50_000 - p) < 6 * sd + 1e-9


def test_driver_with_suspects_follows_the_stream(er1k):
    """With probabilistic suspects the stream is the probabilistic sampler's
    kept walks in attempt order: R_t of the returned iteration is the first
    N_t of one sampling run."""
    wl, g = er1k
    rng = np.random.default_rng(4)
    sus = np.sort(rng.choice(g.n, 60, replace=False)).astype(np.int32)
    p = rng.uniform(0, 1, 60).astype(np.float32)
    r = sas.stop_and_stare(g, sus, cpu.MODE_NODES, wl.k, 0.1, None, wl.seed, chunk=1 << 12, p=p)
    whole = g.sample_suspects(sus, p, cpu.MODE_NODES, r["attempts_rp"], 0, wl.seed)
    assert whole.n_walks == 2 * r["n_t"]
    o = whole.off[: r["n_t"] + 1].astype(np.int64)
    sel, gains = cpu.greedy_csr(g.n, o.astype(np.uint64), whole.ids[:o[-1]], wl.k)
    assert np.array_equal(sel, r["selected"]) and np.array_equal(gains, r["gains"])
