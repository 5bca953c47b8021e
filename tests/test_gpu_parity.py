"""GPU parity: the HIP path through the C ABI against the CPU oracle,
element by element (bit-exact: all quantities are integers)."""
import numpy as np
import pytest

from oracle import cpu
from tiny import catalogue, csc_from_edges, random_tiny

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CAT = catalogue()
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
    assert got.stats["hits"] == ref.hits, label
    assert got.stats["dead_ends"] == ref.dead_ends, label
    assert got.stats["cycles"] == ref.cycles, label
    assert got.stats["steps"] == ref.steps, label
    assert got.stats["evaluations"] >= got.stats["steps"], label
    assert np.array_equal(got.attempt, ref.attempt), label
    assert np.array_equal(got.off, ref.off), label
    assert np.array_equal(got.ids, ref.ids), label


# ------------------------------------------------------------------ ingest
@pytest.mark.parametrize("case", CAT, ids=[c[0] for c in CAT])
def test_thresholds_match_oracle(sia, case):
    name, n, edges, src = case
    col, row, w = csc_from_edges(n, edges)
    g = sia.Graph(col, row, w)
    assert np.array_equal(g.thresholds(), cpu.Graph(col, row, w).thr), name
    gd = sia.Graph(torch.from_numpy(col).cuda(), torch.from_numpy(row).cuda(),
                   torch.from_numpy(w).cuda())
    assert np.array_equal(gd.thresholds(), cpu.Graph(col, row, w).thr), name


def test_thresholds_big_columns_and_device_inputs(sia):
    # one column above the one-workgroup threshold, plus ragged small ones
    rng = np.random.default_rng(1)
    n = 40000
    degs = rng.integers(0, 5, n)
    degs[7] = 70_001
    degs[123] = 16_385
    col = np.zeros(n + 1, np.int64)
    col[1:] = np.cumsum(degs)
    m = int(col[-1])
    row = rng.integers(0, n, m).astype(np.int32)
    w = np.empty(m, np.float32)
    for v in range(n):
        d = degs[v]
        if d:
            x = rng.uniform(0.01, 1, d)
            w[col[v]:col[v + 1]] = (x * rng.uniform(0.2, 1.0) / x.sum()).astype(np.float32)
    ref = cpu.Graph(col, row, w).thr
    g = sia.Graph(torch.from_numpy(col).cuda(), torch.from_numpy(row).cuda(), torch.from_numpy(w).cuda())
    assert np.array_equal(g.thresholds(), ref)


def compact_case(seed=7, n=3000):
    """A graph with w = 1/d_in (fp32) in every column: ragged small columns,
    in-degree-1 columns and one column above the one-workgroup size."""
    rng = np.random.default_rng(seed)
    degs = rng.integers(0, 7, n)
    degs[5] = 20_000
    degs[9] = degs[11] = 1
    col = np.zeros(n + 1, np.int64)
    col[1:] = np.cumsum(degs)
    m = int(col[-1])
    row = rng.integers(0, n, m).astype(np.int32)
    w = np.empty(m, np.float32)
    for v in range(n):
        if degs[v]:
            w[col[v]:col[v + 1]] = np.float32(1.0) / np.float32(degs[v])
    return col, row, w, degs


@pytest.mark.parametrize("perturb", [False, True])
def test_record_format_follows_weights(sia, perturb):
    """w = 1/d_in in every column gives 16-byte records, anything else (here
    one weight of one column moved by one ulp) 32-byte ones; thresholds, walks
    and answers equal the oracle's either way."""
    col, row, w, degs = compact_case()
    if perturb:
        v = int(np.flatnonzero(degs >= 3)[0])
        w[col[v] + 1] = np.nextafter(w[col[v] + 1], np.float32(0))
    g = sia.Graph(col, row, w)
    assert g.arc_bytes == (32 if perturb else 16)
    og = cpu.Graph(col, row, w)
    assert np.array_equal(g.thresholds(), og.thr)
    src = [3, 5, 77, 1234, 2999]
    for mode in ("edges", "nodes"):
        for offset, N in ((0, 40_000), (10 ** 12, 7_777)):
            got = sia.sample(g, src, mode, N, offset, SEED)
            ref = og.sample(np.array(src, np.int32), omode(mode), N, offset, SEED)
            assert_walks_equal(got, ref, (perturb, mode, offset))
        r = sia.solve(g, src, mode, 25, 40_000, 0, SEED)
        o = cpu.solve(og, np.array(src, np.int32), omode(mode), 25, 40_000, 0, SEED)
        assert np.array_equal(r["selected"], o["selected"]), (perturb, mode)
        assert np.array_equal(r["gains"], o["gains"]), (perturb, mode)


@pytest.mark.parametrize("shape", ["geometric", "one_heavy", "zeros", "ramp"])
def test_skewed_weights_search(sia, shape):
    """Weight shapes far from equal (where the interpolated first guess and
    the interpolation steps of the in-edge search miss, and it must bisect):
    walks and answers equal the oracle's."""
    rng = np.random.default_rng({"geometric": 1, "one_heavy": 2, "zeros": 3, "ramp": 4}[shape])
    n = 4000
    degs = rng.integers(0, 40, n)
    degs[17] = 20_000
    degs[18] = 300
    col = np.zeros(n + 1, np.int64)
    col[1:] = np.cumsum(degs)
    m = int(col[-1])
    row = rng.integers(0, n, m).astype(np.int32)
    w = np.zeros(m, np.float32)
    for v in range(n):
        d = int(degs[v])
        if not d:
            continue
        if shape == "geometric":
            x = 0.7 ** np.arange(d)
        elif shape == "one_heavy":
            x = np.full(d, 1e-4)
            x[rng.integers(d)] = 1.0
        elif shape == "zeros":
            x = rng.uniform(0, 1, d) * (rng.uniform(0, 1, d) < 0.3)
            x[rng.integers(d)] += 0.5
        else:
            x = np.arange(1, d + 1, dtype=np.float64) ** 3
        w[col[v]:col[v + 1]] = (x / x.sum() * rng.uniform(0.6, 1.0)).astype(np.float32)
    g = sia.Graph(col, row, w)
    assert g.arc_bytes == 32
    og = cpu.Graph(col, row, w)
    assert np.array_equal(g.thresholds(), og.thr)
    src = sorted(rng.choice(n, size=8, replace=False).tolist())
    for mode in ("edges", "nodes"):
        got = sia.sample(g, src, mode, 60_000, 0, SEED)
        ref = og.sample(np.array(src, np.int32), omode(mode), 60_000, 0, SEED)
        assert_walks_equal(got, ref, (shape, mode))


def test_quantize_exhaustive_all_fp32_in_unit_interval(sia):
    """Every fp32 value in [0, 1] (bit patterns 0 .. 0x3F800000) converts to
    the same integer on the device as in the oracle."""
    end = 0x3F800001
    chunk = 1 << 26
    for base in range(0, end, chunk):
        cnt = min(chunk, end - base)
        bits = torch.arange(base, base + cnt, dtype=torch.int64, device="cuda").to(torch.int32)
        wdev = bits.view(torch.float32)
        qdev = torch.empty(cnt, dtype=torch.int64, device="cuda")
        sia.quantize(wdev, qdev)
        torch.cuda.synchronize()
        got = qdev.cpu().numpy().view(np.uint64)
        ref = cpu.quantize(wdev.cpu().numpy())
        assert np.array_equal(got, ref), hex(base)


def test_invalid_weights_rejected(sia):
    col = np.array([0, 2, 3, 3], np.int64)
    row = np.array([1, 2, 0], np.int32)
    for w in ([0.7, 0.4, 0.5], [np.nan, 0.1, 0.5], [-0.5, 0.1, 0.5], [0.5, 0.5, 1.5]):
        with pytest.raises(sia.SiaError) as e:
            sia.Graph(col, row, np.array(w, np.float32))
        assert e.value.status == -2
        with pytest.raises(sia.SiaError) as e:
            sia.Graph(torch.from_numpy(col).cuda(), torch.from_numpy(row).cuda(),
                      torch.tensor(w, dtype=torch.float32, device="cuda"))
        assert e.value.status == -2
    with pytest.raises(sia.SiaError) as e:
        sia.Graph(torch.tensor([0, 2, 1, 3], device="cuda"),
                  torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda"),
                  torch.tensor([0.1, 0.1, 0.1], device="cuda"))
    assert e.value.status == -1
    with pytest.raises(sia.SiaError) as e:
        sia.Graph(torch.tensor([0, 2, 3, 3], device="cuda"),
                  torch.tensor([1, 5, 0], dtype=torch.int32, device="cuda"),
                  torch.tensor([0.1, 0.1, 0.1], device="cuda"))
    assert e.value.status == -1


# ------------------------------------------------------------------ sampler
@pytest.mark.parametrize("case", CAT, ids=[c[0] for c in CAT])
@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_sample_matches_oracle_tiny(sia, case, mode):
    name, n, edges, src = case
    col, row, w = csc_from_edges(n, edges)
    g = sia.Graph(col, row, w)
    og = cpu.Graph(col, row, w)
    for offset, N in ((0, 20_000), (987_654_321_000, 3_333)):
        got = sia.sample(g, src, mode, N, offset, SEED)
        ref = og.sample(np.array(src, np.int32), omode(mode), N, offset, SEED)
        assert_walks_equal(got, ref, (name, mode, offset))


@pytest.mark.parametrize("mode", ["edges", "nodes"])
@pytest.mark.parametrize("weights", ["inv", "rand"])
def test_long_walks_match_oracle(sia, mode, weights):
    """Walks far longer than the sampler's walk ring (1024 positions) take
    the ring-free paths (two-pointer cycle entry, re-walk emission), shorter
    ones the ring: a chain of 3000 nodes into a source, a 2500-node cycle fed
    by a 1500-node tail, and shortcuts that make lengths of every size."""
    rng = np.random.default_rng(77 if weights == "inv" else 78)
    L, C, T = 3000, 2500, 1500
    n = L + 1 + C + T
    edges = []
    # chain: node i's live in-edge comes from i + 1; node L is the source
    for i in range(L):
        edges.append((i + 1, i, 1.0))
    base = L + 1  # cycle base .. base + C - 1, tail base + C .. n - 1 feeding the cycle
    for i in range(C):
        edges.append((base + (i + 1) % C, base + i, 1.0))
    for i in range(T - 1):
        edges.append((base + C + i + 1, base + C + i, 1.0))
    edges.append((base, base + C + T - 1, 1.0))  # the tail's last node is fed by the cycle
    if weights == "rand":
        # a few extra in-edges with split weights: walks branch between the parts
        extra = rng.choice(n, 200, replace=False)
        rebuilt = []
        touched = set(int(v) for v in extra)
        for (u, v, w) in edges:
            rebuilt.append((u, v, 0.7 if v in touched else w))
        for v in extra:
            u = int(rng.integers(0, n))
            if u != v:
                rebuilt.append((u, int(v), 0.25))
        edges = rebuilt
    col, row, w = csc_from_edges(n, edges)
    g = sia.Graph(col, row, w)
    og = cpu.Graph(col, row, w)
    src = [L]
    got = sia.sample(g, src, mode, 20_000, 0, SEED)
    ref = og.sample(np.array(src, np.int32), omode(mode), 20_000, 0, SEED)
    assert_walks_equal(got, ref, (mode, weights))
    assert ref.cycles > 0 and ref.hits > 0 and int(np.diff(ref.off.astype(np.int64)).max()) > 1024
    g.close()


@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_sample_matches_oracle_random_graphs(sia, mode):
    for seed in range(20):
        n = 30 + seed * 7
        edges = random_tiny(n, 3.0 / n, 500 + seed, "inv" if seed % 2 else "rand", max_deg=6)
        rng = np.random.default_rng(seed)
        src = sorted(rng.choice(n, size=1 + seed % 4, replace=False).tolist())
        col, row, w = csc_from_edges(n, edges)
        g = sia.Graph(col, row, w)
        og = cpu.Graph(col, row, w)
        N = 5000 + 37 * seed
        got = sia.sample(g, src, mode, N, seed * 1000, SEED + seed)
        ref = og.sample(np.array(src, np.int32), omode(mode), N, seed * 1000, SEED + seed)
        assert_walks_equal(got, ref, (seed, mode))


def test_sample_er1k_full(sia):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    col, row, w = wl.host()
    g = sia.Graph(wl.col_off.cuda(), wl.row_idx.cuda(), wl.w.cuda())
    og = cpu.Graph(col, row, w)
    for mode in ("edges", "nodes"):
        got = sia.sample(g, wl.sources, mode, wl.n_attempts, 0, wl.seed)
        ref = og.sample(wl.sources, omode(mode), wl.n_attempts, 0, wl.seed)
        assert_walks_equal(got, ref, mode)


def test_sample_split_equals_whole(sia):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    g = sia.Graph(*wl.host())
    whole = sia.sample(g, wl.sources, "edges", 50_000, 100, 7)
    a = sia.sample(g, wl.sources, "edges", 20_001, 100, 7)
    b = sia.sample(g, wl.sources, "edges", 29_999, 20_101, 7)
    assert np.array_equal(whole.attempt, np.concatenate([a.attempt, b.attempt]))
    assert np.array_equal(whole.ids, np.concatenate([a.ids, b.ids]))
    for key in ("hits", "dead_ends", "cycles", "steps"):
        assert whole.stats[key] == a.stats[key] + b.stats[key]


# ------------------------------------------------------------------ greedy
@pytest.mark.parametrize("seed", range(6))
def test_greedy_matches_oracle(sia, seed):
    rng = np.random.default_rng(seed)
    id_space = [7, 1000, 1025, 70_000, 1_048_577, 3_000_000][seed]
    n_walks = [50, 3000, 4000, 20_000, 50_000, 100_000][seed]
    hot = rng.integers(0, id_space, 64)
    walks = []
    for i in range(n_walks):
        L = min(int(rng.integers(1, 12)), id_space)
        pool = np.unique(np.concatenate([hot[: L // 2], rng.integers(0, id_space, L)]))
        if pool.shape[0] < L:
            pool = rng.choice(id_space, L, replace=False)
        u = rng.permutation(pool)[:L]
        walks.append(u.astype(np.uint32))
    off = np.zeros(n_walks + 1, np.uint64)
    off[1:] = np.cumsum([w.shape[0] for w in walks])
    ids = np.concatenate(walks)
    k = min(id_space, [7, 50, 200, 300, 100, 1000][seed])
    got_sel, got_gain = sia.greedy(id_space, off, ids, k)
    ref_sel, ref_gain = cpu.greedy_csr(id_space, off, ids, k)
    assert np.array_equal(got_sel, ref_sel)
    assert np.array_equal(got_gain, ref_gain)


def test_greedy_recount_when_picks_cover_most_walks(sia):
    """Five hub ids, one of them in 95% of the walks (as the sources are in
    node removal): the rounds that pick them cover far more walks than stay
    uncovered, so the counts are recomputed from the uncovered walks instead
    of decremented; the later rounds then run on the recomputed counts."""
    rng = np.random.default_rng(21)
    id_space, n_walks = 50_000, 40_000
    hubs = rng.choice(id_space, 5, replace=False)
    walks = []
    for i in range(n_walks):
        body = rng.choice(id_space, int(rng.integers(3, 20)), replace=False)
        if rng.random() < 0.95:
            body = np.unique(np.concatenate([body, hubs[rng.integers(0, 5, 1)]]))
        walks.append(rng.permutation(body).astype(np.uint32))
    off = np.zeros(n_walks + 1, np.uint64)
    off[1:] = np.cumsum([w.shape[0] for w in walks])
    ids = np.concatenate(walks)
    got = sia.greedy(id_space, off, ids, 200)
    ref = cpu.greedy_csr(id_space, off, ids, 200)
    assert set(got[0][:5].tolist()) == set(hubs.tolist())
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_greedy_large_id_space(sia):
    """id space above 64^3 (more than 64 top-level entries) with a ragged tail."""
    rng = np.random.default_rng(9)
    id_space = 20_000_003
    n_walks = 30_000
    walks = [np.unique(rng.integers(id_space - 300_000, id_space, rng.integers(1, 9))).astype(np.uint32)
             for _ in range(n_walks)]
    off = np.zeros(n_walks + 1, np.uint64)
    off[1:] = np.cumsum([w.shape[0] for w in walks])
    ids = np.concatenate(walks)
    got = sia.greedy(id_space, off, ids, 300)
    ref = cpu.greedy_csr(id_space, off, ids, 300)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("case", ["ties", "all", "hot"])
def test_greedy_ties_and_many_rounds(sia, case):
    """Many rounds with large tie groups (the pool is rebuilt many times and
    ties are broken by ascending id), every id selected, and a few very hot ids."""
    rng = np.random.default_rng({"ties": 1, "all": 2, "hot": 3}[case])
    if case == "ties":
        id_space, n_walks, k = 40_000, 25_000, 12_000
        walks = [rng.choice(id_space, rng.integers(1, 3), replace=False) for _ in range(n_walks)]
    elif case == "all":
        id_space, n_walks, k = 5_000, 8_000, 5_000
        walks = [rng.choice(id_space, rng.integers(1, 6), replace=False) for _ in range(n_walks)]
    else:
        id_space, n_walks, k = 2_000_000, 10_000, 2000
        hot = rng.choice(id_space, 10, replace=False)
        walks = [np.unique(np.concatenate([hot[rng.integers(0, 10, 2)],
                                           rng.integers(0, id_space, rng.integers(1, 30))]))
                 for _ in range(n_walks)]
    walks = [np.asarray(w, np.uint32) for w in walks]
    off = np.zeros(n_walks + 1, np.uint64)
    off[1:] = np.cumsum([w.shape[0] for w in walks])
    ids = np.concatenate(walks)
    got = sia.greedy(id_space, off, ids, k)
    ref = cpu.greedy_csr(id_space, off, ids, k)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("case", ["many_pools", "collected_then_zero", "nodes_like"])
def test_greedy_zero_gain_tails(sia, case):
    """k far above the number of ids any walk holds: after the last positive
    gain the remaining picks are the lowest unselected ids, taken across
    several pool rebuilds; and a pool whose collected ids fall to zero gain
    mid-pool before the ordered pool of zeros takes over."""
    rng = np.random.default_rng({"many_pools": 4, "collected_then_zero": 5, "nodes_like": 6}[case])
    if case == "many_pools":
        id_space, n_walks, k = 50_000, 300, 20_000
        walks = [rng.choice(id_space, rng.integers(1, 4), replace=False) for _ in range(n_walks)]
    elif case == "collected_then_zero":
        id_space, n_walks, k = 3_000, 600, 3_000
        walks = [rng.choice(id_space, rng.integers(1, 4), replace=False) for _ in range(n_walks)]
    else:
        id_space, n_walks, k = 9_000, 40, 8_999
        walks = [rng.choice(id_space, rng.integers(1, 30), replace=False) for _ in range(n_walks)]
    walks = [np.asarray(w, np.uint32) for w in walks]
    off = np.zeros(n_walks + 1, np.uint64)
    off[1:] = np.cumsum([w.shape[0] for w in walks])
    ids = np.concatenate(walks)
    got = sia.greedy(id_space, off, ids, k)
    ref = cpu.greedy_csr(id_space, off, ids, k)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("layout", ["low_ids", "high_ids", "spread"])
def test_greedy_zero_ties_in_a_large_id_space(sia, layout):
    """Few walks in a 2^22 id space and k well past the ids they hold: the
    zero-count ties are counted only up to the bound where the ids they take
    must end (the lowest unselected ids of count 0), with the walks' ids at the
    bottom of the id space, at its top, or spread over it."""
    rng = np.random.default_rng({"low_ids": 31, "high_ids": 32, "spread": 33}[layout])
    S, n_walks, k = 1 << 22, 500, 6000
    lo, hi = {"low_ids": (0, 3000), "high_ids": (S - 3000, S), "spread": (0, S)}[layout]
    walks = [(lo + rng.choice(hi - lo, int(rng.integers(1, 6)), replace=False)).astype(np.uint32)
             for _ in range(n_walks)]
    off = np.zeros(n_walks + 1, np.uint64)
    off[1:] = np.cumsum([w.shape[0] for w in walks])
    ids = np.concatenate(walks)
    got = sia.greedy(S, off, ids, k)
    ref = cpu.greedy_csr(S, off, ids, k)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_greedy_empty_and_exhaustive(sia):
    sel, gains = sia.greedy(5, np.zeros(1, np.uint64), np.zeros(0, np.uint32), 5)
    assert sel.tolist() == [0, 1, 2, 3, 4] and gains.tolist() == [0] * 5
    off = np.array([0, 2, 3], np.uint64)
    ids = np.array([1, 2, 3], np.uint32)
    sel, gains = sia.greedy(6, off, ids, 6)
    assert sel.tolist() == [1, 3, 0, 2, 4, 5] and gains.tolist() == [1, 1, 0, 0, 0, 0]


@pytest.mark.parametrize("case", ["few_bins", "wide", "many_tiles"])
def test_greedy_counts_exact(sia, case):
    """Walks of one id each: covering an id then lowers no other id's count,
    so the greedy takes ids by count (ties by ascending id, then the lowest
    ids of count 0) and each gain is the id's count -- the counting pass is
    checked id by id.  few_bins: 300 ids, 3*10^6 walks (each range of ids is
    counted by several workgroups); wide: an id space above 2^30 (512 fine
    ranges per coarse range), both ends of it used; many_tiles: 2*10^7 walks
    over 2^24 + 3 ids (the most tiles)."""
    rng = np.random.default_rng({"few_bins": 11, "wide": 12, "many_tiles": 13}[case])
    if case == "few_bins":
        S, k = 300, 300
        ids = np.minimum(rng.zipf(1.3, 3_000_000) - 1, S - 1)
    elif case == "wide":
        S, k = (1 << 30) + 5, 3000
        hot = rng.integers(0, S, 2000)
        ids = np.concatenate([rng.integers(0, S, 1_000_000), hot[rng.integers(0, 2000, 1_000_000)],
                              [0, 0, S - 1, S - 1, S - 1]])
    else:
        S, k = (1 << 24) + 3, 5000
        ids = np.concatenate([rng.integers(0, S, 19_000_000), rng.integers(S - 70_000, S, 1_000_000)])
    ids = rng.permutation(ids).astype(np.uint32)
    off = np.arange(ids.shape[0] + 1, dtype=np.uint64)
    sel, gains = sia.greedy(S, off, ids, k)
    u, c = np.unique(ids, return_counts=True)
    order = np.lexsort((u, -c))
    exp_sel, exp_gain = u[order][:k].astype(np.int64), c[order][:k].astype(np.uint64)
    if exp_sel.shape[0] < k:
        rest = k - exp_sel.shape[0]
        zeros = np.setdiff1d(np.arange(min(S, u.shape[0] + rest)), u)[:rest]
        exp_sel = np.concatenate([exp_sel, zeros])
        exp_gain = np.concatenate([exp_gain, np.zeros(rest, np.uint64)])
    assert np.array_equal(sel, exp_sel)
    assert np.array_equal(gains, exp_gain)


@pytest.mark.parametrize("case", ["width8", "width16"])
def test_greedy_overfull_high_count_bin(sia, case):
    """Algorithm 4 / 7 return k picks for any input.  9000 ids whose counts
    all fall in one wide bin of the count histogram (above the exact counts:
    4096..4103, a bin of 8 counts; or 8192..8207, a bin of 16), more ids than
    the lazy pool holds, with 1000 (500) ids in the bin above: the pool is
    planned from a second histogram of that bin's own counts.  Single-id
    walks, so the picks are the ids by count (ties by ascending id) and each
    gain is the id's count; k runs past the hot ids into a tail of low
    counts."""
    rng = np.random.default_rng({"width8": 41, "width16": 42}[case])
    lo, width, n_hot, n_above = (4096, 8, 9000, 1000) if case == "width8" else (8192, 16, 9000, 500)
    S = 50_000
    hot = rng.choice(S, n_hot + n_above, replace=False)
    cnt = np.concatenate([rng.integers(lo, lo + width, n_hot), rng.integers(lo + width, lo + 2 * width, n_above)])
    cold = rng.integers(0, S, 200_000)
    ids = rng.permutation(np.concatenate([np.repeat(hot, cnt), cold])).astype(np.uint32)
    off = np.arange(ids.shape[0] + 1, dtype=np.uint64)
    k = n_hot + n_above + 500
    print("[parity] overfull bin", case, ids.shape[0], "walks", flush=True)
    sel, gains = sia.greedy(S, off, ids, k)
    u, c = np.unique(ids, return_counts=True)
    order = np.lexsort((u, -c))
    assert np.array_equal(sel, u[order][:k].astype(np.int64))
    assert np.array_equal(gains, c[order][:k].astype(np.uint64))


def test_greedy_overfull_high_count_bin_multi_id_walks(sia):
    """The same shape with walks of four distinct ids (covering a walk lowers
    the counts of its other ids), against the oracle's greedy.  4100 rounds,
    each a random permutation of 9000 ids cut into walks of four, give every
    id the count 4100; 3000 more random walks lift some by a few, so more
    than 8192 ids have counts in 4100..4103 (one wide bin) and a few hundred
    lie in the bin above."""
    rng = np.random.default_rng(43)
    S, n_hot, R = 30_000, 9000, 4100
    hot = rng.choice(S, n_hot, replace=False).astype(np.uint32)
    rounds = rng.permuted(np.tile(np.arange(n_hot, dtype=np.uint32), (R, 1)), axis=1).reshape(-1)
    extra = np.stack([rng.choice(n_hot, 4, replace=False) for _ in range(3000)]).reshape(-1).astype(np.uint32)
    walks = np.concatenate([rounds, extra]).reshape(-1, 4)
    walks = walks[rng.permutation(walks.shape[0])]
    ids = hot[walks.reshape(-1)]
    off = np.arange(0, ids.shape[0] + 1, 4, dtype=np.uint64)
    cnt = np.bincount(ids, minlength=S)[hot]
    assert cnt.min() >= 4100 and cnt.max() < 4112 and (cnt < 4104).sum() > 8192
    k = 150
    print("[parity] overfull bin, multi-id walks", off.shape[0] - 1, flush=True)
    a = sia.greedy(S, off, ids, k)
    b = cpu.greedy_csr(S, off, ids, k)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------------ solve
@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_solve_er1k_matches_oracle(sia, mode):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    col, row, w = wl.host()
    g = sia.Graph(wl.col_off.cuda(), wl.row_idx.cuda(), wl.w.cuda())
    og = cpu.Graph(col, row, w)
    got = sia.solve(g, wl.sources, mode, wl.k, wl.n_attempts, 0, wl.seed, timing=True)
    ref = cpu.solve(og, wl.sources, omode(mode), wl.k, wl.n_attempts, 0, wl.seed)
    assert np.array_equal(got["selected"], ref["selected"])
    assert np.array_equal(got["gains"], ref["gains"])
    st = got["stats"]
    assert st["covered"] == ref["covered"]
    assert st["hits"] == ref["walks"].hits and st["steps"] == ref["walks"].steps
    assert st["spread_est"] == ref["spread"]
    assert st["suspension_est"] == ref["suspension"]
    assert st["suspension_nodes_est"] == ref["suspension_nodes"]
    assert st["ms_sample"] > 0 and st["ms_total"] >= st["ms_sample"]


def test_solve_edge_cases(sia):
    # every non-source but one is a source; k = id space; N = 1
    col, row, w = csc_from_edges(4, [(1, 0, 0.3), (2, 0, 0.3), (3, 0, 0.4)])
    g = sia.Graph(col, row, w)
    og = cpu.Graph(col, row, w)
    for mode, k in (("edges", 3), ("nodes", 4)):
        for N in (1, 2, 1000):
            got = sia.solve(g, [1, 2, 3], mode, k, N, 5, 11)
            ref = cpu.solve(og, [1, 2, 3], omode(mode), k, N, 5, 11)
            assert np.array_equal(got["selected"], ref["selected"]), (mode, N)
            assert np.array_equal(got["gains"], ref["gains"]), (mode, N)
    # all weights zero: every attempt is a dead end after one draw
    col, row, w = csc_from_edges(5, [(1, 0, 0.0), (2, 1, 0.0), (0, 2, 0.0)])
    g = sia.Graph(col, row, w)
    got = sia.solve(g, [4], "edges", 3, 10_000, 0, 3)
    assert got["stats"]["dead_ends"] == 10_000 == got["stats"]["steps"]
    assert got["selected"].tolist() == [0, 1, 2] and got["gains"].tolist() == [0, 0, 0]
    # graph without edges
    g = sia.Graph(np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    got = sia.solve(g, [0], "nodes", 2, 1000, 0, 3)
    assert got["stats"]["dead_ends"] == 1000 and got["selected"].tolist() == [0, 1]


# ---------------------------------------- cyclic walks stopped at detection
SAME_WITHOUT_CYCLE_STEPS = ("attempts", "hits", "dead_ends", "cycles", "walk_ids", "covered", "spread_est",
                            "suspension_est", "suspension_nodes_est")


@pytest.mark.parametrize("weights", ["inv_indeg", "normalized"])
def test_no_cycle_steps_changes_only_the_step_count(sia, weights):
    """SIA_FLAG_NO_CYCLE_STEPS stops a walk that closes a cycle when the cycle
    is detected (Algorithm 1 discards it either way).  Picks, gains and every
    counter but steps and evaluations equal the exact run's and the oracle's;
    the step count loses the cyclic walks' draws, at least one each, and
    keeps the kept walks' draws and at least one per dead end."""
    from paper_1702_05854_amd import workloads
    wl = workloads.load("rmat22", scale=16, weights=weights)
    col, row, w = wl.host()
    g = sia.Graph(col, row, w)
    og = cpu.Graph(col, row, w)
    for mode in ("edges", "nodes"):
        exact = sia.solve(g, wl.sources, mode, 50, 300_000, 77, SEED)
        fast = sia.solve(g, wl.sources, mode, 50, 300_000, 77, SEED, cycle_steps=False)
        ref = cpu.solve(og, wl.sources, omode(mode), 50, 300_000, 77, SEED)
        assert np.array_equal(fast["selected"], ref["selected"]) and np.array_equal(fast["gains"], ref["gains"])
        assert np.array_equal(exact["selected"], ref["selected"])
        e, f = exact["stats"], fast["stats"]
        for key in SAME_WITHOUT_CYCLE_STEPS:
            assert f[key] == e[key], (mode, key)
        assert e["steps"] == ref["walks"].steps and f["hits"] == ref["walks"].hits
        assert f["cycles"] == ref["walks"].cycles > 0
        kept_draws = f["walk_ids"] if mode == "edges" else f["walk_ids"] - f["hits"]
        assert kept_draws + f["dead_ends"] <= f["steps"] <= e["steps"] - f["cycles"], mode
        # 16-byte records search the entry by walking the graph again; 32-byte
        # records bisect their walk ring, which takes no evaluation (walks
        # longer than the ring excepted)
        if g.arc_bytes == 16:
            assert f["evaluations"] < e["evaluations"], mode
        else:
            assert f["evaluations"] <= e["evaluations"], mode
    g.close()


def test_no_cycle_steps_on_a_pure_cycle(sia):
    """Two nodes feeding each other with weight 1 and an isolated source:
    every attempt walks 0 -> 1 -> 0 (or 1 -> 0 -> 1), a cycle after two
    draws.  Exact: 2 steps per attempt; stopped at detection: none.  The
    same on 40-node rings, whose walks visit more nodes than the stack
    detector holds."""
    col, row, w = csc_from_edges(3, [(0, 1, 1.0), (1, 0, 1.0)])
    g = sia.Graph(col, row, w)
    for mode in ("edges", "nodes"):
        exact = sia.solve(g, [2], mode, 1, 5000, 0, SEED)["stats"]
        fast = sia.solve(g, [2], mode, 1, 5000, 0, SEED, cycle_steps=False)["stats"]
        assert exact["cycles"] == fast["cycles"] == 5000 and exact["hits"] == fast["hits"] == 0
        assert exact["steps"] == 10_000 and fast["steps"] == 0
    g.close()
    # 40-node rings walked with increasing ids (the stack overflows and drops
    # the cycle's smallest node, so Brent must end the walks) and with
    # decreasing ids (the stack ends them); node 40 is an isolated source
    for edges in ([((i + 1) % 40, i, 1.0) for i in range(40)], [(i, (i + 1) % 40, 1.0) for i in range(40)]):
        col, row, w = csc_from_edges(41, edges)
        g = sia.Graph(col, row, w)
        for mode in ("edges", "nodes"):
            exact = sia.solve(g, [40], mode, 1, 5000, 0, SEED)["stats"]
            fast = sia.solve(g, [40], mode, 1, 5000, 0, SEED, cycle_steps=False)["stats"]
            assert exact["cycles"] == fast["cycles"] == 5000 and exact["steps"] == 40 * 5000
            assert fast["steps"] == 0 and fast["hits"] == 0
        g.close()
    col, row, w = csc_from_edges(3, [(0, 1, 1.0), (1, 0, 1.0)])
    g = sia.Graph(col, row, w)
    # flag bits the library does not know are refused
    sel, gains, src = np.zeros(1, np.int64), np.zeros(1, np.uint64), np.array([2], np.int32)
    assert sia.lib().sia_solve(g.handle, 0, src.ctypes.data, 1, 1, 100, 0, SEED, sel.ctypes.data,
                               gains.ctypes.data, None, 4, None) == -1
    g.close()


@pytest.mark.parametrize("layout", ["dense", "runs", "ends"])
def test_start_ranks_with_dense_sources(sia, layout):
    """The start of an attempt is the idx-th non-source; its rank among the
    sources is read a bucket block and then 4-entry windows at a time.  Source
    sets with long runs of consecutive ids, almost every node a source, and
    sources at both ends of the id range: walks and answers equal the oracle's."""
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    col, row, w = wl.host()
    n = wl.n
    rng = np.random.default_rng(9)
    if layout == "dense":  # all but 7 nodes
        keep = set(rng.choice(n, size=7, replace=False).tolist())
        src = [v for v in range(n) if v not in keep]
    elif layout == "runs":  # a few long runs of consecutive ids
        src = list(range(0, 90)) + list(range(300, 555)) + list(range(700, 703)) + list(range(960, 1000))
    else:  # the ends of the id range and a few more
        src = [0, 1, 2, n - 3, n - 2, n - 1, 500]
    g = sia.Graph(col, row, w)
    og = cpu.Graph(col, row, w)
    s = np.array(sorted(src), np.int32)
    for mode in ("edges", "nodes"):
        got = sia.sample(g, s, mode, 30_000, 777, SEED)
        ref = og.sample(s, omode(mode), 30_000, 777, SEED)
        assert_walks_equal(got, ref, (layout, mode))
        r = sia.solve(g, s, mode, 10, 30_000, 777, SEED)
        o = cpu.solve(og, s, omode(mode), 10, 30_000, 777, SEED)
        assert np.array_equal(r["selected"], o["selected"]), (layout, mode)
        assert np.array_equal(r["gains"], o["gains"]), (layout, mode)


def test_golden_three_node_law(sia):
    """The hand-derived law of tests/golden/three_node_cycle.json: the HIP
    sampler equals the oracle walk for walk, and its outcome rates match the
    law within sampling error."""
    import json
    import os
    from fractions import Fraction
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "three_node_cycle.json")) as f:
        fx = json.load(f)
    edges = [(int(u), int(v), float(w)) for u, v, w in fx["graph"]["edges_u_v_w"]]
    col, row, w = csc_from_edges(fx["graph"]["n"], edges)
    g = sia.Graph(col, row, w)
    og = cpu.Graph(col, row, w)
    src = np.array(fx["sources"], np.int32)
    N = 1_000_000
    for mode in ("edges", "nodes"):
        got = sia.sample(g, src, mode, N, 0, SEED)
        ref = og.sample(src, omode(mode), N, 0, SEED)
        assert_walks_equal(got, ref, mode)
        for k, c in (("hit", "hits"), ("dead_end", "dead_ends"), ("cycle", "cycles")):
            p = float(Fraction(fx["quantized"][k]))
            assert abs(got.stats[c] - N * p) < 5 * np.sqrt(N * p * (1 - p)) + 1, (mode, k)


def test_probe_gather_measures(sia):
    ind, ms_i = sia.probe_gather(64 << 20, 64, dependent=False)
    dep, ms_d = sia.probe_gather(64 << 20, 64, dependent=True)
    assert ind > 0 and dep > 0 and ms_i > 0 and ms_d > 0


def test_failed_call_leaves_graph_clean(sia):
    """A call that fails part-way (an injected device-allocation failure at
    each allocation site in turn, including those after the query's sources
    are tagged in the graph) leaves the graph as it was: the next solve on it
    equals the oracle's."""
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    col, row, w = wl.host()
    og = cpu.Graph(col, row, w)
    ref = cpu.solve(og, wl.sources, cpu.MODE_EDGES, wl.k, 50_000, 0, wl.seed)
    failures = 0
    for nth in range(1, 16):
        g = sia.Graph(col, row, w)
        sia.inject_alloc_failure(nth)
        try:
            sia.solve(g, wl.sources, "edges", wl.k, 50_000, 0, wl.seed)
        except sia.SiaError as e:
            assert e.status == -3, (nth, e)  # SIA_ENOMEM
            failures += 1
        finally:
            sia.inject_alloc_failure(0)
        got = sia.solve(g, wl.sources, "edges", wl.k, 50_000, 0, wl.seed)
        assert np.array_equal(got["selected"], ref["selected"]), nth
        assert np.array_equal(got["gains"], ref["gains"]), nth
        assert got["stats"]["hits"] == ref["walks"].hits, nth
        g.close()
    assert failures >= 5
