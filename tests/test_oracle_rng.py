"""Pins of the oracle's random stream and start-node mapping.

The oracle's Philox4x64-10 is checked against numpy's independent Philox
(``numpy.random.Philox`` is Philox4x64-10; it increments its 256-bit counter
before each block, so block c is produced from state counter c - 1).
"""
import numpy as np
import pytest

from oracle import cpu

M64 = (1 << 64) - 1


def numpy_block(ctr, key):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64))
    st = bg.state
    c = (sum(int(x) << (64 * i) for i, x in enumerate(ctr)) - 1) % (1 << 256)
    st["state"]["counter"] = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    st["buffer_pos"] = 4
    bg.state = st
    return [int(x) for x in bg.random_raw(4)]


CASES = [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((5, 0, 0, 0), (2017, 123)),
    ((0, 1, 0, 0), (1, 2)),
    ((M64, 7, 9, 11), (M64, 3)),
    ((123456789, M64, 0, M64), (0xDEADBEEF, 0xFEEDFACE12345678)),
]


@pytest.mark.parametrize("ctr,key", CASES)
def test_philox_matches_numpy(ctr, key):
    assert [int(x) for x in cpu.philox4x64_10(ctr, key)] == numpy_block(ctr, key)


def test_philox_random_blocks_match_numpy():
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = tuple(int(x) for x in rng.integers(0, 2**64, 4, dtype=np.uint64))
        key = tuple(int(x) for x in rng.integers(0, 2**64, 2, dtype=np.uint64))
        assert [int(x) for x in cpu.philox4x64_10(ctr, key)] == numpy_block(ctr, key)


def test_node_and_start_draws_are_the_documented_words():
    rng = np.random.default_rng(11)
    for _ in range(100):
        seed = int(rng.integers(0, 2**63))
        a = int(rng.integers(0, 2**40))
        x = int(rng.integers(0, 2**31))
        assert cpu.draw_node(seed, a, x) == numpy_block((x, 0, 0, 0), (seed, a))[0] >> 32
        assert cpu.draw_start_word(seed, a) == numpy_block((0, 1, 0, 0), (seed, a))[0]


def test_scale_u64_is_floor_of_product():
    rng = np.random.default_rng(3)
    vals = [0, 1, M64, M64 - 1, 1 << 63]
    counts = [1, 2, 3, 999, (1 << 31) - 1, (1 << 32) + 5, M64]
    for x in vals + [int(v) for v in rng.integers(0, 2**63, 50)]:
        for c in counts + [int(v) for v in rng.integers(1, 2**40, 5)]:
            assert cpu.scale_u64(x, c) == (x * c) >> 64


def test_start_node_is_indexed_non_source():
    """Every kept walk of a graph where each non-source has one weight-1
    in-edge from a source starts at nonsource[floor(x0 * |V\\X| / 2^64)]."""
    n = 50
    sources = np.array([3, 17, 18, 40], dtype=np.int32)
    src_set = set(sources.tolist())
    nonsrc = [v for v in range(n) if v not in src_set]
    col_off = [0]
    row_idx = []
    for v in range(n):
        if v not in src_set:
            row_idx.append(int(sources[v % len(sources)]))
        col_off.append(len(row_idx))
    w = np.ones(len(row_idx), dtype=np.float32)
    g = cpu.Graph(np.array(col_off), np.array(row_idx), w)
    seed = 99
    walks = g.sample(sources, cpu.MODE_NODES, 5000, offset=10, seed=seed)
    assert walks.hits == 5000  # dead-end chance is 2^-32 per attempt
    for i in range(walks.n_walks):
        a = int(walks.attempt[i])
        x0 = numpy_block((0, 1, 0, 0), (seed, a))[0]
        assert int(walks.walk(i)[0]) == nonsrc[(x0 * len(nonsrc)) >> 64]


def test_start_node_uniform_chi2():
    from scipy.stats import chi2
    n = 40
    sources = np.array([0, 9], dtype=np.int32)
    col_off = [0]
    row_idx = []
    for v in range(n):
        if v not in (0, 9):
            row_idx.append(0)
        col_off.append(len(row_idx))
    g = cpu.Graph(np.array(col_off), np.array(row_idx), np.ones(len(row_idx), np.float32))
    N = 200_000
    walks = g.sample(sources, cpu.MODE_NODES, N, seed=5)
    starts = walks.ids[walks.off[:-1].astype(np.int64)]
    obs = np.bincount(starts, minlength=n)[[v for v in range(n) if v not in (0, 9)]]
    exp = N / (n - 2)
    stat = ((obs - exp) ** 2 / exp).sum()
    assert stat < chi2.ppf(1 - 1e-9, n - 3)
