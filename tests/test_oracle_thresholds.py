"""Pins of the oracle's weight quantisation, threshold tables, validation and
live-edge selection (LT model, Section 2.1; live-edge equivalence)."""
import numpy as np
import pytest

from oracle import cpu, exact
from tiny import catalogue, csc_from_edges

TWO32 = 1 << 32


def rne_from_bits(bits):
    """round-half-even(value * 2^32) for fp32 bit patterns of non-negative
    finite floats, derived from the IEEE-754 fields with integer arithmetic
    only (independent of the oracle's double-precision route)."""
    bits = np.asarray(bits, dtype=np.uint64)
    e = (bits >> np.uint64(23)) & np.uint64(0xFF)
    f = bits & np.uint64(0x7FFFFF)
    normal = e > 0
    M = np.where(normal, f | np.uint64(1 << 23), f)
    # value = M * 2^(E) with E = e - 150 (normal) or -149 (subnormal);
    # value * 2^32 = M * 2^(E + 32)
    sh = np.where(normal, e.astype(np.int64) - 118, np.int64(-117))
    out = np.zeros(bits.shape, dtype=np.uint64)
    left = sh >= 0
    out[left] = M[left] << sh[left].astype(np.uint64)
    r = (~left) & (sh > -64)
    s = (-sh[r]).astype(np.uint64)
    Mr = M[r]
    fl = Mr >> s
    rem = Mr & ((np.uint64(1) << s) - np.uint64(1))
    half = np.uint64(1) << (s - np.uint64(1))
    up = (rem > half) | ((rem == half) & ((fl & np.uint64(1)) == np.uint64(1)))
    out[r] = fl + up.astype(np.uint64)
    return out


def test_hand_cases():
    q = cpu.quantize(np.array([0.5, 1.0, 0.0, 0.25, 2.0**-32, 2.0**-33, 3 * 2.0**-33], np.float32))
    assert q.tolist() == [1 << 31, 1 << 32, 0, 1 << 30, 1, 0, 2]
    rc, thr = cpu.thresholds(np.array([0, 1]), np.array([1.0], np.float32))
    assert rc == 0 and thr.tolist() == [TWO32 - 1]           # w = 1 clamps
    rc, thr = cpu.thresholds(np.array([0, 3]), np.array([0.5, 0.0, 0.25], np.float32))
    assert rc == 0 and thr.tolist() == [1 << 31, 1 << 31, 3 << 30]  # zero weight: equal thresholds
    third = np.float32(1.0) / np.float32(3.0)
    rc, thr = cpu.thresholds(np.array([0, 3]), np.array([third] * 3, np.float32))
    qt = exact.quantize_exact(third)
    assert 3 * qt > TWO32 and rc == 0
    assert thr.tolist() == [qt, 2 * qt, TWO32 - 1]


def test_quantize_exhaustive_exponent_slices():
    """All fp32 values in selected binades (incl. subnormals, the rounding
    boundary binades and [0.5, 1]) match the integer derivation."""
    for e in [0, 1, 95, 96, 97, 117, 118, 119, 126]:
        bits = (np.uint64(e) << np.uint64(23)) | np.arange(1 << 23, dtype=np.uint64)
        w = bits.astype(np.uint32).view(np.float32)
        assert np.array_equal(cpu.quantize(w), rne_from_bits(bits)), e
    one = np.array([1.0], np.float32)
    assert cpu.quantize(one)[0] == rne_from_bits(one.view(np.uint32).astype(np.uint64))[0]


def test_quantize_random_sample_and_fractions():
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 0x3F800001, 2_000_000, dtype=np.int64).astype(np.uint64)
    w = bits.astype(np.uint32).view(np.float32)
    q = cpu.quantize(w)
    assert np.array_equal(q, rne_from_bits(bits))
    for x in w[:2000]:
        assert exact.quantize_exact(float(x)) == int(cpu.quantize(np.array([x]))[0])


def test_invalid_weights_rejected():
    col = np.array([0, 2])
    for bad in ([np.nan, 0.1], [-0.0001, 0.5], [1.5, 0.0], [0.7, 0.4]):
        rc, _ = cpu.thresholds(col, np.array(bad, np.float32))
        assert rc == -2, bad


@pytest.mark.parametrize("d", [1, 3, 7, 1000, 65537, 1_000_003])
def test_inv_degree_weights_accepted(d):
    w = np.full(d, np.float32(1.0) / np.float32(d), np.float32)
    rc, thr = cpu.thresholds(np.array([0, d]), w)
    assert rc == 0
    assert np.all(np.diff(thr.astype(np.int64)) >= 0)


def test_thresholds_match_fraction_derivation_on_catalogue():
    for name, n, edges, _ in catalogue():
        col, row, w = csc_from_edges(n, edges)
        rc, thr = cpu.thresholds(col, w)
        assert rc == 0
        assert thr.tolist() == exact.quantized_thresholds(col, w), name


def brute_select(thr, r):
    for j, t in enumerate(thr):
        if t > r:
            return j
    return -1


def test_select_edge_boundaries():
    rng = np.random.default_rng(5)
    cols = [
        [1 << 31, 1 << 31, 3 << 30],
        [TWO32 - 1],
        [0, 0, 5, 5, 5, 6, TWO32 - 1],
        [7],
        sorted(rng.integers(0, TWO32, 40).tolist()),
        sorted(rng.integers(0, 1000, 300).tolist()),
    ]
    for thr in cols:
        probes = {0, TWO32 - 1}
        for t in thr:
            probes |= {max(t - 1, 0), t, min(t + 1, TWO32 - 1)}
        probes |= set(int(x) for x in rng.integers(0, TWO32, 200))
        for r in sorted(probes):
            assert cpu.select_edge(thr, r) == brute_select(thr, r), (thr[:5], r)
    assert cpu.select_edge([], 0) == -1
