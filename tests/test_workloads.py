"""The input generators are device-independent: the integer hash they draw
from matches the published SplitMix64 finaliser, and every generator gives
the same graph on the CPU and on the GPU (bit for bit), so a digest the
oracle computes on a CPU-generated graph holds for the graph the GPU tests
generate on the device."""
import random

import numpy as np
import pytest
import torch

from paper_1702_05854_amd import workloads as W

M64 = (1 << 64) - 1


def splitmix64_finaliser(z):
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_mix64_is_the_splitmix64_finaliser_with_wrapping_int64():
    rng = random.Random(7)
    xs = [rng.getrandbits(64) for _ in range(20000)] + [0, 1, M64, 1 << 63, (1 << 63) - 1]
    t = torch.tensor([W._i64(x) for x in xs], dtype=torch.int64)
    got = W.mix64(t).tolist()
    assert all((g & M64) == splitmix64_finaliser(x) for g, x in zip(got, xs))
    # SplitMix64's first outputs from state 0 (state += gamma, then finalise)
    s = 0
    first = []
    for _ in range(3):
        s = (s + 0x9E3779B97F4A7C15) & M64
        first.append(splitmix64_finaliser(s))
    assert first[0] == 0xE220A8397B1DCDAF


def test_permutation_and_draws_are_valid():
    p = W.random_permutation(1000, 3, 1, "cpu")
    assert torch.equal(torch.sort(p).values, torch.arange(1000))
    h = W.hash64(5, 0, torch.arange(1 << 16, dtype=torch.int64))
    hi = W._shr(h, 32)
    assert int(hi.min()) >= 0 and int(hi.max()) < (1 << 32)
    x = W._below(hi, 10)
    counts = torch.bincount(x, minlength=10).numpy()
    assert counts.sum() == 1 << 16 and np.all(np.abs(counts - 6553.6) < 6 * np.sqrt(6553.6))


@pytest.mark.parametrize("name,kw", [("er1k", {}), ("rmat22", dict(scale=12)),
                                     ("rmat22", dict(scale=12, weights="normalized"))])
def test_generators_are_deterministic(name, kw):
    a = W.load(name, **kw)
    b = W.load(name, **kw)
    for x, y in zip(a.host(), b.host()):
        assert np.array_equal(x, y)
    col_off, row_idx, w = a.host()
    assert col_off[0] == 0 and col_off[-1] == row_idx.shape[0] and np.all(np.diff(col_off) >= 0)
    assert np.all((w > 0) & (w <= 1))


@pytest.mark.gpu
@pytest.mark.parametrize("name,kw", [
    ("er1k", dict(n=20_000, m=160_000)),
    ("cl1m", dict(n=50_000, m=400_000)),
    ("rmat22", dict(scale=16)),
    ("rmat26", dict(scale=16, ef=24)),
])
def test_cpu_and_gpu_generate_the_same_graph(name, kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[workloads]", name, kw, flush=True)
    a = W.load(name, device="cpu", **kw)
    b = W.load(name, device="cuda", **kw)
    for x, y, what in zip(a.host(), b.host(), ("col_off", "row_idx", "w")):
        assert x.dtype == y.dtype and np.array_equal(x, y), (name, what)
    assert np.array_equal(a.sources, b.sources)
