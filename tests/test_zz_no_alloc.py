"""The allocation-free greedy (sia_greedy_noalloc, scratch in a static device
array) gives exactly sia_greedy's answer, on two calls in a row (the second
smaller, so it reuses the array the first left behind), in both modes; and
it rejects inputs beyond its scratch limit and malformed walks."""
import numpy as np
import pytest

from oracle import cpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sia():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05854_amd import sia as _sia
    _sia.lib()
    return _sia


def walks_of(mode, n_attempts):
    from paper_1702_05854_amd import workloads
    wl = workloads.load("er1k")
    og = cpu.Graph(*wl.host())
    w = og.sample(wl.sources, cpu.MODE_EDGES if mode == "edges" else cpu.MODE_NODES, n_attempts, 0, wl.seed)
    return (og.m if mode == "edges" else og.n), w.off, w.ids


def device(off, ids):
    return (torch.from_numpy(off.astype(np.int64)).cuda(), torch.from_numpy(ids.astype(np.int32)).cuda())


def check_equal(sia, S, off, ids, k):
    want_sel, want_gain = sia.greedy(S, off, ids, k)
    d_off, d_ids = device(off, ids)
    sel, gains = sia.greedy_noalloc(S, d_off, d_ids, k)
    torch.cuda.synchronize()
    assert np.array_equal(sel.cpu().numpy(), want_sel)
    assert np.array_equal(gains.cpu().numpy().astype(np.uint64), want_gain)


@pytest.mark.parametrize("mode", ["edges", "nodes"])
def test_noalloc_equals_greedy_twice(sia, mode):
    S, off, ids = walks_of(mode, 200_000)
    print("[noalloc]", mode, off.shape[0] - 1, "walks", ids.shape[0], "ids", flush=True)
    check_equal(sia, S, off, ids, 300)
    # a second, smaller call right after: fewer walks, a smaller k
    nw = (off.shape[0] - 1) // 7
    off2 = off[: nw + 1].copy()
    check_equal(sia, S, off2, ids[: int(off2[-1])], 40)


def test_noalloc_zero_gain_tail_and_no_walks(sia):
    """k beyond the touched ids (zero-gain rounds take the lowest unselected
    ids), and a call with no walks at all."""
    S, off, ids = walks_of("edges", 3000)
    check_equal(sia, S, off, ids, 2000)
    check_equal(sia, 500, np.zeros(1, np.uint64), np.zeros(0, np.uint32), 7)


def test_noalloc_rejects_oversize_and_malformed(sia):
    d_off, d_ids = device(np.array([0, 2], np.uint64), np.array([1, 3], np.uint32))
    with pytest.raises(sia.SiaError) as e:  # 4 bytes of counts per id of a 2^30 id space exceed 64 MiB
        sia.greedy_noalloc(1 << 30, d_off, d_ids, 5)
    assert e.value.status == -1 and "scratch" in str(e.value)
    with pytest.raises(sia.SiaError) as e:  # id 3 outside [0, 3)
        sia.greedy_noalloc(3, d_off, d_ids, 1)
    assert e.value.status == -1
    d_off2, _ = device(np.array([0, 2, 1], np.uint64), np.zeros(0, np.uint32))
    with pytest.raises(sia.SiaError):
        sia.greedy_noalloc(10, d_off2, d_ids, 1)
    # still usable afterwards
    S, off, ids = walks_of("nodes", 20_000)
    check_equal(sia, S, off, ids, 25)
