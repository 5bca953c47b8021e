"""Pins of the oracle's candidate-set greedy: the definition written out by
brute force on small inputs, and C = every id reducing to the plain greedy."""
import numpy as np
import pytest

from oracle import candidates, cpu


def brute_greedy(walks, k, cand):
    """Algorithm 4 / 7 over C as defined: k rounds, each taking the candidate
    not chosen yet whose uncovered walks are most numerous (lowest id on a
    tie), then covering them."""
    chosen, gains = [], []
    covered = [False] * len(walks)
    for _ in range(k):
        best, best_gain = None, -1
        for e in sorted(cand):
            if e in chosen:
                continue
            g = sum(1 for i, w in enumerate(walks) if not covered[i] and e in w)
            if g > best_gain:
                best, best_gain = e, g
        chosen.append(best)
        gains.append(best_gain)
        for i, w in enumerate(walks):
            if best in w:
                covered[i] = True
    return chosen, gains


def csr(walks):
    off = np.concatenate([[0], np.cumsum([len(w) for w in walks])]).astype(np.uint64)
    ids = np.concatenate([np.asarray(w, np.uint32) for w in walks]) if walks else np.zeros(0, np.uint32)
    return off, ids


@pytest.mark.parametrize("seed", range(8))
def test_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    S = int(rng.integers(5, 40))
    walks = [sorted(set(rng.integers(0, S, int(rng.integers(1, 6))).tolist())) for _ in range(int(rng.integers(0, 60)))]
    cand = rng.choice(S, int(rng.integers(1, S + 1)), replace=False)
    k = int(rng.integers(1, cand.shape[0] + 1))
    sel, gains = candidates.greedy_candidates(S, *csr(walks), k, cand)
    want_sel, want_gains = brute_greedy([set(w) for w in walks], k, cand.tolist())
    assert sel.tolist() == want_sel and gains.tolist() == want_gains


def test_every_id_a_candidate_is_the_plain_greedy():
    rng = np.random.default_rng(3)
    S = 500
    walks = [rng.choice(S, int(rng.integers(1, 8)), replace=False) for _ in range(2000)]
    off, ids = csr(walks)
    a = candidates.greedy_candidates(S, off, ids, 60, rng.permutation(S))
    b = cpu.greedy_csr(S, off, ids, 60)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_rejects_bad_candidate_sets():
    off, ids = csr([[1, 2], [3]])
    for cand, k in (([1, 1], 1), ([7], 1), ([-1], 1), ([1, 2], 3)):
        with pytest.raises(ValueError):
            candidates.greedy_candidates(5, off, ids, k, cand)
