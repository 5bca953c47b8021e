"""Greedy restricted to a candidate set C on the CPU oracle.

TEST INFRASTRUCTURE ONLY (test suite, smoke check, CPU-baseline leg).

Definitions "edge_remove" / "node_remove" draw the k ids from C (a subset of
E or V), and Algorithms 4 / 7 take the argmax over C minus the ids already
chosen.  Whether a walk is covered by ids of C depends only on the ids of C
it holds, so each walk keeps its candidate ids, renumbered by their rank in
C in ascending order (the lowest id still wins a tie, and the lowest
unselected candidates follow once every gain is zero), and the plain greedy
of the oracle runs on the ranks.
"""
import numpy as np

from . import cpu


def greedy_candidates(id_space, off, ids, k, candidates):
    cand = np.asarray(candidates, np.int64)
    srt = np.unique(cand)
    if srt.shape[0] != cand.shape[0] or srt[0] < 0 or srt[-1] >= id_space or k > srt.shape[0]:
        raise ValueError("candidates must be distinct ids in [0, id_space), at least k of them")
    rank = np.full(id_space, -1, np.int64)
    rank[srt] = np.arange(srt.shape[0])
    off = np.asarray(off, np.int64)
    ids = np.asarray(ids, np.int64)
    n_walks = off.shape[0] - 1
    walk_of = np.repeat(np.arange(n_walks), np.diff(off))
    r = rank[ids]
    keep = r >= 0
    lens = np.bincount(walk_of[keep], minlength=n_walks)
    off2 = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    sel, gains = cpu.greedy_csr(srt.shape[0], off2, r[keep].astype(np.uint32), k)
    return srt[sel], gains


def solve_candidates(graph, sources, mode, k, n_attempts, offset, seed, candidates):
    """Sample as cpu.solve, then the greedy over the candidates."""
    walks = graph.sample(sources, mode, n_attempts, offset, seed)
    id_space = graph.m if mode == cpu.MODE_EDGES else graph.n
    sel, gains = greedy_candidates(id_space, walks.off, walks.ids, k, candidates)
    return dict(walks=walks, selected=sel, gains=gains, covered=int(gains.sum()))
