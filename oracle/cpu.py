"""ctypes binding of the plain C oracle (``sia_oracle.c``).

TEST INFRASTRUCTURE ONLY (test suite, smoke check, CPU-baseline leg).  The
arithmetic lives in the C file; this module only marshals numpy arrays.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

MODE_EDGES = 0
MODE_NODES = 1

_lib = None


class _Walks(C.Structure):
    _fields_ = [
        ("n_walks", C.c_uint64),
        ("n_ids", C.c_uint64),
        ("attempt", C.POINTER(C.c_uint64)),
        ("off", C.POINTER(C.c_uint64)),
        ("ids", C.POINTER(C.c_uint32)),
        ("attempts", C.c_uint64),
        ("hits", C.c_uint64),
        ("steps", C.c_uint64),
        ("dead_ends", C.c_uint64),
        ("cycles", C.c_uint64),
        ("cap_walks", C.c_uint64),
        ("cap_ids", C.c_uint64),
    ]


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        p = C.c_void_p
        L.orc_philox4x64_10.argtypes = [p, p, p]
        L.orc_draw_node.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32]
        L.orc_draw_node.restype = C.c_uint32
        L.orc_draw_start_word.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_draw_start_word.restype = C.c_uint64
        L.orc_quantize.argtypes = [p, C.c_int64, p]
        L.orc_thresholds.argtypes = [C.c_int64, p, p, p]
        L.orc_select_edge.argtypes = [C.c_int64, C.c_int64, p, C.c_uint32]
        L.orc_select_edge.restype = C.c_int64
        L.orc_scale_u64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_scale_u64.restype = C.c_uint64
        L.orc_sample_range.argtypes = [C.c_int64, p, p, p, p, C.c_int64, C.c_int,
                                       C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(_Walks)]
        L.orc_sample_list.argtypes = [C.c_int64, p, p, p, p, C.c_int64, C.c_int,
                                      p, C.c_uint64, C.c_uint64, C.POINTER(_Walks)]
        L.orc_walks_free.argtypes = [C.POINTER(_Walks)]
        L.orc_draw_node_word.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32]
        L.orc_draw_node_word.restype = C.c_uint64
        L.orc_coin_thresholds.argtypes = [p, C.c_int64, p]
        L.orc_sample_suspects_range.argtypes = [C.c_int64, p, p, p, p, p, C.c_int64, C.c_int,
                                                C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(_Walks)]
        L.orc_sample_suspects_list.argtypes = [C.c_int64, p, p, p, p, p, C.c_int64, C.c_int,
                                               p, C.c_uint64, C.c_uint64, C.POINTER(_Walks)]
        L.orc_count.argtypes = [C.c_int64, C.c_uint64, p, p, p]
        L.orc_greedy.argtypes = [C.c_int64, C.c_uint64, p, p, C.c_int64, p, p]
        L.orc_estimates.argtypes = [C.c_int64, C.c_int64, C.c_uint64, C.c_uint64, C.c_uint64,
                                    C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def philox4x64_10(counter, key):
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(ctr), _ptr(k), _ptr(out))
    return out


def draw_node(seed, attempt, node):
    return int(lib().orc_draw_node(seed, attempt, node))


def draw_start_word(seed, attempt):
    return int(lib().orc_draw_start_word(seed, attempt))


def draw_node_word(seed, attempt, node):
    """Word 0 of the block with counter (node,0,0,0): high half = live-edge
    draw, low half = seed coin."""
    return int(lib().orc_draw_node_word(seed, attempt, node))


def coin_thresholds(p):
    """pq = min(round-half-even(p * 2^32), 2^32 - 1) per suspect."""
    p = np.ascontiguousarray(p, dtype=np.float32)
    out = np.zeros(p.shape[0], dtype=np.uint32)
    _check(lib().orc_coin_thresholds(_ptr(p), p.shape[0], _ptr(out)), "coin thresholds")
    return out


def scale_u64(x0, count):
    return int(lib().orc_scale_u64(x0, count))


def quantize(w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    q = np.zeros(w.shape[0], dtype=np.uint64)
    _check(lib().orc_quantize(_ptr(w), w.shape[0], _ptr(q)), "quantize")
    return q


def thresholds(col_off, w):
    col_off = np.ascontiguousarray(col_off, dtype=np.int64)
    w = np.ascontiguousarray(w, dtype=np.float32)
    thr = np.zeros(w.shape[0], dtype=np.uint32)
    rc = lib().orc_thresholds(col_off.shape[0] - 1, _ptr(col_off), _ptr(w), _ptr(thr))
    return rc, thr


def select_edge(thr_col, r):
    thr_col = np.ascontiguousarray(thr_col, dtype=np.uint32)
    return int(lib().orc_select_edge(0, thr_col.shape[0], _ptr(thr_col), r))


class Walks:
    """Accepted walks in CSR form plus the run's counters."""

    def __init__(self, s: _Walks):
        nw, ni = int(s.n_walks), int(s.n_ids)
        self.attempt = np.ctypeslib.as_array(s.attempt, (nw,)).copy() if nw else np.zeros(0, np.uint64)
        self.off = (np.ctypeslib.as_array(s.off, (nw + 1,)).copy() if nw
                    else np.zeros(1, np.uint64))
        self.ids = np.ctypeslib.as_array(s.ids, (ni,)).copy() if ni else np.zeros(0, np.uint32)
        self.attempts = int(s.attempts)
        self.hits = int(s.hits)
        self.steps = int(s.steps)
        self.dead_ends = int(s.dead_ends)
        self.cycles = int(s.cycles)

    @property
    def n_walks(self):
        return self.attempt.shape[0]

    def walk(self, i):
        return self.ids[int(self.off[i]):int(self.off[i + 1])]


class Graph:
    """Host CSC graph + the oracle's own threshold table."""

    def __init__(self, col_off, row_idx, w):
        self.col_off = np.ascontiguousarray(col_off, dtype=np.int64)
        self.row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.float32)
        self.n = self.col_off.shape[0] - 1
        self.m = self.row_idx.shape[0]
        rc, self.thr = thresholds(self.col_off, self.w)
        _check(rc, "thresholds")

    @classmethod
    def from_tables(cls, col_off, row_idx, thr):
        """A graph whose threshold table was computed by this oracle before
        (the arrays may be read-only memory maps; they are not copied)."""
        g = cls.__new__(cls)
        g.col_off = np.ascontiguousarray(col_off, dtype=np.int64)
        g.row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
        g.thr = np.ascontiguousarray(thr, dtype=np.uint32)
        g.w = None
        g.n = g.col_off.shape[0] - 1
        g.m = g.row_idx.shape[0]
        return g

    def _sample(self, sources, mode, seed, attempts=None, n_attempts=0, offset=0):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        s = _Walks()
        L = lib()
        if attempts is None:
            rc = L.orc_sample_range(self.n, _ptr(self.col_off), _ptr(self.row_idx), _ptr(self.thr),
                                    _ptr(src), src.shape[0], mode, n_attempts, offset, seed,
                                    C.byref(s))
        else:
            at = np.ascontiguousarray(attempts, dtype=np.uint64)
            rc = L.orc_sample_list(self.n, _ptr(self.col_off), _ptr(self.row_idx), _ptr(self.thr),
                                   _ptr(src), src.shape[0], mode, _ptr(at), at.shape[0], seed,
                                   C.byref(s))
        try:
            _check(rc, "sample")
            return Walks(s)
        finally:
            L.orc_walks_free(C.byref(s))

    def _sample_suspects(self, suspects, p, mode, seed, attempts=None, n_attempts=0, offset=0):
        sus = np.ascontiguousarray(suspects, dtype=np.int32)
        pr = np.ascontiguousarray(p, dtype=np.float32)
        assert sus.shape == pr.shape
        s = _Walks()
        L = lib()
        if attempts is None:
            rc = L.orc_sample_suspects_range(self.n, _ptr(self.col_off), _ptr(self.row_idx), _ptr(self.thr),
                                             _ptr(sus), _ptr(pr), sus.shape[0], mode, n_attempts, offset,
                                             seed, C.byref(s))
        else:
            at = np.ascontiguousarray(attempts, dtype=np.uint64)
            rc = L.orc_sample_suspects_list(self.n, _ptr(self.col_off), _ptr(self.row_idx), _ptr(self.thr),
                                            _ptr(sus), _ptr(pr), sus.shape[0], mode, _ptr(at), at.shape[0],
                                            seed, C.byref(s))
        try:
            _check(rc, "sample (suspects)")
            return Walks(s)
        finally:
            L.orc_walks_free(C.byref(s))

    def sample_suspects(self, suspects, p, mode, n_attempts, offset=0, seed=0):
        """Attempts with probabilistic suspects (suspects[i] a seed with
        probability p[i]); start uniform over V."""
        return self._sample_suspects(suspects, p, mode, seed, n_attempts=n_attempts, offset=offset)

    def sample_suspects_list(self, suspects, p, mode, attempts, seed=0):
        return self._sample_suspects(suspects, p, mode, seed, attempts=attempts)

    def sample(self, sources, mode, n_attempts, offset=0, seed=0):
        return self._sample(sources, mode, seed, n_attempts=n_attempts, offset=offset)

    def sample_list(self, sources, mode, attempts, seed=0):
        return self._sample(sources, mode, seed, attempts=attempts)


def count(id_space, walks: Walks):
    cnt = np.zeros(id_space, dtype=np.uint32)
    off = np.ascontiguousarray(walks.off, dtype=np.uint64)
    ids = np.ascontiguousarray(walks.ids, dtype=np.uint32)
    _check(lib().orc_count(id_space, walks.n_walks, _ptr(off), _ptr(ids), _ptr(cnt)), "count")
    return cnt


def greedy_csr(id_space, off, ids, k):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    sel = np.zeros(k, dtype=np.int64)
    gains = np.zeros(k, dtype=np.uint64)
    _check(lib().orc_greedy(id_space, off.shape[0] - 1, _ptr(off), _ptr(ids), k, _ptr(sel),
                            _ptr(gains)), "greedy")
    return sel, gains


def greedy(id_space, walks: Walks, k):
    return greedy_csr(id_space, walks.off, walks.ids, k)


def estimates(n, n_sources, n_attempts, hits, covered, sources_selected=0):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().orc_estimates(n, n_sources, n_attempts, hits, covered, sources_selected,
                        C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def solve_suspects(graph: Graph, suspects, p, mode, k, n_attempts, offset=0, seed=0):
    """The whole path with probabilistic suspects: sample (start uniform over
    V), count, greedy; estimates I(V_I) ~ n hits / N and D(T) ~ n Cov(T) / N
    (a removed seed's own walk <v_1> is one of the covered walks)."""
    walks = graph.sample_suspects(suspects, p, mode, n_attempts, offset, seed)
    id_space = graph.m if mode == MODE_EDGES else graph.n
    sel, gains = greedy(id_space, walks, k)
    covered = int(gains.sum())
    spread, susp, _ = estimates(graph.n, 0, n_attempts, walks.hits, covered, 0)
    return dict(walks=walks, selected=sel, gains=gains, covered=covered, spread=spread, suspension=susp)


def solve(graph: Graph, sources, mode, k, n_attempts, offset=0, seed=0):
    """The whole path on the CPU: sample, count, greedy, estimates."""
    walks = graph.sample(sources, mode, n_attempts, offset, seed)
    id_space = graph.m if mode == MODE_EDGES else graph.n
    sel, gains = greedy(id_space, walks, k)
    covered = int(gains.sum())
    n_src = len(sources)
    src_sel = int(np.isin(sel, np.asarray(sources)).sum()) if mode == MODE_NODES else 0
    spread, susp, susp_n = estimates(graph.n, n_src, n_attempts, walks.hits, covered, src_sel)
    return dict(walks=walks, selected=sel, gains=gains, covered=covered, spread=spread,
                suspension=susp, suspension_nodes=susp_n)
