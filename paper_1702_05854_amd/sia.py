"""Thin ctypes binding of ``libsia.so`` (the C ABI in ``include/sia.h``).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device arrays are torch tensors on a ROCm device (their
``data_ptr()`` is passed through); host arrays are numpy arrays.  The stream
is ``torch.cuda.current_stream().cuda_stream`` unless one is given.

The library must be built (``python -m paper_1702_05854_amd.build``); loading
fails loudly when it is missing -- there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsia.so")

EDGES = 0
NODES = 1
MODES = {"edges": EDGES, "nodes": NODES, EDGES: EDGES, NODES: NODES}
FLAG_TIMING = 1           # SIA_FLAG_TIMING
FLAG_NO_CYCLE_STEPS = 2   # SIA_FLAG_NO_CYCLE_STEPS

STATUS = {0: "SIA_OK", -1: "SIA_EINVAL", -2: "SIA_EWEIGHTS", -3: "SIA_ENOMEM",
          -4: "SIA_EDEVICE", -5: "SIA_ENOTREADY", -6: "SIA_ECANCELLED", -7: "SIA_EBUSY"}


class SiaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Stats(C.Structure):
    _fields_ = [("attempts", C.c_uint64), ("hits", C.c_uint64), ("dead_ends", C.c_uint64),
                ("cycles", C.c_uint64), ("steps", C.c_uint64), ("evaluations", C.c_uint64),
                ("walk_ids", C.c_uint64), ("covered", C.c_uint64),
                ("spread_est", C.c_double), ("suspension_est", C.c_double),
                ("suspension_nodes_est", C.c_double),
                ("ms_sample", C.c_float), ("ms_count", C.c_float), ("ms_greedy", C.c_float),
                ("ms_total", C.c_float)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SasInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("t", C.c_int32), ("n_t", C.c_uint64),
                ("attempts_r", C.c_uint64), ("attempts_rp", C.c_uint64), ("cov_r", C.c_uint64),
                ("cov_rp", C.c_uint64), ("attempts_sampled", C.c_uint64), ("eps_t", C.c_double),
                ("lambda_", C.c_double), ("lambda1", C.c_double), ("n_max", C.c_double),
                ("t_max", C.c_int32), ("reserved", C.c_int32), ("spread_est", C.c_double),
                ("suspension_est", C.c_double), ("suspension_nodes_est", C.c_double),
                ("ms_total", C.c_float), ("reserved2", C.c_float)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("reserved")}


class Query(C.Structure):
    _fields_ = [("mode", C.c_int32), ("flags", C.c_int32), ("sources", C.c_void_p),
                ("n_sources", C.c_int64), ("k", C.c_int64), ("n_attempts", C.c_uint64),
                ("attempt_offset", C.c_uint64), ("seed", C.c_uint64)]


class BatchConfig(C.Structure):
    _fields_ = [("sampler_blocks_per_cu", C.c_int32), ("refill_chunk", C.c_uint32),
                ("wave_attempts", C.c_uint64), ("min_share", C.c_uint64),
                ("use_graph", C.c_int32), ("greedy_mode", C.c_int32), ("greedy_cus", C.c_int32),
                ("greedy_batch", C.c_uint32), ("hist_blocks", C.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TicketInfo(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_sampled", C.c_double),
                ("t_done", C.c_double), ("waves", C.c_uint32), ("reruns", C.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchStats(C.Structure):
    _fields_ = [(name, C.c_uint64) for name in (
        "submitted", "completed", "failed", "cancelled", "waves", "graph_replays",
        "greedy_launches", "greedy_jobs", "reruns", "evictions", "walk_bytes", "walk_bytes_peak",
        "walk_budget")] + [("slots", C.c_uint32), ("busy_slots", C.c_uint32),
                           ("pending", C.c_uint32), ("reserved", C.c_uint32),
                           ("sample_busy_s", C.c_double), ("greedy_busy_s", C.c_double),
                           ("greedy_index_s", C.c_double), ("config", BatchConfig)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}
        d["config"] = self.config.as_dict()
        return d


class _Walks(C.Structure):
    _fields_ = [("n_walks", C.c_uint64), ("n_ids", C.c_uint64),
                ("attempt", C.POINTER(C.c_uint64)), ("off", C.POINTER(C.c_uint64)),
                ("ids", C.POINTER(C.c_uint32)), ("stats", Stats)]


BATCH_SYMBOLS = ("sia_batch_create", "sia_batch_destroy", "sia_batch_submit", "sia_batch_poll",
                 "sia_batch_wait", "sia_batch_cancel", "sia_batch_stats_get", "sia_batch_tune")

_lib = None


def lib():
    """Load libsia.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1702_05854_amd.build`")
        L = C.CDLL(LIB_PATH)
        p, i64, u64, i32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_int
        L.sia_version.restype = C.c_char_p
        L.sia_last_error.restype = C.c_char_p
        L.sia_check_query.argtypes = [i64, i64, i32, p, i64, i64, u64, u64]
        L.sia_graph_create.argtypes = [i64, i64, p, p, p, i32, p, C.POINTER(p)]
        L.sia_graph_destroy.argtypes = [p]
        L.sia_graph_info.argtypes = [p, C.POINTER(i64), C.POINTER(i64)]
        L.sia_graph_thresholds.argtypes = [p, p, p]
        L.sia_graph_arc_bytes.argtypes = [p, C.POINTER(C.c_uint32)]
        L.sia_quantize.argtypes = [p, p, u64, p]
        L.sia_sample.argtypes = [p, i32, p, i64, u64, u64, u64, C.POINTER(_Walks), p]
        L.sia_walks_free.argtypes = [C.POINTER(_Walks)]
        L.sia_walks_free.restype = None
        L.sia_greedy.argtypes = [i64, p, p, u64, i64, p, p, p]
        L.sia_solve.argtypes = [p, i32, p, i64, i64, u64, u64, u64, p, p, C.POINTER(Stats), i32, p]
        L.sia_batch_create.argtypes = [p, u64, C.c_int32, C.POINTER(BatchConfig), C.POINTER(p)]
        L.sia_batch_destroy.argtypes = [p]
        L.sia_batch_submit.argtypes = [p, C.POINTER(Query), C.POINTER(u64)]
        L.sia_batch_poll.argtypes = [p, u64, p, p, C.POINTER(Stats), C.POINTER(TicketInfo)]
        L.sia_batch_wait.argtypes = [p, u64, i64, p, p, C.POINTER(Stats), C.POINTER(TicketInfo)]
        L.sia_batch_cancel.argtypes = [p, u64]
        L.sia_batch_stats_get.argtypes = [p, C.POINTER(BatchStats)]
        L.sia_batch_tune.argtypes = [p, C.POINTER(Query), C.c_double, C.POINTER(BatchConfig)]
        L.sia_solve_candidates.argtypes = [p, i32, p, i64, p, i64, i64, u64, u64, u64, p, p,
                                           C.POINTER(Stats), i32, p]
        L.sia_evaluate.argtypes = [p, i32, p, i64, p, i64, u64, u64, u64, C.POINTER(Stats), p]
        L.sia_sas_solve.argtypes = [p, i32, p, i64, i64, C.c_double, C.c_double, u64, u64, p, p,
                                    C.POINTER(SasInfo), p]
        L.sia_sas_solve_suspects.argtypes = [p, i32, p, p, i64, i64, C.c_double, C.c_double, u64, u64, p, p,
                                             C.POINTER(SasInfo), p]
        L.sia_sas_solve_suspects.restype = C.c_int
        L.sia_sample_suspects.argtypes = [p, i32, p, p, i64, u64, u64, u64, C.POINTER(_Walks), p]
        L.sia_sample_suspects.restype = C.c_int
        L.sia_solve_suspects.argtypes = [p, i32, p, p, i64, i64, u64, u64, u64, p, p, C.POINTER(Stats), i32, p]
        L.sia_solve_suspects.restype = C.c_int
        L.sia_greedy_noalloc.argtypes = [i64, p, p, u64, i64, p, p, p]
        L.sia_greedy_noalloc.restype = C.c_int
        L.sia_test_fail_alloc.argtypes = [C.c_uint32]
        L.sia_test_fail_alloc.restype = None
        L.sia_sas_params.argtypes = [i64, i64, C.c_double, C.c_double, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.sia_sas_check.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_double, C.c_double,
                                    C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.sia_probe_gather.argtypes = [u64, C.c_uint32, i32, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), p]
        for name in ("sia_check_query", "sia_graph_create", "sia_graph_destroy", "sia_graph_info",
                     "sia_graph_thresholds", "sia_graph_arc_bytes", "sia_quantize", "sia_sample",
                     "sia_greedy",
                     "sia_solve", "sia_solve_candidates", "sia_sas_solve", "sia_evaluate",
                     "sia_sas_params", "sia_sas_check", "sia_probe_gather") + BATCH_SYMBOLS:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SiaError(rc, lib().sia_last_error().decode())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def check_query(n, m, mode, sources, k, n_attempts, attempt_offset=0):
    src = _host(sources, np.int32)
    _check(lib().sia_check_query(n, m, MODES[mode], _hptr(src), src.shape[0], k, n_attempts,
                                 attempt_offset))


class Graph:
    """A device-resident graph (ingest + LT threshold tables built on the GPU).

    ``col_off`` int64[n+1], ``row_idx`` int32[m], ``w`` float32[m]: either all
    torch tensors on the current ROCm device, or host arrays (numpy / CPU
    tensors)."""

    def __init__(self, col_off, row_idx, w, stream=None):
        self._h = C.c_void_p()
        on_dev = hasattr(col_off, "is_cuda") and col_off.is_cuda
        if on_dev:
            import torch
            col_off = col_off.to(torch.int64).contiguous()
            row_idx = row_idx.to(torch.int32).contiguous()
            w = w.to(torch.float32).contiguous()
            n, m = col_off.numel() - 1, row_idx.numel()
            args = [C.c_void_p(col_off.data_ptr()), C.c_void_p(row_idx.data_ptr()),
                    C.c_void_p(w.data_ptr())]
        else:
            col_off = _host(col_off.cpu().numpy() if hasattr(col_off, "cpu") else col_off, np.int64)
            row_idx = _host(row_idx.cpu().numpy() if hasattr(row_idx, "cpu") else row_idx, np.int32)
            w = _host(w.cpu().numpy() if hasattr(w, "cpu") else w, np.float32)
            n, m = col_off.shape[0] - 1, row_idx.shape[0]
            args = [_hptr(col_off), _hptr(row_idx), _hptr(w)]
        _check(lib().sia_graph_create(n, m, *args, 1 if on_dev else 0, _stream(stream),
                                      C.byref(self._h)))
        self.n, self.m = n, m

    def close(self):
        if self._h:
            _check(lib().sia_graph_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    @property
    def arc_bytes(self):
        """Bytes per stored in-edge record: 16 (every column w = 1/d_in) or 32."""
        v = C.c_uint32()
        _check(lib().sia_graph_arc_bytes(self._h, C.byref(v)))
        return v.value

    def thresholds(self, stream=None):
        thr = np.zeros(self.m, dtype=np.uint32)
        _check(lib().sia_graph_thresholds(self._h, _hptr(thr), _stream(stream)))
        return thr


class Walks:
    """Kept walks in CSR form (sorted by attempt id) plus the run's counters."""

    def __init__(self, attempt, off, ids, stats):
        self.attempt, self.off, self.ids, self.stats = attempt, off, ids, stats

    @property
    def n_walks(self):
        return self.attempt.shape[0]

    def walk(self, i):
        return self.ids[int(self.off[i]):int(self.off[i + 1])]


def _walks_of(w):
    L = lib()
    try:
        nw, ni = int(w.n_walks), int(w.n_ids)
        attempt = np.ctypeslib.as_array(w.attempt, (nw,)).copy() if nw else np.zeros(0, np.uint64)
        off = np.ctypeslib.as_array(w.off, (nw + 1,)).copy()
        ids = np.ctypeslib.as_array(w.ids, (ni,)).copy() if ni else np.zeros(0, np.uint32)
        return Walks(attempt, off, ids, w.stats.as_dict())
    finally:
        L.sia_walks_free(C.byref(w))


def sample(graph: Graph, sources, mode, n_attempts, attempt_offset=0, seed=2017, stream=None):
    src = _host(sources, np.int32)
    w = _Walks()
    _check(lib().sia_sample(graph.handle, MODES[mode], _hptr(src), src.shape[0], n_attempts,
                            attempt_offset, seed, C.byref(w), _stream(stream)))
    return _walks_of(w)


def sample_suspects(graph: Graph, suspects, p, mode, n_attempts, attempt_offset=0, seed=2017, stream=None):
    """Kept walks with probabilistic suspects (sia_sample_suspects)."""
    sus = _host(suspects, np.int32)
    pr = _host(p, np.float32)
    assert sus.shape == pr.shape
    w = _Walks()
    _check(lib().sia_sample_suspects(graph.handle, MODES[mode], _hptr(sus), _hptr(pr), sus.shape[0], n_attempts,
                                     attempt_offset, seed, C.byref(w), _stream(stream)))
    return _walks_of(w)


def solve_suspects(graph: Graph, suspects, p, mode, k, n_attempts, attempt_offset=0, seed=2017, timing=False,
                   stream=None, cycle_steps=True):
    """The whole path with probabilistic suspects (sia_solve_suspects)."""
    sus = _host(suspects, np.int32)
    pr = _host(p, np.float32)
    assert sus.shape == pr.shape
    sel = np.zeros(k, dtype=np.int64)
    gains = np.zeros(k, dtype=np.uint64)
    st = Stats()
    _check(lib().sia_solve_suspects(graph.handle, MODES[mode], _hptr(sus), _hptr(pr), sus.shape[0], k, n_attempts,
                                    attempt_offset, seed, _hptr(sel), _hptr(gains), C.byref(st),
                                    _flags(timing, cycle_steps), _stream(stream)))
    return dict(selected=sel, gains=gains, stats=st.as_dict())


def greedy(id_space, walk_off, ids, k, stream=None):
    off = _host(walk_off, np.uint64)
    ids = _host(ids, np.uint32)
    sel = np.zeros(k, dtype=np.int64)
    gains = np.zeros(k, dtype=np.uint64)
    _check(lib().sia_greedy(id_space, _hptr(off), _hptr(ids), off.shape[0] - 1, k, _hptr(sel),
                            _hptr(gains), _stream(stream)))
    return sel, gains


def greedy_noalloc(id_space, walk_off, ids, k, stream=None):
    """The greedy of ``greedy`` on walks in device memory, through the entry
    point that allocates no device memory itself (sia_greedy_noalloc).
    walk_off / ids: device tensors (int64 or uint64 offsets, int32 ids);
    returns device tensors (selected int64[k], gains int64[k] holding the
    uint64 gains)."""
    import torch
    assert walk_off.is_cuda and ids.is_cuda and walk_off.dtype == torch.int64 and ids.dtype == torch.int32
    sel = torch.empty(k, dtype=torch.int64, device=walk_off.device)
    gains = torch.empty(k, dtype=torch.int64, device=walk_off.device)
    _check(lib().sia_greedy_noalloc(id_space, C.c_void_p(walk_off.data_ptr()), C.c_void_p(ids.data_ptr()),
                                    walk_off.numel() - 1, k, C.c_void_p(sel.data_ptr()),
                                    C.c_void_p(gains.data_ptr()), _stream(stream)))
    return sel, gains


def _flags(timing, cycle_steps):
    return (FLAG_TIMING if timing else 0) | (0 if cycle_steps else FLAG_NO_CYCLE_STEPS)


def solve(graph: Graph, sources, mode, k, n_attempts, attempt_offset=0, seed=2017, timing=False,
          stream=None, candidates=None, cycle_steps=True):
    """The whole path for one query; candidates (ids the picks are drawn
    from) calls sia_solve_candidates.  cycle_steps=False passes
    SIA_FLAG_NO_CYCLE_STEPS: walks that close a cycle stop at detection and
    stats["steps"] leaves out their draws; every other output is the same."""
    src = _host(sources, np.int32)
    sel = np.zeros(k, dtype=np.int64)
    gains = np.zeros(k, dtype=np.uint64)
    st = Stats()
    if candidates is None:
        _check(lib().sia_solve(graph.handle, MODES[mode], _hptr(src), src.shape[0], k, n_attempts,
                               attempt_offset, seed, _hptr(sel), _hptr(gains), C.byref(st),
                               _flags(timing, cycle_steps), _stream(stream)))
    else:
        cand = _host(candidates, np.int64)
        _check(lib().sia_solve_candidates(graph.handle, MODES[mode], _hptr(src), src.shape[0],
                                          _hptr(cand), cand.shape[0], k, n_attempts, attempt_offset,
                                          seed, _hptr(sel), _hptr(gains), C.byref(st),
                                          _flags(timing, cycle_steps), _stream(stream)))
    return dict(selected=sel, gains=gains, stats=st.as_dict())


def evaluate(graph: Graph, sources, mode, selected, n_attempts, attempt_offset=0, seed=2017,
             stream=None):
    """Counters and estimates of a chosen set on its own sample (sia_evaluate)."""
    src = _host(sources, np.int32)
    sel = _host(selected, np.int64)
    st = Stats()
    _check(lib().sia_evaluate(graph.handle, MODES[mode], _hptr(src), src.shape[0], _hptr(sel), sel.shape[0],
                              n_attempts, attempt_offset, seed, C.byref(st), _stream(stream)))
    return st.as_dict()


def sas_solve(graph: Graph, sources, mode, k, eps=0.1, delta=None, seed=2017,
              max_attempts=(1 << 32) - 1, stream=None):
    """eSIA / nSIA with the sample count chosen by Stop-and-Stare (see
    sia_sas_solve in include/sia.h); delta defaults to 1/n."""
    src = _host(sources, np.int32)
    if delta is None:
        delta = 1.0 / graph.n
    sel = np.zeros(k, dtype=np.int64)
    gains = np.zeros(k, dtype=np.uint64)
    info = SasInfo()
    _check(lib().sia_sas_solve(graph.handle, MODES[mode], _hptr(src), src.shape[0], k, float(eps),
                               float(delta), seed, max_attempts, _hptr(sel), _hptr(gains),
                               C.byref(info), _stream(stream)))
    return dict(selected=sel, gains=gains, info=info.as_dict())


def inject_alloc_failure(nth):
    """Fault injection (sia_test_fail_alloc): the nth device allocation from
    now fails with SIA_ENOMEM; 0 disables."""
    lib().sia_test_fail_alloc(int(nth))


def sas_solve_suspects(graph: Graph, suspects, p, mode, k, eps=0.1, delta=None, seed=2017,
                       max_attempts=(1 << 32) - 1, stream=None):
    """Stop-and-Stare with probabilistic suspects (sia_sas_solve_suspects);
    delta defaults to 1/n."""
    sus = _host(suspects, np.int32)
    pr = _host(p, np.float32)
    if delta is None:
        delta = 1.0 / graph.n
    sel = np.zeros(k, dtype=np.int64)
    gains = np.zeros(k, dtype=np.uint64)
    info = SasInfo()
    _check(lib().sia_sas_solve_suspects(graph.handle, MODES[mode], _hptr(sus), _hptr(pr), sus.shape[0], k,
                                        float(eps), float(delta), seed, max_attempts, _hptr(sel), _hptr(gains),
                                        C.byref(info), _stream(stream)))
    return dict(selected=sel, gains=gains, info=info.as_dict())


def sas_params(id_space, k, eps, delta):
    """Lambda, Lambda_1, N_max and t_max of the Stop-and-Stare driver
    (sia_sas_params; host arithmetic)."""
    lam, lam1, n_max, t_max = C.c_double(), C.c_double(), C.c_double(), C.c_int32()
    _check(lib().sia_sas_params(id_space, k, float(eps), float(delta), C.byref(lam), C.byref(lam1),
                                C.byref(n_max), C.byref(t_max)))
    return dict(lam=lam.value, lam1=lam1.value, n_max=n_max.value, t_max=t_max.value)


def sas_check(cov_r, cov_rp, n_rp, t, eps, lam1):
    """Check as the driver evaluates it (sia_sas_check): (passed, terms)
    with terms = (eps_1, eps_2, eps_3, eps_t), all NaN below Lambda_1."""
    terms = (C.c_double * 4)()
    passed = C.c_int32()
    _check(lib().sia_sas_check(float(cov_r), float(cov_rp), float(n_rp), t, float(eps), float(lam1), terms,
                               C.byref(passed)))
    return bool(passed.value), tuple(terms)


def _query(sources, mode, k, n_attempts, attempt_offset, seed, cycle_steps=True):
    src = _host(sources, np.int32)
    q = Query(MODES[mode], _flags(False, cycle_steps), src.ctypes.data, src.shape[0], k, n_attempts,
              attempt_offset, seed)
    return q, src  # src keeps the array alive while q is used


class Batch:
    """Queries served together on one graph (see sia_batch_* in include/sia.h).

    ``submit`` queues a query and returns its ticket; ``poll`` returns None
    while it runs, ``wait`` blocks.  A finished ticket yields
    ``dict(selected, gains, stats, info)``; a failed or cancelled one raises
    SiaError with its status."""

    def __init__(self, graph: Graph, walk_budget_bytes=8 << 30, max_slots=31, **config):
        self._h = C.c_void_p()
        cfg = BatchConfig(**config)
        _check(lib().sia_batch_create(graph.handle, walk_budget_bytes, max_slots, C.byref(cfg),
                                      C.byref(self._h)))
        self.graph = graph  # the graph must outlive the batch
        self._k = {}

    def submit(self, sources, mode, k, n_attempts, attempt_offset=0, seed=2017, cycle_steps=True):
        q, src = _query(sources, mode, k, n_attempts, attempt_offset, seed, cycle_steps)
        t = C.c_uint64()
        _check(lib().sia_batch_submit(self._h, C.byref(q), C.byref(t)))
        self._k[t.value] = k
        return t.value

    def _take(self, fn, ticket, *extra):
        k = self._k.get(ticket, 1)  # an unknown ticket is rejected by the library
        sel = np.zeros(k, dtype=np.int64)
        gains = np.zeros(k, dtype=np.uint64)
        st, info = Stats(), TicketInfo()
        rc = fn(self._h, ticket, *extra, _hptr(sel), _hptr(gains), C.byref(st), C.byref(info))
        if rc == -5:  # SIA_ENOTREADY
            return None
        if rc != -1:  # the ticket was released (finished, failed or cancelled)
            self._k.pop(ticket, None)
        _check(rc)
        return dict(selected=sel, gains=gains, stats=st.as_dict(), info=info.as_dict())

    def poll(self, ticket):
        return self._take(lib().sia_batch_poll, ticket)

    def wait(self, ticket, timeout_ms=-1):
        return self._take(lib().sia_batch_wait, ticket, timeout_ms)

    def cancel(self, ticket):
        _check(lib().sia_batch_cancel(self._h, ticket))

    def stats(self):
        s = BatchStats()
        _check(lib().sia_batch_stats_get(self._h, C.byref(s)))
        return s.as_dict()

    def tune(self, sources, mode, n_attempts, attempt_offset=0, seed=2017, target_ms=50.0, k=0,
             cycle_steps=True):
        q, src = _query(sources, mode, k, n_attempts, attempt_offset, seed, cycle_steps)
        cfg = BatchConfig()
        _check(lib().sia_batch_tune(self._h, C.byref(q), target_ms, C.byref(cfg)))
        return cfg.as_dict()

    def close(self):
        if self._h:
            _check(lib().sia_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def probe_gather(array_bytes=2 << 30, loads_per_lane=512, dependent=False, stream=None):
    """Random-gather ceiling (measuring hook): (lines per second, launch ms)."""
    rate, ms = C.c_double(), C.c_double()
    _check(lib().sia_probe_gather(array_bytes, loads_per_lane, 1 if dependent else 0, C.byref(rate),
                                  C.byref(ms), _stream(stream)))
    return rate.value, ms.value


def quantize(w_dev, q_dev, stream=None):
    """Device conversion q = round-half-even(w * 2^32) (test hook)."""
    _check(lib().sia_quantize(C.c_void_p(w_dev.data_ptr()), C.c_void_p(q_dev.data_ptr()),
                              w_dev.numel(), _stream(stream)))


def version():
    return lib().sia_version().decode()
