"""The C ABI library loads, exports every declared symbol, and its host-side
argument checks answer without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1702_05854_amd import sia

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sia.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sia.LIB_PATH):
        from paper_1702_05854_amd import build
        build.build()
    return sia.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sia_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("sia_graph_create", "sia_graph_destroy", "sia_sample", "sia_greedy", "sia_solve",
              "sia_last_error", "sia_check_query", "sia_graph_thresholds"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert L.sia_version().decode().startswith("sia")


def test_check_query_rejects_bad_arguments(L):
    src = [1, 5, 9]
    ok = dict(n=100, m=500, mode="edges", sources=src, k=10, n_attempts=1000, attempt_offset=0)
    sia.check_query(**ok)
    sia.check_query(**{**ok, "k": 0})                 # sampling-only queries
    bad = [
        {"n": 1}, {"n": 1 << 31}, {"m": -1}, {"sources": [1, 1]}, {"sources": [100]},
        {"sources": [-1]}, {"sources": list(range(100))}, {"k": 501}, {"mode": "nodes", "k": 101},
        {"n_attempts": 0}, {"n_attempts": 1 << 32}, {"attempt_offset": (1 << 64) - 10},
    ]
    for b in bad:
        with pytest.raises(sia.SiaError) as e:
            sia.check_query(**{**ok, **b})
        assert e.value.status == -1, b
        assert L.sia_last_error().decode() != ""


def test_graph_create_rejects_bad_structure_on_host(L):
    h = C.c_void_p()
    def create(col, row, w, n=None):
        col = np.asarray(col, np.int64)
        row = np.asarray(row, np.int32)
        w = np.asarray(w, np.float32)
        n = len(col) - 1 if n is None else n
        return L.sia_graph_create(n, len(row), col.ctypes.data_as(C.c_void_p),
                                  row.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p),
                                  0, None, C.byref(h))
    assert create([1, 1, 2], [0, 1], [0.5, 0.5]) == -1       # col_off[0] != 0
    assert create([0, 2, 1], [0, 1], [0.5, 0.5]) == -1       # decreasing
    assert create([0, 1, 1], [0, 1], [0.5, 0.5]) == -1       # col_off[n] != m
    assert create([0, 1, 2], [0, 7], [0.5, 0.5]) == -1       # row out of range
    assert create([0, 1], [0], [0.5], n=1) == -1             # n < 2
    assert L.sia_graph_create(3, 0, None, None, None, 0, None, C.byref(h)) == -1
    assert not h.value
    assert "row_idx" in L.sia_last_error().decode() or L.sia_last_error()


def test_greedy_rejects_bad_arguments(L):
    off = np.array([0, 2], np.uint64)
    ids = np.array([0, 9], np.uint32)
    with pytest.raises(sia.SiaError):
        sia.greedy(5, off, ids, 2, stream=0)                       # id 9 outside [0, 5)
    with pytest.raises(sia.SiaError):
        sia.greedy(10, off, ids, 11, stream=0)                     # k > id_space


def test_batch_entry_points_reject_null_handles(L):
    out = C.c_void_p()
    assert L.sia_batch_create(None, 1 << 30, 4, None, C.byref(out)) == -1
    assert not out.value
    q = sia.Query()
    t = C.c_uint64()
    assert L.sia_batch_submit(None, C.byref(q), C.byref(t)) == -1
    assert L.sia_batch_poll(None, 1, None, None, None, None) == -1
    assert L.sia_batch_wait(None, 1, 0, None, None, None, None) == -1
    assert L.sia_batch_cancel(None, 1) == -1
    assert L.sia_batch_stats_get(None, None) == -1
    assert L.sia_batch_tune(None, None, 1.0, None) == -1
    assert "NULL" in L.sia_last_error().decode()
    assert L.sia_batch_destroy(None) == 0


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and offsets."""
    import subprocess
    structs = {"sia_stats": sia.Stats, "sia_query": sia.Query, "sia_batch_config": sia.BatchConfig,
               "sia_ticket_info": sia.TicketInfo, "sia_batch_stats": sia.BatchStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c_layout = {tuple(l.split()[:2]): int(l.split()[2]) for l in got if l}
    for cname, py in structs.items():
        assert c_layout[(cname, "size")] == C.sizeof(py), cname
        for field, _ in py._fields_:
            assert c_layout[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_probe_gather_rejects_bad_arguments(L):
    rate, ms = C.c_double(), C.c_double()
    assert L.sia_probe_gather(0, 512, 0, C.byref(rate), C.byref(ms), None) == -1
    assert L.sia_probe_gather(1 << 30, 7, 0, C.byref(rate), C.byref(ms), None) == -1
    assert L.sia_probe_gather(1 << 30, 512, 0, None, None, None) == -1


def test_sas_solve_rejects_null_graph_on_host(L):
    info = sia.SasInfo()
    sel = np.zeros(4, np.int64)
    gains = np.zeros(4, np.uint64)
    src = np.array([1, 2], np.int32)
    rc = L.sia_sas_solve(None, 0, src.ctypes.data, 2, 4, 0.1, 1e-3, 1, 1000, sel.ctypes.data,
                         gains.ctypes.data, C.byref(info), None)
    assert rc == -1 and L.sia_last_error().decode() != ""
