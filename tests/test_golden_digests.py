"""The full-size digests under tests/golden/ (written by
make_fullsize_digest.py from the oracle alone) are self-consistent: the
counters partition the attempts, every kept walk holds at least one id, the
greedy's gains never increase and sum to the covered count, the picks are
distinct edge ids, and covered never exceeds the kept walks."""
import json
import os

import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", ["rmat24", "rmat26"])
def test_digest_is_consistent(name):
    with open(os.path.join(HERE, f"{name}_digest.json")) as f:
        D = json.load(f)
    C = D["counters"]
    assert C["attempts"] == D["n_attempts"] == C["hits"] + C["dead_ends"] + C["cycles"]
    # edges: a kept walk of t draws holds t >= 1 ids; every attempt draws at least once
    assert C["walk_ids"] >= C["hits"] and C["steps"] >= C["walk_ids"] + C["dead_ends"] + C["cycles"]
    sel, gains = D["selected"], D["gains"]
    assert len(sel) == len(gains) == D["k"] and len(set(sel)) == D["k"]
    assert all(0 <= x < D["m"] for x in sel)
    assert all(a >= b for a, b in zip(gains, gains[1:]))
    assert sum(gains) == D["covered"] <= C["hits"]
    assert set(D["sha256"]) >= {"attempt", "off", "ids", "counts", "col_off", "row_idx", "w"}
