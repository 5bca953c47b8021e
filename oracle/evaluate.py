"""Out-of-sample evaluation of a chosen set on the CPU oracle.

TEST INFRASTRUCTURE ONLY (test suite, smoke check, CPU-baseline leg).

The experiments score a solution T by an estimate of its influence
suspension D(T) (Section 6.1).  Here the estimate comes from HSAWs on a
sample of its own: by Theorem "lem:rr_edge" / "lem:rr_node", D(T) equals
|V\\X| times the probability that an attempt's walk is an HSAW holding an id
of T, so D^ = |V\\X| * covered / N over N attempts.
"""
import numpy as np

from . import cpu, sas


def evaluate(graph, sources, mode, selected, n_attempts, offset=0, seed=0):
    walks = graph.sample(sources, mode, n_attempts, offset, seed)
    id_space = graph.m if mode == cpu.MODE_EDGES else graph.n
    covered = sas.coverage(walks.off, walks.ids, np.asarray(selected, np.int64), id_space)
    src_sel = int(np.isin(selected, np.asarray(sources)).sum()) if mode == cpu.MODE_NODES else 0
    spread, susp, susp_n = cpu.estimates(graph.n, len(sources), n_attempts, walks.hits, covered, src_sel)
    return dict(walks=walks, covered=covered, spread=spread, suspension=susp, suspension_nodes=susp_n)
