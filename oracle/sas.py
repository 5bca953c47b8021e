"""Stop-and-Stare driver of eSIA (Algorithm 6 with Check, Algorithm 5) and
nSIA (Algorithm 9 with CheckNode, Algorithm 8) on the CPU oracle.

TEST INFRASTRUCTURE ONLY (test suite, smoke check, CPU-baseline leg).

The driver doubles the number of accepted walks (HSAWs) each iteration t:
the greedy picks a candidate from the first N_t accepted walks R_t and the
candidate's coverage is verified on the next N_t accepted walks R'_t; it
stops when Check passes or when |R_t| reaches N_max.

Readings of the paper (where its text is garbled or leaves a choice):
* the stream R_1, R_2, ... is the accepted walks in attempt-id order, so
  R_t and R'_t are fixed by (seed, sources) and every attempt's walk is the
  same as in a single sampling run;
* N_t = ceil(Lambda * 2^(t-1)) and |R'_t| = N_t (Algorithm 6 defines R'_t
  as the walks after R_t up to index Lambda * 2^t);
* t_max: its displayed formula takes ln(delta/3) < 0; the lemma bounding the
  iterations uses Upsilon(eps, delta/3) = (2 + 2eps/3) ln(3/delta) / eps^2,
  so t_max = ceil(log2(2 N_max / Upsilon));
* ln C(m, k) is evaluated with lgamma;
* N_max uses m for edges (equation "guard") and n for nodes ("nguard");
  the rest is the same for both (Check and CheckNode are the same test).
"""
import math

import numpy as np

from . import cpu


def ln_binom(a, b):
    """ln C(a, b) through the log-gamma function."""
    return math.lgamma(a + 1) - math.lgamma(b + 1) - math.lgamma(a - b + 1)


def params(id_space, k, eps, delta):
    """Lambda (equation "lambda"), Lambda_1 ("lambda_1"), N_max ("guard" /
    "nguard", id_space = m or n) and t_max (lemma on the iteration count)."""
    c = 2.0 + 2.0 * eps / 3.0
    e1 = 1.0 - 1.0 / math.e
    n_max = (2.0 - 1.0 / math.e) ** 2 * c * id_space * (math.log(6.0 / delta) + ln_binom(id_space, k)) / (
        k * eps * eps)
    upsilon = c * math.log(3.0 / delta) / (eps * eps)
    t_max = max(1, math.ceil(math.log2(2.0 * n_max / upsilon)))
    lam = c * math.log(3.0 * t_max / delta) / (eps * eps)
    lam1 = 1.0 + (1.0 + eps) * c * math.log(3.0 * t_max / delta) / (eps * eps)
    return dict(lam=lam, lam1=lam1, n_max=n_max, t_max=t_max, upsilon=upsilon, e1=e1)


def check_terms(cov_r, cov_rp, n_rp, t, eps, lam1):
    """The quantities Check (Algorithm 5 / 8) forms: None below the Lambda_1
    cut-off (Cov_{R'_t} < Lambda_1), else (eps_1, eps_2, eps_3, eps_t)."""
    if cov_rp < lam1:
        return None
    e = 1.0 - 1.0 / math.e
    scale = n_rp * (1.0 + eps) / (2.0 ** (t - 1) * cov_rp)
    eps1 = cov_r / cov_rp - 1.0
    eps2 = eps * math.sqrt(scale)
    eps3 = eps * math.sqrt(scale * (e - eps) / (1.0 + eps / 3.0))
    eps_t = (eps1 + eps2 + eps1 * eps2) * (e - eps) + e * eps3
    return eps1, eps2, eps3, eps_t


def check(cov_r, cov_rp, n_rp, t, eps, lam1):
    """Check (Algorithm 5 / 8): (passed, eps_t); eps_t is None when the
    coverage on R'_t is below Lambda_1."""
    terms = check_terms(cov_r, cov_rp, n_rp, t, eps, lam1)
    if terms is None:
        return False, None
    return terms[3] <= eps, terms[3]


def coverage(off, ids, chosen, id_space):
    """Number of walks (CSR off / ids) holding at least one chosen id."""
    mark = np.zeros(id_space, bool)
    mark[np.asarray(chosen, np.int64)] = True
    off = np.asarray(off, np.int64)
    hit = mark[np.asarray(ids, np.int64)]
    n = off.shape[0] - 1
    if n == 0:
        return 0
    per = np.add.reduceat(hit.astype(np.int64), off[:-1]) if hit.shape[0] else np.zeros(n, np.int64)
    per[off[:-1] == off[1:]] = 0  # (a kept walk always holds an id; guards reduceat on empties)
    return int((per > 0).sum())


class _Stream:
    """Accepted walks in attempt-id order, sampled in growing attempt ranges."""

    def __init__(self, graph, sources, mode, seed, chunk, p=None):
        self.g, self.src, self.mode, self.seed, self.p = graph, sources, mode, seed, p
        self.chunk = chunk
        self.end = 0  # attempts [0, end) sampled
        self.attempt = np.zeros(0, np.uint64)
        self.lens = np.zeros(0, np.int64)
        self.ids = np.zeros(0, np.uint32)

    def ensure(self, n_walks, max_attempts):
        while self.attempt.shape[0] < n_walks:
            if self.end >= max_attempts:
                return False
            c = min(self.chunk, max_attempts - self.end)
            if self.p is None:
                w = self.g.sample(self.src, self.mode, c, self.end, self.seed)
            else:
                w = self.g.sample_suspects(self.src, self.p, self.mode, c, self.end, self.seed)
            self.attempt = np.concatenate([self.attempt, w.attempt])
            self.lens = np.concatenate([self.lens, np.diff(w.off.astype(np.int64))])
            self.ids = np.concatenate([self.ids, w.ids])
            self.end += c
            self.chunk *= 2
        return True

    def slice(self, a, b):
        """Walks a .. b-1 of the stream as (off, ids)."""
        starts = np.concatenate([[0], np.cumsum(self.lens)])
        off = (starts[a:b + 1] - starts[a]).astype(np.uint64)
        return off, self.ids[starts[a]:starts[b]]


def stop_and_stare(graph, sources, mode, k, eps=0.1, delta=None, seed=0, max_attempts=1 << 40,
                   chunk=1 << 16, p=None):
    """eSIA (mode = cpu.MODE_EDGES) or nSIA (cpu.MODE_NODES) with a sample
    count chosen by Stop-and-Stare.  Returns the candidate of the last
    iteration with the iteration's figures.  With p, sources are suspects
    with those probabilities (the HSAW stream of the probabilistic
    sampler)."""
    id_space = graph.m if mode == cpu.MODE_EDGES else graph.n
    if delta is None:
        delta = 1.0 / graph.n
    P = params(id_space, k, eps, delta)
    st = _Stream(graph, sources, mode, seed, chunk, p)
    t = 0
    while True:
        t += 1
        n_t = math.ceil(P["lam"] * 2.0 ** (t - 1))
        if not st.ensure(2 * n_t, max_attempts):
            return dict(status="attempts", t=t, n_t=n_t, params=P)
        off, ids = st.slice(0, n_t)
        sel, gains = cpu.greedy_csr(id_space, off, ids, k)
        offp, idsp = st.slice(n_t, 2 * n_t)
        cov_r = int(gains.sum())
        cov_rp = coverage(offp, idsp, sel, id_space)
        passed, eps_t = check(cov_r, cov_rp, n_t, t, eps, P["lam1"])
        if passed or n_t >= P["n_max"]:
            a_r = int(st.attempt[n_t - 1]) + 1       # R_t = accepted walks of attempts [0, a_r)
            a_rp = int(st.attempt[2 * n_t - 1]) + 1  # R'_t: attempts [a_r, a_rp)
            return dict(status="passed" if passed else "n_max", t=t, n_t=n_t, selected=sel, gains=gains,
                        cov_r=cov_r, cov_rp=cov_rp, eps_t=eps_t, attempts_r=a_r, attempts_rp=a_rp,
                        params=P)
