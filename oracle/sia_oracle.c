/*
 * sia_oracle.c -- plain single-threaded CPU oracle for HSAW sampling,
 * coverage counting and greedy max-coverage (eSIA / nSIA hot path).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check
 * and the benchmark's CPU-baseline leg may load or call this library.  The
 * product path (the HIP library) never calls it, and the two share no
 * code: this file includes nothing from the package and the package
 * includes nothing from here.
 *
 * Everything is written for clarity, not speed: one attempt at a time, a
 * per-node "last visited by attempt" stamp array as the visited set, a
 * bisection for the live in-edge, and a greedy that rescans every touched
 * id each round.
 *
 * Paper: Nguyen, Cano, Dinh, Vu, "Blocking Self-avoiding Walks Stops
 * Cyber-epidemics: A Scalable GPU-based Approach", KDD 2017
 * (arXiv 1702.05854).  Passages are cited by section / definition /
 * algorithm / equation.
 *
 * Readings where the paper is silent or garbled:
 *  R1  Live-edge selection is discretised: weight w_j becomes the integer
 *      q_j = round-half-even(w_j * 2^32); thresholds are the per-column
 *      running sums clamped to 2^32-1; the draw r (32 bits) selects the
 *      first in-edge j with thr_j > r, and r >= thr_last means "no edge".
 *  R2  The random stream is Philox4x64-10 keyed by (seed, attempt id a).
 *      The start draw is 64-bit word 0 of the block with counter (0,1,0,0);
 *      the live in-edge of node x is chosen by the high 32 bits of word 0 of
 *      the block with counter (x,0,0,0).  A walk visits each node at most
 *      once before it stops, so every draw it uses is fresh -- the law of
 *      Algorithm 1 -- while the walk of an attempt is a fixed function of
 *      (seed, a): the live-edge sample graph of that attempt, read lazily.
 *  R3  The start node is uniform over the non-sources V\X: it is the
 *      floor(x0 * |V\X| / 2^64)-th non-source in ascending id order.
 *  R4  Suspect probabilities are p == 1 (a deterministic source set X);
 *      the edge is appended after it is selected (Algorithm 2 order).
 *  R5  Greedy ties go to the lowest id; once every marginal gain is zero
 *      the round takes the lowest id not yet selected, so exactly k ids
 *      are always returned.
 *
 * Probabilistic suspects (Section 2.2: V_I = (V_I, p), a seed set X drawn
 * with probability given by equation "prob_src_set"; Algorithm 1's suspect
 * test, a suspect u the walk meets is a seed with probability p(u)), in place
 * of R3 and R4:
 *  R6  p is discretised as the weights are: pq = min(round-half-even(p *
 *      2^32), 2^32 - 1); node x is a seed in attempt a when the low 32 bits
 *      of its draw word (word 0 of counter (x,0,0,0), whose high half picks
 *      its live in-edge) are below pq(x).  One coin per node and attempt, so
 *      the seeds of an attempt are one draw of X.
 *  R7  The start is uniform over all of V, floor(x0 * n / 2^64), as
 *      Algorithm 1 picks it; a start that is a seed gives the walk <v_1>
 *      (no edge).
 *  R8  A node is tested when the walk arrives at it: a node already on the
 *      walk ends it as a cycle (its coin came up "not a seed" on the first
 *      visit, so the order of the two tests does not matter), else a seed
 *      ends it as a kept walk, else its live in-edge is drawn.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status codes (mirrors the meaning, not the code, of the library's) */
#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EWEIGHTS -2
#define ORC_ENOMEM -3

#define ORC_MODE_EDGES 0
#define ORC_MODE_NODES 1

#define ORC_DEAD_END 0
#define ORC_CYCLE 1
#define ORC_HIT 2

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC 2011).  Round: two 64x64->128 products of the
 * even counter words with the multipliers, the high halves xored with the
 * odd words and the round key, then the words permuted; the key is bumped
 * by the Weyl constants between rounds.                                 */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                       uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(PHILOX_M0, c0, &hi0, &lo0);
        mul128(PHILOX_M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draws of attempt a (reading R2). */
uint64_t orc_draw_start_word(uint64_t seed, uint64_t attempt)
{
    uint64_t key[2] = {seed, attempt};
    uint64_t ctr[4] = {0, 1, 0, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return out[0];
}

uint32_t orc_draw_node(uint64_t seed, uint64_t attempt, uint32_t node)
{
    uint64_t key[2] = {seed, attempt};
    uint64_t ctr[4] = {node, 0, 0, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return (uint32_t)(out[0] >> 32);
}

/* Word 0 of the block with counter (x,0,0,0): high half = live-edge draw
 * of node x, low half = its seed coin (readings R2, R6). */
uint64_t orc_draw_node_word(uint64_t seed, uint64_t attempt, uint32_t node)
{
    uint64_t key[2] = {seed, attempt};
    uint64_t ctr[4] = {node, 0, 0, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return out[0];
}

/* ------------------------------------------------------------------ */
/* Thresholds (LT model, Section 2.1; live-edge rule, reading R1).      */
/* ------------------------------------------------------------------ */

/* q = round-half-even(w * 2^32).  (double)w is exact, scaling by 2^32 is
 * exact, and llrint rounds half to even in the default rounding mode.   */
int orc_quantize(const float *w, int64_t count, uint64_t *q_out)
{
    for (int64_t i = 0; i < count; ++i) {
        float x = w[i];
        if (!(x >= 0.0f && x <= 1.0f)) /* also rejects NaN */
            return ORC_EWEIGHTS;
        q_out[i] = (uint64_t)llrint(ldexp((double)x, 32));
    }
    return ORC_OK;
}

/* Weight validation: the LT model needs sum_u w(u,v) <= 1 for every v
 * (Section 2.1).  The check is made on the integer table: with real weights
 * summing to at most 1, fp32 rounding adds at most 2^-24 (2^8 units of q)
 * and the rounding of each q_j at most 1/2, so a column is rejected when
 *     sum_j q_j > 2^32 + 2^12 + floor(deg / 2).
 * Every weight must lie in [0,1] (NaN rejected).                        */
int orc_thresholds(int64_t n, const int64_t *col_off, const float *w,
                   uint32_t *thr_out)
{
    if (n < 1 || col_off[0] != 0)
        return ORC_EINVAL;
    for (int64_t v = 0; v < n; ++v) {
        int64_t lo = col_off[v], hi = col_off[v + 1];
        if (hi < lo)
            return ORC_EINVAL;
        uint64_t run = 0;
        for (int64_t j = lo; j < hi; ++j) {
            float x = w[j];
            if (!(x >= 0.0f && x <= 1.0f))
                return ORC_EWEIGHTS;
            uint64_t qj = (uint64_t)llrint(ldexp((double)x, 32));
            run += qj;
            thr_out[j] = run > 0xFFFFFFFFULL ? 0xFFFFFFFFU : (uint32_t)run;
        }
        if (run > (1ULL << 32) + (1ULL << 12) + (uint64_t)(hi - lo) / 2)
            return ORC_EWEIGHTS;
    }
    return ORC_OK;
}

/* First in-edge j in [lo,hi) with thr[j] > r, or -1 for "no live edge"
 * (deg 0 or r >= thr[hi-1]).  Bisection over the non-decreasing column. */
int64_t orc_select_edge(int64_t lo, int64_t hi, const uint32_t *thr, uint32_t r)
{
    if (lo == hi || r >= thr[hi - 1])
        return -1;
    int64_t a = lo, b = hi - 1; /* answer in [a, b]; thr[b] > r */
    while (a < b) {
        int64_t mid = a + (b - a) / 2;
        if (thr[mid] > r)
            b = mid;
        else
            a = mid + 1;
    }
    return a;
}

/* ------------------------------------------------------------------ */
/* Start node (reading R3).                                              */
/* ------------------------------------------------------------------ */

/* floor(x0 * count / 2^64) */
uint64_t orc_scale_u64(uint64_t x0, uint64_t count)
{
    unsigned __int128 p = (unsigned __int128)x0 * (unsigned __int128)count;
    return (uint64_t)(p >> 64);
}

/* ------------------------------------------------------------------ */
/* Sampling (Definition "HSAW", Algorithm 1, Algorithm 2).              */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t n_walks;   /* accepted walks */
    uint64_t n_ids;     /* total ids over accepted walks */
    uint64_t *attempt;  /* [n_walks] attempt id of each accepted walk */
    uint64_t *off;      /* [n_walks+1] offsets into ids */
    uint32_t *ids;      /* [n_ids] edge positions (edges) or nodes (nodes) */
    uint64_t attempts, hits, steps, dead_ends, cycles;
    uint64_t cap_walks, cap_ids; /* internal */
} orc_walks;

typedef struct {
    int64_t n;
    const int64_t *col_off;
    const int32_t *row_idx;
    const uint32_t *thr;
    int mode;
    uint64_t seed;
    uint8_t *is_source;    /* [n] */
    int32_t *nonsource;    /* [n_ns] ascending */
    int64_t n_ns;
    uint64_t *stamp;       /* [n] attempt+1 that last put the node on its path */
    int32_t *path_nodes;   /* [n] */
    uint32_t *path_edges;  /* [n] */
} sampler_t;

static int walks_push(orc_walks *out, uint64_t attempt, const uint32_t *ids,
                      uint64_t len)
{
    if (out->n_walks + 1 > out->cap_walks) {
        uint64_t cap = out->cap_walks ? out->cap_walks * 2 : 1024;
        uint64_t *na = realloc(out->attempt, cap * sizeof(uint64_t));
        if (!na) return ORC_ENOMEM;
        out->attempt = na;
        uint64_t *no = realloc(out->off, (cap + 1) * sizeof(uint64_t));
        if (!no) return ORC_ENOMEM;
        out->off = no;
        out->cap_walks = cap;
    }
    if (out->n_ids + len > out->cap_ids) {
        uint64_t cap = out->cap_ids ? out->cap_ids : 4096;
        while (cap < out->n_ids + len) cap *= 2;
        uint32_t *ni = realloc(out->ids, cap * sizeof(uint32_t));
        if (!ni) return ORC_ENOMEM;
        out->ids = ni;
        out->cap_ids = cap;
    }
    out->attempt[out->n_walks] = attempt;
    out->off[out->n_walks] = out->n_ids;
    memcpy(out->ids + out->n_ids, ids, len * sizeof(uint32_t));
    out->n_ids += len;
    out->n_walks += 1;
    out->off[out->n_walks] = out->n_ids;
    return ORC_OK;
}

/* One attempt: a random SAW from a uniform non-source start, followed
 * backwards along the live in-edge of each node (Algorithm 1, inner loop;
 * Algorithm 2, loop body).  Returns the outcome; on a hit fills *len ids. */
static int walk_one(sampler_t *S, uint64_t a, uint64_t *steps_out, uint64_t *len)
{
    uint64_t idx = orc_scale_u64(orc_draw_start_word(S->seed, a), (uint64_t)S->n_ns);
    int32_t v = S->nonsource[idx];
    uint64_t tag = a + 1;
    uint64_t n_nodes = 0, n_edges = 0, s = 0;
    S->path_nodes[n_nodes++] = v;
    S->stamp[v] = tag;
    for (;;) {
        uint32_t r = orc_draw_node(S->seed, a, (uint32_t)v);
        s += 1;
        int64_t j = orc_select_edge(S->col_off[v], S->col_off[v + 1], S->thr, r);
        if (j < 0) { *steps_out = s; return ORC_DEAD_END; }
        int32_t u = S->row_idx[j];
        S->path_edges[n_edges++] = (uint32_t)j;
        if (S->stamp[u] == tag) { *steps_out = s; return ORC_CYCLE; }
        if (S->is_source[u]) {
            S->path_nodes[n_nodes++] = u;
            *steps_out = s;
            *len = (S->mode == ORC_MODE_EDGES) ? n_edges : n_nodes;
            return ORC_HIT;
        }
        S->stamp[u] = tag;
        S->path_nodes[n_nodes++] = u;
        v = u;
    }
}

static int sampler_setup(sampler_t *S, int64_t n, const int64_t *col_off,
                         const int32_t *row_idx, const uint32_t *thr,
                         const int32_t *sources, int64_t n_sources, int mode,
                         uint64_t seed)
{
    memset(S, 0, sizeof(*S));
    if (n < 2 || n_sources < 1 || n_sources >= n) return ORC_EINVAL;
    if (mode != ORC_MODE_EDGES && mode != ORC_MODE_NODES) return ORC_EINVAL;
    S->n = n; S->col_off = col_off; S->row_idx = row_idx; S->thr = thr;
    S->mode = mode; S->seed = seed;
    S->is_source = calloc((size_t)n, 1);
    S->stamp = calloc((size_t)n, sizeof(uint64_t));
    S->path_nodes = malloc((size_t)n * sizeof(int32_t));
    S->path_edges = malloc((size_t)n * sizeof(uint32_t));
    if (!S->is_source || !S->stamp || !S->path_nodes || !S->path_edges)
        return ORC_ENOMEM;
    for (int64_t i = 0; i < n_sources; ++i) {
        int32_t x = sources[i];
        if (x < 0 || x >= n || S->is_source[x]) return ORC_EINVAL;
        S->is_source[x] = 1;
    }
    S->n_ns = n - n_sources;
    S->nonsource = malloc((size_t)S->n_ns * sizeof(int32_t));
    if (!S->nonsource) return ORC_ENOMEM;
    int64_t c = 0;
    for (int64_t v = 0; v < n; ++v)
        if (!S->is_source[v]) S->nonsource[c++] = (int32_t)v;
    return ORC_OK;
}

static void sampler_free(sampler_t *S)
{
    free(S->is_source); free(S->stamp); free(S->path_nodes);
    free(S->path_edges); free(S->nonsource);
}

static int sample_one_into(sampler_t *S, uint64_t a, orc_walks *out)
{
    uint64_t steps = 0, len = 0;
    int outcome = walk_one(S, a, &steps, &len);
    out->attempts += 1;
    out->steps += steps;
    if (outcome == ORC_DEAD_END) { out->dead_ends += 1; return ORC_OK; }
    if (outcome == ORC_CYCLE) { out->cycles += 1; return ORC_OK; }
    out->hits += 1;
    const uint32_t *ids = (S->mode == ORC_MODE_EDGES)
                              ? S->path_edges
                              : (const uint32_t *)S->path_nodes;
    return walks_push(out, a, ids, len);
}

/* Attempts attempt_offset .. attempt_offset+n_attempts-1, in order. */
int orc_sample_range(int64_t n, const int64_t *col_off, const int32_t *row_idx,
                     const uint32_t *thr, const int32_t *sources,
                     int64_t n_sources, int mode, uint64_t n_attempts,
                     uint64_t attempt_offset, uint64_t seed, orc_walks *out)
{
    memset(out, 0, sizeof(*out));
    sampler_t S;
    int rc = sampler_setup(&S, n, col_off, row_idx, thr, sources, n_sources,
                           mode, seed);
    for (uint64_t i = 0; rc == ORC_OK && i < n_attempts; ++i)
        rc = sample_one_into(&S, attempt_offset + i, out);
    sampler_free(&S);
    return rc;
}

/* The listed attempts, in the given order. */
int orc_sample_list(int64_t n, const int64_t *col_off, const int32_t *row_idx,
                    const uint32_t *thr, const int32_t *sources,
                    int64_t n_sources, int mode, const uint64_t *attempt_ids,
                    uint64_t count, uint64_t seed, orc_walks *out)
{
    memset(out, 0, sizeof(*out));
    sampler_t S;
    int rc = sampler_setup(&S, n, col_off, row_idx, thr, sources, n_sources,
                           mode, seed);
    for (uint64_t i = 0; rc == ORC_OK && i < count; ++i)
        rc = sample_one_into(&S, attempt_ids[i], out);
    sampler_free(&S);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Probabilistic suspects (readings R6-R8).                             */
/* ------------------------------------------------------------------ */

/* pq = min(round-half-even(p * 2^32), 2^32 - 1) for p in [0, 1]. */
int orc_coin_thresholds(const float *p, int64_t count, uint32_t *pq_out)
{
    for (int64_t i = 0; i < count; ++i) {
        float x = p[i];
        if (!(x >= 0.0f && x <= 1.0f))
            return ORC_EINVAL;
        uint64_t q = (uint64_t)llrint(ldexp((double)x, 32));
        pq_out[i] = q > 0xFFFFFFFFULL ? 0xFFFFFFFFU : (uint32_t)q;
    }
    return ORC_OK;
}

typedef struct {
    int64_t n;
    const int64_t *col_off;
    const int32_t *row_idx;
    const uint32_t *thr;
    int mode;
    uint64_t seed;
    uint8_t *is_suspect;   /* [n] */
    uint32_t *coin_thr;    /* [n] pq of each suspect */
    uint64_t *stamp;       /* [n] attempt+1 that last put the node on its path */
    int32_t *path_nodes;   /* [n] */
    uint32_t *path_edges;  /* [n] */
} psampler_t;

static void psampler_free(psampler_t *S)
{
    free(S->is_suspect); free(S->coin_thr); free(S->stamp);
    free(S->path_nodes); free(S->path_edges);
}

static int psampler_setup(psampler_t *S, int64_t n, const int64_t *col_off,
                          const int32_t *row_idx, const uint32_t *thr,
                          const int32_t *suspects, const float *p,
                          int64_t n_suspects, int mode, uint64_t seed)
{
    memset(S, 0, sizeof(*S));
    if (n < 1 || n_suspects < 0 || n_suspects > n) return ORC_EINVAL;
    if (mode != ORC_MODE_EDGES && mode != ORC_MODE_NODES) return ORC_EINVAL;
    S->n = n; S->col_off = col_off; S->row_idx = row_idx; S->thr = thr;
    S->mode = mode; S->seed = seed;
    S->is_suspect = calloc((size_t)n, 1);
    S->coin_thr = calloc((size_t)n, sizeof(uint32_t));
    S->stamp = calloc((size_t)n, sizeof(uint64_t));
    S->path_nodes = malloc((size_t)n * sizeof(int32_t));
    S->path_edges = malloc((size_t)n * sizeof(uint32_t));
    if (!S->is_suspect || !S->coin_thr || !S->stamp || !S->path_nodes || !S->path_edges)
        return ORC_ENOMEM;
    for (int64_t i = 0; i < n_suspects; ++i) {
        int32_t x = suspects[i];
        if (x < 0 || x >= n || S->is_suspect[x]) return ORC_EINVAL;
        int rc = orc_coin_thresholds(&p[i], 1, &S->coin_thr[x]);
        if (rc != ORC_OK) return rc;
        S->is_suspect[x] = 1;
    }
    return ORC_OK;
}

/* Is x a seed in attempt a (reading R6)? */
static int is_seed(const psampler_t *S, uint64_t a, int32_t x)
{
    if (!S->is_suspect[x]) return 0;
    uint32_t coin = (uint32_t)orc_draw_node_word(S->seed, a, (uint32_t)x);
    return coin < S->coin_thr[x];
}

/* One attempt (Algorithm 1 with suspect coins, readings R6-R8). */
static int pwalk_one(psampler_t *S, uint64_t a, uint64_t *steps_out, uint64_t *len)
{
    uint64_t idx = orc_scale_u64(orc_draw_start_word(S->seed, a), (uint64_t)S->n);
    int32_t v = (int32_t)idx;
    uint64_t tag = a + 1;
    uint64_t n_nodes = 0, n_edges = 0, s = 0;
    S->path_nodes[n_nodes++] = v;
    S->stamp[v] = tag;
    for (;;) {
        if (is_seed(S, a, v)) {
            *steps_out = s;
            *len = (S->mode == ORC_MODE_EDGES) ? n_edges : n_nodes;
            return ORC_HIT;
        }
        uint32_t r = orc_draw_node(S->seed, a, (uint32_t)v);
        s += 1;
        int64_t j = orc_select_edge(S->col_off[v], S->col_off[v + 1], S->thr, r);
        if (j < 0) { *steps_out = s; return ORC_DEAD_END; }
        int32_t u = S->row_idx[j];
        S->path_edges[n_edges++] = (uint32_t)j;
        if (S->stamp[u] == tag) { *steps_out = s; return ORC_CYCLE; }
        S->stamp[u] = tag;
        S->path_nodes[n_nodes++] = u;
        v = u;
    }
}

static int psample_one_into(psampler_t *S, uint64_t a, orc_walks *out)
{
    uint64_t steps = 0, len = 0;
    int outcome = pwalk_one(S, a, &steps, &len);
    out->attempts += 1;
    out->steps += steps;
    if (outcome == ORC_DEAD_END) { out->dead_ends += 1; return ORC_OK; }
    if (outcome == ORC_CYCLE) { out->cycles += 1; return ORC_OK; }
    out->hits += 1;
    const uint32_t *ids = (S->mode == ORC_MODE_EDGES)
                              ? S->path_edges
                              : (const uint32_t *)S->path_nodes;
    return walks_push(out, a, ids, len);
}

/* Attempts attempt_offset .. attempt_offset+n_attempts-1 with suspects
 * suspects[i] of probability p[i] (distinct ids, any order). */
int orc_sample_suspects_range(int64_t n, const int64_t *col_off, const int32_t *row_idx,
                              const uint32_t *thr, const int32_t *suspects, const float *p,
                              int64_t n_suspects, int mode, uint64_t n_attempts,
                              uint64_t attempt_offset, uint64_t seed, orc_walks *out)
{
    memset(out, 0, sizeof(*out));
    psampler_t S;
    int rc = psampler_setup(&S, n, col_off, row_idx, thr, suspects, p, n_suspects, mode, seed);
    for (uint64_t i = 0; rc == ORC_OK && i < n_attempts; ++i)
        rc = psample_one_into(&S, attempt_offset + i, out);
    psampler_free(&S);
    return rc;
}

/* The listed attempts, in the given order. */
int orc_sample_suspects_list(int64_t n, const int64_t *col_off, const int32_t *row_idx,
                             const uint32_t *thr, const int32_t *suspects, const float *p,
                             int64_t n_suspects, int mode, const uint64_t *attempt_ids,
                             uint64_t count, uint64_t seed, orc_walks *out)
{
    memset(out, 0, sizeof(*out));
    psampler_t S;
    int rc = psampler_setup(&S, n, col_off, row_idx, thr, suspects, p, n_suspects, mode, seed);
    for (uint64_t i = 0; rc == ORC_OK && i < count; ++i)
        rc = psample_one_into(&S, attempt_ids[i], out);
    psampler_free(&S);
    return rc;
}

void orc_walks_free(orc_walks *w)
{
    free(w->attempt); free(w->off); free(w->ids);
    memset(w, 0, sizeof(*w));
}

/* ------------------------------------------------------------------ */
/* Coverage counts: Cov of a single id = number of kept walks holding it
 * (symbol table, Cov_R).  A simple walk holds each id at most once.     */
/* ------------------------------------------------------------------ */
int orc_count(int64_t id_space, uint64_t n_walks, const uint64_t *off,
              const uint32_t *ids, uint32_t *cnt_out)
{
    memset(cnt_out, 0, (size_t)id_space * sizeof(uint32_t));
    for (uint64_t w = 0; w < n_walks; ++w)
        for (uint64_t e = off[w]; e < off[w + 1]; ++e) {
            if ((int64_t)ids[e] >= id_space) return ORC_EINVAL;
            cnt_out[ids[e]] += 1;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Greedy max-coverage (Algorithm 4 for edges, Algorithm 7 for nodes):
 * k rounds, each taking the id of largest marginal coverage on the kept
 * walks (lowest id on ties, reading R5), then marking its walks covered. */
/* ------------------------------------------------------------------ */
int orc_greedy(int64_t id_space, uint64_t n_walks, const uint64_t *off,
               const uint32_t *ids, int64_t k, int64_t *selected,
               uint64_t *gains)
{
    if (k < 1 || k > id_space) return ORC_EINVAL;
    uint32_t *cnt = malloc((size_t)id_space * sizeof(uint32_t));
    uint8_t *chosen = calloc((size_t)id_space, 1);
    uint8_t *covered = calloc(n_walks ? (size_t)n_walks : 1, 1);
    uint32_t *touched = malloc((off[n_walks] + 1) * sizeof(uint32_t));
    if (!cnt || !chosen || !covered || !touched) {
        free(cnt); free(chosen); free(covered); free(touched);
        return ORC_ENOMEM;
    }
    int rc = orc_count(id_space, n_walks, off, ids, cnt);
    /* the ids with a positive count, ascending: only they can have gain */
    uint64_t n_touched = 0;
    for (int64_t id = 0; rc == ORC_OK && id < id_space; ++id)
        if (cnt[id] > 0) touched[n_touched++] = (uint32_t)id;
    int64_t next_zero = 0; /* lowest id that may still be unselected */
    for (int64_t round = 0; rc == ORC_OK && round < k; ++round) {
        int64_t best = -1;
        uint32_t best_cnt = 0;
        for (uint64_t t = 0; t < n_touched; ++t) {
            uint32_t id = touched[t];
            if (!chosen[id] && cnt[id] > best_cnt) {
                best_cnt = cnt[id];
                best = id;
            }
        }
        if (best < 0) { /* every gain is zero */
            while (chosen[next_zero]) ++next_zero;
            best = next_zero;
            best_cnt = 0;
        }
        chosen[best] = 1;
        selected[round] = best;
        gains[round] = best_cnt;
        if (best_cnt == 0) continue;
        for (uint64_t w = 0; w < n_walks; ++w) {
            if (covered[w]) continue;
            int holds = 0;
            for (uint64_t e = off[w]; e < off[w + 1]; ++e)
                if ((int64_t)ids[e] == best) { holds = 1; break; }
            if (!holds) continue;
            covered[w] = 1;
            for (uint64_t e = off[w]; e < off[w + 1]; ++e) cnt[ids[e]] -= 1;
        }
    }
    free(cnt); free(chosen); free(covered); free(touched);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Estimates (Theorem "lem:rr_edge" / "lem:rr_node" with p == 1): with N
 * attempts from uniform non-source starts, each attempt is the HSAW of
 * its start in a live-edge sample (walk uniqueness), so
 *   I(X)   ~ |X| + |V\X| * hits / N
 *   D(T)   ~ |V\X| * Cov(T) / N
 * and a removed source also stops its own infection (+|T & X| for nodes). */
/* ------------------------------------------------------------------ */
void orc_estimates(int64_t n, int64_t n_sources, uint64_t n_attempts,
                   uint64_t hits, uint64_t covered, int64_t sources_selected,
                   double *spread, double *suspension, double *suspension_nodes)
{
    double n_ns = (double)(n - n_sources);
    *spread = (double)n_sources + n_ns * (double)hits / (double)n_attempts;
    *suspension = n_ns * (double)covered / (double)n_attempts;
    *suspension_nodes = *suspension + (double)sources_selected;
}
