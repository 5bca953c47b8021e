/*
 * sia.h -- C ABI of the MI355X (gfx950) HSAW spread-interdiction library.
 *
 * Method: Nguyen, Cano, Dinh, Vu, "Blocking Self-avoiding Walks Stops
 * Cyber-epidemics: A Scalable GPU-based Approach" (KDD 2017,
 * arXiv 1702.05854).  The library runs the data-parallel hot path of eSIA
 * (Algorithm 6, edges) and nSIA (Algorithm 9, nodes) for a fixed sample
 * count: sample Hitting Self-avoiding Walks (HSAWs) under the Linear
 * Threshold model, count how many kept walks hold each edge / node, and pick
 * k of them greedily by marginal coverage.
 *
 * Conventions for every entry point:
 *  - Every call returns sia_status; 0 is success.  On failure a message for
 *    the calling thread is available from sia_last_error().
 *  - "device pointer" = memory the HIP runtime allocated on the current
 *    device; "host pointer" = ordinary CPU memory.  The caller owns every
 *    array it passes; the library never frees caller memory.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *    ordered on that stream; calls that return host results synchronise it
 *    before returning.
 *  - Graph: n nodes 0..n-1, m directed edges in in-edge CSC order.  Column v
 *    lists the in-edges (u,v) of v at positions col_off[v] .. col_off[v+1]-1;
 *    row_idx[j] is u, w[j] is the LT weight w(u,v).  An edge id is its CSC
 *    position j.  Limits: 2 <= n < 2^31, 0 <= m < 2^32.
 *  - Random stream: Philox4x64-10 keyed by (seed, attempt id).  The start
 *    draw of attempt a is 64-bit word 0 of the block with counter (0,1,0,0);
 *    the live in-edge of node x in attempt a is chosen by the high 32 bits of
 *    word 0 of the block with counter (x,0,0,0).  Results therefore depend
 *    only on (graph, sources, mode, k, attempt range, seed).
 */
#ifndef SIA_H
#define SIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIA_OK = 0,
    SIA_EINVAL = -1,     /* malformed argument or graph structure */
    SIA_EWEIGHTS = -2,   /* a weight outside [0,1]/NaN, or an in-weight sum above 1 */
    SIA_ENOMEM = -3,     /* device or host allocation failed */
    SIA_EDEVICE = -4,    /* HIP runtime error */
    SIA_ENOTREADY = -5,  /* batch: the query has not finished yet */
    SIA_ECANCELLED = -6, /* batch: the query was cancelled */
    SIA_EBUSY = -7       /* batch: resource held (tag bits, or tuning while busy) */
} sia_status;

/*
 * Flags of the solve calls (argument `flags` of sia_solve,
 * sia_solve_candidates and sia_solve_suspects; sia_query.flags of a batch).
 *  SIA_FLAG_TIMING           record HIP events around the phases into stats
 *                            (solve calls; 1 keeps its old meaning of
 *                            "timing requested")
 *  SIA_FLAG_NO_CYCLE_STEPS   stop a walk that closes a cycle as soon as the
 *                            cycle is detected.  Algorithm 1 discards such a
 *                            walk, and which attempts end in a cycle does not
 *                            change; only its exact length is not found (the
 *                            search for where it entered the cycle is skipped).
 *                            stats.steps then leaves out the draws of those
 *                            walks; every other output is identical.
 */
#define SIA_FLAG_TIMING 1
#define SIA_FLAG_NO_CYCLE_STEPS 2

typedef enum {
    SIA_EDGES = 0, /* eSIA: ids are CSC edge positions (Definition "edge_remove") */
    SIA_NODES = 1  /* nSIA: ids are node ids (Definition "node_remove") */
} sia_mode;

typedef struct sia_graph sia_graph; /* opaque; device-resident, immutable */

/* Counters and estimates of one run.  Integer fields are exact. */
typedef struct {
    uint64_t attempts;     /* walk attempts made (N) */
    uint64_t hits;         /* attempts that ended at a source: kept HSAWs */
    uint64_t dead_ends;    /* attempts that found no live in-edge */
    uint64_t cycles;       /* attempts whose walk returned to a visited node */
    uint64_t steps;        /* live-edge draws of the plain walk (Algorithm 1):
                              a hit or dead end after t draws counts t; a walk
                              whose t-th draw repeats a node counts t (0 under
                              SIA_FLAG_NO_CYCLE_STEPS) */
    uint64_t evaluations;  /* live-edge evaluations the device performed
                              (cycle detection and re-walks make it >= steps) */
    uint64_t walk_ids;     /* ids over all kept walks */
    uint64_t covered;      /* kept walks hit by the selected set, = sum of gains */
    double spread_est;     /* |X| + |V\X| * hits / N  (expected spread, p == 1) */
    double suspension_est; /* |V\X| * covered / N  (Theorem "lem:rr_edge") */
    double suspension_nodes_est; /* suspension_est + |selected & X| (nodes) */
    float ms_sample;       /* device time of the sampling kernel (HIP events,
                              on hip_stream), 0 without SIA_FLAG_TIMING */
    float ms_count;        /* coverage counting and greedy set-up */
    float ms_greedy;       /* greedy: pool rebuilds, walk lists of pool
                              ids, rounds */
    float ms_total;        /* whole call on the device */
} sia_stats;

/* Kept walks returned by sia_sample, in CSR form, allocated by the library
 * in host memory; release with sia_walks_free. */
typedef struct {
    uint64_t n_walks;  /* kept HSAWs */
    uint64_t n_ids;
    uint64_t *attempt; /* [n_walks] attempt id of each kept walk, ascending */
    uint64_t *off;     /* [n_walks+1] offsets into ids */
    uint32_t *ids;     /* [n_ids] edges: CSC positions j_1..j_{l-1} (walk
                          order from the start); nodes: v_1..v_l */
    sia_stats stats;
} sia_walks;

/* Library version string. */
const char *sia_version(void);

/* Message for the last failed call on this thread ("" if none). */
const char *sia_last_error(void);

/* Test hook (fault injection on the host): the nth device allocation the
 * library makes from now on fails as if the device were out of memory
 * (SIA_ENOMEM from the call making it); 0 disables.  Allocations that reuse
 * a buffer large enough do not count.  Process-wide. */
void sia_test_fail_alloc(uint32_t nth);

/*
 * Check the query arguments of sia_solve / sia_sample on the host without
 * touching the GPU (also done inside those calls).
 *   n, m             graph sizes
 *   mode             SIA_EDGES or SIA_NODES
 *   sources          host pointer, n_sources node ids (any order); must be
 *                    distinct, in [0,n), with 1 <= n_sources <= n-1
 *   k                budget; 1 <= k <= m (edges) or <= n (nodes); k = 0 is
 *                    accepted here when the caller does not select (sampling)
 *   n_attempts       1 <= n_attempts < 2^32
 *   attempt_offset   first attempt id; offset + n_attempts must not overflow
 * Returns SIA_OK or SIA_EINVAL.
 */
sia_status sia_check_query(int64_t n, int64_t m, int mode, const int32_t *sources,
                           int64_t n_sources, int64_t k, uint64_t n_attempts,
                           uint64_t attempt_offset);

/*
 * Ingest a graph (a1): copy it into library-owned HBM and build, for every
 * column v, the integer live-edge table of the LT model (Section 2.1, the
 * live-edge equivalence): q_j = round-half-even(w_j * 2^32), thr_j = the
 * running sum of q over the column, clamped to 2^32 - 1.  Edge j is live
 * with probability (thr_j - thr_{j-1}) / 2^32, no edge with
 * (2^32 - thr_last) / 2^32.
 *   col_off   int64[n+1], col_off[0] = 0, non-decreasing, col_off[n] = m
 *   row_idx   int32[m] in [0,n)
 *   w         float[m] in [0,1]; each column's sum must be <= 1 + 2^-20
 *             (the LT constraint up to fp32 rounding)
 *   inputs_on_device  0: the three arrays are host pointers (validated on
 *             the host, then copied); 1: device pointers (validated by a
 *             kernel).  The caller may free them when the call returns.
 *   out       receives the handle (NULL on failure).
 * Errors: SIA_EINVAL (structure), SIA_EWEIGHTS (weights), SIA_ENOMEM,
 * SIA_EDEVICE.
 */
sia_status sia_graph_create(int64_t n, int64_t m, const int64_t *col_off,
                            const int32_t *row_idx, const float *w,
                            int inputs_on_device, void *hip_stream,
                            sia_graph **out);

/* Release a graph and all its device memory (NULL is a no-op). */
sia_status sia_graph_destroy(sia_graph *g);

/* n and m of a graph (either pointer may be NULL). */
sia_status sia_graph_info(const sia_graph *g, int64_t *n, int64_t *m);

/* Bytes of the per-in-edge record the graph was stored with: 16 when every
 * column carries the weights w = 1/d_in of its node (the setting of the
 * paper's experiments, Section 6.1), checked exactly on the quantised
 * weights at ingest -- the live in-edge then follows from the draw and the
 * in-degree alone; 32 otherwise (each record holds its threshold interval).
 * Results do not depend on it.  Test and reporting hook. */
sia_status sia_graph_arc_bytes(const sia_graph *g, uint32_t *arc_bytes);

/* Copy the threshold table thr[m] (see sia_graph_create) to host memory
 * thr_host (caller-allocated, m entries).  Test hook. */
sia_status sia_graph_thresholds(const sia_graph *g, uint32_t *thr_host, void *hip_stream);

/* Device conversion q[i] = round-half-even(w[i] * 2^32) for count values
 * (w, q device pointers; w in [0,1], other values give q = 0).  Exposes the
 * ingest kernel's conversion for exhaustive checks.  Test hook. */
sia_status sia_quantize(const float *w_dev, uint64_t *q_dev, uint64_t count, void *hip_stream);

/*
 * Sample HSAWs (Algorithm 1 semantics, Definition "self_walk"): for every
 * attempt a in [attempt_offset, attempt_offset + n_attempts): start at the
 * floor(x0 * |V\X| / 2^64)-th non-source node in ascending id order and
 * follow the live in-edge of each node until the walk reaches a source
 * (kept), finds no live edge (dead end) or returns to a node already on it
 * (cycle).  Kept walks go to *out (library-allocated host memory).
 *   sources    host pointer, see sia_check_query
 *   out        filled on success; free with sia_walks_free
 */
sia_status sia_sample(const sia_graph *g, int mode, const int32_t *sources,
                      int64_t n_sources, uint64_t n_attempts, uint64_t attempt_offset,
                      uint64_t seed, sia_walks *out, void *hip_stream);

/* Free the arrays of a sia_walks filled by sia_sample (NULL-safe). */
void sia_walks_free(sia_walks *w);

/*
 * Greedy max-coverage (Algorithm 4 / Algorithm 7) on given walks: k rounds,
 * each taking the id with the largest number of not-yet-covered walks
 * holding it (ties: lowest id), then covering those walks.  Rounds where
 * every gain is zero take the lowest id not yet selected, so exactly k ids
 * are returned.
 *   id_space   ids are in [0, id_space); 1 <= k <= id_space
 *   walk_off   host uint64[n_walks+1], ids host uint32[walk_off[n_walks]];
 *              each walk holds an id at most once
 *   selected   host int64[k] (out), gains host uint64[k] (out)
 */
sia_status sia_greedy(int64_t id_space, const uint64_t *walk_off, const uint32_t *ids,
                      uint64_t n_walks, int64_t k, int64_t *selected, uint64_t *gains,
                      void *hip_stream);

/*
 * sia_greedy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same greedy, the same answer, with every array in device memory and
 * no hipMalloc / hipFree.  The buffers its kernels need (walk lengths,
 * coverage counts, the greedy's state, pool, walk lists and counting
 * partition) come from one static device array of 64 MiB per device,
 * reserved while the library is loaded and shared by every call on that
 * device: calls that overlap on one device race and must be serialised by
 * the caller (each call starts from cleared state).
 *   id_space   ids are in [0, id_space); 1 <= k <= id_space
 *   walk_off   device uint64[n_walks+1] (walk_off[0] = 0, non-decreasing);
 *              ids device uint32[walk_off[n_walks]], each walk holding an id
 *              at most once
 *   selected   device int64[k] (out); gains device uint64[k] (out)
 * Limit: about 8.2 id_space + 10 n_ids + 16 n_walks + 16 k bytes plus 3 MB
 * of scratch must fit in 64 MiB (for example id_space = 10^6, 3.5 * 10^6
 * ids in 5 * 10^5 walks); larger inputs are rejected with SIA_EINVAL and a
 * message giving the bytes needed.  Malformed walks (decreasing offsets, an
 * id outside the id space): SIA_EINVAL.  Synchronises hip_stream (it reads
 * the walk count and the greedy's progress back to the host).
 */
sia_status sia_greedy_noalloc(int64_t id_space, const uint64_t *walk_off, const uint32_t *ids,
                              uint64_t n_walks, int64_t k, int64_t *selected, uint64_t *gains,
                              void *hip_stream);

/*
 * The whole hot path for one query (eSIA / nSIA with a fixed sample count):
 * sample as sia_sample, count coverage, greedy as sia_greedy over the kept
 * walks, and the estimates of Theorem "lem:rr_edge" / "lem:rr_node".
 *   selected   host int64[k] (out); gains host uint64[k] (out)
 *   stats      host (out, may be NULL)
 *   flags      SIA_FLAG_TIMING | SIA_FLAG_NO_CYCLE_STEPS (0: neither); other
 *              bits: SIA_EINVAL
 */
sia_status sia_solve(const sia_graph *g, int mode, const int32_t *sources,
                     int64_t n_sources, int64_t k, uint64_t n_attempts,
                     uint64_t attempt_offset, uint64_t seed, int64_t *selected,
                     uint64_t *gains, sia_stats *stats, int flags, void *hip_stream);

/*
 * sia_solve with a candidate set C (Definitions "edge_remove" /
 * "node_remove": the k ids are chosen from C within E or V; Algorithm 4 / 7
 * take the argmax over C minus the ids already chosen).  Coverage and the
 * estimates are as in sia_solve; ties go to the lowest candidate id, and
 * once every gain is zero the lowest unselected candidates follow.
 *   candidates  host int64[n_candidates]: distinct ids in [0, m) (edges) or
 *               [0, n) (nodes), any order; k <= n_candidates
 * Errors as sia_solve (SIA_EINVAL for a NULL, repeated or out-of-range
 * candidate, or fewer candidates than k).
 */
sia_status sia_solve_candidates(const sia_graph *g, int mode, const int32_t *sources,
                                int64_t n_sources, const int64_t *candidates,
                                int64_t n_candidates, int64_t k, uint64_t n_attempts,
                                uint64_t attempt_offset, uint64_t seed, int64_t *selected,
                                uint64_t *gains, sia_stats *stats, int flags,
                                void *hip_stream);

/*
 * Probabilistic suspects (Section 2.2: V_I = (V_I, p); a seed set X is drawn
 * with probability prod_{u in X} p(u) prod_{v in V_I \ X} (1 - p(v)),
 * equation "prob_src_set"; Algorithm 1's suspect test makes a suspect u met by
 * the walk a seed with probability p(u)).
 * Each attempt draws its own X: suspect x is a seed in attempt a when the
 * low 32 bits of x's draw word (word 0 of counter (x,0,0,0), whose high half
 * picks x's live in-edge) are below min(round-half-even(p(x) 2^32), 2^32-1).
 * The start is uniform over all of V, floor(x0 * n / 2^64); the walk stops
 * at the first seed it arrives at (the start included: a seed start gives the
 * walk <v_1> with no edge), at a node already on it, or where no in-edge is
 * live.  Estimates: I(V_I) ~ n hits / N, D(T) ~ n Cov(T) / N (Theorems
 * "lem:rr_edge" / "lem:rr_node").
 *   suspects  host int32[n_suspects], distinct, in [0,n); 1 <= n_suspects <= n
 *   p         host float[n_suspects] in [0,1] (NaN rejected)
 * Other arguments and outputs as sia_sample / sia_solve; stats.spread_est,
 * suspension_est and suspension_nodes_est follow the estimates above.
 * Errors as sia_sample / sia_solve (SIA_EINVAL for the suspects or p).
 */
sia_status sia_sample_suspects(const sia_graph *g, int mode, const int32_t *suspects, const float *p,
                               int64_t n_suspects, uint64_t n_attempts, uint64_t attempt_offset,
                               uint64_t seed, sia_walks *out, void *hip_stream);
sia_status sia_solve_suspects(const sia_graph *g, int mode, const int32_t *suspects, const float *p,
                              int64_t n_suspects, int64_t k, uint64_t n_attempts, uint64_t attempt_offset,
                              uint64_t seed, int64_t *selected, uint64_t *gains, sia_stats *stats,
                              int flags, void *hip_stream);

/* Figures of a Stop-and-Stare run (sia_sas_solve). */
typedef struct {
    int32_t status;        /* 1: Check passed at iteration t; 0: |R_t| reached
                              N_max first; -1: max_attempts ran out first */
    int32_t t;             /* iterations run (the last one's figures follow) */
    uint64_t n_t;          /* |R_t| = |R'_t| = ceil(Lambda * 2^(t-1)) HSAWs */
    uint64_t attempts_r;   /* R_t = the HSAWs of attempts [0, attempts_r) */
    uint64_t attempts_rp;  /* R'_t = the HSAWs of attempts [attempts_r, attempts_rp) */
    uint64_t cov_r;        /* Cov_{R_t}(selected) = sum of the gains */
    uint64_t cov_rp;       /* Cov_{R'_t}(selected): walks of R'_t holding a selected id */
    uint64_t attempts_sampled; /* attempts the driver sampled in all */
    double eps_t;          /* Check's bound at the last iteration (NaN when
                              Cov_{R'_t} < Lambda_1, where it is not formed) */
    double lambda;         /* equation "lambda" */
    double lambda1;        /* equation "lambda_1" */
    double n_max;          /* equation "guard" (edges) / "nguard" (nodes) */
    int32_t t_max;         /* ceil(log2(2 N_max / Upsilon(eps, delta/3))) */
    int32_t reserved;
    double spread_est;     /* |X| + |V\X| * n_t / attempts_r */
    double suspension_est; /* |V\X| * cov_r / attempts_r */
    double suspension_nodes_est; /* suspension_est + |selected & X| (nodes) */
    float ms_total;        /* wall time of the call */
    float reserved2;
} sia_sas_info;

/*
 * eSIA (Algorithm 6, mode SIA_EDGES) / nSIA (Algorithm 9, SIA_NODES): the
 * Stop-and-Stare driver over the hot path.  The HSAW stream R_1, R_2, ...
 * is the kept walks in attempt-id order (attempts 0, 1, 2, ... of seed).
 * Iteration t takes the first N_t = ceil(Lambda 2^(t-1)) HSAWs as R_t and
 * the next N_t as R'_t, picks k ids by the greedy on R_t and verifies them
 * on R'_t with Check (Algorithm 5 / 8); it stops when Check passes or
 * N_t >= N_max.  t_max reads the iteration lemma's Upsilon(eps, delta/3)
 * (the displayed formula takes the logarithm of delta/3); the parameters
 * and Check are those of sia_sas_params and sia_sas_check.  The driver
 * samples the attempts [0, end) once, in growing chunks, into a device
 * store of kept walks; a walk is a function of its attempt id, so R_t is
 * the stored walks with attempt id below a bound A and R'_t those in
 * [A, A'), the bounds being the N_t-th and 2 N_t-th smallest stored
 * attempt ids plus one.  Walks are never sampled twice.
 *   eps        in (0, 1 - 1/e); delta in (0, 1) (the paper uses 1/n)
 *   max_attempts  in [1, 2^32): the attempts the stream may use
 *   selected   host int64[k] (out), gains host uint64[k] (out): the last
 *              iteration's candidate; not written when status is -1 (then
 *              info holds status, t and n_t of the iteration that could not
 *              get its 2 N_t HSAWs, the parameters and attempts_sampled)
 *   info       host (out)
 * Errors as sia_solve.
 */
sia_status sia_sas_solve(const sia_graph *g, int mode, const int32_t *sources,
                         int64_t n_sources, int64_t k, double eps, double delta,
                         uint64_t seed, uint64_t max_attempts, int64_t *selected,
                         uint64_t *gains, sia_sas_info *info, void *hip_stream);

/* sia_sas_solve with probabilistic suspects (suspects and p as in
 * sia_sample_suspects): the HSAW stream is the kept walks of attempts
 * 0, 1, 2, ... with a start uniform over V; spread_est = n n_t / attempts_r,
 * suspension_est = suspension_nodes_est = n cov_r / attempts_r. */
sia_status sia_sas_solve_suspects(const sia_graph *g, int mode, const int32_t *suspects, const float *p,
                                  int64_t n_suspects, int64_t k, double eps, double delta, uint64_t seed,
                                  uint64_t max_attempts, int64_t *selected, uint64_t *gains,
                                  sia_sas_info *info, void *hip_stream);

/*
 * The parameters sia_sas_solve uses, for id space S = id_space (m for
 * edges, equation "guard"; n for nodes, equation "nguard"), budget k,
 * eps in (0, 1 - 1/e) and delta in (0, 1):
 *   n_max   = (2 - 1/e)^2 (2 + 2eps/3) S (ln(6/delta) + ln C(S,k)) / (k eps^2)
 *   t_max   = ceil(log2(2 n_max / Upsilon)), Upsilon = (2 + 2eps/3) ln(3/delta) / eps^2
 *             (the lemma bounding the iterations), at least 1
 *   lambda  = (2 + 2eps/3) ln(3 t_max / delta) / eps^2        (equation "lambda")
 *   lambda1 = 1 + (1 + eps) lambda                            (equation "lambda_1")
 * ln C(S,k) is taken through lgamma in double precision.  Host arithmetic
 * only (no device work); every output pointer may be NULL.  Errors:
 * SIA_EINVAL (k outside [1, id_space], eps or delta out of range).
 */
sia_status sia_sas_params(int64_t id_space, int64_t k, double eps, double delta, double *lambda,
                          double *lambda1, double *n_max, int32_t *t_max);

/*
 * Check (Algorithm 5 / 8) as sia_sas_solve evaluates it at iteration t:
 * with Cov' = cov_rp the coverage on R'_t, |R'_t| = n_rp, Cov = cov_r the
 * coverage on R_t and s = n_rp (1 + eps) / (2^(t-1) Cov'):
 *   eps_1 = Cov / Cov' - 1,  eps_2 = eps sqrt(s),
 *   eps_3 = eps sqrt(s (1 - 1/e - eps) / (1 + eps/3)),
 *   eps_t = (eps_1 + eps_2 + eps_1 eps_2)(1 - 1/e - eps) + (1 - 1/e) eps_3.
 *   terms   host double[4] (out): eps_1, eps_2, eps_3, eps_t; all NaN when
 *           Cov' < lambda1 (Check then fails without forming them)
 *   passed  host (out): 1 when Cov' >= lambda1 and eps_t <= eps, else 0
 * Host arithmetic only.  Errors: SIA_EINVAL (NULL output, t outside
 * [1, 1024), cov_rp or n_rp not positive, cov_r negative, eps out of
 * range).
 */
sia_status sia_sas_check(double cov_r, double cov_rp, double n_rp, int32_t t, double eps, double lambda1,
                         double *terms, int32_t *passed);

/*
 * Evaluate a chosen set on its own sample (the out-of-sample estimate the
 * experiments use to score solutions, Section 6.1, here from HSAWs instead
 * of the external estimator the paper cites): sample attempts
 * [attempt_offset, attempt_offset + n_attempts) of seed as sia_sample and
 * count the kept walks holding at least one selected id.
 *   selected  host int64[k] ids in [0, m) (edges) or [0, n) (nodes)
 *   stats     host (out): the sampler's counters, covered = walks hit by the
 *             set, and the estimates of sia_solve (suspension_est =
 *             |V\X| * covered / N); times are 0
 * Errors as sia_solve.
 */
sia_status sia_evaluate(const sia_graph *g, int mode, const int32_t *sources,
                        int64_t n_sources, const int64_t *selected, int64_t k,
                        uint64_t n_attempts, uint64_t attempt_offset, uint64_t seed,
                        sia_stats *stats, void *hip_stream);

/*
 * Measuring hook (not part of the method): the device's random-gather
 * ceiling.  Fills a device array of array_bytes (1 MiB .. 16 GiB) and times
 * one launch, at full occupancy, in which every lane makes loads_per_lane
 * 4-byte loads at pseudo-random positions (each its own 128-byte line):
 * independent loads (dependent = 0) or a chain where each load's value is
 * the next position (dependent != 0, a walk's access pattern).
 *   lines_per_s  out: loads (lines) completed per second
 *   ms           out (may be NULL): launch time
 * The array is freed before returning.  Errors: SIA_EINVAL, SIA_ENOMEM,
 * SIA_EDEVICE.
 */
sia_status sia_probe_gather(uint64_t array_bytes, uint32_t loads_per_lane, int dependent,
                            double *lines_per_s, double *ms, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched and served queries.  Not part of the paper's method (which runs
 * one query per launch); the answers are identical to sia_solve's for the
 * same query.
 *
 * A batch owns up to 31 query slots on one graph.  Queries are submitted at
 * any time and admitted in arrival order as a slot and walk-buffer memory
 * become free.  Every sampling launch takes a share of the attempts of every
 * admitted query (one persistent launch, queries told apart by a per-slot
 * source tag bit in the node records); a query whose attempts are all
 * sampled moves to the greedy, which runs the greedies of all such queries
 * in shared launches, either between sampling launches (default) or on a
 * second stream beside them.  Host threads of the batch drive the device;
 * the calls below only queue work and read results, and are safe from any
 * thread.
 *
 * Walk buffers: each slot keeps its kept walks (20 bytes per walk + 4 per
 * id) in device memory counted against walk_budget_bytes.  A launch gives a
 * query at most the share its buffer has room for (estimated from the rates
 * seen so far); a share whose walks outgrow the buffer is discarded and
 * sampled again with a buffer of the exact size, so results never depend on
 * the budget.  The greedy's index (about 12 bytes per id of the id space per
 * running greedy) is outside the budget.
 * ---------------------------------------------------------------------- */
typedef struct sia_batch sia_batch; /* opaque */

/* One query: the arguments of sia_solve. */
typedef struct {
    int32_t mode;            /* SIA_EDGES or SIA_NODES */
    int32_t flags;           /* 0 or SIA_FLAG_NO_CYCLE_STEPS */
    const int32_t *sources;  /* host; copied by sia_batch_submit */
    int64_t n_sources;
    int64_t k;               /* >= 1 */
    uint64_t n_attempts;
    uint64_t attempt_offset;
    uint64_t seed;
} sia_query;

/* Launch shape of a batch (0 in any field = the default). */
typedef struct {
    int32_t sampler_blocks_per_cu; /* persistent sampler workgroups per CU
                                      (default: as many as fit) */
    uint32_t refill_chunk;         /* attempts a sampler wave takes per refill
                                      (default 256) */
    uint64_t wave_attempts;        /* attempts per sampling launch, shared by
                                      the admitted queries (default 2^23) */
    uint64_t min_share;            /* smallest share of a launch one query
                                      gets (default 2^16) */
    int32_t use_graph;             /* nonzero: each sampling launch is a replay
                                      of one captured hipGraph (table and
                                      counter uploads, kernel, read-back) */
    int32_t greedy_mode;           /* 0: time-sliced -- the greedy of finished
                                      queries runs between sampling launches
                                      in batches of greedy_batch (sooner when
                                      sampling would wait for it); 1:
                                      concurrent -- a second thread runs each
                                      finished query's greedy at once on its
                                      own stream, beside the sampling */
    int32_t greedy_cus;            /* greedy_mode 1 only: CUs given to the
                                      greedy stream alone (CU-masked streams;
                                      the sampler gets the rest); 0: both
                                      streams use every CU */
    uint32_t greedy_batch;         /* greedy_mode 0: finished queries per
                                      greedy launch (default 32) */
    uint32_t hist_blocks;          /* histogram tiling of the greedy's pool
                                      rebuilds: workgroups for one query's
                                      histogram (default: one per CU) */
} sia_batch_config;

/* Timeline of one query, in seconds since sia_batch_create (host steady
 * clock). */
typedef struct {
    double t_submit;
    double t_admit;    /* took a slot */
    double t_sampled;  /* last share sampled */
    double t_done;     /* greedy finished */
    uint32_t waves;    /* sampling launches it took part in */
    uint32_t reruns;   /* shares sampled again after outgrowing the buffer */
} sia_ticket_info;

/* Counters of a batch. */
typedef struct {
    uint64_t submitted, completed, failed, cancelled;
    uint64_t waves;           /* sampling launches */
    uint64_t graph_replays;   /* of those, replays of the captured graph */
    uint64_t greedy_launches; /* shared greedy runs */
    uint64_t greedy_jobs;     /* queries they served */
    uint64_t reruns;
    uint64_t evictions;       /* queries restarted to free walk memory */
    uint64_t walk_bytes;      /* walk-buffer memory held now */
    uint64_t walk_bytes_peak;
    uint64_t walk_budget;
    uint32_t slots, busy_slots, pending, reserved;
    double sample_busy_s;     /* host wall time inside sampling launches */
    double greedy_busy_s;     /* host wall time inside greedy launches */
    double greedy_index_s;    /* of which: device time of counts + index */
    sia_batch_config config;  /* the shape in use */
} sia_batch_stats;

/*
 * Create a batch on graph g (whose device must be current or is made
 * current for the batch's threads).
 *   walk_budget_bytes  device memory for walk buffers (>= 1 MiB)
 *   max_slots          1..31 concurrent queries; takes that many source-tag
 *                      bits of the graph (SIA_EBUSY if other batches hold
 *                      them).  sia_solve on the same graph stays available.
 *   config             NULL for defaults
 * The graph must outlive the batch.
 */
sia_status sia_batch_create(const sia_graph *g, uint64_t walk_budget_bytes, int32_t max_slots,
                            const sia_batch_config *config, sia_batch **out);

/* Stop the batch (queries not finished are dropped), join its threads and
 * free its memory.  NULL is a no-op. */
sia_status sia_batch_destroy(sia_batch *b);

/* Queue a query; *ticket identifies it.  The query is checked as in
 * sia_check_query (SIA_EINVAL, nothing queued). */
sia_status sia_batch_submit(sia_batch *b, const sia_query *q, uint64_t *ticket);

/*
 * Result of a ticket.  SIA_ENOTREADY while it runs.  Once finished the
 * outputs are filled (selected / gains: host arrays of the query's k
 * entries; stats, info may be NULL), the ticket is released and the
 * query's status is returned: SIA_OK, SIA_ECANCELLED, or the error that
 * ended it (message via sia_last_error).  Unknown ticket: SIA_EINVAL.
 */
sia_status sia_batch_poll(sia_batch *b, uint64_t ticket, int64_t *selected, uint64_t *gains,
                          sia_stats *stats, sia_ticket_info *info);

/* As sia_batch_poll, blocking up to timeout_ms (< 0: no limit). */
sia_status sia_batch_wait(sia_batch *b, uint64_t ticket, int64_t timeout_ms, int64_t *selected,
                          uint64_t *gains, sia_stats *stats, sia_ticket_info *info);

/* Cancel a ticket: a queued query leaves at once, a sampling one at the end
 * of the current launch, a query in the greedy when the greedy ends.  Its
 * poll then returns SIA_ECANCELLED.  Finished or unknown tickets:
 * SIA_EINVAL. */
sia_status sia_batch_cancel(sia_batch *b, uint64_t ticket);

/* Counters and the launch shape in use. */
sia_status sia_batch_stats_get(sia_batch *b, sia_batch_stats *out);

/*
 * Autotune the launch shapes on a probe query: sample its attempts once per
 * candidate (workgroups per CU x refill chunk), with the probe's flags (set
 * SIA_FLAG_NO_CYCLE_STEPS when the queries to be served will), and keep the
 * fastest; size
 * wave_attempts for launches of about target_ms; then run the greedy on the
 * probe's walks (k = the probe's k, or 1000 if 0) once per histogram tiling
 * candidate and keep the fastest.  The batch must be idle (no unfinished
 * ticket), else SIA_EBUSY.  *chosen (may be NULL) receives the new shape.
 */
sia_status sia_batch_tune(sia_batch *b, const sia_query *probe, double target_ms,
                          sia_batch_config *chosen);

#ifdef __cplusplus
}
#endif
#endif /* SIA_H */
