// Coverage counts and greedy max-coverage (Algorithm 4 for edges, Algorithm 7
// for nodes) over the kept walks of one or more queries ("jobs").
//
//   cnt[id] = number of not-yet-covered walks holding id (Cov of one id),
//             exact between launches of the rounds kernel (inside one, the
//             pool's counts are kept in LDS and the walks it covers are taken
//             off cnt after it ends); 0xFFFFFFFF once id is selected;
//   key(id) = ((cnt+1) << 32) | (2^32-1-id) for an unselected id, 0 once
//             selected: the largest key is the largest marginal gain with the
//             lowest id on ties, and once every gain is zero the lowest id not
//             selected yet (exactly k picks).
//
// Lazy greedy.  Covering walks only lowers counts, so a key computed once is
// an upper bound forever.  A pool holds the ids whose keys may be the
// largest, and tau bounds the key of every id outside the pool.  One
// workgroup per job runs rounds back to back: take the pool's keys from its
// exact counts, and while the best exceeds tau it is the true argmax of the
// round -- record it, mark its walks covered and decrement the counts of
// their pool ids.  When the best no longer exceeds tau, grid-wide kernels rebuild
// the pool from the current counts: a histogram of counts, read on the
// device, chooses the threshold, and ties at the threshold are taken by
// ascending id (ordered compaction).  The result is exactly the greedy of
// Algorithm 4 / 7.
//
// Walk lists.  Covering needs the walks holding the chosen id, and only pool
// ids can be chosen, so with each pool the lists of its ids that still hold
// uncovered walks are built (a bitmap marks them; one pass over the
// uncovered walks appends each walk to the lists of its marked ids), and
// their transpose: for each listed walk, the pool positions of its ids, so
// that covering a walk touches only its pool ids.  No inverted index over
// the whole id space is built.
//
// Every kernel takes the job table; blockIdx.y (blockIdx.x for the
// one-workgroup kernels) selects the job, so the greedies of a batch of
// queries advance in the same launches, and a job that is finished returns
// at once.
#include "common.hpp"

#include <algorithm>
#include <cstddef>

namespace sia {

namespace {

constexpr int kWave = 64;
constexpr uint32_t kSelected = 0xFFFFFFFFu;
constexpr uint32_t kScanTile = 4096;  // 256 threads x 16

// Count histogram: counts 0..4095 exactly; above, 512 bins per octave.
constexpr uint32_t kExact = 4096;
constexpr uint32_t kPerOctave = 512;
constexpr uint32_t kBins = kExact + 20 * kPerOctave;  // octaves 2^12 .. 2^31
constexpr uint32_t kPoolTarget = 4096;
constexpr uint32_t kPoolMax = 8192;        // the lazy rounds keep the pool in LDS
constexpr uint32_t kFilterBits = 17;       // LDS bit filter of pool ids (false positives <= 1/16)
// Coverage counting by id ranges (k_bin_sort .. k_bin_count): fine bins of
// 2^kCountSpanLog ids (the LDS counters of one workgroup); up to
// kCountTilesMax tiles of the walk ids.
constexpr uint32_t kCountSpanLog = 14;  // LDS counters of one counting pass
constexpr uint32_t kCountSpan = 1u << kCountSpanLog;
constexpr uint32_t kCountTilesMax = 512;
constexpr uint64_t kCountTileMin = 32768;
constexpr uint32_t kCoarseLog = 8;          // first level: at most 256 coarse bins
constexpr uint32_t kCoarseMax = 1u << kCoarseLog;
constexpr uint32_t kFineLog = 10;           // fine bins per coarse bin: id spaces up to 2^32
constexpr uint32_t kFineMax = 1u << kFineLog;
constexpr uint32_t kChunk = 8192;           // second level: ids sorted per LDS chunk
static_assert(kCountSpanLog + kCoarseLog + kFineLog >= 32, "two levels span a 32-bit id space");
constexpr uint32_t kFilterWords = (1u << kFilterBits) / 32;

enum PlanKind : uint32_t { PLAN_COLLECT = 0, PLAN_TIES = 1, PLAN_REFINE = 2 };
// An overfull wide bin (one above the exact counts) is split by one or two
// further histograms of its own counts, kRefineBins sub-bins each.
constexpr uint32_t kRefineLog = 13;
constexpr uint32_t kRefineBins = 1u << kRefineLog;

// Per-job state, written by the plan / collect / lazy kernels.
struct GreedyState {
    uint32_t rounds;    // rounds completed so far
    uint32_t error;     // nonzero: the job stopped (no valid input sets it)
    uint32_t plan;      // PlanKind of the current pool
    uint32_t c_min;     // pool holds every unselected id with cnt >= c_min (0: none)
    uint32_t pool_n;    // ids collected that way
    uint32_t c_tie;     // PLAN_TIES: the tied count
    uint32_t n_tie;     // PLAN_TIES: tied ids taken, lowest ids first
    uint32_t leftover;  // PLAN_TIES: tied ids were left out
    uint32_t next_id;   // PLAN_TIES: lowest tied id left out
    uint32_t plist_total;  // ids' list entries of the current pool
    uint64_t tau;       // bound on keys outside the pool (without left-out ties)
    uint32_t n_claimed;     // walks covered so far (entries of the claimed list)
    uint32_t claimed_done;  // of them, already taken off the global counts
    uint32_t marked;        // rounds whose picks are marked selected in the global counts
    uint32_t r_lo;          // PLAN_REFINE: lowest count of the range being split
    uint32_t r_shift;       //   sub-bins of 2^r_shift counts
    uint32_t r_nbins;       //   sub-bins covering the range (<= kRefineBins)
    uint32_t r_above;       //   unselected ids with a count above the range
    uint32_t wp_total;      // entries of the per-walk pool lists handed out so far
};

static_assert(sizeof(GreedyState) % 8 == 0, "GreedyState is cleared in 8-byte words");

struct GreedyJob {
    uint32_t *cnt;
    uint32_t *pidx;     // id_space: pool position of a marked id
    uint32_t *plist;    // n_ids: walk lists of the marked pool ids
    uint32_t *pstart;   // kPoolMax + 1: list starts (pool order)
    uint32_t *pfill;    // kPoolMax: list fill counters
    uint32_t *bitmap;   // ceil(id_space / 32): marked ids
    uint32_t *claimed;  // n_walks: covered walks in the order they were covered
    uint64_t *wst;      // n_walks: walk state, see kCovered
    uint16_t *wpool;    // n_ids: pool positions of the listed walks' marked ids, walk by walk
    const uint64_t *walk_off;
    const uint32_t *walk_len;
    const uint32_t *ids;
    uint64_t S;         // id space
    uint64_t n_walks;
    uint64_t n_ids;
    int64_t k;
    uint32_t c_rbits;   // counting: ids per bin = 2^c_rbits
    uint32_t c_bins;    // counting: bins over [0, S)
    uint32_t c_fbits;   // counting: fine bins per coarse bin = 2^c_fbits
    uint32_t c_coarse;  // counting: coarse bins
    uint32_t c_tiles;   // counting: tiles of the walk ids
    uint32_t c_parts;   // counting: workgroups per fine bin (> 1: they add into cnt)
    uint32_t c_chunks_max;  // counting: bound on the chunks of all coarse bins
    uint32_t c_pad;
    uint64_t c_tile_len;
    uint32_t *coffs;    // c_tiles x (c_coarse + 1): where each tile's coarse bins start in plist
    uint32_t *ctab;     // c_coarse x c_tiles pairs: segment start in the bin, in plist
    uint32_t *cn;       // c_coarse: ids per coarse bin
    uint32_t *cchunk;   // c_coarse + 1: first chunk of each coarse bin
    uint32_t *coffs2;   // c_chunks_max x (2^c_fbits + 1): fine-bin starts in a chunk
    uint32_t *cbuf;     // c_chunks_max x kChunk: chunks sorted by fine bin
    const uint32_t *cand;  // candidate bitmap over [0, S) (NULL: every id)
    int64_t *sel;       // k
    uint64_t *gain;     // k
    uint32_t *hist;     // kBins
    uint32_t *pool;     // kPoolMax
    uint32_t *tiles;    // ceil(S / kScanTile)
    GreedyState *st;
};

// Device view of a job with its arrays in the global address space (see gp).

struct GJob {
    GLOBAL uint32_t *cnt;
    GLOBAL uint32_t *pidx;
    GLOBAL uint32_t *plist;
    GLOBAL uint32_t *pstart;
    GLOBAL uint32_t *pfill;
    GLOBAL uint32_t *bitmap;
    GLOBAL uint32_t *claimed;
    GLOBAL uint64_t *wst;
    GLOBAL uint16_t *wpool;
    const GLOBAL uint64_t *walk_off;
    const GLOBAL uint32_t *walk_len;
    const GLOBAL uint32_t *ids;
    uint64_t S, n_walks, n_ids;
    int64_t k;
    uint32_t c_rbits, c_bins, c_fbits, c_coarse, c_tiles, c_parts, c_chunks_max;
    uint64_t c_tile_len;
    GLOBAL uint32_t *coffs;
    GLOBAL uint32_t *ctab;
    GLOBAL uint32_t *cn;
    GLOBAL uint32_t *cchunk;
    GLOBAL uint32_t *coffs2;
    GLOBAL uint32_t *cbuf;
    const GLOBAL uint32_t *cand;
    GLOBAL int64_t *sel;
    GLOBAL uint64_t *gain;
    GLOBAL uint32_t *hist;
    GLOBAL uint32_t *pool;
    GLOBAL uint32_t *tiles;
    GLOBAL GreedyState *st;
};

__device__ __forceinline__ GJob view(const GreedyJob &j)
{
    GJob J;
    J.cnt = gp(j.cnt);
    J.pidx = gp(j.pidx);
    J.plist = gp(j.plist);
    J.pstart = gp(j.pstart);
    J.pfill = gp(j.pfill);
    J.bitmap = gp(j.bitmap);
    J.claimed = gp(j.claimed);
    J.wst = gp(j.wst);
    J.wpool = gp(j.wpool);
    J.walk_off = gp(j.walk_off);
    J.walk_len = gp(j.walk_len);
    J.ids = gp(j.ids);
    J.S = j.S;
    J.n_walks = j.n_walks;
    J.n_ids = j.n_ids;
    J.k = j.k;
    J.c_rbits = j.c_rbits;
    J.c_bins = j.c_bins;
    J.c_fbits = j.c_fbits;
    J.c_coarse = j.c_coarse;
    J.c_tiles = j.c_tiles;
    J.c_parts = j.c_parts;
    J.c_chunks_max = j.c_chunks_max;
    J.c_tile_len = j.c_tile_len;
    J.coffs = gp(j.coffs);
    J.ctab = gp(j.ctab);
    J.cn = gp(j.cn);
    J.cchunk = gp(j.cchunk);
    J.coffs2 = gp(j.coffs2);
    J.cbuf = gp(j.cbuf);
    J.cand = j.cand ? gp(j.cand) : nullptr;
    J.sel = gp(j.sel);
    J.gain = gp(j.gain);
    J.hist = gp(j.hist);
    J.pool = gp(j.pool);
    J.tiles = gp(j.tiles);
    J.st = gp(j.st);
    return J;
}

// agent-scope relaxed atomics on global memory
__device__ __forceinline__ uint32_t g_add(GLOBAL uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t g_or(GLOBAL uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t g_and(GLOBAL uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t g_add64(GLOBAL uint64_t *p, uint64_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t g_or64(GLOBAL uint64_t *p, uint64_t v)
{
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t g_and64(GLOBAL uint64_t *p, uint64_t v)
{
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Walk state, one 64-bit word per walk, so that one atomic claims a walk and
// returns its pool list: bit 63 the walk is covered; bits 32..62 the marked
// pool ids it holds (0 for walks in no list); bits 0..31 the end of its pool
// positions in wpool (their start until the lists are filled).
constexpr uint64_t kCovered = 1ull << 63;
constexpr uint64_t kWsCountOne = 1ull << 32;
__device__ __forceinline__ uint32_t ws_count(uint64_t s) { return static_cast<uint32_t>(s >> 32) & 0x7FFFFFFFu; }

__device__ __forceinline__ uint32_t count_bin(uint32_t c)
{
    if (c < kExact) return c;
    const uint32_t L = 32u - __clz(c);  // bit length, 13..32
    return kExact + (L - 13u) * kPerOctave + ((c >> (L - 10u)) & (kPerOctave - 1u));
}

// lowest count of bin b
__device__ __forceinline__ uint64_t bin_lo(uint32_t b)
{
    if (b < kExact) return b;
    const uint32_t o = (b - kExact) / kPerOctave, r = (b - kExact) % kPerOctave;
    const uint32_t L = o + 13;  // bit length
    return (static_cast<uint64_t>(kPerOctave + r)) << (L - 10);
}

__device__ __forceinline__ uint64_t key_of(uint32_t c, uint32_t id)
{
    return c == kSelected ? 0ull : ((static_cast<uint64_t>(c) + 1ull) << 32) | (0xFFFFFFFFu - id);
}

__device__ __forceinline__ bool job_done(const GJob &J)
{
    return J.st->error != 0 || static_cast<int64_t>(J.st->rounds) >= J.k;
}

__device__ __forceinline__ uint64_t n_tiles_of(uint64_t S) { return (S + kScanTile - 1) / kScanTile; }

__device__ __forceinline__ uint32_t pool_size(const GLOBAL GreedyState *st)
{
    return st->pool_n + (st->plan == PLAN_TIES ? st->n_tie : 0u);
}

// block-wide exclusive scan of one value per thread (T threads; sh holds T/64)
template <int T>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    constexpr int W = T / kWave;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(x, d, kWave);
        if (lane >= d) x += o;
    }
    if (lane == kWave - 1) sh[wid] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int k = 0; k < W; ++k) {
        if (k < wid) before += sh[k];
        total += sh[k];
    }
    __syncthreads();
    return before + x - v;
}

__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *sh, uint32_t &total)
{
    return block_excl_scan<256>(v, sh, total);
}

// exclusive scan of tiles[0 .. n) in place, one 256-thread workgroup
__device__ void scan_tiles_256(GLOBAL uint32_t *tiles, uint64_t n)
{
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (uint64_t base = 0; base < n; base += 256) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < n ? tiles[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan_256(v, sh, total);
        if (i < n) tiles[i] = carry + ex;
        carry += total;
    }
}

// ---------------------------------------------------------------- set-up
// Zero the per-job state, histogram, walk states and, when the counting
// pass adds partial counts, the counts (else it writes every count).  A
// kernel rather than memsets, so a captured graph holds no memset nodes.
__global__ void k_init(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    const uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = t; i < J.n_walks; i += stride) J.wst[i] = 0;
    if (J.c_parts > 1)
        for (uint64_t i = t; i < J.S; i += stride) J.cnt[i] = 0;
    for (uint64_t i = t; i < kBins; i += stride) J.hist[i] = 0;
    for (uint64_t i = t; i < (J.S + 31) / 32; i += stride) J.bitmap[i] = 0;
    if (t == 0) {
        GLOBAL uint64_t *w = reinterpret_cast<GLOBAL uint64_t *>(J.st);
        for (uint32_t i = 0; i < sizeof(GreedyState) / 8; ++i) w[i] = 0;
    }
}

// ---------------------------------------------------------------- coverage counts
// cnt[id] = number of kept walks holding id (the initial Cov of each id),
// taken without global atomics: random atomics over an id space of 10^8 ids
// and more miss every cache.  The id space is cut into fine bins of 2^rbits
// ids (one LDS pass each for id spaces up to 2^32), grouped into at most
// kCoarseMax coarse bins of 2^fbits fine bins.  The ids are partitioned in
// two levels, each narrow enough that the lines being written stay in L2
// until they are whole (a single 2^14-way scatter wrote every 4-byte id as a
// separate partial line):
//   k_bin_sort   each tile of the walk ids is split by coarse bin into plist
//                (unused until the first pool is filled); coffs records where
//                each of the tile's coarse bins starts;
//   k_bin_plan   per coarse bin: where its segment of each tile starts in the
//                bin's concatenation (ctab) and its size (cn);
//   k_bin_bases  chunks of kChunk ids per coarse bin, numbered (cchunk);
//   k_bin_sort2  each chunk is sorted by fine bin in LDS and written whole
//                to its kChunk slots of cbuf; coffs2 records the fine bins;
//   k_bin_count  one workgroup per fine bin counts its run of every chunk of
//                its coarse bin in LDS (kCountSpan ids per pass) and writes
//                the count of every id of the bin, so cnt needs no clearing.
//                When the fine bins are too few to fill the GPU, each bin's
//                chunks are split among c_parts workgroups that add their
//                counts (cnt is then cleared by k_init).

// last index i in [0, n) with pre[i] <= x (pre ascending, pre[0] <= x)
__device__ __forceinline__ uint32_t last_le(const uint32_t *pre, uint32_t n, uint32_t x)
{
    uint32_t a = 0, z = n;
    while (z - a > 1) {
        const uint32_t m = (a + z) >> 1;
        if (pre[m] <= x) a = m;
        else z = m;
    }
    return a;
}

template <int T>
__global__ __launch_bounds__(T) void k_bin_sort(const GreedyJob *jobs)
{
    constexpr int U = 8;  // loads in flight per lane
    static_assert(kCoarseMax <= T, "one coarse bin per thread");
    __shared__ uint32_t h[kCoarseMax];
    __shared__ uint32_t sh[T / kWave];
    const GJob J = view(jobs[blockIdx.y]);
    const uint32_t w = blockIdx.x;
    if (w >= J.c_tiles) return;  // uniform per block
    const uint64_t lo = min(J.n_ids, w * J.c_tile_len), hi = min(J.n_ids, lo + J.c_tile_len);
    const uint32_t C = J.c_coarse, sft = J.c_rbits + J.c_fbits;
    if (threadIdx.x < kCoarseMax) h[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += U * T) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = i + u * T < hi ? J.ids[i + u * T] : 0u;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * T < hi) atomicAdd(&h[v[u] >> sft], 1u);
    }
    __syncthreads();
    const uint32_t mine = threadIdx.x < C ? h[threadIdx.x] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<T>(mine, sh, total);  // ends with a barrier
    GLOBAL uint32_t *offs = J.coffs + static_cast<uint64_t>(w) * (C + 1);
    if (threadIdx.x < C) {
        h[threadIdx.x] = ex;
        offs[threadIdx.x] = static_cast<uint32_t>(lo) + ex;
    }
    if (threadIdx.x == 0) offs[C] = static_cast<uint32_t>(hi);
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += U * T) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = i + u * T < hi ? J.ids[i + u * T] : 0u;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u * T < hi) J.plist[lo + atomicAdd(&h[v[u] >> sft], 1u)] = v[u];
    }
}

template <int T>
__global__ __launch_bounds__(T) void k_bin_plan(const GreedyJob *jobs)
{
    static_assert(kCountTilesMax <= T, "one tile per thread");
    __shared__ uint32_t sh[T / kWave];
    const GJob J = view(jobs[blockIdx.y]);
    const uint32_t c = blockIdx.x;
    if (c >= J.c_coarse) return;  // uniform per block
    const uint32_t nt = J.c_tiles, C = J.c_coarse;
    uint32_t len = 0, at = 0;
    if (threadIdx.x < nt) {
        const GLOBAL uint32_t *o = J.coffs + static_cast<uint64_t>(threadIdx.x) * (C + 1) + c;
        at = o[0];
        len = o[1] - at;
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan<T>(len, sh, total);
    if (threadIdx.x < nt) {
        GLOBAL uint32_t *row = J.ctab + 2ull * (static_cast<uint64_t>(c) * nt + threadIdx.x);
        row[0] = ex;  // start in the coarse bin's concatenation
        row[1] = at;  // start in plist
    }
    if (threadIdx.x == 0) J.cn[c] = total;
}

template <int T>
__global__ __launch_bounds__(T) void k_bin_bases(const GreedyJob *jobs)
{
    static_assert(kCoarseMax <= T, "one coarse bin per thread");
    __shared__ uint32_t sh[T / kWave];
    const GJob J = view(jobs[blockIdx.y]);
    const uint32_t C = J.c_coarse;
    const uint32_t n = threadIdx.x < C ? (J.cn[threadIdx.x] + kChunk - 1) / kChunk : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_scan<T>(n, sh, total);
    if (threadIdx.x < C) J.cchunk[threadIdx.x] = ex;
    if (threadIdx.x == 0) J.cchunk[C] = total;
}

template <int T>
__global__ __launch_bounds__(T) void k_bin_sort2(const GreedyJob *jobs)
{
    constexpr int U = kChunk / T;  // every load of the chunk in flight at once
    static_assert(kChunk % T == 0 && kFineMax % T == 0, "chunk and fine bins per thread");
    __shared__ uint32_t vpre[kCountTilesMax], vphys[kCountTilesMax];
    __shared__ uint32_t base[kCoarseMax + 1];
    __shared__ uint32_t fh[kFineMax];
    __shared__ uint32_t wr[2];  // tiles holding the chunk's first and last id
    __shared__ uint32_t sh[T / kWave];
    const GJob J = view(jobs[blockIdx.y]);
    const uint32_t g = blockIdx.x;
    if (g >= J.c_chunks_max) return;  // uniform per block
    const uint32_t C = J.c_coarse, nt = J.c_tiles, F = 1u << J.c_fbits;
    for (uint32_t t = threadIdx.x; t <= C; t += T) base[t] = J.cchunk[t];
    for (uint32_t f = threadIdx.x; f < kFineMax; f += T) fh[f] = 0;
    __syncthreads();
    if (g >= base[C]) return;  // uniform: past the last chunk
    const uint32_t c = last_le(base, C + 1, g);  // coarse bin of chunk g
    const uint32_t v0 = (g - base[c]) * kChunk;
    const uint32_t n = min(kChunk, J.cn[c] - v0);
    for (uint32_t t = threadIdx.x; t < nt; t += T) {
        const GLOBAL uint32_t *row = J.ctab + 2ull * (static_cast<uint64_t>(c) * nt + t);
        vpre[t] = row[0];
        vphys[t] = row[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        wr[0] = last_le(vpre, nt, v0);
        wr[1] = last_le(vpre, nt, v0 + n - 1);
    }
    __syncthreads();
    // the chunk spans tiles w0 .. w1 of its coarse bin (a few, unless they are tiny)
    const uint32_t w0 = wr[0], nw = wr[1] - w0 + 1;
    const uint32_t rb = J.c_rbits;
    uint32_t x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t i = threadIdx.x + u * T;
        x[u] = 0u;
        if (i < n) {
            const uint32_t v = v0 + i;
            const uint32_t w = w0 + last_le(vpre + w0, nw, v);
            x[u] = J.plist[vphys[w] + (v - vpre[w])];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (threadIdx.x + u * T < n) atomicAdd(&fh[(x[u] >> rb) & (F - 1)], 1u);
    __syncthreads();
    // exclusive scan of fh[0 .. F); thread t holds fine bins [t*kPer, (t+1)*kPer)
    constexpr uint32_t kPer = kFineMax / T;
    const uint32_t f0 = threadIdx.x * kPer;
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) mine += f0 + r < F ? fh[f0 + r] : 0u;
    uint32_t total;
    uint32_t run = block_excl_scan<T>(mine, sh, total);  // ends with a barrier
    GLOBAL uint32_t *offs = J.coffs2 + static_cast<uint64_t>(g) * (F + 1);
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t f = f0 + r;
        if (f < F) {
            const uint32_t c = fh[f];
            fh[f] = run;
            offs[f] = run;
            run += c;
        }
    }
    if (threadIdx.x == 0) offs[F] = n;
    __syncthreads();
    GLOBAL uint32_t *out = J.cbuf + static_cast<uint64_t>(g) * kChunk;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (threadIdx.x + u * T < n) out[atomicAdd(&fh[(x[u] >> rb) & (F - 1)], 1u)] = x[u];
}

template <int T>
__global__ __launch_bounds__(T) void k_bin_count(const GreedyJob *jobs)
{
    constexpr int U = 4;
    __shared__ uint32_t lc[kCountSpan];
    __shared__ uint32_t sat[T], spre[T];  // a batch of chunks: run start in cbuf, prefix
    __shared__ uint32_t sh[T / kWave];
    const GJob J = view(jobs[blockIdx.y]);
    const uint32_t P = J.c_parts, b = blockIdx.x / P, part = blockIdx.x % P;
    if (b >= J.c_bins) return;  // uniform per block
    const uint32_t F = 1u << J.c_fbits, c = b >> J.c_fbits, f = b & (F - 1);
    const uint32_t g0 = J.cchunk[c], g1 = J.cchunk[c + 1];
    // this workgroup's chunks: [ga, gb)
    const uint32_t ga = g0 + static_cast<uint32_t>(static_cast<uint64_t>(g1 - g0) * part / P);
    const uint32_t gb = g0 + static_cast<uint32_t>(static_cast<uint64_t>(g1 - g0) * (part + 1) / P);
    const uint64_t lo_id = static_cast<uint64_t>(b) << J.c_rbits;
    const uint64_t span = min(static_cast<uint64_t>(1) << J.c_rbits, J.S - lo_id);
    for (uint64_t s0 = 0; s0 < span; s0 += kCountSpan) {
        for (uint32_t j = threadIdx.x; j < kCountSpan; j += T) lc[j] = 0;
        __syncthreads();
        const uint64_t first = lo_id + s0;
        for (uint32_t gq = ga; gq < gb; gq += T) {
            const uint32_t nb = min(static_cast<uint32_t>(T), gb - gq);
            uint32_t len = 0;
            if (threadIdx.x < nb) {
                const uint32_t g = gq + threadIdx.x;
                const GLOBAL uint32_t *o = J.coffs2 + static_cast<uint64_t>(g) * (F + 1) + f;
                const uint32_t r0 = o[0];
                len = o[1] - r0;
                sat[threadIdx.x] = r0;
            }
            uint32_t total;
            const uint32_t ex = block_excl_scan<T>(len, sh, total);  // ends with a barrier
            if (threadIdx.x < nb) spre[threadIdx.x] = ex;
            __syncthreads();
            for (uint32_t e = threadIdx.x; e < total; e += U * T) {
                uint32_t v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t x = e + u * T;
                    v[u] = 0u;
                    if (x < total) {
                        const uint32_t k = last_le(spre, nb, x);
                        v[u] = J.cbuf[static_cast<uint64_t>(gq + k) * kChunk + sat[k] + (x - spre[k])];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t r = static_cast<uint64_t>(v[u]) - first;  // wraps when below
                    if (e + u * T < total && r < kCountSpan) atomicAdd(&lc[r], 1u);
                }
            }
            __syncthreads();  // the batch tables are rewritten next
        }
        const uint64_t n = min<uint64_t>(kCountSpan, span - s0);
        if (P == 1) {
            for (uint32_t j = threadIdx.x; j < n; j += T) J.cnt[first + j] = lc[j];
        } else {
            for (uint32_t j = threadIdx.x; j < n; j += T)
                if (lc[j]) g_add(&J.cnt[first + j], lc[j]);
        }
        __syncthreads();
    }
}

// Candidate sets (C within E or V, Definitions "edge_remove" / "node_remove"):
// an id outside C is marked selected once counted, so no pool, histogram or
// tie plan ever holds it and the greedy picks only from C.
__global__ __launch_bounds__(256) void k_apply_cand(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    if (!J.cand) return;  // uniform per block
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < J.S; i += stride)
        if (!((J.cand[i >> 5] >> (i & 31)) & 1u)) J.cnt[i] = kSelected;
}

// ---------------------------------------------------------------- pool rebuild
template <int T>
__global__ __launch_bounds__(T) void k_hist(const GreedyJob *jobs)
{
    constexpr int U = 8;              // loads in flight per lane
    constexpr uint32_t kBallot = 4;   // counts below this are tallied by wave ballots
    __shared__ uint32_t h[kBins];
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J)) return;  // uniform per block
    for (uint32_t i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    // whole-block tiles of U*T counts, so every lane of a wave takes part in each ballot
    for (uint64_t base = blockIdx.x * static_cast<uint64_t>(U * T); base < J.S;
         base += static_cast<uint64_t>(gridDim.x) * U * T) {
        uint32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + u * T + threadIdx.x;
            c[u] = i < J.S ? J.cnt[i] : kSelected;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (uint32_t v = 0; v < kBallot; ++v) {
                const uint64_t m = __ballot(c[u] == v);
                if (lane == 0 && m) atomicAdd(&h[v], static_cast<uint32_t>(__popcll(m)));
            }
            if (c[u] != kSelected && c[u] >= kBallot) atomicAdd(&h[count_bin(c[u])], 1u);
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kBins; b += blockDim.x)
        if (h[b]) g_add(&J.hist[b], h[b]);
}

// The plan for a pool once the crossing bin is known: ab unselected ids lie
// above it, h_b in it, its counts are [c_lo, c_lo + 2^shift).  If ab + h_b
// fit the pool (and the bin is not count 0), the pool is every id with cnt
// >= c_lo.  A single count c = c_lo gives a tie plan: every id above c plus
// the lowest-id ones at c, up to kPoolTarget.  A wider bin that overfills
// the pool is split by a histogram of its own counts (PLAN_REFINE).
__device__ void set_plan(GLOBAL GreedyState *st, uint64_t c_lo, uint32_t shift, uint32_t ab, uint32_t h_b)
{
    const uint64_t ge = static_cast<uint64_t>(ab) + h_b;
    st->pool_n = 0;
    st->next_id = 0;
    if (ge <= kPoolMax && c_lo > 0) {
        st->plan = PLAN_COLLECT;
        st->c_min = static_cast<uint32_t>(c_lo);
        st->n_tie = 0;
        st->leftover = 0;
        st->tau = (c_lo << 32) | 0xFFFFFFFFull;  // bound for every count <= c_lo - 1
    } else if (shift == 0) {
        const uint32_t c = static_cast<uint32_t>(c_lo);
        const uint32_t R = static_cast<uint32_t>(std::min<uint64_t>(kPoolTarget, ge) - ab);
        st->plan = PLAN_TIES;
        st->c_min = ab ? c + 1 : 0;
        st->c_tie = c;
        st->n_tie = R;
        st->leftover = ge > static_cast<uint64_t>(ab) + R;
        st->tau = c ? (static_cast<uint64_t>(c) << 32) | 0xFFFFFFFFull : 0ull;
    } else {
        const uint32_t sub = shift > kRefineLog ? shift - kRefineLog : 0u;
        st->plan = PLAN_REFINE;
        st->r_lo = static_cast<uint32_t>(c_lo);
        st->r_shift = sub;
        st->r_nbins = 1u << (shift - sub);
        st->r_above = ab;
        st->n_tie = 0;
    }
}

// log2 of the width of histogram bin b (0 for the exact counts)
__device__ __forceinline__ uint32_t bin_shift(uint32_t b)
{
    return b < kExact ? 0u : (b - kExact) / kPerOctave + 3u;
}

// Choose the next pool from the histogram (and clear it for the next
// rebuild).  b* = the highest bin with at least kPoolTarget unselected ids at
// or above it (bin 0 if there are fewer); set_plan turns it into a pool.
// One workgroup per job.
template <int T>
__global__ __launch_bounds__(T) void k_plan(const GreedyJob *jobs)
{
    constexpr uint32_t kPer = (kBins + T - 1) / T;
    constexpr int kWaves = T / kWave;
    __shared__ uint32_t h[kBins];
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t found, bstar, ab_sh;
    const GJob J = view(jobs[blockIdx.x]);
    if (job_done(J)) return;  // uniform per block
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (uint32_t b = threadIdx.x; b < kBins; b += T) {
        h[b] = J.hist[b];
        J.hist[b] = 0;
    }
    if (threadIdx.x == 0) found = 0;
    __syncthreads();
    // thread t owns bins [t*kPer, t*kPer + kPer)
    const uint32_t b0 = threadIdx.x * kPer;
    uint32_t mine = 0;
    for (uint32_t i = 0; i < kPer; ++i)
        if (b0 + i < kBins) mine += h[b0 + i];
    uint32_t x = mine;  // inclusive suffix sum within the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_down(x, d, kWave);
        if (lane + d < kWave) x += o;
    }
    if (lane == 0) wsum[wid] = x;
    __syncthreads();
    uint32_t above = x - mine;  // ids in bins >= b0 + kPer
    for (int w = wid + 1; w < kWaves; ++w) above += wsum[w];
    // the suffix sum crosses kPoolTarget at exactly one bin (if at all)
    for (int i = static_cast<int>(kPer) - 1; i >= 0; --i) {
        const uint32_t b = b0 + i;
        if (b >= kBins) continue;
        if (above < kPoolTarget && above + h[b] >= kPoolTarget) {
            found = 1;
            bstar = b;
            ab_sh = above;
        }
        above += h[b];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t b = 0, ab = above - h[0];  // thread 0: above == every unselected id
    if (found) {
        b = bstar;
        ab = ab_sh;
    }
    set_plan(J.st, bin_lo(b), bin_shift(b), ab, h[b]);
}

// PLAN_REFINE: histogram of the unselected counts in [r_lo, r_lo +
// r_nbins 2^r_shift), sub-bin (c - r_lo) >> r_shift, into the job's histogram
// array (cleared by the plan kernels).
template <int T>
__global__ __launch_bounds__(T) void k_refine_hist(const GreedyJob *jobs)
{
    constexpr int U = 8;  // loads in flight per lane
    __shared__ uint32_t h[kRefineBins];
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plan != PLAN_REFINE) return;  // uniform per block
    const uint32_t lo = J.st->r_lo, shift = J.st->r_shift, nb = J.st->r_nbins;
    for (uint32_t i = threadIdx.x; i < nb; i += T) h[i] = 0;
    __syncthreads();
    for (uint64_t base = blockIdx.x * static_cast<uint64_t>(U * T); base < J.S;
         base += static_cast<uint64_t>(gridDim.x) * U * T) {
        uint32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + u * T + threadIdx.x;
            c[u] = i < J.S ? J.cnt[i] : kSelected;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (c[u] == kSelected || c[u] < lo) continue;
            const uint32_t sb = (c[u] - lo) >> shift;
            if (sb < nb) atomicAdd(&h[sb], 1u);
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += T)
        if (h[b]) g_add(&J.hist[b], h[b]);
}

// PLAN_REFINE: the sub-bin where the count of ids at or above it (with the
// r_above ids above the range) reaches kPoolTarget -- it exists, since the
// range's bin crossed it -- then set_plan.  One workgroup per job.
template <int T>
__global__ __launch_bounds__(T) void k_refine_plan(const GreedyJob *jobs)
{
    constexpr uint32_t kPer = kRefineBins / T;
    constexpr int kWaves = T / kWave;
    static_assert(kRefineBins % T == 0, "sub-bins per thread");
    __shared__ uint32_t h[kRefineBins];
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t bstar, ab_sh;
    const GJob J = view(jobs[blockIdx.x]);
    if (job_done(J) || J.st->plan != PLAN_REFINE) return;  // uniform per block
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint32_t nb = J.st->r_nbins;
    for (uint32_t b = threadIdx.x; b < kRefineBins; b += T) {
        h[b] = b < nb ? J.hist[b] : 0u;
        if (b < nb) J.hist[b] = 0;
    }
    if (threadIdx.x == 0) {
        bstar = 0;
        ab_sh = J.st->r_above;
    }
    __syncthreads();
    const uint32_t b0 = threadIdx.x * kPer;
    uint32_t mine = 0;
    for (uint32_t i = 0; i < kPer; ++i) mine += h[b0 + i];
    uint32_t x = mine;  // inclusive suffix sum within the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_down(x, d, kWave);
        if (lane + d < kWave) x += o;
    }
    if (lane == 0) wsum[wid] = x;
    __syncthreads();
    uint32_t above = J.st->r_above + x - mine;
    for (int w = wid + 1; w < kWaves; ++w) above += wsum[w];
    for (int i = static_cast<int>(kPer) - 1; i >= 0; --i) {
        const uint32_t b = b0 + i;
        if (above < kPoolTarget && above + h[b] >= kPoolTarget) {
            bstar = b;
            ab_sh = above;
        }
        above += h[b];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    GLOBAL GreedyState *st = J.st;
    const uint32_t shift = st->r_shift;
    set_plan(st, static_cast<uint64_t>(st->r_lo) + (static_cast<uint64_t>(bstar) << shift), shift, ab_sh,
             h[bstar]);
}

// Pool += every unselected id with cnt >= c_min.
__global__ __launch_bounds__(256) void k_collect(const GreedyJob *jobs)
{
    constexpr int U = 8;  // loads in flight per lane
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J)) return;
    const uint32_t c_min = J.st->c_min;
    if (c_min == 0) return;
    for (uint64_t base = blockIdx.x * static_cast<uint64_t>(U * blockDim.x); base < J.S;
         base += static_cast<uint64_t>(gridDim.x) * U * blockDim.x) {
        uint32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + u * blockDim.x + threadIdx.x;
            c[u] = i < J.S ? J.cnt[i] : kSelected;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] != kSelected && c[u] >= c_min)
                J.pool[g_add(&J.st->pool_n, 1u)] = static_cast<uint32_t>(base + u * blockDim.x + threadIdx.x);
    }
}

// Tiles the tie scan must count.  Ties at count 0 (the pool has room for
// more than the ids that hold a count, as small queries give) take the
// lowest unselected ids of count 0, and the first n_tie + 1 of them lie below
// n_tie + 1 + n_ids + rounds: no more ids than n_ids hold a count and no more
// than rounds are selected (unless a candidate set marks its excluded ids
// selected too).  Past that the tiles need no scan.
__device__ __forceinline__ uint64_t tie_tiles(const GJob &J)
{
    const GLOBAL GreedyState *st = J.st;
    const uint64_t all = n_tiles_of(J.S);
    if (st->c_tie != 0 || J.cand) return all;
    return min(all, n_tiles_of(static_cast<uint64_t>(st->n_tie) + 1 + J.n_ids + st->rounds));
}

// Ties: per tile of 4096 ids, how many have cnt == c_tie.  Each workgroup
// takes tiles gridDim.x apart, up to the job's tie_tiles (later tiles are
// neither counted nor read).
__global__ __launch_bounds__(256) void k_tie_count(const GreedyJob *jobs)
{
    __shared__ uint32_t sh[4];
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plan != PLAN_TIES) return;  // uniform per block
    const uint32_t c = J.st->c_tie;
    const uint64_t lim = tie_tiles(J);
    for (uint64_t b = blockIdx.x; b < lim; b += gridDim.x) {
        const uint64_t base = b * kScanTile + threadIdx.x * 16ull;
        uint32_t k = 0;
        for (int i = 0; i < 16; ++i)
            if (base + i < J.S && J.cnt[base + i] == c) ++k;
        uint32_t total;
        block_excl_scan_256(k, sh, total);  // ends with a barrier
        if (threadIdx.x == 0) J.tiles[b] = total;
    }
}

__global__ __launch_bounds__(256) void k_tie_scan(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plan != PLAN_TIES) return;  // uniform per block
    scan_tiles_256(J.tiles, tie_tiles(J));
}

// Ties: the first n_tie ids (ascending) with cnt == c_tie go to the pool after
// the collected ones; the next tied id is recorded in next_id.  Tiles as in
// k_tie_count; a tile whose first tied id ranks past n_tie is skipped.
__global__ __launch_bounds__(256) void k_tie_emit(const GreedyJob *jobs)
{
    __shared__ uint32_t sh[4];
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plan != PLAN_TIES) return;  // uniform per block
    const uint32_t R = J.st->n_tie, c = J.st->c_tie;
    const uint32_t pool_base = J.st->pool_n;  // complete: written by an earlier kernel
    const uint64_t lim = tie_tiles(J);
    for (uint64_t b = blockIdx.x; b < lim; b += gridDim.x) {
        const uint32_t first = J.tiles[b];
        if (first > R) continue;  // uniform per block
        const uint64_t base = b * kScanTile + threadIdx.x * 16ull;
        uint32_t k = 0;
        for (int i = 0; i < 16; ++i)
            if (base + i < J.S && J.cnt[base + i] == c) ++k;
        uint32_t total;
        uint32_t q = first + block_excl_scan_256(k, sh, total);  // ends with a barrier
        for (int i = 0; i < 16; ++i) {
            if (base + i < J.S && J.cnt[base + i] == c) {
                if (q < R) J.pool[pool_base + q] = static_cast<uint32_t>(base + i);
                else if (q == R) J.st->next_id = static_cast<uint32_t>(base + i);
                ++q;
            }
        }
    }
}

// ---------------------------------------------------------------- walk lists of the pool
// Mark every pool id that still holds uncovered walks (bitmap bit and its
// pool position) and lay out its list: pstart = exclusive prefix over the
// pool of those counts.  One workgroup per job.  Counts do not change until
// the lists are filled.
// One bit per hash value of the pool's ids: a clear bit proves an id is not
// in the pool, so most ids need no further lookup.
__device__ __forceinline__ uint32_t filter_hash(uint32_t x)
{
    return (x * 0x9E3779B1u) >> (32 - kFilterBits);
}

__device__ __forceinline__ bool filter_has(const uint32_t *filt, uint32_t x)
{
    const uint32_t h = filter_hash(x);
    return (filt[h >> 5] >> (h & 31)) & 1u;
}

// Build the filter of the pool's P ids in LDS (all threads of the block).
__device__ __forceinline__ void filter_build(uint32_t *filt, const GLOBAL uint32_t *pool, uint32_t P)
{
    for (uint32_t i = threadIdx.x; i < kFilterWords; i += blockDim.x) filt[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
        const uint32_t h = filter_hash(pool[i]);
        atomicOr(&filt[h >> 5], 1u << (h & 31));
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_pool_mark(const GreedyJob *jobs)
{
    __shared__ uint32_t sh[1024 / kWave];
    const GJob J = view(jobs[blockIdx.x]);
    if (job_done(J)) return;  // uniform per block
    GLOBAL GreedyState *st = J.st;
    const uint32_t P = pool_size(st);
    uint32_t carry = 0;
    for (uint32_t base = 0; base < P; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        uint32_t c = 0;
        if (i < P) {
            const uint32_t id = J.pool[i];
            const uint32_t v = J.cnt[id];
            if (v != kSelected && v > 0) {
                c = v;
                J.pidx[id] = i;
                g_or(&J.bitmap[id >> 5], 1u << (id & 31));
            }
        }
        uint32_t total;
        const uint32_t ex = block_excl_scan<1024>(c, sh, total);
        if (i < P) {
            J.pstart[i] = carry + ex;
            J.pfill[i] = 0;
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        J.pstart[P] = carry;
        st->plist_total = carry;
        st->wp_total = 0;
    }
}

// Fill the lists: one wave per uncovered walk; each of its ids that is
// marked gets the walk appended to its list (ids outside the LDS filter of the
// pool skip the bitmap).
__global__ __launch_bounds__(256) void k_pool_fill(const GreedyJob *jobs)
{
    constexpr int T = 256, U = 8;  // U id loads in flight per lane
    __shared__ uint32_t filt[kFilterWords];
    __shared__ uint32_t start[T];  // a batch of walks: first position in the batch
    __shared__ uint64_t woff[T];   //                   and offset into ids
    __shared__ uint32_t wid[T];
    __shared__ uint32_t sh[T / kWave];
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plist_total == 0) return;  // uniform per block
    filter_build(filt, J.pool, pool_size(J.st));
    // batches of T walks; the ids of a batch's uncovered walks are laid end
    // to end and every thread takes positions, finding each one's walk by
    // binary search, so all of a thread's id loads are independent
    for (uint64_t w0 = blockIdx.x * static_cast<uint64_t>(T); w0 < J.n_walks;
         w0 += static_cast<uint64_t>(gridDim.x) * T) {
        const uint64_t w = w0 + threadIdx.x;
        uint32_t len = 0;
        uint64_t off = 0;
        if (w < J.n_walks) {
            const uint64_t o = J.walk_off[w];
            const uint32_t l = J.walk_len[w];
            if (!(J.wst[w] & kCovered)) {
                off = o;
                len = l;
            }
        }
        uint32_t total;
        const uint32_t ex = block_excl_scan<T>(len, sh, total);  // ends with a barrier
        start[threadIdx.x] = ex;
        woff[threadIdx.x] = off;
        wid[threadIdx.x] = static_cast<uint32_t>(w);
        __syncthreads();
        // each thread takes U consecutive positions: one search for the
        // first, then the walk index only moves forward
        for (uint32_t f0 = 0; f0 < total; f0 += U * T) {
            const uint32_t fb = f0 + threadIdx.x * U;
            uint32_t x[U], k[U];
            uint32_t kk = fb < total ? last_le(start, T, fb) : 0u;  // empty (covered) walks share their start
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t f = fb + u;
                x[u] = 0u;
                k[u] = 0u;
                if (f < total) {
                    while (kk + 1 < static_cast<uint32_t>(T) && start[kk + 1] <= f) ++kk;
                    k[u] = kk;
                    x[u] = J.ids[woff[kk] + (f - start[kk])];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (fb + u < total && filter_has(filt, x[u]) &&
                    (J.bitmap[x[u] >> 5] & (1u << (x[u] & 31)))) {
                    const uint32_t i = J.pidx[x[u]];
                    J.plist[J.pstart[i] + g_add(&J.pfill[i], 1u)] = wid[k[u]];
                }
            }
        }
        __syncthreads();  // the batch tables are rewritten next
    }
}

// Per-walk pool lists: the transpose of the pool ids' walk lists.  For every
// walk in some list, the pool positions of its marked ids, so that covering
// a walk decrements its pool ids' counts without reading its ids or looking
// them up.  The lists are counted, given their ranges of wpool (one atomic
// per block of 2048 walks), filled, and after the rounds their counts are
// cleared again.  One wave per pool id's list (count, fill, clear); eight
// consecutive walks per thread (ranges).
__global__ __launch_bounds__(256) void k_wp_count(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plist_total == 0) return;  // uniform per block
    const uint32_t P = pool_size(J.st);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < P; i += waves)
        for (uint32_t e = J.pstart[i] + lane; e < J.pstart[i + 1]; e += kWave) g_add64(&J.wst[J.plist[e]], kWsCountOne);
}

__global__ __launch_bounds__(256) void k_wp_alloc(const GreedyJob *jobs)
{
    constexpr uint32_t T = 256, kPer = 8;  // consecutive walks per thread
    __shared__ uint32_t wsum[T / kWave];
    __shared__ uint32_t bbase;
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plist_total == 0) return;  // uniform per block
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint64_t span = static_cast<uint64_t>(T) * kPer;
    // one atomic per block and span: the ranges of T * kPer walks at a time
    for (uint64_t base = blockIdx.x * span; base < J.n_walks; base += static_cast<uint64_t>(gridDim.x) * span) {
        const uint64_t w0 = base + static_cast<uint64_t>(threadIdx.x) * kPer;
        uint64_t ws[kPer];
        uint32_t c[kPer], mine = 0;
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            ws[j] = w0 + j < J.n_walks ? J.wst[w0 + j] : 0ull;
            c[j] = ws_count(ws[j]);
            mine += c[j];
        }
        uint32_t incl = mine;  // inclusive scan of the wave's sums
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += o;
        }
        if (lane == kWave - 1) wsum[wid] = incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (uint32_t w = 0; w < T / kWave; ++w) {
                const uint32_t v = wsum[w];
                wsum[w] = tot;
                tot += v;
            }
            bbase = tot ? g_add(&J.st->wp_total, tot) : 0u;
        }
        __syncthreads();
        uint32_t at = bbase + wsum[wid] + incl - mine;  // the walks' ranges start here; the fill advances them
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            if (c[j]) J.wst[w0 + j] = (ws[j] & ~0xFFFFFFFFull) | at;  // (no other writer now)
            at += c[j];
        }
        __syncthreads();  // wsum and bbase are rewritten next
    }
}

__global__ __launch_bounds__(256) void k_wp_fill(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    if (job_done(J) || J.st->plist_total == 0) return;  // uniform per block
    const uint32_t P = pool_size(J.st);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < P; i += waves)
        for (uint32_t e = J.pstart[i] + lane; e < J.pstart[i + 1]; e += kWave)
            J.wpool[static_cast<uint32_t>(g_add64(&J.wst[J.plist[e]], 1ull))] = static_cast<uint16_t>(i);
}

// after the rounds: the next pool's lists count from zero
__global__ __launch_bounds__(256) void k_wp_clear(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    if (J.st->error != 0 || J.st->plist_total == 0) return;  // (runs after the job's last rounds too)
    const uint32_t P = pool_size(J.st);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < P; i += waves)
        for (uint32_t e = J.pstart[i] + lane; e < J.pstart[i + 1]; e += kWave)
            g_and64(&J.wst[J.plist[e]], kCovered | 0xFFFFFFFFull);
}

// ---------------------------------------------------------------- lazy rounds
// One workgroup of T threads per job: rounds [rounds, k) while the pool
// certifies the pick.
//
// The pool lives in LDS for the whole launch: its ids and their exact counts
// (a walk covered now never holds an id chosen in an earlier round, so chosen
// entries are never decremented).  A round's argmax is then an LDS scan.  The global counts are not touched
// here: each covered walk is appended to the claimed list, and k_uncover
// (all CUs) takes the list's walks off the global counts after the launch,
// before k_mark marks this launch's picks selected.  Each pool id's list
// range sits in registers of the thread that holds the id.
//
// Covering: each pass claims up to T of the chosen id's walks (one list
// entry per thread); block scans rank the claimed walks and lay their pool
// positions (the per-walk pool lists) end to end; every thread reads the
// positions at its slots (finding each one's walk by binary search over the
// claimed walks' first slots in LDS) and decrements those LDS counts.
//
// Zero gains.  When the best key of the pool has gain 0, every unselected id
// of the pool has count 0 (and the plan is a tie at count 0, so every id
// outside the pool has count 0 and, if tied ids were left out, an id >=
// next_id).  The remaining rounds take the pool's unselected ids in ascending
// order below next_id, all in one pass: directly when the pool is already
// that ordered list (nothing collected above count 0), else after an LDS sort.
template <int T>
__global__ __launch_bounds__(T) void k_lazy(const GreedyJob *jobs)
{
    constexpr int kWaves = T / kWave;
    constexpr int kPer = kPoolMax / T;
    // each wave's best key and its list range, double-buffered by round parity
    // (a wave can be one round ahead of the slowest reader, not two)
    __shared__ uint64_t shk[2][kWaves];
    __shared__ uint32_t shlo[2][kWaves], shhi[2][kWaves], shpos[2][kWaves];
    __shared__ uint32_t sh32[kWaves];
    __shared__ uint32_t start[T];        // a pass's walks: first flattened slot
    __shared__ uint32_t woff[T];         //                 and start in wpool
    __shared__ uint32_t pcnt[kPoolMax];  // exact counts of the pool's ids
    __shared__ uint32_t pids[kPoolMax];
    __shared__ uint32_t sortbuf[kPoolMax];  // zero-gain tail: the open pool ids, sorted
    const GJob J = view(jobs[blockIdx.x]);
    if (job_done(J)) return;  // uniform per block
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    GLOBAL GreedyState *st = J.st;
    const bool ties = st->plan == PLAN_TIES;
    const uint32_t P = pool_size(st);
    const uint64_t tau = ties && st->leftover
                             ? ((static_cast<uint64_t>(st->c_tie) + 1) << 32) | (0xFFFFFFFFu - st->next_id)
                             : st->tau;
    const bool ordered_zeros = ties && st->c_tie == 0 && st->pool_n == 0;
    uint32_t pid[kPer], plo[kPer], phi[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const uint32_t i = threadIdx.x + j * T;
        pid[j] = plo[j] = phi[j] = 0;
        if (i < P) {
            const uint32_t x = J.pool[i];
            pid[j] = x;
            pids[i] = x;
            pcnt[i] = J.cnt[x];
            plo[j] = J.pstart[i];
            phi[j] = J.pstart[i + 1];
        }
    }
    __syncthreads();
    const int64_t r0 = st->rounds;
    int64_t r = r0;
    uint32_t cbase = st->n_claimed;  // uniform: next entry of the claimed list
    for (; r < J.k; ++r) {
        // exact keys of the pool; the largest is this round's pick if it beats
        // tau.  The key and the list range of each wave's best travel together,
        // so every thread ends the reduction knowing the pick's list.
        uint64_t best = 0;
        uint32_t blo = 0, bhi = 0, bpos = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = threadIdx.x + j * T;
            if (i < P) {
                const uint64_t key = key_of(pcnt[i], pid[j]);
                if (key > best) {
                    best = key;
                    blo = plo[j];
                    bhi = phi[j];
                    bpos = i;
                }
            }
        }
        const int par = static_cast<int>(r & 1);
        // wave maximum of the 64-bit keys from two 32-bit wave reductions (the
        // device library's, across lanes without LDS): the count part, then
        // the id part among the lanes that hold that count
        const uint32_t mh = __ockl_wfred_max_u32(static_cast<uint32_t>(best >> 32));
        const uint32_t ml = __ockl_wfred_max_u32(static_cast<uint32_t>(best >> 32) == mh ? static_cast<uint32_t>(best) : 0u);
        const uint64_t wbest = (static_cast<uint64_t>(mh) << 32) | ml;
        // keys are distinct (an id is in the pool once), so one lane holds a
        // nonzero wave maximum; lane 0 reports a wave without keys
        if (wbest != 0 ? best == wbest : lane == 0) {
            shk[par][wid] = wbest;
            shlo[par][wid] = blo;
            shhi[par][wid] = bhi;
            shpos[par][wid] = bpos;
        }
        __syncthreads();
        // the waves' keys first, then only the winning wave's range and position
        int bw = 0;
        best = shk[par][0];
#pragma unroll 3
        for (int w = 1; w < kWaves; ++w) {
            const uint64_t kw = shk[par][w];
            if (kw > best) {
                best = kw;
                bw = w;
            }
        }
        const uint32_t lo = shlo[par][bw], hi = shhi[par][bw];
        const uint32_t cpos = shpos[par][bw];  // the pick's list range and pool position
        if (best <= tau) break;  // uniform: every thread saw the same values
        const uint32_t id = 0xFFFFFFFFu - static_cast<uint32_t>(best);
        const uint32_t g = static_cast<uint32_t>(best >> 32) - 1u;
        if (g == 0 && ordered_zeros) {
            const uint64_t need = static_cast<uint64_t>(J.k - r);
            uint64_t taken = 0;
            for (uint32_t b0 = 0; b0 < P && taken < need; b0 += T) {
                const uint32_t i = b0 + threadIdx.x;
                const bool open = i < P && pcnt[i] != kSelected;
                uint32_t total;
                const uint64_t rank = taken + block_excl_scan<T>(open ? 1u : 0u, sh32, total);
                if (open && rank < need) {
                    J.sel[r + rank] = pids[i];
                    J.gain[r + rank] = 0;
                    pcnt[i] = kSelected;
                }
                taken += total;
            }
            r += static_cast<int64_t>(taken < need ? taken : need);
            break;
        }
        // the owner marks the pick (only the owner reads its count in later
        // argmaxes; the covering below skips the pick's own id)
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t i = threadIdx.x + j * T;
            if (i < P && pid[j] == id) pcnt[i] = kSelected;  // the pool holds each id once
        }
        if (threadIdx.x == 0) {
            J.sel[r] = id;
            J.gain[r] = g;
        }
        if (g == 0) {
            __syncthreads();  // every thread reads the marks below
            // Every unselected pool id has count 0, and so has every id
            // outside the pool (this is a tie plan at count 0: all ids with a
            // count were collected), whose ids are all >= next_id when tied
            // ids were left out.  The picks are the pool's unselected ids in
            // ascending order, below next_id: sort them and take them.  (The
            // id just chosen is the first.)
            uint32_t *buf = sortbuf;
            uint32_t N = 1;
            while (N < P) N <<= 1;
            for (uint32_t i = threadIdx.x; i < N; i += T)
                buf[i] = (i < P && (pcnt[i] != kSelected || pids[i] == id)) ? pids[i] : 0xFFFFFFFFu;
            __syncthreads();
            for (uint32_t kk = 2; kk <= N; kk <<= 1) {
                for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (uint32_t i = threadIdx.x; i < N; i += T) {
                        const uint32_t o = i ^ jj;
                        if (o > i) {
                            const uint32_t a = buf[i], b = buf[o];
                            if ((a > b) == ((i & kk) == 0)) {
                                buf[i] = b;
                                buf[o] = a;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            const uint32_t bound = st->leftover ? st->next_id : 0xFFFFFFFFu;
            const uint64_t need = static_cast<uint64_t>(J.k - r);
            uint32_t taken = 0;  // sorted: the valid picks are a prefix
            {
                uint32_t a = 0, b = N;  // first position whose id >= bound
                while (a < b) {
                    const uint32_t m = (a + b) >> 1;
                    if (buf[m] < bound) a = m + 1;
                    else b = m;
                }
                taken = static_cast<uint32_t>(a < need ? a : need);
            }
            for (uint32_t i = threadIdx.x; i < taken; i += T) {
                J.sel[r + i] = buf[i];
                J.gain[r + i] = 0;
            }
            r += taken;
            break;
        }
        for (uint32_t b0 = lo; b0 < hi; b0 += T) {
            const uint32_t p = b0 + threadIdx.x;
            uint32_t len = 0, w = 0, off = 0;
            if (p < hi) {
                w = J.plist[p];
                // one atomic claims the walk and returns its pool list, which
                // holds the pick's own position, so len >= 1
                const uint64_t old = g_or64(&J.wst[w], kCovered);
                if (!(old & kCovered)) {
                    len = ws_count(old);
                    off = static_cast<uint32_t>(old) - len;
                }
            }
            uint32_t n_new;
            const uint32_t rank = block_excl_scan<T>(len ? 1u : 0u, sh32, n_new);  // ends with a barrier
            if (len) {
                start[rank] = len;
                woff[rank] = off;
                J.claimed[cbase + rank] = w;
            }
            cbase += n_new;
            __syncthreads();
            const uint32_t mylen = threadIdx.x < n_new ? start[threadIdx.x] : 0u;
            uint32_t total;
            const uint32_t first = block_excl_scan<T>(mylen, sh32, total);  // ends with a barrier
            start[threadIdx.x] = first;  // first slot of claimed walk threadIdx.x
            __syncthreads();
            // slots f = threadIdx.x + u*T, kSpan at a time: every load of a
            // group is issued before its LDS updates
            constexpr uint32_t kSpan = 8;
            for (uint32_t f0 = threadIdx.x; f0 < total; f0 += kSpan * T) {
                uint32_t x[kSpan];
#pragma unroll
                for (uint32_t u = 0; u < kSpan; ++u) {
                    const uint32_t f = f0 + u * T;
                    x[u] = cpos;
                    if (f < total) {
                        // the last claimed walk whose first slot is <= f holds f
                        uint32_t a = 0, b = n_new - 1;
                        while (a < b) {
                            const uint32_t m = (a + b + 1) >> 1;
                            if (start[m] <= f) a = m;
                            else b = m - 1;
                        }
                        x[u] = J.wpool[woff[a] + (f - start[a])];
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < kSpan; ++u)
                    if (x[u] != cpos) atomicSub(&pcnt[x[u]], 1u);
            }
            __syncthreads();  // LDS counts final and LDS free before the next pass / round
        }
    }
    if (threadIdx.x == 0) {
        st->rounds = static_cast<uint32_t>(r);
        st->n_claimed = cbase;
    }
    // unmark the pool (the next rebuild marks its own)
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        if (threadIdx.x + j * T < P) g_and(&J.bitmap[pid[j] >> 5], ~(1u << (pid[j] & 31)));
}

// After a k_lazy launch, cnt must again hold, for every unselected id, the
// number of uncovered walks holding it.  Either the walks the launch covered
// are taken off (k_uncover), or, when they outweigh the walks still
// uncovered (queries whose picks cover most walks, as node removal of
// well-hit sources does), the counts are recomputed from the uncovered walks
// (k_recount_zero, then k_recount_add).  Estimated work in atomics: an id of
// a walk costs one, clearing an id and testing a walk a sixteenth.
__device__ __forceinline__ bool recount_cheaper(const GJob &J, const GLOBAL GreedyState *st)
{
    if (J.n_walks == 0) return false;
    const double per_walk = static_cast<double>(J.n_ids) / static_cast<double>(J.n_walks);
    const double covered_now = static_cast<double>(st->n_claimed - st->claimed_done);
    const double open = static_cast<double>(J.n_walks - st->n_claimed);
    return open * per_walk + (static_cast<double>(J.S) + static_cast<double>(J.n_walks)) / 16.0 <
           covered_now * per_walk;
}

// Take the walks covered by the last k_lazy launch off the global counts:
// one wave per claimed walk, its lanes along the walk's ids.  The picks'
// own counts drop too; k_mark overwrites them next.
__global__ __launch_bounds__(256) void k_uncover(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    const GLOBAL GreedyState *st = J.st;
    if (recount_cheaper(J, st)) return;  // uniform per block
    const uint32_t lo = st->claimed_done, hi = st->n_claimed;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    for (uint64_t c = lo + (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave; c < hi;
         c += waves) {
        const uint32_t w = J.claimed[c];
        const uint64_t o = J.walk_off[w];
        const uint32_t L = J.walk_len[w];
        if (J.cand) {
            // ids outside the candidate set are marked selected: leave them so
            for (uint32_t e = lane; e < L; e += kWave) {
                const uint32_t x = J.ids[o + e];
                if (J.cnt[x] != kSelected) g_add(&J.cnt[x], 0xFFFFFFFFu);
            }
        } else {
            for (uint32_t e = lane; e < L; e += kWave) g_add(&J.cnt[J.ids[o + e]], 0xFFFFFFFFu);
        }
    }
}

// Recount, first pass: every unselected id's count to zero (selected ids,
// and ids outside a candidate set, keep their mark).
__global__ __launch_bounds__(256) void k_recount_zero(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    if (!recount_cheaper(J, J.st)) return;  // uniform per block
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < J.S; i += stride)
        if (J.cnt[i] != kSelected) J.cnt[i] = 0;
}

// Recount, second pass: each wave tests 64 walks at a time and adds the ids
// of the uncovered ones, its lanes along each walk.  No uncovered walk holds
// a selected id; ids outside a candidate set keep their mark.
__global__ __launch_bounds__(256) void k_recount_add(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.y]);
    if (!recount_cheaper(J, J.st)) return;  // uniform per block
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    for (uint64_t base = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave * kWave;
         base < J.n_walks; base += waves * kWave) {
        const uint64_t w = base + lane;
        uint64_t open = __ballot(w < J.n_walks && !(J.wst[w] & kCovered));
        while (open != 0) {
            const uint64_t v = base + static_cast<uint64_t>(__ffsll(static_cast<long long>(open)) - 1);
            open &= open - 1;
            const uint64_t o = J.walk_off[v];
            const uint32_t L = J.walk_len[v];
            for (uint32_t e = lane; e < L; e += kWave) {
                const uint32_t x = J.ids[o + e];
                if (J.cnt[x] != kSelected) g_add(&J.cnt[x], 1u);
            }
        }
    }
}

// Mark the picks of the rounds since the last call selected in the global
// counts (after k_uncover or the recount) and retire the claimed entries.
__global__ __launch_bounds__(256) void k_mark(const GreedyJob *jobs)
{
    const GJob J = view(jobs[blockIdx.x]);
    GLOBAL GreedyState *st = J.st;
    const uint32_t from = st->marked, r = st->rounds, claimed = st->n_claimed;
    for (uint32_t q = from + threadIdx.x; q < r; q += blockDim.x) J.cnt[J.sel[q]] = kSelected;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->marked = r;
        st->claimed_done = claimed;
    }
}

unsigned grid_for(uint64_t items, unsigned block, unsigned cap)
{
    uint64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(std::min<uint64_t>(g, cap));
}

uint64_t al256(uint64_t b) { return (b + 255) / 256 * 256; }

// Counting plan of a job: fine bins of 2^rbits ids (rbits = kCountSpanLog,
// so each is one LDS pass) in at most kCoarseMax coarse bins of at most
// kFineMax fine bins, tiles of at least kCountTileMin walk ids, and, when
// there are fewer than kCountBinsFull fine bins, several workgroups per fine
// bin.
constexpr uint32_t kCountBinsFull = 256;
struct CountPlan {
    uint32_t rbits, bins, fbits, coarse, tiles, parts, chunks_max;
    uint64_t tile_len;
    // scratch words: coffs, ctab, cn, cchunk, coffs2, cbuf
    uint64_t w_offs, w_tab, w_cn, w_chunk, w_offs2, w_buf;
};
uint32_t ceil_log2(uint64_t x)
{
    uint32_t L = 0;
    while ((uint64_t(1) << L) < x) ++L;
    return L;
}
CountPlan count_plan(uint64_t S, uint64_t n_ids)
{
    CountPlan P;
    P.rbits = kCountSpanLog;
    P.bins = static_cast<uint32_t>((S + (uint64_t(1) << P.rbits) - 1) >> P.rbits);
    const uint32_t Lb = ceil_log2(P.bins);
    P.fbits = Lb > kCoarseLog ? Lb - kCoarseLog : 0u;
    P.coarse = (P.bins + (1u << P.fbits) - 1) >> P.fbits;
    P.tiles = static_cast<uint32_t>(
        std::min<uint64_t>(kCountTilesMax, std::max<uint64_t>(1, (n_ids + kCountTileMin - 1) / kCountTileMin)));
    P.tile_len = (n_ids + P.tiles - 1) / P.tiles;
    P.parts = P.bins >= kCountBinsFull ? 1u : (2 * kCountBinsFull + P.bins - 1) / P.bins;
    // each coarse bin ends in at most one partial chunk
    P.chunks_max = static_cast<uint32_t>((n_ids + kChunk - 1) / kChunk + P.coarse);
    P.w_offs = static_cast<uint64_t>(P.tiles) * (P.coarse + 1);
    P.w_tab = 2ull * P.coarse * P.tiles;
    P.w_cn = P.coarse;
    P.w_chunk = P.coarse + 1;
    P.w_offs2 = static_cast<uint64_t>(P.chunks_max) * ((1u << P.fbits) + 1);
    P.w_buf = static_cast<uint64_t>(P.chunks_max) * kChunk;
    return P;
}

// Carve a job's buffers from its scratch block (layout of greedy_scratch_bytes).
GreedyJob carve(const GreedyInput &g)
{
    char *p = static_cast<char *>(g.scratch);
    const uint64_t S = g.id_space;
    GreedyJob J{};
    auto take = [&p](uint64_t bytes) {
        char *q = p;
        p += al256(bytes);
        return q;
    };
    J.pidx = reinterpret_cast<uint32_t *>(take(4 * S));
    J.plist = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(g.n_ids, 1)));
    J.pstart = reinterpret_cast<uint32_t *>(take(4 * (kPoolMax + 1)));
    J.pfill = reinterpret_cast<uint32_t *>(take(4 * kPoolMax));
    J.bitmap = reinterpret_cast<uint32_t *>(take(4 * ((S + 31) / 32)));
    J.claimed = reinterpret_cast<uint32_t *>(take(4 * std::max<uint64_t>(g.n_walks, 1)));
    J.wst = reinterpret_cast<uint64_t *>(take(8 * std::max<uint64_t>(g.n_walks, 1)));
    J.wpool = reinterpret_cast<uint16_t *>(take(2 * std::max<uint64_t>(g.n_ids, 1)));
    J.sel = reinterpret_cast<int64_t *>(take(8 * g.k));
    J.gain = reinterpret_cast<uint64_t *>(take(8 * g.k));
    J.hist = reinterpret_cast<uint32_t *>(take(4 * kBins));
    J.pool = reinterpret_cast<uint32_t *>(take(4 * kPoolMax));
    J.tiles = reinterpret_cast<uint32_t *>(take(4 * ((S + kScanTile - 1) / kScanTile)));
    const CountPlan P = count_plan(S, g.n_ids);
    J.coffs = reinterpret_cast<uint32_t *>(take(4 * P.w_offs));
    J.ctab = reinterpret_cast<uint32_t *>(take(4 * P.w_tab));
    J.cn = reinterpret_cast<uint32_t *>(take(4 * P.w_cn));
    J.cchunk = reinterpret_cast<uint32_t *>(take(4 * P.w_chunk));
    J.coffs2 = reinterpret_cast<uint32_t *>(take(4 * P.w_offs2));
    J.cbuf = reinterpret_cast<uint32_t *>(take(4 * P.w_buf));
    J.c_rbits = P.rbits;
    J.c_bins = P.bins;
    J.c_fbits = P.fbits;
    J.c_coarse = P.coarse;
    J.c_tiles = P.tiles;
    J.c_parts = P.parts;
    J.c_chunks_max = P.chunks_max;
    J.c_tile_len = P.tile_len;
    J.cnt = g.cnt;
    J.cand = g.cand;
    J.walk_off = g.walk_off;
    J.walk_len = g.walk_len;
    J.ids = g.ids;
    J.S = S;
    J.n_walks = g.n_walks;
    J.n_ids = g.n_ids;
    J.k = g.k;
    return J;
}

}  // namespace

// ---------------------------------------------------------------- host side
namespace {
uint64_t count_scratch_bytes(uint64_t S, uint64_t n_ids)
{
    const CountPlan P = count_plan(S, n_ids);
    return al256(4 * P.w_offs) + al256(4 * P.w_tab) + al256(4 * P.w_cn) + al256(4 * P.w_chunk) +
           al256(4 * P.w_offs2) + al256(4 * P.w_buf);
}
}  // namespace

size_t greedy_scratch_bytes(uint64_t id_space, uint64_t n_walks, uint64_t n_ids, int64_t k)
{
    const uint64_t S = id_space;
    return al256(4 * S) + al256(4 * std::max<uint64_t>(n_ids, 1)) + al256(4 * (kPoolMax + 1)) +
           al256(4 * kPoolMax) + al256(4 * ((S + 31) / 32)) +
           al256(4 * std::max<uint64_t>(n_walks, 1)) + al256(8 * std::max<uint64_t>(n_walks, 1)) +
           al256(2 * std::max<uint64_t>(n_ids, 1)) +
           2 * al256(8 * static_cast<uint64_t>(k)) +
           al256(4 * kBins) + al256(4 * kPoolMax) + al256(4 * ((S + kScanTile - 1) / kScanTile)) +
           count_scratch_bytes(S, n_ids);
}

// job table: n_jobs GreedyJob records, then their n_jobs states (one copy
// reads every state back)
size_t greedy_job_table_bytes(uint32_t n_jobs)
{
    return al256(sizeof(GreedyJob) * n_jobs) + sizeof(GreedyState) * n_jobs;
}

void run_greedy_jobs(std::vector<GreedyInput> &in, void *d_job_table, hipStream_t s, bool timing,
                     GreedyResult *res, unsigned hist_base)
{
    const uint32_t Q = static_cast<uint32_t>(in.size());
    if (!Q) return;
    uint64_t max_S = 0, max_walks = 0;
    uint32_t max_bins = 1, max_ctiles = 1, max_coarse = 1, max_chunks = 1;
    std::vector<GreedyJob> jobs(Q);
    for (uint32_t q = 0; q < Q; ++q) {
        GreedyInput &g = in[q];
        SIA_REQUIRE(g.n_ids < 0xFFFFFFFFull && g.n_walks < 0xFFFFFFFFull, SIA_EINVAL,
                    "too many walk ids for 32-bit inverted index offsets");
        SIA_REQUIRE(g.k >= 1 && static_cast<uint64_t>(g.k) <= g.id_space, SIA_EINVAL,
                    "k must be in [1, id space]");
        SIA_REQUIRE(g.cnt && g.scratch && g.selected && g.gains, SIA_EINVAL, "greedy job buffers");
        jobs[q] = carve(g);
        if (g.out_on_device) {  // the rounds write the caller's device arrays
            jobs[q].sel = g.selected;
            jobs[q].gain = g.gains;
        }
        g.rounds_seen = 0;
        max_S = std::max(max_S, g.id_space);
        max_walks = std::max(max_walks, g.n_walks);
        max_bins = std::max(max_bins, jobs[q].c_bins * jobs[q].c_parts);
        max_ctiles = std::max(max_ctiles, jobs[q].c_tiles);
        max_coarse = std::max(max_coarse, jobs[q].c_coarse);
        max_chunks = std::max(max_chunks, jobs[q].c_chunks_max);
    }
    const unsigned cus = static_cast<unsigned>(device_cu_count());
    const unsigned tiles = static_cast<unsigned>((max_S + kScanTile - 1) / kScanTile);
    GreedyJob *d_jobs = static_cast<GreedyJob *>(d_job_table);
    GreedyState *d_states = reinterpret_cast<GreedyState *>(static_cast<char *>(d_job_table) +
                                                            al256(sizeof(GreedyJob) * Q));
    for (uint32_t q = 0; q < Q; ++q) jobs[q].st = d_states + q;

    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (timing) {
        for (auto &e : ev) SIA_HIP(hipEventCreate(&e));
        SIA_HIP(hipEventRecord(ev[0], s));
    }
    SIA_HIP(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(GreedyJob) * Q, hipMemcpyHostToDevice, s));
    const uint64_t init_items = std::max<uint64_t>({max_walks, max_S, kBins});
    hipLaunchKernelGGL(k_init, dim3(grid_for(init_items, 256, cus * 8), Q), dim3(256), 0, s, d_jobs);
    hipLaunchKernelGGL(k_bin_sort<1024>, dim3(max_ctiles, Q), dim3(1024), 0, s, d_jobs);
    hipLaunchKernelGGL(k_bin_plan<512>, dim3(max_coarse, Q), dim3(512), 0, s, d_jobs);
    hipLaunchKernelGGL(k_bin_bases<256>, dim3(1, Q), dim3(256), 0, s, d_jobs);
    hipLaunchKernelGGL(k_bin_sort2<256>, dim3(max_chunks, Q), dim3(256), 0, s, d_jobs);
    hipLaunchKernelGGL(k_bin_count<1024>, dim3(max_bins, Q), dim3(1024), 0, s, d_jobs);
    bool any_cand = false;
    for (uint32_t q = 0; q < Q; ++q) any_cand = any_cand || in[q].cand != nullptr;
    if (any_cand)
        hipLaunchKernelGGL(k_apply_cand, dim3(grid_for(max_S, 256, cus * 8), Q), dim3(256), 0, s, d_jobs);
    SIA_HIP(hipGetLastError());
    if (timing) SIA_HIP(hipEventRecord(ev[1], s));

    // pool rebuilds + certified rounds; groups of generations between host checks
    constexpr unsigned T = 1024;
    // histogram tiling: hist_base workgroups for one job (default: one per CU),
    // shared out when several jobs run
    const unsigned base = hist_base ? hist_base : cus;
    const unsigned hist_blocks =
        std::min(grid_for(max_S, T * 8, base), std::max(1u, base / std::min<unsigned>(Q, 8)));
    const unsigned collect_blocks = grid_for(max_S, 256 * 8, cus * 4);
    const unsigned fill_blocks = grid_for(max_walks, 256, cus * 8);
    const unsigned alloc_blocks = grid_for(max_walks, 256 * 8, cus * 8);  // 8 walks per thread
    const unsigned list_blocks = grid_for(static_cast<uint64_t>(kPoolMax) * kWave, 256, cus * 2);  // a wave per list
    const unsigned zero_blocks = grid_for(max_S, 256, cus * 8);
    const unsigned tie_blocks = std::max(1u, std::min(tiles, static_cast<unsigned>(cus) * 8));  // tiles apart
    const unsigned recount_blocks = grid_for(max_walks, 256, cus * 8);  // a wave per 64 walks
    std::vector<GreedyState> hs(Q);
    for (int group = 1;; group = std::min(group * 2, 8)) {
        for (int gen = 0; gen < group; ++gen) {
            hipLaunchKernelGGL(k_hist<T>, dim3(hist_blocks, Q), dim3(T), 0, s, d_jobs);
            hipLaunchKernelGGL(k_plan<T>, dim3(Q), dim3(T), 0, s, d_jobs);
            for (int level = 0; level < 2; ++level) {  // bins of up to 2^22 counts: two splits at most
                hipLaunchKernelGGL(k_refine_hist<T>, dim3(hist_blocks, Q), dim3(T), 0, s, d_jobs);
                hipLaunchKernelGGL(k_refine_plan<T>, dim3(Q), dim3(T), 0, s, d_jobs);
            }
            hipLaunchKernelGGL(k_collect, dim3(collect_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_tie_count, dim3(tie_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_tie_scan, dim3(1, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_tie_emit, dim3(tie_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_pool_mark, dim3(Q), dim3(1024), 0, s, d_jobs);
            hipLaunchKernelGGL(k_pool_fill, dim3(fill_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_wp_count, dim3(list_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_wp_alloc, dim3(alloc_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_wp_fill, dim3(list_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_lazy<T>, dim3(Q), dim3(T), 0, s, d_jobs);
            hipLaunchKernelGGL(k_wp_clear, dim3(list_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_uncover, dim3(cus * 4, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_recount_zero, dim3(zero_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_recount_add, dim3(recount_blocks, Q), dim3(256), 0, s, d_jobs);
            hipLaunchKernelGGL(k_mark, dim3(Q), dim3(256), 0, s, d_jobs);
            SIA_HIP(hipGetLastError());
        }
        SIA_HIP(hipMemcpyAsync(hs.data(), d_states, sizeof(GreedyState) * Q, hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (uint32_t q = 0; q < Q; ++q) {
            SIA_REQUIRE(hs[q].error == 0 && hs[q].plan != PLAN_REFINE, SIA_EDEVICE,
                        "greedy pool plan left unresolved");
            const bool finished = static_cast<int64_t>(hs[q].rounds) >= in[q].k;
            // every rebuild certifies at least one pick, so an unfinished job
            // always advances
            SIA_REQUIRE(finished || hs[q].rounds > in[q].rounds_seen, SIA_EDEVICE,
                        "greedy made no progress");
            in[q].rounds_seen = hs[q].rounds;
            all = all && finished;
        }
        if (all) break;
    }
    if (timing) SIA_HIP(hipEventRecord(ev[2], s));
    for (uint32_t q = 0; q < Q; ++q) {
        if (in[q].out_on_device) continue;
        SIA_HIP(hipMemcpyAsync(in[q].selected, jobs[q].sel, sizeof(int64_t) * in[q].k,
                               hipMemcpyDeviceToHost, s));
        SIA_HIP(hipMemcpyAsync(in[q].gains, jobs[q].gain, sizeof(uint64_t) * in[q].k,
                               hipMemcpyDeviceToHost, s));
    }
    SIA_HIP(hipStreamSynchronize(s));
    if (timing) {
        SIA_HIP(hipEventElapsedTime(&res->ms_count, ev[0], ev[1]));
        SIA_HIP(hipEventElapsedTime(&res->ms_greedy, ev[1], ev[2]));
        for (auto &e : ev) SIA_HIP(hipEventDestroy(e));
    }
}

GreedyResult run_greedy(Workspace &ws, int64_t id_space, uint64_t n_walks, uint64_t n_ids,
                        int64_t k, int64_t *selected, uint64_t *gains, hipStream_t s, bool timing,
                        const uint32_t *cand)
{
    const uint64_t S = static_cast<uint64_t>(id_space);
    ws.greedy.ensure(greedy_scratch_bytes(S, n_walks, n_ids, k));
    ws.jobs.ensure(greedy_job_table_bytes(1));
    ws.cnt.ensure(sizeof(uint32_t) * std::max<uint64_t>(S, 1));
    std::vector<GreedyInput> in(1);
    GreedyInput &g = in[0];
    g.walk_off = ws.walk_off.as<uint64_t>();
    g.walk_len = ws.walk_len.as<uint32_t>();
    g.ids = ws.ids.as<uint32_t>();
    g.id_space = S;
    g.n_walks = n_walks;
    g.n_ids = n_ids;
    g.k = k;
    g.cnt = ws.cnt.as<uint32_t>();
    g.scratch = ws.greedy.ptr;
    g.cand = cand;
    g.selected = selected;
    g.gains = gains;
    GreedyResult res;
    run_greedy_jobs(in, ws.jobs.ptr, s, timing, &res);
    return res;
}

}  // namespace sia
