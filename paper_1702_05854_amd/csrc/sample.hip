// HSAW sampler (Algorithm 1 semantics; Definition "self_walk").
//
// Attempt a starts at the floor(x0 * |V\X| / 2^64)-th non-source and follows
// the live in-edge of each node until it reaches a source (kept walk), finds
// no live edge (dead end) or comes back to a node it already visited (cycle).
// The live in-edge of node x in attempt a is drawn from Philox keyed by
// (seed, a) with counter (x,0,0,0), so within one attempt the walk is the
// iteration of a fixed function f_a -- the live-edge sample graph of that
// attempt, read lazily.  Two consequences shape the kernel:
//
//  * Exact self-avoidance needs no visited set.  A walk that revisits a node
//    is on a cycle of f_a and never leaves it; Brent's cycle detection finds
//    the cycle length lambda in O(1) state, and the first-repeat step of the
//    plain walk, mu + lambda, follows from a two-pointer pass from the start
//    (the paper's heuristics had false negatives because its draws depended
//    on the step, not the node).  A query that does not need the step count
//    of cyclic walks (SIA_FLAG_NO_CYCLE_STEPS) ends such a walk as soon as a
//    repeat is seen, with no entry search; its lanes also run Nivasch's stack
//    detector (a 16-entry stack per lane in LDS), which sees the repeat
//    within one lap of the cycle where Brent may take two.
//  * With 32-byte records (the format that searches), each wave keeps a ring
//    of what its lanes evaluated: position t of a lane's walk goes to row
//    it0 + t (it0: the iteration of its first evaluation).  A lane evaluates
//    in consecutive iterations, so a row is mostly the same iteration of all
//    64 lanes and is written whole.  With the cycle length lambda known, the
//    entry mu is the first position i with x_i == x_{i+lambda} -- false
//    before mu, true from mu on -- found by bisection over the ring (two
//    4-byte reads per probe instead of walking the graph again), and a kept
//    walk's ids are copied from the ring.  Walks longer than the ring, and
//    every walk with 16-byte records, use a two-pointer pass from the start
//    and a re-walk instead.  Coverage counts are taken afterwards, in one
//    pass over the written ids (atomics here would compete with the gathers).
//
// One launch samples a wave: attempt ranges of up to 31 queries ("slots",
// each with its own sources, seed, mode and output buffers) laid end to end.
// One lane per attempt; persistent waves refill idle lanes from a global
// counter in chunks and find the slot of each attempt in a small table kept
// in LDS; kept walks are appended with one pair of atomics per slot per
// wave.  A query with probabilistic suspects (a per-node coin threshold
// array) starts uniformly over V and, at a tagged node, reads its threshold
// in the next iteration: the node is a seed when the low half of its draw
// word is below it (a seed start gives a walk without edges).  Every
// iteration a lane computes one Philox block (its start draw, or the draw of
// the node it evaluates) and issues at most one 16-byte gather:
// mostly the in-edge record the draw selects, which says whether the evaluated
// node is a source and carries the next node's offset and degree -- so a step
// costs one random line.  With 32-byte records (any weights) the record sits
// at the interpolated position of the draw and its threshold interval
// certifies the choice (else a bracketed search); with 16-byte records
// (w = 1/d_in everywhere) the position is floor(r / q(d)) exactly and needs
// no certificate.  Node records are read only where a walk (re)starts and,
// for their source tag, at nodes without a live edge; a starting walk reads
// its rank among the sources from its query's tables a block at a time.  A
// single query is a wave of one slot, so every call goes through this kernel.
#include "common.hpp"
#include "philox.hpp"

#include <algorithm>
#include <cstddef>

namespace sia {

namespace {

constexpr int kWave = 64;

enum Phase : uint32_t {
    PH_START = 0,   // start draw; its bucket pair of the start tables
    PH_DETECT = 1,  // walk with Brent's cycle detection
    PH_MU_POS = 2,  // cycle found: advance the second pointer lambda steps
    PH_MU_A = 3,    // advance the first pointer
    PH_MU_B = 4,    // advance the second pointer, compare
    PH_EMIT = 5,    // kept walk: re-walk and write its ids
    PH_SRC = 6,     // start: the rank of the start among the sources, a 4-entry window at a time
    PH_MU_RING = 7, // cycle found: bisect the ring for the entry mu
    PH_EMIT_RING = 8  // kept walk: copy its ids from the ring
};

constexpr uint32_t kRingCells = kRingRows / 4;  // a lane's 16-byte cells: positions 4c .. 4c+3
// Depth of each lane's LDS stack of the stack cycle detector (Nivasch, IPL
// 2004) used when cyclic walks stop at detection; a power of two.
constexpr uint32_t kStack = 16;
constexpr uint32_t kCellMask = kRingCells - 1;
constexpr uint32_t kEmitPerIter = 4;  // ids a lane copies from the ring per iteration

struct WaveArgs {
    const NodeRec *nodes;
    const void *arcs;              // ArcRec[m] or ArcRec16[m]
    const SlotDev *slots;
    uint32_t n_slots;
    uint32_t chunk;                // attempts taken per refill
    const WaveTable *table;
    uint64_t guard_evals;          // no walk may need more evaluations than this
    uint32_t *ring;                // kRingRows x 64 words per wave of the grid (NULL: no ring)
};

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    uint32_t lo = __shfl(static_cast<uint32_t>(v), src, kWave);
    uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), src, kWave);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Whole 32-byte record load through a global pointer (two 16-byte loads).
__device__ __forceinline__ ArcRec load_arc(const GLOBAL ArcRec *p)
{
    const GLOBAL u32x4 *q = reinterpret_cast<const GLOBAL u32x4 *>(p);
    const u32x4 lo = q[0], hi = q[1];
    return ArcRec{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
}

// Compact format: the quantum of a node with in-degree d (>= 1) kept in 32
// bits (d = 1 has q = 2^32, kept as 2^32 - 1: the live draws r < 2^32 - 1
// then still give index 0), and its last threshold min(d * q, 2^32 - 1).
__device__ __forceinline__ void compact_node(uint32_t d, uint32_t &q, uint32_t &thr_last)
{
    const uint64_t q64 = d ? inv_indeg_quantum(d) : 0;
    const uint64_t t = static_cast<uint64_t>(d) * q64;
    q = static_cast<uint32_t>(q64 > 0xFFFFFFFFull ? 0xFFFFFFFFull : q64);
    thr_last = static_cast<uint32_t>(t > 0xFFFFFFFFull ? 0xFFFFFFFFull : t);
}

// floor(r / q) for q >= 1: a float estimate, corrected exactly.
__device__ __forceinline__ uint32_t quantum_index(uint32_t r, uint32_t q)
{
    uint32_t j = __float2uint_rz(static_cast<float>(r) * __builtin_amdgcn_rcpf(static_cast<float>(q)));
    while (static_cast<uint64_t>(j) * q > r) --j;
    while (static_cast<uint64_t>(j + 1) * q <= r) ++j;
    return j;
}

__device__ __forceinline__ uint32_t pick4(const u32x4 &v, uint32_t i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// Interpolation guess for the in-edge that is live for draw r at a node with
// deg in-edges and last threshold thr_last > r: r * deg / thr_last, exact for
// equal weights.
__device__ __forceinline__ uint32_t guess_of(uint32_t r, uint32_t deg, uint32_t thr_last)
{
    const float scale = static_cast<float>(deg) * __builtin_amdgcn_rcpf(static_cast<float>(thr_last));
    const uint32_t g = __float2uint_rz(static_cast<float>(r) * scale);
    return g >= deg ? deg - 1 : g;
}

// Index of the live in-edge (the first with thr_hi > r) among the deg arcs at
// base, given E = arcs[base + g] for the interpolation guess g (r < thr_last):
// g itself when E's interval holds r; else a search of the side E points to
// that keeps the exact thresholds at both ends of its bracket (each probe's
// interval gives them) and interpolates within it for the first kInterp
// probes (close to linear cumulative weights converge in two or three), then
// bisects (bounded in the worst case).  E ends as the chosen arc.
__device__ __forceinline__ uint32_t settle_arc(const GLOBAL ArcRec *arcs, uint32_t base, uint32_t deg,
                                               uint32_t thr_last, uint32_t g, uint32_t r, ArcRec &E)
{
    if (E.thr_lo <= r && r < E.thr_hi) return g;
    constexpr int kInterp = 3;
    uint32_t lo, hi, tlo, thi;  // answer in [lo, hi]; thr_{lo-1} = tlo <= r < thi = thr_hi
    if (E.thr_hi <= r) {
        lo = g + 1;
        hi = deg - 1;
        tlo = E.thr_hi;
        thi = thr_last;
    } else {
        lo = 0;
        hi = g - 1;
        tlo = 0;
        thi = E.thr_lo;
    }
    for (int step = 0; lo < hi; ++step) {
        uint32_t m;
        if (step < kInterp) {
            const float f = static_cast<float>(r - tlo) * __builtin_amdgcn_rcpf(static_cast<float>(thi - tlo));
            m = lo + __float2uint_rz(f * static_cast<float>(hi - lo + 1));
            m = m > hi ? hi : m;
        } else {
            m = lo + ((hi - lo) >> 1);
        }
        E = load_arc(arcs + base + m);
        if (E.thr_lo <= r && r < E.thr_hi) return m;
        if (E.thr_hi <= r) {
            lo = m + 1;
            tlo = E.thr_hi;
        } else {
            hi = m - 1;
            thi = E.thr_lo;
        }
    }
    E = load_arc(arcs + base + lo);
    return lo;
}

template <bool kCompact>
__global__ __launch_bounds__(256, 5) void k_sample(const WaveArgs A)
{
    __shared__ SlotDev sl[kMaxSlots + 1];
    __shared__ uint64_t ip[kMaxItems + 1];
    __shared__ uint64_t il[kMaxItems];
    __shared__ uint32_t is[kMaxItems];
    // per-slot counters of this workgroup: hits, dead ends, cycles, steps, evaluations, faults
    __shared__ unsigned long long acc[kMaxSlots + 1][6];
    // each lane's detector stack, entry e of thread i at stk[e][i] (bank-conflict free)
    __shared__ uint32_t stk[kStack][256];
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t n_items = A.table->n_items;
    for (uint32_t i = threadIdx.x; i < A.n_slots; i += blockDim.x) sl[i] = A.slots[i];
    for (uint32_t i = threadIdx.x; i <= n_items; i += blockDim.x) ip[i] = A.table->prefix[i];
    for (uint32_t i = threadIdx.x; i < n_items; i += blockDim.x) {
        il[i] = A.table->local[i];
        is[i] = A.table->slot[i];
    }
    for (uint32_t i = threadIdx.x; i < A.n_slots * 6; i += blockDim.x) acc[i / 6][i % 6] = 0;
    __syncthreads();
    const uint64_t total = ip[n_items];
    uint64_t *next = const_cast<uint64_t *>(&A.table->next[0]);
    // this lane's column of its wave's ring: cells of 4 positions, the 64
    // lanes' cells of one cell row side by side (1 KB).  Only the 32-byte
    // record format keeps a ring: with 16-byte records an evaluation is one
    // line, and the ring's stores cost more time than the evaluations they
    // save (rmat24: 145 against 136 ms with 19% fewer evaluations; the
    // billion-edge graph's 32-byte records: 927 against 1192 ms)
    GLOBAL uint32_t *ring = (!kCompact && A.ring) ? gp(A.ring) + (static_cast<uint64_t>(blockIdx.x) * (blockDim.x / kWave) +
                                                   threadIdx.x / kWave) * (kRingRows * kWave) + 4 * lane
                                   : nullptr;
    // word of virtual position v (= it0 + position) in the ring
    auto ring_word = [&](uint32_t v) { return ring + static_cast<uint64_t>((v >> 2) & kCellMask) * (4 * kWave) + (v & 3u); };
    // the cell being filled; written whole when its last position is, or
    // when the walk needs the ring read back
    uint32_t rb0 = 0, rb1 = 0, rb2 = 0, rb3 = 0;
    auto ring_put = [&](uint32_t v, uint32_t val) {
        const uint32_t c = v & 3u;
        rb0 = c == 0 ? val : rb0;
        rb1 = c == 1 ? val : rb1;
        rb2 = c == 2 ? val : rb2;
        rb3 = c == 3 ? val : rb3;
        if (c == 3) {
            const u32x4 cell = {rb0, rb1, rb2, rb3};
            *reinterpret_cast<GLOBAL u32x4 *>(ring_word(v & ~3u)) = cell;
        }
    };
    auto ring_flush = [&](uint32_t v_last) {  // the cell holding v_last, unless already written
        if ((v_last & 3u) != 3u) {
            const u32x4 cell = {rb0, rb1, rb2, rb3};
            *reinterpret_cast<GLOBAL u32x4 *>(ring_word(v_last & ~3u)) = cell;
        }
    };
    uint32_t iter = 0;  // wave-uniform iteration count

    // wave-uniform work state
    uint64_t chunk_next = 0, chunk_end = 0;
    bool exhausted = false;
    // lane state
    bool active = false, fetch = false;  // fetch: load cur's node record next iteration
    uint64_t a = 0, out_pos = 0, seed = 0;
    uint32_t slot = 0, mode = SIA_EDGES, tag_mask = 0;
    bool psus = false;  // the lane's query has probabilistic suspects
    // Stack detector (walks of queries that stop cyclic walks at detection):
    // the walk's nodes that no later node undercuts, increasing from the
    // bottom; a node equal to the top after popping the larger ones was
    // visited before.  The cycle's smallest node is never popped once pushed,
    // so its second visit is caught -- within one lap past the first repeat
    // instead of Brent's up to two.  A full stack drops its bottom (a ring:
    // sb is the bottom's slot); what it then misses Brent still catches.
    bool use_stack = false;
    uint32_t sd = 0, sb = 0, stop = 0;  // depth, bottom slot, top value
    bool ck = false;    // cur is a suspect: its coin threshold is read with this evaluation
    uint32_t phase = PH_START, x1 = 0, cur = 0, tort = 0, power = 1, lam = 0, t = 0, lambda = 0,
             cnt = 0, pa = 0, pb = 0, evals = 0, ptort = 0, mbase = 0,
             it0 = 0;  // iteration of the walk's first evaluation (its ring row)
    // (off, deg, thr_last, compact quantum) of the pointers' nodes: c for cur
    // (and pb in the cycle-entry search), p for pa
    uint32_t c_off = 0, c_deg = 0, c_thr = 0, c_q = 0, p_off = 0, p_deg = 0, p_thr = 0, p_q = 0;

    for (;; ++iter) {
        // ---- refill idle lanes with new attempts (converged section)
        uint64_t idle = __ballot(!active);
        while (idle != 0 && !exhausted) {
            if (chunk_next >= chunk_end) {
                uint64_t base = 0;
                if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long *>(next),
                                                static_cast<unsigned long long>(A.chunk));
                base = shfl_u64(base, 0);
                if (base >= total) {
                    exhausted = true;
                    break;
                }
                chunk_next = base;
                chunk_end = min(base + A.chunk, total);
            }
            const uint32_t need = static_cast<uint32_t>(__popcll(idle));
            const uint64_t avail = chunk_end - chunk_next;
            const uint32_t take = static_cast<uint32_t>(min(static_cast<uint64_t>(need), avail));
            const uint32_t rank = lanes_below(idle);
            if (!active && rank < take) {
                const uint64_t gidx = chunk_next + rank;
                uint32_t it = 0;
                while (it + 1 < n_items && ip[it + 1] <= gidx) ++it;
                slot = is[it];
                const SlotDev &S = sl[slot];
                a = S.attempt_base + il[it] + (gidx - ip[it]);
                seed = S.seed;
                mode = S.mode;
                tag_mask = S.tag_mask;
                psus = S.coin_thr != nullptr;
                use_stack = !S.cycle_steps;
                sd = 0;
                sb = 0;
                ck = false;
                phase = PH_START;
                fetch = false;
                evals = 0;
                active = true;
            }
            chunk_next += take;
            idle = __ballot(!active);
        }
        if (__ballot(active) == 0) break;

        // ---- stage 1: choose this iteration's draw and its one gather
        bool hit_now = false, do_eval = false, live = false, fetch_now = false, tag_only = false,
             starting = false, in_src = false;
        uint32_t y = 0, r = 0, yoff = 0, ydeg = 0, ylast = 0, g = 0;
        NodeRec R = {0u, 0u, 0u, 0u};
        ArcRec E = {};
        ArcRec16 E16 = {};
        if (active) {
            if (fetch) {  // the record of a (re)started walk's first node
                y = cur;
                fetch_now = true;
            } else if (phase == PH_START) {
                starting = true;
            } else if (phase == PH_SRC) {
                in_src = true;
            } else {
                do_eval = true;
                if (phase == PH_DETECT) {
                    y = cur;
                    if (t > 0 && !ck) {  // (a coin retry evaluates a position already checked)
                        ++lam;
                        if (cur == tort) {  // Brent: cycle of length lam (tort is never a source)
                            // The tortoise sits at positions 2^j - 1 with a window of
                            // 2^j.  If lam fits half the final window, the previous
                            // tortoise (position power/2 - 1) was off the cycle --
                            // else its window would have found it -- so the cycle
                            // entry mu is past it, not anywhere from x1 on.
                            const bool past = lam <= (power >> 1);
                            lambda = lam;
                            const uint32_t lo = past ? (power >> 1) : 0u;  // mu in [lo, t - lam]
                            do_eval = false;
                            if (!sl[slot].cycle_steps) {
                                // the walk is discarded whatever its length: done
                                atomicAdd(&acc[slot][2], 1ull);
                                atomicAdd(&acc[slot][4], static_cast<unsigned long long>(evals));
                                active = false;
                            } else if (ring && ((it0 + t - 1u) >> 2) - ((it0 + lo) >> 2) < kRingCells) {
                                // the cells of positions lo .. t-1 are all in the ring
                                ring_flush(it0 + t - 1u);
                                mbase = lo;
                                cnt = t - lam;  // the tortoise's position: on the cycle
                                phase = PH_MU_RING;
                            } else {
                                cnt = lam;
                                mbase = past ? (power >> 1) - 1u : 0u;
                                pa = past ? ptort : x1;
                                pb = pa;
                                phase = PH_MU_POS;
                                y = pa;
                                fetch_now = true;  // both pointers start from this record
                            }
                        } else if (lam == power) {
                            ptort = tort;
                            tort = cur;
                            power <<= 1;
                            lam = 0;
                        }
                    }
                } else if (phase == PH_MU_A) {
                    y = pa;
                } else if (phase == PH_EMIT) {
                    y = cur;
                } else if (phase == PH_MU_RING) {
                    // bisect [mbase, cnt] for mu, the first position i with
                    // x_i == x_{i+lambda} (compared as the ring's entries:
                    // equal chosen in-edges mean equal nodes)
                    do_eval = false;
                    if (mbase == cnt) {
                        atomicAdd(&acc[slot][2], 1ull);
                        atomicAdd(&acc[slot][3], static_cast<unsigned long long>(mbase) + lambda);
                        atomicAdd(&acc[slot][4], static_cast<unsigned long long>(evals));
                        active = false;
                    } else {
                        const uint32_t mid = (mbase + cnt) >> 1;  // mid + lambda <= t - 1
                        const uint32_t va = *ring_word(it0 + mid);
                        const uint32_t vb = *ring_word(it0 + mid + lambda);
                        if (va == vb) cnt = mid;
                        else mbase = mid + 1u;
                    }
                } else if (phase == PH_EMIT_RING) {
                    // copy positions pa .. cnt-1 of the walk, a few per iteration
                    do_eval = false;
                    const SlotDev &S = sl[slot];
                    uint32_t v[kEmitPerIter];
#pragma unroll
                    for (uint32_t e = 0; e < kEmitPerIter; ++e)
                        v[e] = pa + e < cnt ? *ring_word(it0 + pa + e) : 0u;
#pragma unroll
                    for (uint32_t e = 0; e < kEmitPerIter; ++e)
                        if (pa + e < cnt) gp(S.ids)[out_pos + e] = v[e];
                    const uint32_t n_copied = min(kEmitPerIter, cnt - pa);
                    out_pos += n_copied;
                    pa += n_copied;
                    if (pa == cnt) {
                        if (mode == SIA_NODES) gp(S.ids)[out_pos++] = cur;  // the source reached
                        atomicAdd(&acc[slot][4], static_cast<unsigned long long>(evals));
                        active = false;
                    }
                } else {
                    y = pb;
                }
            }
        }
        // one Philox block per lane and iteration: the start draw (counter
        // (0,1)) or the draw of node y (counter (y,0)); computed by every lane
        // so the wave runs the rounds once
        const uint64_t word = philox_word0(starting ? 0u : y, starting ? 1u : 0u, seed, a);
        if (active) {
            if (starting) {
                // the start is the idx-th non-source: idx + #{i : t_i <= idx}, from
                // the bucket block now (done when the next t exceeds idx) and
                // 4-entry windows of t in PH_SRC
                x1 = static_cast<uint32_t>(__umul64hi(word, sl[slot].n_ns));  // idx (< n)
            } else if (do_eval) {
                const bool pside = phase == PH_MU_A;
                yoff = pside ? p_off : c_off;
                ydeg = pside ? p_deg : c_deg;
                const uint32_t ythr = pside ? p_thr : c_thr;
                ylast = ythr;
                r = static_cast<uint32_t>(word >> 32);
                live = ydeg != 0 && r < ythr;
                if (live) {
                    if constexpr (kCompact) g = min(quantum_index(r, pside ? p_q : c_q), ydeg - 1u);
                    else g = guess_of(r, ydeg, ythr);
                } else {
                    tag_only = phase == PH_DETECT && t > 0;
                }
                if (phase == PH_DETECT) {
                    if (t == 0) it0 = iter;
                    // the walk's position t goes to ring row it0 + t, stored beside
                    // this iteration's gather so the two are in flight together
                    // (an evaluation this iteration cancels -- a source reached,
                    // a coin to read first -- leaves a row no position uses, or
                    // one its retry rewrites with the same value)
                    if (ring && live && (kCompact || mode == SIA_NODES))
                        ring_put(it0 + t, mode == SIA_EDGES ? yoff + g : y);
                }
            }
            // one 16-byte gather instruction per iteration: the node record (a
            // walk's first node, or the tag of a node without a live edge) or
            // the selected in-edge record (its first half for 32-byte records)
            // (or, for a starting walk, a 16-byte block of its query's bucket or t table)
            const GLOBAL u32x4 *src = nullptr;
            if (fetch_now || tag_only) {
                src = reinterpret_cast<const GLOBAL u32x4 *>(gp(A.nodes) + y);
            } else if (live) {
                if constexpr (kCompact)
                    src = reinterpret_cast<const GLOBAL u32x4 *>(gp(static_cast<const ArcRec16 *>(A.arcs)) + yoff + g);
                else
                    src = reinterpret_cast<const GLOBAL u32x4 *>(gp(static_cast<const ArcRec *>(A.arcs)) + yoff + g);
            } else if (starting && !psus) {
                src = reinterpret_cast<const GLOBAL u32x4 *>(gp(sl[slot].bucket) +
                                                              ((2u * (x1 >> sl[slot].bucket_shift)) & ~3u));
            } else if (in_src) {
                src = reinterpret_cast<const GLOBAL u32x4 *>(gp(sl[slot].src_t) + (cnt & ~3u));
            }
            // compact records are loaded non-temporally: the line is not read
            // again soon, and keeping it out of the caches' recent set leaves
            // them to the hot small tables (6% faster on rmat24).  A 32-byte
            // record's line is read again at once (its second half, search
            // probes), so it is cached normally (non-temporal: 10% slower).
            u32x4 v = {0u, 0u, 0u, 0u};
            if (src) {
                if constexpr (kCompact) v = __builtin_nontemporal_load(src);
                else v = *src;
            }
            const uint32_t cthr = (do_eval && ck) ? gp(sl[slot].coin_thr)[cur] : 0u;
            // the stack detector runs while the gather is in flight (a walk it
            // ends leaves that one record unused)
            if (use_stack && do_eval && phase == PH_DETECT && !ck) {
                while (sd && stop > cur) {
                    --sd;
                    stop = sd ? stk[(sb + sd - 1u) & (kStack - 1u)][threadIdx.x] : 0u;
                }
                if (sd && stop == cur) {  // a repeat: a cycle, the walk is discarded
                    do_eval = false;
                    atomicAdd(&acc[slot][2], 1ull);
                    atomicAdd(&acc[slot][4], static_cast<unsigned long long>(evals));
                    active = false;
                } else {
                    if (sd == kStack) sb = (sb + 1u) & (kStack - 1u);
                    else ++sd;
                    stk[(sb + sd - 1u) & (kStack - 1u)][threadIdx.x] = cur;
                    stop = cur;
                }
            }
            if (fetch_now || tag_only) {
                R = NodeRec{v.x, v.y, v.z, v.w};
            } else if (live) {
                if constexpr (kCompact) {
                    E16 = ArcRec16{v.x, v.y, v.z, v.w};
                } else {
                    const u32x4 h = src[1];
                    E = ArcRec{v.x, v.y, v.z, v.w, h.x, h.y, h.z, h.w};
                }
            } else if (starting || in_src) {
                const SlotDev &D = sl[slot];
                uint32_t c = 0;
                bool more = false;  // the next window of t is needed
                if (psus) {  // uniform over V: the start is idx itself
                } else if (starting) {  // the bucket's pair: the count below it, the next t
                    const uint32_t k = (2u * (x1 >> D.bucket_shift)) & 3u;
                    c = pick4(v, k);
                    more = c < D.n_src && pick4(v, k + 1u) <= x1;
                } else {
                    c = cnt;
                    const uint32_t end = (c | 3u) + 1u;
                    while (c < end && c < D.n_src && pick4(v, c & 3u) <= x1) ++c;
                    more = c == end && c < D.n_src;
                }
                if (more) {
                    cnt = c;
                    phase = PH_SRC;
                } else {  // start at x1 = idx + c: fetch its record next
                    x1 += c;
                    cur = x1;
                    tort = x1;
                    power = 1;
                    lam = 0;
                    t = 0;
                    phase = PH_DETECT;
                    fetch = true;
                }
            }
            if (do_eval && phase == PH_DETECT) {
                if (ck) {  // a suspect: a seed when its coin is below the threshold
                    ck = false;
                    if (static_cast<uint32_t>(word) < cthr) {
                        hit_now = true;
                        do_eval = false;
                    }
                } else if (t > 0) {
                    const uint32_t tag = live ? (kCompact ? E16.head_tag : E.head_tag) : R.tag;
                    if (tag & tag_mask) {
                        do_eval = false;
                        if (psus) ck = true;  // its coin decides, with its threshold, next iteration
                        else hit_now = true;  // reached a source: kept walk
                    } else if (t > A.guard_evals) {  // unreachable for a correct walk
                        atomicAdd(&acc[slot][5], 1ull);
                        active = false;
                        do_eval = false;
                    }
                }
            }
            if (fetch_now && psus && phase == PH_DETECT && t == 0 && (R.tag & tag_mask))
                ck = true;  // the start is a suspect: its coin comes first
            if (fetch_now) {
                c_off = R.off;
                c_deg = R.deg;
                c_thr = R.thr_last;
                if constexpr (kCompact) compact_node(R.deg, c_q, c_thr);
                if (phase == PH_MU_POS) {
                    p_off = c_off;
                    p_deg = c_deg;
                    p_thr = c_thr;
                    p_q = c_q;
                }
                fetch = false;
            }
        }

        // ---- stage 2: reserve output for kept walks, one pair of atomics per slot (converged)
        uint64_t hm = __ballot(hit_now);
        while (hm) {
            const int leader = __ffsll(static_cast<long long>(hm)) - 1;
            const uint32_t s_lead = __shfl(slot, leader, kWave);
            const bool mine = hit_now && slot == s_lead;
            const uint64_t mm = __ballot(mine);
            const uint32_t len = mine ? (mode == SIA_EDGES ? t : t + 1u) : 0u;
            const uint32_t incl = wave_incl_scan_u32(len, lane);
            const uint32_t total_len = __shfl(incl, kWave - 1, kWave);
            uint64_t wbase = 0, ibase = 0;
            if (lane == leader) {
                GLOBAL uint64_t *ctr = gp(sl[s_lead].counters);
                wbase = __hip_atomic_fetch_add(&ctr[ST_WALKS], static_cast<uint64_t>(__popcll(mm)),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ibase = __hip_atomic_fetch_add(&ctr[ST_IDS], static_cast<uint64_t>(total_len),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            wbase = shfl_u64(wbase, leader);
            ibase = shfl_u64(ibase, leader);
            if (mine) {
                const SlotDev &S = sl[slot];
                atomicAdd(&acc[slot][0], 1ull);
                atomicAdd(&acc[slot][3], static_cast<unsigned long long>(t));
                const uint64_t widx = wbase + lanes_below(mm);
                const uint64_t ioff = ibase + incl - len;
                if (widx < S.walk_cap && ioff + len <= S.id_cap) {
                    gp(S.walk_attempt)[widx] = a;
                    gp(S.walk_off)[widx] = ioff;
                    gp(S.walk_len)[widx] = len;
                    out_pos = ioff;
                    if (mode == SIA_NODES) gp(S.ids)[out_pos++] = x1;
                    if (t == 0) {  // a seed start: the walk <x1>, nothing more to write
                        atomicAdd(&acc[slot][4], static_cast<unsigned long long>(evals));
                        active = false;
                    } else if (ring && ((it0 + t - 1u) >> 2) - (it0 >> 2) < kRingCells) {
                        // positions 0 .. t-1 sit in the ring: edges copy all
                        // of them, nodes positions 1 .. t-1 and then the
                        // source reached (cur)
                        ring_flush(it0 + t - 1u);
                        phase = PH_EMIT_RING;
                        pa = mode == SIA_NODES ? 1u : 0u;
                        cnt = t;
                    } else {
                        phase = PH_EMIT;
                        cur = x1;
                        fetch = true;
                        cnt = t;
                    }
                } else {
                    gp(S.counters)[ST_OVERFLOW] = 1;
                    atomicAdd(&acc[slot][4], static_cast<unsigned long long>(evals));
                    active = false;
                }
            }
            hm &= ~mm;
        }

        // ---- stage 3: one live-edge evaluation per evaluating lane
        if (do_eval) {
            uint32_t j = 0, u = 0;
            if (live) {
                uint32_t uo, ud, ut, uq = 0;
                if constexpr (kCompact) {
                    j = yoff + g;
                    u = E16.row;
                    uo = E16.u_off;
                    ud = E16.u_deg;
                    compact_node(ud, uq, ut);
                } else {
                    j = yoff + settle_arc(gp(static_cast<const ArcRec *>(A.arcs)), yoff, ydeg, ylast, g, r, E);
                    u = E.row;
                    uo = E.u_off;
                    ud = E.u_deg;
                    ut = E.u_thr;
                }
                if (phase == PH_MU_A) {
                    p_off = uo;
                    p_deg = ud;
                    p_thr = ut;
                    p_q = uq;
                } else {
                    c_off = uo;
                    c_deg = ud;
                    c_thr = ut;
                    c_q = uq;
                }
            }
            ++evals;
            bool done = false;
            if (phase == PH_DETECT) {
                if constexpr (!kCompact)  // (the searched in-edge is known only now)
                    if (ring && live && mode == SIA_EDGES)
                        ring_put(it0 + t, j);
                ++t;
                if (!live) {
                    atomicAdd(&acc[slot][1], 1ull);
                    atomicAdd(&acc[slot][3], static_cast<unsigned long long>(t));
                    done = true;
                } else {
                    cur = u;
                }
            } else if (!live) {  // re-walks retrace live edges only
                atomicAdd(&acc[slot][5], 1ull);
                done = true;
            } else if (phase == PH_MU_POS) {
                pb = u;
                if (--cnt == 0) {
                    if (pa == pb) {  // the search start lies on the cycle: mu = mbase (= 0)
                        atomicAdd(&acc[slot][2], 1ull);
                        atomicAdd(&acc[slot][3], static_cast<unsigned long long>(mbase) + lambda);
                        done = true;
                    } else {
                        phase = PH_MU_A;
                    }
                }
            } else if (phase == PH_MU_A) {
                pa = u;
                phase = PH_MU_B;
            } else if (phase == PH_MU_B) {
                pb = u;
                ++cnt;
                if (pa == pb) {  // first repeat after mu + lambda draws, mu = mbase + cnt
                    atomicAdd(&acc[slot][2], 1ull);
                    atomicAdd(&acc[slot][3], static_cast<unsigned long long>(mbase) + cnt + lambda);
                    done = true;
                } else if (cnt > t) {
                    atomicAdd(&acc[slot][5], 1ull);
                    done = true;
                } else {
                    phase = PH_MU_A;
                }
            } else {  // PH_EMIT
                const SlotDev &S = sl[slot];
                const uint32_t id = (mode == SIA_EDGES) ? j : u;
                gp(S.ids)[out_pos++] = id;
                cur = u;
                if (--cnt == 0) done = true;
            }
            if (done) {
                atomicAdd(&acc[slot][4], static_cast<unsigned long long>(evals));
                active = false;
            }
        }
    }

    // ---- fold this workgroup's per-slot counters into the global ones
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < A.n_slots * 6; i += blockDim.x) {
        const unsigned long long v = acc[i / 6][i % 6];
        if (!v) continue;
        const int map[6] = {ST_HITS, ST_DEAD, ST_CYCLE, ST_STEPS, ST_EVALS, ST_FAULTS};
        __hip_atomic_fetch_add(gp(sl[i / 6].counters) + map[i % 6], static_cast<uint64_t>(v),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Set (or clear) bit mask in the tag of every source and in the head_tag
// copy of each of its in-edge records (word tag_words[j * stride] of record j);
// one wave per source.
__global__ __launch_bounds__(256) void k_tag_sources(const int32_t *src, uint32_t n_src, NodeRec *nodes,
                                                     uint32_t *tag_words, uint32_t stride, uint32_t mask,
                                                     int set)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    for (uint64_t w = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave; w < n_src;
         w += waves) {
        const uint32_t v = static_cast<uint32_t>(src[w]);
        const uint32_t off = nodes[v].off, deg = nodes[v].deg;
        for (uint32_t i = lane; i < deg; i += kWave) {
            uint32_t *p = tag_words + static_cast<uint64_t>(off + i) * stride;
            if (set) atomicOr(p, mask);
            else atomicAnd(p, ~mask);
        }
        if (lane == 0) {
            if (set) atomicOr(&nodes[v].tag, mask);
            else atomicAnd(&nodes[v].tag, ~mask);
        }
    }
}

// coin_thr[ids[i]] = q[i]: the seed thresholds of a query's suspects (the
// other entries are never read: only tagged nodes look theirs up)
__global__ __launch_bounds__(256) void k_scatter_coin(const int32_t *ids, const uint32_t *q, uint32_t count,
                                                      uint32_t *coin_thr)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) gp(coin_thr)[gp(ids)[i]] = gp(q)[i];
}

int max_blocks_per_cu(bool compact)
{
    static int per_cu[2] = {0, 0};
    int &v = per_cu[compact ? 1 : 0];
    if (!v) {
        int b = 0;
        if (compact) SIA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_sample<true>, 256, 0));
        else SIA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_sample<false>, 256, 0));
        v = std::max(1, b);
    }
    return v;
}

bool compact_arcs(const sia_graph *g) { return g->arc_bytes == sizeof(ArcRec16); }

}  // namespace

int sampler_max_blocks_per_cu(const sia_graph *g) { return max_blocks_per_cu(compact_arcs(g)); }

void fill_wave_table(WaveTable &t, const WaveItem *items, uint32_t n_items, uint32_t n_slots)
{
    SIA_REQUIRE(n_slots >= 1 && n_slots <= kMaxSlots + 1 && n_items >= 1 && n_items <= kMaxItems,
                SIA_EINVAL, "bad wave shape");
    t = WaveTable{};
    uint64_t run = 0;
    for (uint32_t i = 0; i < n_items; ++i) {
        SIA_REQUIRE(items[i].slot < n_slots, SIA_EINVAL, "wave item names a missing slot");
        t.prefix[i] = run;
        t.local[i] = items[i].local_start;
        t.slot[i] = items[i].slot;
        run += items[i].count;
    }
    t.prefix[n_items] = run;
    t.n_items = n_items;
}

void tag_sources(const sia_graph *g, const int32_t *d_src, uint32_t n_src, uint32_t mask, bool set,
                 hipStream_t s)
{
    if (!n_src) return;
    const unsigned blocks = static_cast<unsigned>(
        std::min<uint64_t>((static_cast<uint64_t>(n_src) + 3) / 4, static_cast<uint64_t>(device_cu_count()) * 16));
    uint32_t *words = g->arcs.as<uint32_t>();
    uint32_t stride;
    if (compact_arcs(g)) {
        words += offsetof(ArcRec16, head_tag) / sizeof(uint32_t);
        stride = sizeof(ArcRec16) / sizeof(uint32_t);
    } else {
        words += offsetof(ArcRec, head_tag) / sizeof(uint32_t);
        stride = sizeof(ArcRec) / sizeof(uint32_t);
    }
    hipLaunchKernelGGL(k_tag_sources, dim3(blocks), dim3(256), 0, s, d_src, n_src,
                       const_cast<NodeRec *>(g->nodes.as<NodeRec>()), words, stride, mask, set ? 1 : 0);
    SIA_HIP(hipGetLastError());
}

size_t sampler_ring_bytes(const sia_graph *g)
{
    if (compact_arcs(g)) return 0;  // (no ring with 16-byte records)
    const uint64_t waves = static_cast<uint64_t>(max_blocks_per_cu(compact_arcs(g))) * device_cu_count() * (256 / kWave);
    return static_cast<size_t>(waves * kRingRows * kWave * sizeof(uint32_t));
}

void launch_wave(const sia_graph *g, const SlotDev *d_slots, uint32_t n_slots,
                 const WaveTable *d_table, const SamplerConfig &cfg, uint32_t *ring, hipStream_t s)
{
    SIA_REQUIRE(n_slots >= 1 && n_slots <= kMaxSlots + 1, SIA_EINVAL, "bad wave shape");
    SIA_REQUIRE(cfg.chunk >= 1 && cfg.chunk <= (1u << 20), SIA_EINVAL, "bad refill chunk");
    const bool compact = compact_arcs(g);
    const int per_cu = cfg.blocks_per_cu > 0 ? std::min(cfg.blocks_per_cu, max_blocks_per_cu(compact))
                                             : max_blocks_per_cu(compact);
    WaveArgs A;
    A.nodes = g->nodes.as<NodeRec>();
    A.arcs = g->arcs.ptr;
    A.slots = d_slots;
    A.n_slots = n_slots;
    A.chunk = cfg.chunk;
    A.table = d_table;
    A.guard_evals = 3 * static_cast<uint64_t>(g->n) + 8;
    A.ring = ring;  // sized by sampler_ring_bytes for the largest grid
    const int cus = cfg.cus > 0 ? std::min(cfg.cus, device_cu_count()) : device_cu_count();
    if (compact) hipLaunchKernelGGL(k_sample<true>, dim3(per_cu * cus), dim3(256), 0, s, A);
    else hipLaunchKernelGGL(k_sample<false>, dim3(per_cu * cus), dim3(256), 0, s, A);
    SIA_HIP(hipGetLastError());
}

namespace {
// Clears a query's source-tag bit on every exit from the sampler, thrown
// errors included: a tag left set would make later queries on the graph
// treat those nodes as sources.
struct SourceTagScope {
    const sia_graph *g;
    const int32_t *d_src;
    uint32_t n_src, mask;
    hipStream_t s;
    SourceTagScope(const sia_graph *g_, const int32_t *d_src_, uint32_t n_src_, uint32_t mask_, hipStream_t s_)
        : g(g_), d_src(d_src_), n_src(n_src_), mask(mask_), s(s_)
    {
        tag_sources(g, d_src, n_src, mask, true, s);
    }
    ~SourceTagScope()
    {
        try {
            tag_sources(g, d_src, n_src, mask, false, s);
            (void)hipStreamSynchronize(s);
        } catch (...) {
            // the device already failed; nothing more can be undone here
        }
    }
    SourceTagScope(const SourceTagScope &) = delete;
    SourceTagScope &operator=(const SourceTagScope &) = delete;
};
}  // namespace

SampleResult run_sampler(sia_graph *g, int mode, const SourceTables &st, uint64_t n_attempts,
                         uint64_t attempt_offset, uint64_t seed, hipStream_t s, bool timing,
                         bool cycle_steps)
{
    Workspace &ws = g->ws;
    const uint32_t n_src = static_cast<uint32_t>(st.sorted.size());
    const uint32_t mask = 1u << kSoloBit;

    ws.src_sorted.ensure(sizeof(int32_t) * n_src);
    ws.src_t.ensure(sizeof(uint32_t) * st.t.size());
    ws.bucket.ensure(sizeof(uint32_t) * st.bucket.size());
    ws.counters.ensure(sizeof(uint64_t) * ST_COUNT + sizeof(SlotDev) + sizeof(WaveTable) + 256);
    ws.ring.ensure(sampler_ring_bytes(g));
    SIA_HIP(hipMemcpyAsync(ws.src_sorted.ptr, st.sorted.data(), sizeof(int32_t) * n_src,
                           hipMemcpyHostToDevice, s));
    SIA_HIP(hipMemcpyAsync(ws.src_t.ptr, st.t.data(), sizeof(uint32_t) * st.t.size(),
                           hipMemcpyHostToDevice, s));
    SIA_HIP(hipMemcpyAsync(ws.bucket.ptr, st.bucket.data(), sizeof(uint32_t) * st.bucket.size(),
                           hipMemcpyHostToDevice, s));
    if (st.probabilistic) {
        ws.coin_thr.ensure(sizeof(uint32_t) * static_cast<uint64_t>(g->n));
        ws.coin_src.ensure(sizeof(uint32_t) * n_src);
        SIA_HIP(hipMemcpyAsync(ws.coin_src.ptr, st.coin.data(), sizeof(uint32_t) * n_src, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_scatter_coin, dim3((n_src + 255) / 256), dim3(256), 0, s, ws.src_sorted.as<int32_t>(),
                           ws.coin_src.as<uint32_t>(), n_src, ws.coin_thr.as<uint32_t>());
        SIA_HIP(hipGetLastError());
    }
    const SourceTagScope tags(g, ws.src_sorted.as<int32_t>(), n_src, mask, s);
    char *cbase = ws.counters.as<char>();
    uint64_t *d_counters = reinterpret_cast<uint64_t *>(cbase);
    SlotDev *d_slot = reinterpret_cast<SlotDev *>(cbase + sizeof(uint64_t) * ST_COUNT);
    WaveTable *d_table = reinterpret_cast<WaveTable *>(
        cbase + ((sizeof(uint64_t) * ST_COUNT + sizeof(SlotDev) + 255) / 256) * 256);

    // The first call on a graph sizes the walk buffers from a pilot of this
    // query's first attempts (its output is discarded), so a cold query does
    // not run the full launch twice.
    const uint64_t kPilot = uint64_t(1) << 16;
    bool pilot = !ws.walk_cap && n_attempts > kPilot;
    if (!ws.walk_cap) {
        ws.walk_cap = std::min<uint64_t>(n_attempts, std::max<uint64_t>(1u << 20, n_attempts / 16));
        ws.id_cap = std::max<uint64_t>(1u << 24, ws.walk_cap * 32);
    }

    SampleResult res;
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
        const uint64_t launch_attempts = pilot ? kPilot : n_attempts;
        ws.walk_attempt.ensure(sizeof(uint64_t) * ws.walk_cap);
        ws.walk_off.ensure(sizeof(uint64_t) * ws.walk_cap);
        ws.walk_len.ensure(sizeof(uint32_t) * ws.walk_cap);
        ws.ids.ensure(sizeof(uint32_t) * ws.id_cap);
        SIA_HIP(hipMemsetAsync(d_counters, 0, sizeof(uint64_t) * ST_COUNT, s));

        SlotDev S{};
        S.seed = seed;
        S.attempt_base = attempt_offset;
        S.n_ns = st.n_ns;
        S.src_t = ws.src_t.as<uint32_t>();
        S.bucket = ws.bucket.as<uint32_t>();
        S.n_src = n_src;
        S.bucket_shift = st.shift;
        S.tag_mask = mask;
        S.mode = static_cast<uint32_t>(mode);
        S.walk_attempt = ws.walk_attempt.as<uint64_t>();
        S.walk_off = ws.walk_off.as<uint64_t>();
        S.walk_len = ws.walk_len.as<uint32_t>();
        S.ids = ws.ids.as<uint32_t>();
        S.walk_cap = ws.walk_cap;
        S.id_cap = ws.id_cap;
        S.counters = d_counters;
        S.coin_thr = st.probabilistic ? ws.coin_thr.as<uint32_t>() : nullptr;
        S.cycle_steps = cycle_steps ? 1u : 0u;
        SIA_HIP(hipMemcpyAsync(d_slot, &S, sizeof(S), hipMemcpyHostToDevice, s));
        const WaveItem item{0u, 0u, launch_attempts};
        WaveTable table;
        fill_wave_table(table, &item, 1, 1);
        SIA_HIP(hipMemcpyAsync(d_table, &table, sizeof(table), hipMemcpyHostToDevice, s));

        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            SIA_HIP(hipEventCreate(&e0));
            SIA_HIP(hipEventCreate(&e1));
            SIA_HIP(hipEventRecord(e0, s));
        }
        launch_wave(g, d_slot, 1, d_table, SamplerConfig{}, ws.ring.as<uint32_t>(), s);
        if (timing) SIA_HIP(hipEventRecord(e1, s));

        uint64_t h[ST_COUNT];
        SIA_HIP(hipMemcpyAsync(h, d_counters, sizeof(h), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        if (timing) {
            SIA_HIP(hipEventElapsedTime(&res.ms, e0, e1));
            SIA_HIP(hipEventDestroy(e0));
            SIA_HIP(hipEventDestroy(e1));
        }
        if (h[ST_FAULTS]) throw Error{SIA_EDEVICE, "sampler consistency check failed"};
        if (pilot) {
            // room for the whole query at the pilot's rates, plus 25% and slack
            const double scale = 1.25 * static_cast<double>(n_attempts) / static_cast<double>(kPilot);
            ws.walk_cap = std::max<uint64_t>(ws.walk_cap, static_cast<uint64_t>(scale * h[ST_WALKS]) + 4096);
            ws.id_cap = std::max<uint64_t>(ws.id_cap, static_cast<uint64_t>(scale * h[ST_IDS]) + 65536);
            ws.walk_cap = std::min<uint64_t>(ws.walk_cap, n_attempts);
            pilot = false;
            --attempt;  // the pilot is not one of the tries
            continue;
        }
        res.walks = h[ST_WALKS];
        res.ids = h[ST_IDS];
        res.hits = h[ST_HITS];
        res.dead = h[ST_DEAD];
        res.cycles = h[ST_CYCLE];
        res.steps = h[ST_STEPS];
        res.evals = h[ST_EVALS];
        ok = !h[ST_OVERFLOW];
        if (!ok) {  // the counters say exactly how much room the walks need: rerun once
            ws.walk_cap = std::max(ws.walk_cap, h[ST_WALKS]);
            ws.id_cap = std::max(ws.id_cap, h[ST_IDS] + 1);
        }
    }
    SIA_REQUIRE(ok, SIA_EDEVICE, "sampler output did not fit after resizing");
    return res;
}

}  // namespace sia
