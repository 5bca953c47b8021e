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
//    on the step, not the node).
//  * A kept walk is re-walked to emit its ids, so no per-lane path storage
//    is needed either; coverage counts are incremented as the ids are
//    written.
//
// One lane per attempt; persistent waves refill idle lanes from a global
// attempt counter in chunks; kept walks are appended with one pair of
// atomics per wave.  Every iteration a lane computes one Philox block (its
// start draw, or the draw of the node it evaluates) and, when evaluating,
// gathers the 16-byte node record (which also carries the source tag) and
// one or two 8-byte edge records (threshold + tail).
#include "common.hpp"
#include "philox.hpp"

#include <algorithm>

namespace sia {

namespace {

constexpr int kWave = 64;
constexpr uint64_t kChunk = 256;

enum Phase : uint32_t {
    PH_START = 0,   // compute the start node
    PH_DETECT = 1,  // walk with Brent's cycle detection
    PH_MU_POS = 2,  // cycle found: advance the second pointer lambda steps
    PH_MU_A = 3,    // advance the first pointer
    PH_MU_B = 4,    // advance the second pointer, compare
    PH_EMIT = 5     // kept walk: re-walk and write its ids
};

struct SampleArgs {
    const NodeRec *nodes;
    const EdgeRec *edges;
    const uint32_t *src_t;    // t_i = s_i - i over sorted sources
    const uint32_t *bucket;   // bucket[b] = #{i : t_i < b << bucket_shift}
    uint32_t n_src;
    uint32_t bucket_shift;
    uint32_t tag;             // source tag of this query in NodeRec::tag
    uint64_t n_ns;
    uint64_t seed;
    uint64_t attempt_offset;
    uint64_t n_attempts;
    uint64_t guard_evals;     // no walk may need more evaluations than this
    uint64_t *stats;
    uint64_t *walk_attempt;
    uint64_t *walk_off;
    uint32_t *walk_len;
    uint32_t *ids;
    uint32_t *cnt;            // coverage counts (nullptr: not counted)
    uint64_t walk_cap;
    uint64_t id_cap;
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

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), d, kWave);
        uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), d, kWave);
        v += (static_cast<uint64_t>(hi) << 32) | lo;
    }
    return v;
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

// First in-edge j of the node with record R whose threshold exceeds r, or
// false for "no live edge" (no in-edge, or r >= thr_last).  The first probe
// is the interpolation guess r * deg / thr_last, certified by
// thr[g-1] <= r < thr[g]; otherwise bisection on the side the probe points to.
__device__ __forceinline__ bool select_edge(const EdgeRec *__restrict__ edges, const NodeRec &R,
                                            uint32_t r, uint32_t &j, uint32_t &u)
{
    if (R.deg == 0 || r >= R.thr_last) return false;
    const float scale = static_cast<float>(R.deg) * __builtin_amdgcn_rcpf(static_cast<float>(R.thr_last));
    uint32_t g = __float2uint_rz(static_cast<float>(r) * scale);
    if (g >= R.deg) g = R.deg - 1;
    const uint32_t base = R.off;
    EdgeRec e = edges[base + g];
    const uint32_t prev = g ? edges[base + g - 1].thr : 0u;
    if (e.thr > r && prev <= r) {
        j = base + g;
        u = e.row;
        return true;
    }
    uint32_t lo, hi;  // answer in [lo, hi]; thr[hi] > r
    if (e.thr <= r) {
        lo = g + 1;
        hi = R.deg - 1;
    } else {
        lo = 0;
        hi = g - 1;
    }
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (edges[base + mid].thr > r) hi = mid;
        else lo = mid + 1;
    }
    e = edges[base + lo];
    j = base + lo;
    u = e.row;
    return true;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_sample(const SampleArgs A)
{
    const int lane = threadIdx.x & (kWave - 1);
    // wave-uniform work state
    uint64_t chunk_next = 0, chunk_end = 0;
    bool exhausted = false;
    // lane state
    bool active = false;
    uint64_t a = 0, out_pos = 0;
    uint32_t phase = PH_START, x1 = 0, cur = 0, tort = 0, power = 1, lam = 0, t = 0, lambda = 0,
             cnt = 0, pa = 0, pb = 0;
    uint32_t hits = 0, dead = 0, cycles = 0, faults = 0;
    uint64_t steps = 0, evals = 0;

    for (;;) {
        // ---- refill idle lanes with new attempts (converged section)
        uint64_t idle = __ballot(!active);
        while (idle != 0 && !exhausted) {
            if (chunk_next >= chunk_end) {
                uint64_t base = 0;
                if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long *>(&A.stats[ST_NEXT]),
                                                static_cast<unsigned long long>(kChunk));
                base = shfl_u64(base, 0);
                if (base >= A.n_attempts) {
                    exhausted = true;
                    break;
                }
                chunk_next = base;
                chunk_end = min(base + kChunk, A.n_attempts);
            }
            const uint32_t need = static_cast<uint32_t>(__popcll(idle));
            const uint64_t avail = chunk_end - chunk_next;
            const uint32_t take = static_cast<uint32_t>(min(static_cast<uint64_t>(need), avail));
            const uint32_t rank = lanes_below(idle);
            if (!active && rank < take) {
                a = A.attempt_offset + chunk_next + rank;
                phase = PH_START;
                active = true;
            }
            chunk_next += take;
            idle = __ballot(!active);
        }
        if (__ballot(active) == 0) break;

        // ---- stage 1: choose this iteration's draw; start draws; load the record
        bool hit_now = false, do_eval = false;
        uint32_t y = 0;
        NodeRec R = {0u, 0u, 0u, 0u};
        uint64_t word = 0;
        if (active) {
            if (phase == PH_DETECT) {
                y = cur;
                if (t > 0) {
                    ++lam;
                    if (cur == tort) {  // Brent: cycle of length lam (tort is never a source)
                        lambda = lam;
                        cnt = lam;
                        pa = x1;
                        pb = x1;
                        phase = PH_MU_POS;
                        y = pb;
                    } else if (lam == power) {
                        tort = cur;
                        power <<= 1;
                        lam = 0;
                    }
                }
            } else if (phase == PH_MU_A) {
                y = pa;
            } else if (phase == PH_EMIT) {
                y = cur;
            } else {
                y = pb;
            }
            word = phase == PH_START ? philox_word0(0, 1, A.seed, a) : philox_word0(y, 0, A.seed, a);
            if (phase == PH_START) {
                const uint64_t idx = __umul64hi(word, A.n_ns);
                uint32_t c = A.bucket[idx >> A.bucket_shift];
                while (c < A.n_src && A.src_t[c] <= idx) ++c;
                x1 = static_cast<uint32_t>(idx + c);
                cur = x1;
                tort = x1;
                power = 1;
                lam = 0;
                t = 0;
                phase = PH_DETECT;
            } else {
                R = A.nodes[y];
                do_eval = true;
                if (phase == PH_DETECT && t > 0 && R.tag == A.tag) {
                    hit_now = true;
                    do_eval = false;
                } else if (phase == PH_DETECT && t > A.guard_evals) {  // unreachable for a correct walk
                    ++faults;
                    active = false;
                    do_eval = false;
                }
            }
        }

        // ---- stage 2: reserve output for kept walks (converged section)
        const uint64_t hm = __ballot(hit_now);
        if (hm) {
            const uint32_t len = hit_now ? (MODE == SIA_EDGES ? t : t + 1u) : 0u;
            const uint32_t incl = wave_incl_scan_u32(len, lane);
            const uint32_t total = __shfl(incl, kWave - 1, kWave);
            uint64_t wbase = 0, ibase = 0;
            if (lane == 0) {
                wbase = atomicAdd(reinterpret_cast<unsigned long long *>(&A.stats[ST_WALKS]),
                                  static_cast<unsigned long long>(__popcll(hm)));
                ibase = atomicAdd(reinterpret_cast<unsigned long long *>(&A.stats[ST_IDS]),
                                  static_cast<unsigned long long>(total));
            }
            wbase = shfl_u64(wbase, 0);
            ibase = shfl_u64(ibase, 0);
            if (hit_now) {
                ++hits;
                steps += t;
                const uint64_t widx = wbase + lanes_below(hm);
                const uint64_t ioff = ibase + incl - len;
                if (widx < A.walk_cap && ioff + len <= A.id_cap) {
                    A.walk_attempt[widx] = a;
                    A.walk_off[widx] = ioff;
                    A.walk_len[widx] = len;
                    out_pos = ioff;
                    if (MODE == SIA_NODES) {
                        A.ids[out_pos++] = x1;
                        if (A.cnt) atomicAdd(&A.cnt[x1], 1u);
                    }
                    phase = PH_EMIT;
                    cur = x1;
                    cnt = t;
                } else {
                    A.stats[ST_OVERFLOW] = 1;
                    active = false;
                }
            }
        }

        // ---- stage 3: one live-edge evaluation per evaluating lane
        if (do_eval) {
            uint32_t j = 0, u = 0;
            const bool live = select_edge(A.edges, R, static_cast<uint32_t>(word >> 32), j, u);
            ++evals;
            if (phase == PH_DETECT) {
                ++t;
                if (!live) {
                    ++dead;
                    steps += t;
                    active = false;
                } else {
                    cur = u;
                }
            } else if (!live) {  // re-walks retrace live edges only
                ++faults;
                active = false;
            } else if (phase == PH_MU_POS) {
                pb = u;
                if (--cnt == 0) {
                    if (pa == pb) {  // the start lies on the cycle: mu = 0
                        ++cycles;
                        steps += lambda;
                        active = false;
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
                if (pa == pb) {  // first repeat after mu + lambda draws
                    ++cycles;
                    steps += static_cast<uint64_t>(cnt) + lambda;
                    active = false;
                } else if (cnt > t) {
                    ++faults;
                    active = false;
                } else {
                    phase = PH_MU_A;
                }
            } else {  // PH_EMIT
                const uint32_t id = (MODE == SIA_EDGES) ? j : u;
                A.ids[out_pos++] = id;
                if (A.cnt) atomicAdd(&A.cnt[id], 1u);
                cur = u;
                if (--cnt == 0) active = false;
            }
        }
    }

    // ---- fold the lane counters into the global ones (one atomic per wave)
    const uint64_t s_hits = wave_sum_u64(hits), s_dead = wave_sum_u64(dead),
                   s_cyc = wave_sum_u64(cycles), s_steps = wave_sum_u64(steps),
                   s_evals = wave_sum_u64(evals), s_faults = wave_sum_u64(faults);
    if (lane == 0) {
        auto add = [&](int slot, uint64_t v) {
            if (v) atomicAdd(reinterpret_cast<unsigned long long *>(&A.stats[slot]),
                             static_cast<unsigned long long>(v));
        };
        add(ST_HITS, s_hits);
        add(ST_DEAD, s_dead);
        add(ST_CYCLE, s_cyc);
        add(ST_STEPS, s_steps);
        add(ST_EVALS, s_evals);
        add(ST_FAULTS, s_faults);
    }
}

__global__ void k_tag_sources(const int32_t *src, uint32_t n_src, NodeRec *nodes, uint32_t tag)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_src) nodes[src[i]].tag = tag;
}

__global__ void k_clear_tags(NodeRec *nodes, uint64_t n)
{
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) nodes[i].tag = 0;
}

template <int MODE>
int persistent_blocks()
{
    static int blocks = 0;
    if (!blocks) {
        int per_cu = 0;
        SIA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sample<MODE>, 256, 0));
        blocks = std::max(1, per_cu) * device_cu_count();
    }
    return blocks;
}

}  // namespace

SampleResult run_sampler(sia_graph *g, int mode, const SourceTables &st, uint64_t n_attempts,
                         uint64_t attempt_offset, uint64_t seed, hipStream_t s, bool timing,
                         bool count_ids)
{
    Workspace &ws = g->ws;
    const uint32_t n_src = static_cast<uint32_t>(st.sorted.size());
    const uint64_t id_space = mode == SIA_EDGES ? static_cast<uint64_t>(g->m) : static_cast<uint64_t>(g->n);

    ws.src_sorted.ensure(sizeof(int32_t) * n_src);
    ws.src_t.ensure(sizeof(uint32_t) * n_src);
    ws.bucket.ensure(sizeof(uint32_t) * st.bucket.size());
    ws.counters.ensure(sizeof(uint64_t) * ST_COUNT);
    SIA_HIP(hipMemcpyAsync(ws.src_sorted.ptr, st.sorted.data(), sizeof(int32_t) * n_src,
                           hipMemcpyHostToDevice, s));
    SIA_HIP(hipMemcpyAsync(ws.src_t.ptr, st.t.data(), sizeof(uint32_t) * n_src,
                           hipMemcpyHostToDevice, s));
    SIA_HIP(hipMemcpyAsync(ws.bucket.ptr, st.bucket.data(), sizeof(uint32_t) * st.bucket.size(),
                           hipMemcpyHostToDevice, s));
    // a fresh tag per query marks exactly its sources
    if (++g->tag == 0) {
        hipLaunchKernelGGL(k_clear_tags, dim3(device_cu_count() * 8), dim3(256), 0, s,
                           g->nodes.as<NodeRec>(), static_cast<uint64_t>(g->n));
        SIA_HIP(hipGetLastError());
        g->tag = 1;
    }
    hipLaunchKernelGGL(k_tag_sources, dim3((n_src + 255) / 256), dim3(256), 0, s,
                       ws.src_sorted.as<int32_t>(), n_src, g->nodes.as<NodeRec>(), g->tag);
    SIA_HIP(hipGetLastError());
    if (count_ids) ws.cnt.ensure(sizeof(uint32_t) * std::max<uint64_t>(id_space, 1));

    if (!ws.walk_cap) {
        ws.walk_cap = std::min<uint64_t>(n_attempts, std::max<uint64_t>(1u << 20, n_attempts / 16));
        ws.id_cap = std::max<uint64_t>(1u << 24, ws.walk_cap * 32);
    }

    SampleResult res;
    for (int attempt = 0; attempt < 2; ++attempt) {
        ws.walk_attempt.ensure(sizeof(uint64_t) * ws.walk_cap);
        ws.walk_off.ensure(sizeof(uint64_t) * ws.walk_cap);
        ws.walk_len.ensure(sizeof(uint32_t) * ws.walk_cap);
        ws.ids.ensure(sizeof(uint32_t) * ws.id_cap);
        SIA_HIP(hipMemsetAsync(ws.counters.ptr, 0, sizeof(uint64_t) * ST_COUNT, s));
        if (count_ids) SIA_HIP(hipMemsetAsync(ws.cnt.ptr, 0, sizeof(uint32_t) * id_space, s));

        SampleArgs A;
        A.nodes = g->nodes.as<NodeRec>();
        A.edges = g->edges.as<EdgeRec>();
        A.src_t = ws.src_t.as<uint32_t>();
        A.bucket = ws.bucket.as<uint32_t>();
        A.n_src = n_src;
        A.bucket_shift = st.shift;
        A.tag = g->tag;
        A.n_ns = st.n_ns;
        A.seed = seed;
        A.attempt_offset = attempt_offset;
        A.n_attempts = n_attempts;
        A.guard_evals = 3 * static_cast<uint64_t>(g->n) + 8;
        A.stats = ws.counters.as<uint64_t>();
        A.walk_attempt = ws.walk_attempt.as<uint64_t>();
        A.walk_off = ws.walk_off.as<uint64_t>();
        A.walk_len = ws.walk_len.as<uint32_t>();
        A.ids = ws.ids.as<uint32_t>();
        A.cnt = count_ids ? ws.cnt.as<uint32_t>() : nullptr;
        A.walk_cap = ws.walk_cap;
        A.id_cap = ws.id_cap;

        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            SIA_HIP(hipEventCreate(&e0));
            SIA_HIP(hipEventCreate(&e1));
            SIA_HIP(hipEventRecord(e0, s));
        }
        if (mode == SIA_EDGES)
            hipLaunchKernelGGL(k_sample<SIA_EDGES>, dim3(persistent_blocks<SIA_EDGES>()), dim3(256),
                               0, s, A);
        else
            hipLaunchKernelGGL(k_sample<SIA_NODES>, dim3(persistent_blocks<SIA_NODES>()), dim3(256),
                               0, s, A);
        SIA_HIP(hipGetLastError());
        if (timing) SIA_HIP(hipEventRecord(e1, s));

        uint64_t h[ST_COUNT];
        SIA_HIP(hipMemcpyAsync(h, ws.counters.ptr, sizeof(h), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        if (timing) {
            SIA_HIP(hipEventElapsedTime(&res.ms, e0, e1));
            SIA_HIP(hipEventDestroy(e0));
            SIA_HIP(hipEventDestroy(e1));
        }
        SIA_REQUIRE(h[ST_FAULTS] == 0, SIA_EDEVICE, "sampler consistency check failed");
        res.walks = h[ST_WALKS];
        res.ids = h[ST_IDS];
        res.hits = h[ST_HITS];
        res.dead = h[ST_DEAD];
        res.cycles = h[ST_CYCLE];
        res.steps = h[ST_STEPS];
        res.evals = h[ST_EVALS];
        if (!h[ST_OVERFLOW]) return res;
        // The counters say exactly how much room the walks need: rerun once.
        ws.walk_cap = std::max(ws.walk_cap, h[ST_WALKS]);
        ws.id_cap = std::max(ws.id_cap, h[ST_IDS] + 1);
    }
    throw Error{SIA_EDEVICE, "sampler output did not fit after resizing"};
}

}  // namespace sia
