// Coverage counts and greedy max-coverage (Algorithm 4 for edges, Algorithm 7
// for nodes) over the kept walks.
//
//   cnt[id] = number of not-yet-covered walks holding id (Cov of one id),
//             exact at all times; 0xFFFFFFFF once id is selected;
//   inv     = inverted index id -> walks, a counting sort driven by cnt;
//   key(id) = ((cnt+1) << 32) | (2^32-1-id) for an unselected id, 0 once
//             selected: the largest key is the largest marginal gain with the
//             lowest id on ties, and once every gain is zero the lowest id not
//             selected yet (exactly k picks).
//
// Lazy greedy.  Covering walks only lowers counts, so a key computed once is
// an upper bound forever.  A pool holds the ids whose keys may be the
// largest, and tau bounds the key of every id outside the pool.  One
// workgroup then runs rounds back to back: recompute the pool's keys from the
// exact counts, and if the best exceeds tau it is the true argmax of the
// round -- record it, mark its walks covered and decrement the counts of
// their ids.  When the best no longer exceeds tau, grid-wide kernels rebuild
// the pool from the current counts (a histogram of counts chooses the
// threshold; ties at the threshold are resolved by ascending id).  The
// result is exactly the greedy of Algorithm 4 / 7.
#include "common.hpp"

#include <algorithm>
#include <cstddef>

namespace sia {

namespace {

constexpr int kWave = 64;
constexpr uint32_t kSelected = 0xFFFFFFFFu;
constexpr uint32_t kScanTile = 4096;  // 256 threads x 16

struct GreedyState {
    uint32_t pool_n;    // ids in the pool
    uint32_t next_id;   // first tied id left out of the pool (tie case)
    uint32_t rounds;    // rounds completed so far
    uint32_t error;
};

// Count histogram: counts 0..4095 exactly; above, 512 bins per octave.
constexpr uint32_t kExact = 4096;
constexpr uint32_t kPerOctave = 512;
constexpr uint32_t kBins = kExact + 20 * kPerOctave;  // octaves 2^12 .. 2^31

__device__ __forceinline__ uint32_t count_bin(uint32_t c)
{
    if (c < kExact) return c;
    const uint32_t L = 32u - __clz(c);  // bit length, 13..32
    return kExact + (L - 13u) * kPerOctave + ((c >> (L - 10u)) & (kPerOctave - 1u));
}

__device__ __forceinline__ uint64_t key_of(uint32_t c, uint32_t id)
{
    return c == kSelected ? 0ull : ((static_cast<uint64_t>(c) + 1ull) << 32) | (0xFFFFFFFFu - id);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), d, kWave);
        uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), d, kWave);
        uint64_t o = (static_cast<uint64_t>(hi) << 32) | lo;
        v = o > v ? o : v;
    }
    return v;
}

__global__ void k_count(const uint32_t *ids, uint64_t n_ids, uint32_t *cnt)
{
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < n_ids; i += stride) atomicAdd(&cnt[ids[i]], 1u);
}

// ---- inclusive scan of cnt[0..S) into out[0..S) (uint32; totals < 2^32)
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *sh, uint32_t &total)
{
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
    for (int k = 0; k < 4; ++k) {
        if (k < wid) before += sh[k];
        total += sh[k];
    }
    __syncthreads();
    return before + x - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *in, uint64_t count,
                                                     uint32_t *tile_sums)
{
    __shared__ uint32_t sh[4];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile + threadIdx.x * 16ull;
    uint32_t s = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < count) s += in[base + i];
    uint32_t total;
    block_excl_scan_256(s, sh, total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_tiles(uint32_t *tile_sums, uint64_t n_tiles)
{
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (uint64_t base = 0; base < n_tiles; base += 256) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < n_tiles ? tile_sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan_256(v, sh, total);
        if (i < n_tiles) tile_sums[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(256) void k_scan_down(const uint32_t *in, uint64_t count,
                                                   const uint32_t *tile_offs, uint32_t *out)
{
    __shared__ uint32_t sh[4];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile + threadIdx.x * 16ull;
    uint32_t v[16];
    uint32_t s = 0;
    for (int i = 0; i < 16; ++i) {
        v[i] = base + i < count ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = tile_offs[blockIdx.x] + block_excl_scan_256(s, sh, total);
    for (int i = 0; i < 16; ++i) {
        run += v[i];
        if (base + i < count) out[base + i] = run;
    }
}

// ---- inverted index: cur[id] counts down from the inclusive prefix sum to
// the start of id's list; walk w is listed under each of its ids.  One wave
// per walk.
__global__ __launch_bounds__(256) void k_fill(const uint64_t *walk_off, const uint32_t *walk_len,
                                              uint64_t n_walks, const uint32_t *ids, uint32_t *cur,
                                              uint32_t *inv)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    for (uint64_t w = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave;
         w < n_walks; w += waves) {
        const uint64_t o = walk_off[w];
        const uint32_t L = walk_len[w];
        for (uint32_t e = lane; e < L; e += kWave) {
            const uint32_t p = atomicSub(&cur[ids[o + e]], 1u) - 1u;
            inv[p] = static_cast<uint32_t>(w);
        }
    }
}

// ---- pool rebuild
__global__ __launch_bounds__(1024) void k_hist(const uint32_t *cnt, uint64_t S, uint32_t *hist)
{
    __shared__ uint32_t h[kBins];
    for (uint32_t i = threadIdx.x; i < kBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < S; i += stride) {
        const uint32_t c = cnt[i];
        if (c != kSelected) atomicAdd(&h[count_bin(c)], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kBins; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Pool += every unselected id with cnt >= c_min (c_min >= 1).
__global__ void k_collect(const uint32_t *cnt, uint64_t S, uint32_t c_min, uint32_t *pool,
                          GreedyState *st)
{
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < S; i += stride) {
        const uint32_t c = cnt[i];
        if (c != kSelected && c >= c_min) pool[atomicAdd(&st->pool_n, 1u)] = static_cast<uint32_t>(i);
    }
}

// Ties: per tile of 4096 ids, how many have cnt == c.
__global__ __launch_bounds__(256) void k_tie_count(const uint32_t *cnt, uint64_t S, uint32_t c,
                                                   uint32_t *tile_counts)
{
    __shared__ uint32_t sh[4];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile + threadIdx.x * 16ull;
    uint32_t k = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < S && cnt[base + i] == c) ++k;
    uint32_t total;
    block_excl_scan_256(k, sh, total);
    if (threadIdx.x == 0) tile_counts[blockIdx.x] = total;
}

// Ties: the first R ids (ascending) with cnt == c go to pool[pool_base ..];
// the (R+1)-th one is recorded in st->next_id.
__global__ __launch_bounds__(256) void k_tie_emit(const uint32_t *cnt, uint64_t S, uint32_t c,
                                                  const uint32_t *tile_offs, uint32_t R,
                                                  uint32_t pool_base, uint32_t *pool, GreedyState *st)
{
    __shared__ uint32_t sh[4];
    if (tile_offs[blockIdx.x] > R) return;  // uniform per block
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile + threadIdx.x * 16ull;
    uint32_t k = 0;
    for (int i = 0; i < 16; ++i)
        if (base + i < S && cnt[base + i] == c) ++k;
    uint32_t total;
    uint32_t q = tile_offs[blockIdx.x] + block_excl_scan_256(k, sh, total);
    for (int i = 0; i < 16; ++i) {
        if (base + i < S && cnt[base + i] == c) {
            if (q < R) pool[pool_base + q] = static_cast<uint32_t>(base + i);
            else if (q == R) st->next_id = static_cast<uint32_t>(base + i);
            ++q;
        }
    }
}

// ---- lazy rounds: one workgroup, rounds [st->rounds, k) while certified
constexpr int kLazyThreads = 1024;

__device__ __forceinline__ uint32_t load_count(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kLazyThreads) void k_lazy(uint32_t *cnt, const uint32_t *pool,
                                                       uint64_t tau, int64_t k, int64_t *sel,
                                                       uint64_t *gain, const uint32_t *cur,
                                                       const uint32_t *inv, const uint64_t *walk_off,
                                                       const uint32_t *walk_len, const uint32_t *ids,
                                                       uint32_t *covered, GreedyState *st)
{
    __shared__ uint64_t sh[kLazyThreads / kWave];
    __shared__ uint32_t queue[kLazyThreads];
    __shared__ uint32_t qn;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    constexpr int kWaves = kLazyThreads / kWave;
    const uint32_t P = st->pool_n;
    int64_t r = st->rounds;
    for (; r < k; ++r) {
        // exact keys of the pool; the largest is this round's pick if it beats tau
        uint64_t best = 0;
        for (uint32_t i = threadIdx.x; i < P; i += kLazyThreads) {
            const uint32_t id = pool[i];
            const uint64_t key = key_of(load_count(&cnt[id]), id);
            best = key > best ? key : best;
        }
        best = wave_max_u64(best);
        if (lane == 0) sh[wid] = best;
        if (threadIdx.x == 0) qn = 0;
        __syncthreads();
        best = sh[0];
        for (int w = 1; w < kWaves; ++w) best = sh[w] > best ? sh[w] : best;
        if (best <= tau) break;  // uniform: every thread saw the same values
        const uint32_t id = 0xFFFFFFFFu - static_cast<uint32_t>(best);
        const uint32_t g = static_cast<uint32_t>(best >> 32) - 1u;
        if (threadIdx.x == 0) {
            sel[r] = id;
            gain[r] = g;
            atomicExch(&cnt[id], kSelected);
        }
        if (g > 0) {
            const uint32_t lo = cur[id], hi = cur[id + 1];
            for (uint32_t b0 = lo; b0 < hi; b0 += kLazyThreads) {
                const uint32_t p = b0 + threadIdx.x;
                if (p < hi) {
                    const uint32_t w = inv[p];
                    if (atomicExch(&covered[w], 1u) == 0u) queue[atomicAdd(&qn, 1u)] = w;
                }
                __syncthreads();
                const uint32_t n = qn;
                for (uint32_t qi = wid; qi < n; qi += kWaves) {
                    const uint32_t w = queue[qi];
                    const uint64_t o = walk_off[w];
                    const uint32_t L = walk_len[w];
                    for (uint32_t e = lane; e < L; e += kWave) {
                        const uint32_t x = ids[o + e];
                        if (x != id) atomicSub(&cnt[x], 1u);
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) qn = 0;
                __syncthreads();
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) st->rounds = static_cast<uint32_t>(r);
}

unsigned grid_for(uint64_t items, unsigned block, unsigned cap)
{
    uint64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(std::min<uint64_t>(g, cap));
}

}  // namespace

namespace {

uint64_t bin_lo(uint32_t b)
{
    if (b < kExact) return b;
    const uint32_t o = (b - kExact) / kPerOctave, r = (b - kExact) % kPerOctave;
    const uint32_t L = o + 13;  // bit length
    return (static_cast<uint64_t>(kPerOctave + r)) << (L - 10);
}

constexpr uint64_t kPoolTarget = 4096;
constexpr uint64_t kPoolMax = 16384;

}  // namespace

GreedyResult run_greedy(Workspace &ws, int64_t id_space, uint64_t n_walks, uint64_t n_ids,
                        int64_t k, int64_t *selected, uint64_t *gains, hipStream_t s, bool timing,
                        bool counts_ready)
{
    SIA_REQUIRE(n_ids < 0xFFFFFFFFull && n_walks < 0xFFFFFFFFull, SIA_EINVAL,
                "too many walk ids for 32-bit inverted index offsets");
    const uint64_t S = static_cast<uint64_t>(id_space);
    const uint64_t n_tiles = (S + kScanTile - 1) / kScanTile;
    const int cus = device_cu_count();

    ws.cnt.ensure(sizeof(uint32_t) * S);
    ws.cur.ensure(sizeof(uint32_t) * (S + 1));
    ws.inv.ensure(sizeof(uint32_t) * std::max<uint64_t>(n_ids, 1));
    ws.covered.ensure(sizeof(uint32_t) * std::max<uint64_t>(n_walks, 1));
    ws.lvl1.ensure(sizeof(uint32_t) * (kBins + kPoolMax));   // histogram + pool
    ws.sel.ensure(sizeof(int64_t) * k);
    ws.gain.ensure(sizeof(uint64_t) * k);
    ws.scan_tmp.ensure(sizeof(uint32_t) * n_tiles + sizeof(GreedyState) + 64);
    uint32_t *tiles = ws.scan_tmp.as<uint32_t>();
    GreedyState *st = reinterpret_cast<GreedyState *>(
        ws.scan_tmp.as<char>() + ((sizeof(uint32_t) * n_tiles + 63) / 64) * 64);
    uint32_t *hist = ws.lvl1.as<uint32_t>();
    uint32_t *pool = hist + kBins;
    uint32_t *cnt = ws.cnt.as<uint32_t>(), *cur = ws.cur.as<uint32_t>();
    const uint32_t *ids = ws.ids.as<uint32_t>();

    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (timing) {
        for (auto &e : ev) SIA_HIP(hipEventCreate(&e));
        SIA_HIP(hipEventRecord(ev[0], s));
    }
    // counts (unless the sampler already produced them)
    if (!counts_ready) SIA_HIP(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * S, s));
    if (n_ids && !counts_ready) {
        hipLaunchKernelGGL(k_count, dim3(grid_for(n_ids, 256, cus * 64)), dim3(256), 0, s, ids,
                           n_ids, cnt);
        SIA_HIP(hipGetLastError());
    }
    // inverted index
    hipLaunchKernelGGL(k_scan_reduce, dim3(n_tiles), dim3(256), 0, s, cnt, S, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(256), 0, s, tiles, n_tiles);
    hipLaunchKernelGGL(k_scan_down, dim3(n_tiles), dim3(256), 0, s, cnt, S, tiles, cur);
    SIA_HIP(hipGetLastError());
    SIA_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(cur + S), static_cast<int>(n_ids), 1, s));
    if (n_walks) {
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n_walks * kWave, 256, cus * 32)), dim3(256), 0, s,
                           ws.walk_off.as<uint64_t>(), ws.walk_len.as<uint32_t>(), n_walks, ids,
                           cur, ws.inv.as<uint32_t>());
        SIA_HIP(hipGetLastError());
    }
    SIA_HIP(hipMemsetAsync(ws.covered.ptr, 0, sizeof(uint32_t) * std::max<uint64_t>(n_walks, 1), s));
    SIA_HIP(hipMemsetAsync(st, 0, sizeof(GreedyState), s));
    if (timing) SIA_HIP(hipEventRecord(ev[1], s));

    std::vector<uint32_t> h(kBins);
    GreedyState hs{};
    int64_t done = 0;
    while (done < k) {
        // ---- rebuild the pool from the current counts
        SIA_HIP(hipMemsetAsync(hist, 0, sizeof(uint32_t) * kBins, s));
        hipLaunchKernelGGL(k_hist, dim3(cus), dim3(1024), 0, s, cnt, S, hist);
        SIA_HIP(hipGetLastError());
        SIA_HIP(hipMemcpyAsync(h.data(), hist, sizeof(uint32_t) * kBins, hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        // highest bin b* with at least kPoolTarget ids at or above it (or bin 0)
        uint64_t above = 0;
        int64_t bstar = kBins - 1;
        for (; bstar > 0; --bstar) {
            if (above + h[bstar] >= kPoolTarget) break;
            above += h[bstar];
        }
        const uint64_t ge = above + h[bstar];
        uint64_t tau;
        uint32_t pool_n;
        SIA_HIP(hipMemsetAsync(st, 0, offsetof(GreedyState, rounds), s));  // pool_n, next_id
        if (ge <= kPoolMax && bstar > 0) {
            const uint64_t c_lo = bin_lo(static_cast<uint32_t>(bstar));
            hipLaunchKernelGGL(k_collect, dim3(cus * 8), dim3(256), 0, s, cnt, S,
                               static_cast<uint32_t>(c_lo), pool, st);
            tau = (c_lo << 32) | 0xFFFFFFFFull;  // bound for every count <= c_lo - 1
            pool_n = static_cast<uint32_t>(ge);
        } else {
            // ties at an exact count c: all ids above c, then the lowest-id ones at c
            SIA_REQUIRE(bstar < static_cast<int64_t>(kExact), SIA_EDEVICE,
                        "greedy pool: more tied high counts than the pool holds");
            const uint32_t c = static_cast<uint32_t>(bstar);
            const uint32_t R = static_cast<uint32_t>(std::min<uint64_t>(kPoolTarget, ge) - above);
            if (above) {
                hipLaunchKernelGGL(k_collect, dim3(cus * 8), dim3(256), 0, s, cnt, S, c + 1, pool, st);
            }
            hipLaunchKernelGGL(k_tie_count, dim3(n_tiles), dim3(256), 0, s, cnt, S, c, tiles);
            hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(256), 0, s, tiles, n_tiles);
            hipLaunchKernelGGL(k_tie_emit, dim3(n_tiles), dim3(256), 0, s, cnt, S, c, tiles, R,
                               static_cast<uint32_t>(above), pool, st);
            SIA_HIP(hipGetLastError());
            SIA_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
            SIA_HIP(hipStreamSynchronize(s));
            pool_n = static_cast<uint32_t>(above + R);
            tau = ge > above + R ? ((static_cast<uint64_t>(c) + 1) << 32) | (0xFFFFFFFFu - hs.next_id)
                                 : (c ? (static_cast<uint64_t>(c) << 32) | 0xFFFFFFFFull : 0ull);
            SIA_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(&st->pool_n),
                                      static_cast<int>(pool_n), 1, s));
        }
        SIA_HIP(hipGetLastError());
        // ---- certified rounds, back to back
        hipLaunchKernelGGL(k_lazy, dim3(1), dim3(kLazyThreads), 0, s, cnt, pool, tau, k,
                           ws.sel.as<int64_t>(), ws.gain.as<uint64_t>(), cur,
                           ws.inv.as<uint32_t>(), ws.walk_off.as<uint64_t>(),
                           ws.walk_len.as<uint32_t>(), ids, ws.covered.as<uint32_t>(), st);
        SIA_HIP(hipGetLastError());
        SIA_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        SIA_REQUIRE(static_cast<int64_t>(hs.rounds) > done, SIA_EDEVICE, "greedy made no progress");
        done = hs.rounds;
    }
    if (timing) SIA_HIP(hipEventRecord(ev[2], s));
    SIA_HIP(hipMemcpyAsync(selected, ws.sel.ptr, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
    SIA_HIP(hipMemcpyAsync(gains, ws.gain.ptr, sizeof(uint64_t) * k, hipMemcpyDeviceToHost, s));
    SIA_HIP(hipStreamSynchronize(s));
    GreedyResult res;
    if (timing) {
        SIA_HIP(hipEventElapsedTime(&res.ms_count, ev[0], ev[1]));
        SIA_HIP(hipEventElapsedTime(&res.ms_greedy, ev[1], ev[2]));
        for (auto &e : ev) SIA_HIP(hipEventDestroy(e));
    }
    return res;
}

}  // namespace sia
