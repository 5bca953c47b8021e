// Coverage counts and greedy max-coverage (Algorithm 4 for edges, Algorithm 7
// for nodes) over the kept walks.
//
//   cnt[id]  = number of not-yet-covered walks holding id (Cov of one id);
//   inv      = inverted index id -> walks, built by a counting sort driven by
//              cnt (offsets = prefix sums of the initial counts);
//   key(id)  = ((cnt+1) << 32) | (2^32-1-id) for an unselected id, 0 once
//              selected, so the largest key is the largest marginal gain with
//              the lowest id on ties, and zero-gain rounds take the lowest
//              id not selected yet;
//   L1/L2/L3 = maxima of key over 64 ids / 64 L1 entries / 64 L2 entries.
//
// Each round is four kernels.  pick+cover: every workgroup reads L3 and
// derives the same pick; workgroup 0 records it; all waves then take the
// picked id's walks (one wave per walk), mark the uncovered ones and
// decrement the counts of their ids, queueing each touched L1 block once.
// Then one refresh kernel per level: one wave per queued block recomputes its
// maximum and queues the parent block once.  Kernel boundaries order the
// phases (and make the writes of one phase visible to every XCD in the
// next); nothing is read back until the last round.
#include "common.hpp"

#include <algorithm>

namespace sia {

namespace {

constexpr int kWave = 64;
constexpr uint32_t kSelected = 0xFFFFFFFFu;
constexpr uint32_t kScanTile = 4096;  // 256 threads x 16

struct GreedyState {
    uint32_t n_queued[3][2];  // queued blocks per level, by round parity
    uint32_t error;
};

constexpr uint32_t kB = 64;  // fan-in of every level

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

// ---- full build of one level: out[i] = max over in[i*64 .. i*64+63]
// (level 1 reads keys of the counts directly).
__global__ __launch_bounds__(256) void k_build_level(const uint32_t *cnt, const uint64_t *in,
                                                     uint64_t n_in, uint64_t *out, uint64_t n_out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    for (uint64_t i = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave;
         i < n_out; i += waves) {
        const uint64_t c = i * kB + lane;
        uint64_t v = 0;
        if (c < n_in) v = cnt ? key_of(cnt[c], static_cast<uint32_t>(c)) : in[c];
        v = wave_max_u64(v);
        if (lane == 0) out[i] = v;
    }
}

struct Tree {
    uint32_t *cnt;
    uint64_t id_space;
    uint64_t *lvl[3];    // L1, L2, L3 maxima
    uint64_t n[3];       // entries per level
    uint32_t *flag[3];   // block queued this round, per level
    uint32_t *queue[3];  // two queues per level (round parity), n[l] entries each
};

__device__ __forceinline__ void enqueue(const Tree &T, GreedyState *st, int level, uint32_t par,
                                        uint64_t b)
{
    if (T.flag[level][b] == 0u && atomicExch(&T.flag[level][b], 1u) == 0u)
        T.queue[level][par * T.n[level] + atomicAdd(&st->n_queued[level][par], 1u)] =
            static_cast<uint32_t>(b);
}

__global__ __launch_bounds__(256) void k_pick_cover(Tree T, GreedyState *st, int64_t round,
                                                    int64_t *sel, uint64_t *gain, const uint32_t *cur,
                                                    const uint32_t *inv, const uint64_t *walk_off,
                                                    const uint32_t *walk_len, const uint32_t *ids,
                                                    uint32_t *covered)
{
    __shared__ uint64_t sh[4];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const uint32_t par = static_cast<uint32_t>(round & 1);
    // every workgroup derives the same pick from L3
    uint64_t best = 0;
    const uint64_t *l3 = T.lvl[2];
    for (uint64_t i = threadIdx.x; i < T.n[2]; i += blockDim.x) best = l3[i] > best ? l3[i] : best;
    best = wave_max_u64(best);
    if (lane == 0) sh[wid] = best;
    __syncthreads();
    best = sh[0];
    for (int k = 1; k < 4; ++k) best = sh[k] > best ? sh[k] : best;
    if (best == 0) {  // unreachable while rounds < id space; never index with it
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->error = 1;
            sel[round] = -1;
            gain[round] = 0;
        }
        return;
    }
    const uint32_t id = 0xFFFFFFFFu - static_cast<uint32_t>(best);
    const uint32_t g = static_cast<uint32_t>(best >> 32) - 1u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sel[round] = id;
        gain[round] = g;
        T.cnt[id] = kSelected;
        enqueue(T, st, 0, par, id / kB);
        // the queues of the next round start empty
        for (int l = 0; l < 3; ++l) st->n_queued[l][par ^ 1u] = 0;
    }
    if (g == 0) return;
    // cover the picked id's walks: one wave per listed walk
    const uint32_t lo = cur[id], hi = cur[id + 1];
    const uint32_t gw = blockIdx.x * (blockDim.x / kWave) + wid;
    const uint32_t nw = gridDim.x * (blockDim.x / kWave);
    for (uint32_t p = lo + gw; p < hi; p += nw) {
        const uint32_t w = inv[p];
        uint32_t old = 1;
        if (lane == 0) old = atomicExch(&covered[w], 1u);
        old = __shfl(old, 0, kWave);
        if (old != 0u) continue;
        const uint64_t o = walk_off[w];
        const uint32_t L = walk_len[w];
        for (uint32_t e = lane; e < L; e += kWave) {
            const uint32_t x = ids[o + e];
            if (x == id) continue;
            atomicSub(&T.cnt[x], 1u);
            enqueue(T, st, 0, par, x / kB);
        }
    }
}

// Recompute the queued blocks of one level; queue their parents.
__global__ __launch_bounds__(256) void k_refresh(Tree T, GreedyState *st, int64_t round, int level)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t par = static_cast<uint32_t>(round & 1);
    const uint32_t todo = st->n_queued[level][par];
    const uint32_t waves = (gridDim.x * blockDim.x) / kWave;
    const uint64_t n_in = level == 0 ? T.id_space : T.n[level - 1];
    const uint64_t *in = level == 0 ? nullptr : T.lvl[level - 1];
    for (uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < todo; i += waves) {
        const uint64_t b = T.queue[level][par * T.n[level] + i];
        const uint64_t c = b * kB + lane;
        uint64_t v = 0;
        if (c < n_in) v = level == 0 ? key_of(T.cnt[c], static_cast<uint32_t>(c)) : in[c];
        v = wave_max_u64(v);
        if (lane == 0) {
            T.lvl[level][b] = v;
            T.flag[level][b] = 0u;
            if (level < 2) enqueue(T, st, level + 1, par, b / kB);
        }
    }
}

unsigned grid_for(uint64_t items, unsigned block, unsigned cap)
{
    uint64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(std::min<uint64_t>(g, cap));
}

}  // namespace

GreedyResult run_greedy(Workspace &ws, int64_t id_space, uint64_t n_walks, uint64_t n_ids,
                        int64_t k, int64_t *selected, uint64_t *gains, hipStream_t s, bool timing,
                        bool counts_ready)
{
    SIA_REQUIRE(n_ids < 0xFFFFFFFFull && n_walks < 0xFFFFFFFFull, SIA_EINVAL,
                "too many walk ids for 32-bit inverted index offsets");
    const uint64_t S = static_cast<uint64_t>(id_space);
    const uint64_t n1 = (S + kB - 1) / kB, n2 = (n1 + kB - 1) / kB, n3 = (n2 + kB - 1) / kB;
    const uint64_t n_tiles = (S + kScanTile - 1) / kScanTile;
    const int cus = device_cu_count();

    ws.cnt.ensure(sizeof(uint32_t) * S);
    ws.cur.ensure(sizeof(uint32_t) * (S + 1));
    ws.inv.ensure(sizeof(uint32_t) * std::max<uint64_t>(n_ids, 1));
    ws.covered.ensure(sizeof(uint32_t) * std::max<uint64_t>(n_walks, 1));
    ws.lvl1.ensure(sizeof(uint64_t) * (n1 + n2 + n3));
    ws.flag1.ensure(sizeof(uint32_t) * (n1 + n2 + n3));
    ws.dirty1.ensure(sizeof(uint32_t) * 2 * (n1 + n2 + n3));
    ws.sel.ensure(sizeof(int64_t) * k);
    ws.gain.ensure(sizeof(uint64_t) * k);
    ws.scan_tmp.ensure(sizeof(uint32_t) * n_tiles + sizeof(GreedyState) + 64);
    uint32_t *tiles = ws.scan_tmp.as<uint32_t>();
    GreedyState *st = reinterpret_cast<GreedyState *>(
        ws.scan_tmp.as<char>() + ((sizeof(uint32_t) * n_tiles + 63) / 64) * 64);

    Tree T;
    T.cnt = ws.cnt.as<uint32_t>();
    T.id_space = S;
    T.n[0] = n1;
    T.n[1] = n2;
    T.n[2] = n3;
    T.lvl[0] = ws.lvl1.as<uint64_t>();
    T.flag[0] = ws.flag1.as<uint32_t>();
    T.queue[0] = ws.dirty1.as<uint32_t>();
    for (int l = 1; l < 3; ++l) {
        T.lvl[l] = T.lvl[l - 1] + T.n[l - 1];
        T.flag[l] = T.flag[l - 1] + T.n[l - 1];
        T.queue[l] = T.queue[l - 1] + 2 * T.n[l - 1];
    }
    uint32_t *cnt = T.cnt, *cur = ws.cur.as<uint32_t>();
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
    // greedy state
    SIA_HIP(hipMemsetAsync(ws.covered.ptr, 0, sizeof(uint32_t) * std::max<uint64_t>(n_walks, 1), s));
    SIA_HIP(hipMemsetAsync(ws.flag1.ptr, 0, sizeof(uint32_t) * (n1 + n2 + n3), s));
    SIA_HIP(hipMemsetAsync(st, 0, sizeof(GreedyState), s));
    hipLaunchKernelGGL(k_build_level, dim3(grid_for(n1 * kWave, 256, cus * 32)), dim3(256), 0, s,
                       cnt, nullptr, S, T.lvl[0], n1);
    hipLaunchKernelGGL(k_build_level, dim3(grid_for(n2 * kWave, 256, cus * 32)), dim3(256), 0, s,
                       nullptr, T.lvl[0], n1, T.lvl[1], n2);
    hipLaunchKernelGGL(k_build_level, dim3(grid_for(n3 * kWave, 256, cus * 32)), dim3(256), 0, s,
                       nullptr, T.lvl[1], n2, T.lvl[2], n3);
    SIA_HIP(hipGetLastError());
    if (timing) SIA_HIP(hipEventRecord(ev[1], s));

    const unsigned grid = static_cast<unsigned>(cus * 2);
    for (int64_t r = 0; r < k; ++r) {
        hipLaunchKernelGGL(k_pick_cover, dim3(grid), dim3(256), 0, s, T, st, r,
                           ws.sel.as<int64_t>(), ws.gain.as<uint64_t>(), cur,
                           ws.inv.as<uint32_t>(), ws.walk_off.as<uint64_t>(),
                           ws.walk_len.as<uint32_t>(), ids, ws.covered.as<uint32_t>());
        for (int l = 0; l < 3; ++l)
            hipLaunchKernelGGL(k_refresh, dim3(l == 0 ? grid : cus), dim3(256), 0, s, T, st, r, l);
    }
    SIA_HIP(hipGetLastError());
    if (timing) SIA_HIP(hipEventRecord(ev[2], s));
    GreedyState hst;
    SIA_HIP(hipMemcpyAsync(selected, ws.sel.ptr, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
    SIA_HIP(hipMemcpyAsync(gains, ws.gain.ptr, sizeof(uint64_t) * k, hipMemcpyDeviceToHost, s));
    SIA_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    SIA_HIP(hipStreamSynchronize(s));
    SIA_REQUIRE(hst.error == 0, SIA_EDEVICE, "greedy state inconsistent");
    for (int64_t i = 0; i < k; ++i)
        SIA_REQUIRE(selected[i] >= 0, SIA_EDEVICE, "greedy state inconsistent");
    GreedyResult res;
    if (timing) {
        SIA_HIP(hipEventElapsedTime(&res.ms_count, ev[0], ev[1]));
        SIA_HIP(hipEventElapsedTime(&res.ms_greedy, ev[1], ev[2]));
        for (auto &e : ev) SIA_HIP(hipEventDestroy(e));
    }
    return res;
}

}  // namespace sia
