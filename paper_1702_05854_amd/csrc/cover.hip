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
//   lvl1/lvl2 = maxima of key over 1024 ids / 1024 lvl1 entries.
//
// Each round: pick = max over lvl2 (one workgroup), cover = the picked id's
// uncovered walks are marked and their ids' counts decremented (the dirty
// lvl1 blocks are queued), then only the dirty lvl1 / lvl2 maxima are
// recomputed.  All state stays in HBM; the host only launches.
#include "common.hpp"

#include <algorithm>

namespace sia {

namespace {

constexpr int kWave = 64;
constexpr uint32_t kL1 = 1024;  // ids per level-1 block
constexpr uint32_t kL2 = 1024;  // level-1 blocks per level-2 block
constexpr uint32_t kSelected = 0xFFFFFFFFu;
constexpr uint32_t kScanTile = 4096;  // 256 threads x 16

struct GreedyState {
    uint32_t cur_id;
    uint32_t cur_gain;
    uint32_t n_dirty1;
    uint32_t n_dirty2;
};

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
// the start of id's list; walk w is listed under each of its ids.
__global__ void k_fill(const uint64_t *walk_off, const uint32_t *walk_len, uint64_t n_walks,
                       const uint32_t *ids, uint32_t *cur, uint32_t *inv)
{
    uint64_t w = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; w < n_walks; w += stride) {
        const uint64_t o = walk_off[w];
        const uint32_t L = walk_len[w];
        for (uint32_t e = 0; e < L; ++e) {
            const uint32_t p = atomicSub(&cur[ids[o + e]], 1u) - 1u;
            inv[p] = static_cast<uint32_t>(w);
        }
    }
}

// ---- level maxima: one wave per block
__global__ __launch_bounds__(256) void k_lvl1(const uint32_t *cnt, uint64_t id_space, uint64_t n1,
                                              const uint32_t *list, const GreedyState *st,
                                              uint64_t *lvl1, uint32_t *flag1, uint32_t *flag2,
                                              uint32_t *dirty2, GreedyState *st_out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    const uint64_t todo = list ? st->n_dirty1 : n1;
    for (uint64_t i = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave;
         i < todo; i += waves) {
        const uint64_t b = list ? list[i] : i;
        uint64_t best = 0;
        for (uint32_t k = lane; k < kL1; k += kWave) {
            const uint64_t id = b * kL1 + k;
            if (id < id_space) {
                const uint64_t key = key_of(cnt[id], static_cast<uint32_t>(id));
                best = key > best ? key : best;
            }
        }
        best = wave_max_u64(best);
        if (lane == 0) {
            lvl1[b] = best;
            if (list) {
                flag1[b] = 0;
                const uint32_t p = static_cast<uint32_t>(b / kL2);
                if (atomicExch(&flag2[p], 1u) == 0u)
                    dirty2[atomicAdd(&st_out->n_dirty2, 1u)] = p;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_lvl2(const uint64_t *lvl1, uint64_t n1, uint64_t n2,
                                              const uint32_t *list, const GreedyState *st,
                                              uint64_t *lvl2, uint32_t *flag2)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    const uint64_t todo = list ? st->n_dirty2 : n2;
    for (uint64_t i = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave;
         i < todo; i += waves) {
        const uint64_t p = list ? list[i] : i;
        uint64_t best = 0;
        for (uint32_t k = lane; k < kL2; k += kWave) {
            const uint64_t b = p * kL2 + k;
            if (b < n1) best = lvl1[b] > best ? lvl1[b] : best;
        }
        best = wave_max_u64(best);
        if (lane == 0) {
            lvl2[p] = best;
            if (list) flag2[p] = 0;
        }
    }
}

// ---- one greedy round
__global__ __launch_bounds__(1024) void k_pick(const uint64_t *lvl2, uint64_t n2, uint32_t *cnt,
                                               uint32_t *flag1, uint32_t *dirty1, int64_t round,
                                               int64_t *sel, uint64_t *gain, GreedyState *st)
{
    __shared__ uint64_t sh[16];
    uint64_t best = 0;
    for (uint64_t i = threadIdx.x; i < n2; i += blockDim.x) best = lvl2[i] > best ? lvl2[i] : best;
    best = wave_max_u64(best);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < static_cast<int>(blockDim.x / kWave); ++k) best = sh[k] > best ? sh[k] : best;
        best = sh[0] > best ? sh[0] : best;
        if (best == 0) {  // unreachable while rounds < id space; never index with it
            st->cur_gain = 0;
            st->n_dirty1 = 0;
            st->n_dirty2 = 0;
            sel[round] = -1;
            gain[round] = 0;
            return;
        }
        const uint32_t id = 0xFFFFFFFFu - static_cast<uint32_t>(best);
        const uint32_t g = static_cast<uint32_t>(best >> 32) - 1u;
        sel[round] = id;
        gain[round] = g;
        st->cur_id = id;
        st->cur_gain = g;
        cnt[id] = kSelected;
        const uint32_t b = id / kL1;
        flag1[b] = 1;
        dirty1[0] = b;
        st->n_dirty1 = 1;
        st->n_dirty2 = 0;
    }
}

__global__ __launch_bounds__(256) void k_cover(const GreedyState *st_in, const uint32_t *cur,
                                               const uint32_t *inv, const uint64_t *walk_off,
                                               const uint32_t *walk_len, const uint32_t *ids,
                                               uint32_t *covered, uint32_t *cnt, uint32_t *flag1,
                                               uint32_t *dirty1, GreedyState *st)
{
    if (st_in->cur_gain == 0) return;
    const uint32_t id = st_in->cur_id;
    const uint32_t lo = cur[id], hi = cur[id + 1];
    uint32_t p = lo + blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (; p < hi; p += stride) {
        const uint32_t w = inv[p];
        if (atomicExch(&covered[w], 1u) != 0u) continue;
        const uint64_t o = walk_off[w];
        const uint32_t L = walk_len[w];
        for (uint32_t e = 0; e < L; ++e) {
            const uint32_t x = ids[o + e];
            if (x == id) continue;
            atomicSub(&cnt[x], 1u);
            const uint32_t b = x / kL1;
            if (flag1[b] == 0u && atomicExch(&flag1[b], 1u) == 0u)
                dirty1[atomicAdd(&st->n_dirty1, 1u)] = b;
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
                        int64_t k, int64_t *selected, uint64_t *gains, hipStream_t s, bool timing)
{
    SIA_REQUIRE(n_ids < 0xFFFFFFFFull && n_walks < 0xFFFFFFFFull, SIA_EINVAL,
                "too many walk ids for 32-bit inverted index offsets");
    const uint64_t S = static_cast<uint64_t>(id_space);
    const uint64_t n1 = (S + kL1 - 1) / kL1, n2 = (n1 + kL2 - 1) / kL2;
    const uint64_t n_tiles = (S + kScanTile - 1) / kScanTile;
    const int cus = device_cu_count();

    ws.cnt.ensure(sizeof(uint32_t) * S);
    ws.cur.ensure(sizeof(uint32_t) * (S + 1));
    ws.inv.ensure(sizeof(uint32_t) * std::max<uint64_t>(n_ids, 1));
    ws.covered.ensure(sizeof(uint32_t) * std::max<uint64_t>(n_walks, 1));
    ws.lvl1.ensure(sizeof(uint64_t) * n1);
    ws.lvl2.ensure(sizeof(uint64_t) * n2);
    ws.flag1.ensure(sizeof(uint32_t) * n1);
    ws.flag2.ensure(sizeof(uint32_t) * n2);
    ws.dirty1.ensure(sizeof(uint32_t) * n1);
    ws.dirty2.ensure(sizeof(uint32_t) * n2);
    ws.sel.ensure(sizeof(int64_t) * k);
    ws.gain.ensure(sizeof(uint64_t) * k);
    ws.scan_tmp.ensure(sizeof(uint32_t) * n_tiles + sizeof(GreedyState) + 64);
    uint32_t *tiles = ws.scan_tmp.as<uint32_t>();
    GreedyState *st = reinterpret_cast<GreedyState *>(
        ws.scan_tmp.as<char>() + ((sizeof(uint32_t) * n_tiles + 63) / 64) * 64);

    uint32_t *cnt = ws.cnt.as<uint32_t>(), *cur = ws.cur.as<uint32_t>();
    const uint32_t *ids = ws.ids.as<uint32_t>();

    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (timing) {
        for (auto &e : ev) SIA_HIP(hipEventCreate(&e));
        SIA_HIP(hipEventRecord(ev[0], s));
    }
    // counts
    SIA_HIP(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * S, s));
    if (n_ids) {
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
        hipLaunchKernelGGL(k_fill, dim3(grid_for(n_walks, 256, cus * 32)), dim3(256), 0, s,
                           ws.walk_off.as<uint64_t>(), ws.walk_len.as<uint32_t>(), n_walks, ids,
                           cur, ws.inv.as<uint32_t>());
        SIA_HIP(hipGetLastError());
    }
    // greedy state
    SIA_HIP(hipMemsetAsync(ws.covered.ptr, 0, sizeof(uint32_t) * std::max<uint64_t>(n_walks, 1), s));
    SIA_HIP(hipMemsetAsync(ws.flag1.ptr, 0, sizeof(uint32_t) * n1, s));
    SIA_HIP(hipMemsetAsync(ws.flag2.ptr, 0, sizeof(uint32_t) * n2, s));
    hipLaunchKernelGGL(k_lvl1, dim3(grid_for(n1 * kWave, 256, cus * 16)), dim3(256), 0, s, cnt, S,
                       n1, nullptr, st, ws.lvl1.as<uint64_t>(), ws.flag1.as<uint32_t>(),
                       ws.flag2.as<uint32_t>(), ws.dirty2.as<uint32_t>(), st);
    hipLaunchKernelGGL(k_lvl2, dim3(grid_for(n2 * kWave, 256, cus * 16)), dim3(256), 0, s,
                       ws.lvl1.as<uint64_t>(), n1, n2, nullptr, st, ws.lvl2.as<uint64_t>(),
                       ws.flag2.as<uint32_t>());
    SIA_HIP(hipGetLastError());
    if (timing) SIA_HIP(hipEventRecord(ev[1], s));

    const unsigned cover_grid = static_cast<unsigned>(cus * 2);
    const unsigned lvl_grid = static_cast<unsigned>(cus);
    for (int64_t r = 0; r < k; ++r) {
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(1024), 0, s, ws.lvl2.as<uint64_t>(), n2, cnt,
                           ws.flag1.as<uint32_t>(), ws.dirty1.as<uint32_t>(), r,
                           ws.sel.as<int64_t>(), ws.gain.as<uint64_t>(), st);
        hipLaunchKernelGGL(k_cover, dim3(cover_grid), dim3(256), 0, s, st, cur,
                           ws.inv.as<uint32_t>(), ws.walk_off.as<uint64_t>(),
                           ws.walk_len.as<uint32_t>(), ids, ws.covered.as<uint32_t>(), cnt,
                           ws.flag1.as<uint32_t>(), ws.dirty1.as<uint32_t>(), st);
        hipLaunchKernelGGL(k_lvl1, dim3(lvl_grid), dim3(256), 0, s, cnt, S, n1,
                           ws.dirty1.as<uint32_t>(), st, ws.lvl1.as<uint64_t>(),
                           ws.flag1.as<uint32_t>(), ws.flag2.as<uint32_t>(),
                           ws.dirty2.as<uint32_t>(), st);
        hipLaunchKernelGGL(k_lvl2, dim3(lvl_grid), dim3(256), 0, s, ws.lvl1.as<uint64_t>(), n1,
                           n2, ws.dirty2.as<uint32_t>(), st, ws.lvl2.as<uint64_t>(),
                           ws.flag2.as<uint32_t>());
    }
    SIA_HIP(hipGetLastError());
    if (timing) SIA_HIP(hipEventRecord(ev[2], s));
    SIA_HIP(hipMemcpyAsync(selected, ws.sel.ptr, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
    SIA_HIP(hipMemcpyAsync(gains, ws.gain.ptr, sizeof(uint64_t) * k, hipMemcpyDeviceToHost, s));
    SIA_HIP(hipStreamSynchronize(s));
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
