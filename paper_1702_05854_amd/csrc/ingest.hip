// Graph ingest: validation and the integer live-edge tables of the LT model
// (Section 2.1, live-edge equivalence).  For column v with in-edges
// j = lo..hi-1:  q_j = round-half-even(w_j * 2^32),  thr_j = min(sum of q over
// lo..j, 2^32 - 1).  Edge j is live with probability (thr_j - thr_{j-1})/2^32.
//
// Layout built here (device): NodeRec[n] {off, deg, thr_last, source tag 0}
// and one record per in-edge j in CSR order: ArcRec {thr_{j-1}, thr_j, tail u,
// tag 0, u's off / deg / thr_last}, or, when every column has the weights
// w = 1/d_in (checked exactly on the quantised values), the compact
// ArcRec16 {tail u, tag 0, u's off / deg}.  One wave per column (wave-wide
// uint64 prefix sums); columns above kBigDeg in-edges are finished by one
// workgroup each; a last pass copies each tail's node record into its arcs.
#include "common.hpp"

#include <algorithm>

namespace sia {

namespace {

constexpr uint32_t kBigDeg = 16384;
constexpr int kWave = 64;

enum ErrCode : int { E_NONE = 0, E_OFFSETS = 1, E_ROWS = 2, E_WEIGHT_RANGE = 3, E_WEIGHT_SUM = 4 };

__device__ __forceinline__ bool weight_ok(float x) { return x >= 0.0f && x <= 1.0f; }

__device__ __forceinline__ void report(int *err, int code) { atomicCAS(err, 0, code); }

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d)
{
    uint32_t lo = __shfl_up(static_cast<uint32_t>(v), d, kWave);
    uint32_t hi = __shfl_up(static_cast<uint32_t>(v >> 32), d, kWave);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    uint32_t lo = __shfl(static_cast<uint32_t>(v), src, kWave);
    uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), src, kWave);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t o = shfl_up_u64(v, d);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ bool column_sum_ok(uint64_t qsum, uint64_t deg)
{
    // Real weights summing to <= 1: fp32 rounding adds <= 2^8 units, the
    // rounding of each q_j <= 1/2.
    return qsum <= (1ull << 32) + (1ull << 12) + deg / 2;
}

__device__ __forceinline__ NodeRec make_node(uint64_t lo, uint64_t deg, uint64_t qsum)
{
    NodeRec r;
    r.off = static_cast<uint32_t>(lo);
    r.deg = static_cast<uint32_t>(deg);
    r.thr_last = static_cast<uint32_t>(qsum > 0xFFFFFFFFull ? 0xFFFFFFFFull : qsum);
    r.tag = 0;
    return r;
}

__global__ void k_check_offsets(const int64_t *col_off, int64_t n, int64_t m, int *err)
{
    int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) {
        int64_t a = col_off[i], b = col_off[i + 1];
        if (b < a || a < 0 || b > m) report(err, E_OFFSETS);
        if (i == 0 && a != 0) report(err, E_OFFSETS);
        if (i == n - 1 && b != m) report(err, E_OFFSETS);
    }
}

__global__ void k_check_rows(const int32_t *row, int64_t m, int64_t n, int *err)
{
    int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (; i < m; i += stride) {
        int32_t u = row[i];
        if (u < 0 || u >= n) report(err, E_ROWS);
    }
}

__device__ __forceinline__ uint32_t clamp32(uint64_t v)
{
    return static_cast<uint32_t>(v > 0xFFFFFFFFull ? 0xFFFFFFFFull : v);
}

// First half of arc j: its threshold interval [clamp(run - q), clamp(run))
// and tail; the second half (the tail's record) is written by k_arc_tails.
__device__ __forceinline__ void put_arc_head(ArcRec *arcs, int64_t j, uint64_t run, uint64_t q, int32_t u)
{
    uint4 v;
    v.x = clamp32(run - q);
    v.y = clamp32(run);
    v.z = static_cast<uint32_t>(u);
    v.w = 0u;
    *reinterpret_cast<uint4 *>(&arcs[j]) = v;
}

// One wave per column.
__global__ __launch_bounds__(256) void k_thresholds(const int64_t *col_off, const int32_t *row,
                                                    const float *w, int64_t n, NodeRec *nodes,
                                                    ArcRec *arcs, uint32_t *big_list,
                                                    uint32_t *big_count, int *err, int *general)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (static_cast<int64_t>(gridDim.x) * blockDim.x) / kWave;
    for (int64_t v = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave; v < n;
         v += waves) {
        const int64_t lo = col_off[v], hi = col_off[v + 1];
        const uint64_t deg = static_cast<uint64_t>(hi - lo);
        if (deg > kBigDeg) {
            if (lane == 0) big_list[atomicAdd(big_count, 1u)] = static_cast<uint32_t>(v);
            continue;
        }
        const uint64_t qd = deg ? inv_indeg_quantum(static_cast<uint32_t>(deg)) : 0;
        uint64_t carry = 0;
        bool bad = false, mixed = false;
        for (int64_t base = lo; base < hi; base += kWave) {
            const int64_t j = base + lane;
            uint64_t q = 0;
            if (j < hi) {
                const float x = w[j];
                if (!weight_ok(x)) bad = true;
                else q = quantize_weight(x);
                if (q != qd) mixed = true;
            }
            const uint64_t s = wave_incl_scan(q, lane);
            if (j < hi) put_arc_head(arcs, j, carry + s, q, row[j]);
            carry += shfl_u64(s, kWave - 1);
        }
        if (bad) report(err, E_WEIGHT_RANGE);
        if (mixed) atomicOr(general, 1);
        if (lane == 0) {
            if (!column_sum_ok(carry, deg)) report(err, E_WEIGHT_SUM);
            nodes[v] = make_node(static_cast<uint64_t>(lo), deg, carry);
        }
    }
}

// One workgroup (256 threads) per column with more than kBigDeg in-edges.
__global__ __launch_bounds__(256) void k_thresholds_big(const int64_t *col_off, const int32_t *row,
                                                        const float *w, NodeRec *nodes,
                                                        ArcRec *arcs, const uint32_t *big_list,
                                                        const uint32_t *big_count, int *err,
                                                        int *general)
{
    __shared__ uint64_t wave_tot[4];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const uint32_t count = *big_count;
    for (uint32_t b = blockIdx.x; b < count; b += gridDim.x) {
        const uint32_t v = big_list[b];
        const int64_t lo = col_off[v], hi = col_off[v + 1];
        const uint64_t qd = inv_indeg_quantum(static_cast<uint32_t>(hi - lo));
        uint64_t carry = 0;
        bool bad = false, mixed = false;
        for (int64_t base = lo; base < hi; base += blockDim.x) {
            const int64_t j = base + threadIdx.x;
            uint64_t q = 0;
            if (j < hi) {
                const float x = w[j];
                if (!weight_ok(x)) bad = true;
                else q = quantize_weight(x);
                if (q != qd) mixed = true;
            }
            uint64_t s = wave_incl_scan(q, lane);
            if (lane == kWave - 1) wave_tot[wid] = s;
            __syncthreads();
            uint64_t before = 0, total = 0;
            for (int k = 0; k < 4; ++k) {
                if (k < wid) before += wave_tot[k];
                total += wave_tot[k];
            }
            __syncthreads();
            if (j < hi) put_arc_head(arcs, j, carry + before + s, q, row[j]);
            carry += total;
        }
        if (bad) report(err, E_WEIGHT_RANGE);
        if (mixed) atomicOr(general, 1);
        if (threadIdx.x == 0) {
            if (!column_sum_ok(carry, static_cast<uint64_t>(hi - lo))) report(err, E_WEIGHT_SUM);
            nodes[v] = make_node(static_cast<uint64_t>(lo), static_cast<uint64_t>(hi - lo), carry);
        }
    }
}

// Second half of every arc: a copy of its tail's node record.
__global__ __launch_bounds__(256) void k_arc_tails(const NodeRec *nodes, ArcRec *arcs, int64_t m)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; j < m; j += stride) {
        const NodeRec R = nodes[arcs[j].row];
        uint4 v;
        v.x = R.off;
        v.y = R.deg;
        v.z = R.thr_last;
        v.w = 0u;
        *reinterpret_cast<uint4 *>(&arcs[j].u_off) = v;
    }
}

// Compact records (every column has w = 1/d_in): tail, head tag 0 and the
// tail's offset and degree, from the tails the threshold pass wrote.
__global__ __launch_bounds__(256) void k_arc16(const NodeRec *nodes, const ArcRec *arcs, ArcRec16 *out,
                                               int64_t m)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; j < m; j += stride) {
        const uint32_t u = arcs[j].row;
        const NodeRec R = nodes[u];
        uint4 v;
        v.x = u;
        v.y = 0u;
        v.z = R.off;
        v.w = R.deg;
        *reinterpret_cast<uint4 *>(&out[j]) = v;
    }
}

// Threshold table of a compact graph: thr_j = min((j - off + 1) * q(d), 2^32 - 1)
// over each column's in-edges; one wave per column.
__global__ __launch_bounds__(256) void k_compact_thresholds(const NodeRec *nodes, int64_t n, uint32_t *thr)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (static_cast<int64_t>(gridDim.x) * blockDim.x) / kWave;
    for (int64_t v = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) / kWave; v < n;
         v += waves) {
        const NodeRec R = nodes[v];
        if (!R.deg) continue;
        const uint64_t q = inv_indeg_quantum(R.deg);
        for (uint32_t i = lane; i < R.deg; i += kWave)
            thr[static_cast<uint64_t>(R.off) + i] = clamp32(static_cast<uint64_t>(i + 1) * q);
    }
}

__global__ void k_quantize(const float *w, uint64_t *q, uint64_t count)
{
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) {
        const float x = w[i];
        q[i] = weight_ok(x) ? quantize_weight(x) : 0;
    }
}

unsigned grid_for(uint64_t items, unsigned block, unsigned cap)
{
    uint64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(std::min<uint64_t>(g, cap));
}

}  // namespace

void host_check_structure(int64_t n, int64_t m, const int64_t *col_off, const int32_t *row_idx)
{
    SIA_REQUIRE(col_off[0] == 0, SIA_EINVAL, "col_off[0] must be 0");
    for (int64_t v = 0; v < n; ++v)
        SIA_REQUIRE(col_off[v + 1] >= col_off[v], SIA_EINVAL,
                    "col_off must be non-decreasing (column " + std::to_string(v) + ")");
    SIA_REQUIRE(col_off[n] == m, SIA_EINVAL, "col_off[n] must equal m");
    for (int64_t j = 0; j < m; ++j)
        SIA_REQUIRE(row_idx[j] >= 0 && row_idx[j] < n, SIA_EINVAL,
                    "row_idx out of range at edge " + std::to_string(j));
}

int device_cu_count()
{
    int dev = 0, cus = 0;
    SIA_HIP(hipGetDevice(&dev));
    SIA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return cus;
}

void ingest_graph(sia_graph *g, const int64_t *col_off, const int32_t *row_idx, const float *w,
                  bool on_device, hipStream_t s)
{
    const int64_t n = g->n, m = g->m;

    DevBuf staging, scratch;
    const int64_t *d_off = col_off;
    const int32_t *d_row = row_idx;
    const float *d_w = w;
    if (!on_device) {
        const size_t off_b = sizeof(int64_t) * (n + 1), row_b = sizeof(int32_t) * m,
                     w_b = sizeof(float) * m;
        staging.ensure(off_b + row_b + w_b + 64);
        char *base = staging.as<char>();
        SIA_HIP(hipMemcpyAsync(base, col_off, off_b, hipMemcpyHostToDevice, s));
        if (m) {
            SIA_HIP(hipMemcpyAsync(base + off_b, row_idx, row_b, hipMemcpyHostToDevice, s));
            SIA_HIP(hipMemcpyAsync(base + off_b + row_b, w, w_b, hipMemcpyHostToDevice, s));
        }
        d_off = reinterpret_cast<const int64_t *>(base);
        d_row = reinterpret_cast<const int32_t *>(base + off_b);
        d_w = reinterpret_cast<const float *>(base + off_b + row_b);
    }
    // scratch: err (int), big_count (uint32), general (int), big_list (uint32[n])
    scratch.ensure(64 + sizeof(uint32_t) * static_cast<size_t>(n));
    int *d_err = scratch.as<int>();
    uint32_t *d_big_count = reinterpret_cast<uint32_t *>(scratch.as<char>() + 16);
    int *d_general = reinterpret_cast<int *>(scratch.as<char>() + 32);
    uint32_t *d_big = reinterpret_cast<uint32_t *>(scratch.as<char>() + 64);
    SIA_HIP(hipMemsetAsync(scratch.ptr, 0, 64, s));

    g->nodes.ensure(sizeof(NodeRec) * static_cast<size_t>(n));
    g->arcs.ensure(sizeof(ArcRec) * static_cast<size_t>(m > 0 ? m : 1));

    const int cus = device_cu_count();
    if (on_device) {
        hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(n, 256, cus * 16)), dim3(256), 0, s,
                           d_off, n, m, d_err);
        SIA_HIP(hipGetLastError());
        if (m) {
            hipLaunchKernelGGL(k_check_rows, dim3(grid_for(m, 256, cus * 16)), dim3(256), 0, s,
                               d_row, m, n, d_err);
            SIA_HIP(hipGetLastError());
        }
        int err = 0;
        SIA_HIP(hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        SIA_REQUIRE(err != E_OFFSETS, SIA_EINVAL,
                    "col_off must start at 0, be non-decreasing and end at m");
        SIA_REQUIRE(err != E_ROWS, SIA_EINVAL, "row_idx out of range");
    }
    hipLaunchKernelGGL(k_thresholds, dim3(grid_for(static_cast<uint64_t>(n) * kWave, 256, cus * 32)),
                       dim3(256), 0, s, d_off, d_row, d_w, n, g->nodes.as<NodeRec>(),
                       g->arcs.as<ArcRec>(), d_big, d_big_count, d_err, d_general);
    SIA_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_thresholds_big, dim3(cus * 2), dim3(256), 0, s, d_off, d_row, d_w,
                       g->nodes.as<NodeRec>(), g->arcs.as<ArcRec>(), d_big, d_big_count, d_err, d_general);
    SIA_HIP(hipGetLastError());
    int flags[9] = {};  // err at word 0, general at word 8
    SIA_HIP(hipMemcpyAsync(flags, scratch.ptr, sizeof(flags), hipMemcpyDeviceToHost, s));
    SIA_HIP(hipStreamSynchronize(s));
    const int err = flags[0];
    SIA_REQUIRE(err != E_WEIGHT_RANGE, SIA_EWEIGHTS, "a weight is outside [0,1] or NaN");
    SIA_REQUIRE(err != E_WEIGHT_SUM, SIA_EWEIGHTS,
                "a column's in-weights sum above 1 (LT model requires sum <= 1)");
    SIA_REQUIRE(err == E_NONE, SIA_EDEVICE, "ingest failed");
    g->arc_bytes = flags[8] ? sizeof(ArcRec) : sizeof(ArcRec16);
    if (!m) return;
    if (g->arc_bytes == sizeof(ArcRec)) {
        hipLaunchKernelGGL(k_arc_tails, dim3(grid_for(m, 256, cus * 32)), dim3(256), 0, s,
                           g->nodes.as<NodeRec>(), g->arcs.as<ArcRec>(), m);
        SIA_HIP(hipGetLastError());
    } else {
        DevBuf compact;
        compact.ensure(sizeof(ArcRec16) * static_cast<size_t>(m));
        hipLaunchKernelGGL(k_arc16, dim3(grid_for(m, 256, cus * 32)), dim3(256), 0, s,
                           g->nodes.as<NodeRec>(), g->arcs.as<ArcRec>(), compact.as<ArcRec16>(), m);
        SIA_HIP(hipGetLastError());
        SIA_HIP(hipStreamSynchronize(s));
        g->arcs.swap(compact);  // the 32-byte staging records are freed here
    }
    SIA_HIP(hipStreamSynchronize(s));
}

void compact_thresholds(const sia_graph *g, uint32_t *d_thr, hipStream_t s)
{
    const int cus = device_cu_count();
    hipLaunchKernelGGL(k_compact_thresholds, dim3(grid_for(static_cast<uint64_t>(g->n) * kWave, 256, cus * 32)),
                       dim3(256), 0, s, g->nodes.as<NodeRec>(), g->n, d_thr);
    SIA_HIP(hipGetLastError());
}

void quantize_device(const float *w, uint64_t *q, uint64_t count, hipStream_t s)
{
    if (!count) return;
    const int cus = device_cu_count();
    hipLaunchKernelGGL(k_quantize, dim3(grid_for(count, 256, cus * 64)), dim3(256), 0, s, w, q,
                       count);
    SIA_HIP(hipGetLastError());
}

}  // namespace sia
