// sia_greedy_noalloc: the greedy of sia_greedy (Algorithm 4 / 7) on walks
// already in device memory, for callers that cannot allocate device memory.
// Every buffer the greedy's kernels need beyond the caller's inputs and
// outputs (walk lengths, coverage counts, the job record and state, the
// pool, its walk lists and the counting partition) is carved from one
// file-scope device array, `scratch`, of kScratchBytes per device; the call
// makes no hipMalloc / hipFree.  Calls that overlap on one device race on
// that array: the caller serialises them.
#include "common.hpp"

#include <mutex>

namespace sia {
namespace {

constexpr uint64_t kScratchBytes = uint64_t(64) << 20;  // per device, held until the process ends
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, taken once per device with the
// device current (the array's name is only a host-side handle).
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

void *scratch_on_current_device()
{
    int dev = -1;
    SIA_HIP(hipGetDevice(&dev));
    SIA_REQUIRE(dev >= 0 && dev < kMaxDevices, SIA_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        SIA_REQUIRE(e == hipSuccess && p != nullptr, SIA_EDEVICE,
                    std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

uint64_t al256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// len[w] = off[w+1] - off[w]; flags bit 0: off decreasing or a walk longer
// than 2^32 - 1 ids; bit 1: an id outside [0, S).  flags cleared beforehand.
__global__ __launch_bounds__(256) void k_walk_lengths(const uint64_t *off, const uint32_t *ids, uint64_t n_walks,
                                                      uint64_t n_ids, uint64_t S, uint32_t *len, uint32_t *flags)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    uint32_t bad = 0;
    for (uint64_t w = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; w < n_walks; w += stride) {
        const uint64_t a = off[w], b = off[w + 1];
        if (b < a || b - a > 0xFFFFFFFFull) {
            bad |= 1u;
            len[w] = 0;
        } else {
            len[w] = static_cast<uint32_t>(b - a);
        }
    }
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < n_ids; e += stride)
        if (ids[e] >= S) bad |= 2u;
    if (bad) atomicOr(flags, bad);
}

__global__ void k_clear_word(uint32_t *p) { *p = 0; }

}  // namespace
}  // namespace sia

using namespace sia;

extern "C" sia_status sia_greedy_noalloc(int64_t id_space, const uint64_t *walk_off, const uint32_t *ids,
                                         uint64_t n_walks, int64_t k, int64_t *selected, uint64_t *gains,
                                         void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(id_space >= 1 && id_space < (int64_t(1) << 32), SIA_EINVAL, "id_space must be in [1, 2^32)");
        SIA_REQUIRE(k >= 1 && k <= id_space, SIA_EINVAL, "k must be in [1, id_space]");
        SIA_REQUIRE(walk_off != nullptr && selected != nullptr && gains != nullptr, SIA_EINVAL, "NULL argument");
        SIA_REQUIRE(n_walks < 0xFFFFFFFFull, SIA_EINVAL, "n_walks must be below 2^32 - 1");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        unsigned char *base = static_cast<unsigned char *>(scratch_on_current_device());

        uint64_t ends[2] = {0, 0};  // walk_off[0], walk_off[n_walks]
        SIA_HIP(hipMemcpyAsync(&ends[0], walk_off, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipMemcpyAsync(&ends[1], walk_off + n_walks, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        SIA_REQUIRE(ends[0] == 0, SIA_EINVAL, "walk_off[0] must be 0");
        const uint64_t n_ids = ends[1];
        SIA_REQUIRE(n_ids < 0xFFFFFFFFull, SIA_EINVAL, "walk_off[n_walks] must be below 2^32 - 1");
        SIA_REQUIRE(n_ids == 0 || ids != nullptr, SIA_EINVAL, "ids is NULL");
        const uint64_t S = static_cast<uint64_t>(id_space);

        // layout: flags | walk lengths | counts | job table | greedy scratch
        const uint64_t o_len = 256;
        const uint64_t o_cnt = o_len + al256(4 * std::max<uint64_t>(n_walks, 1));
        const uint64_t o_job = o_cnt + al256(4 * S);
        const uint64_t o_grd = o_job + al256(greedy_job_table_bytes(1));
        const uint64_t need = o_grd + al256(greedy_scratch_bytes(S, n_walks, n_ids, k));
        SIA_REQUIRE(need <= kScratchBytes, SIA_EINVAL,
                    "input too large for the allocation-free greedy: it needs " + std::to_string(need) +
                        " bytes of scratch, the limit is " + std::to_string(kScratchBytes) +
                        " (about 8.2 S + 10 n_ids + 16 n_walks + 16 k bytes plus 3 MB)");
        uint32_t *flags = reinterpret_cast<uint32_t *>(base);
        uint32_t *len = reinterpret_cast<uint32_t *>(base + o_len);

        hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, s, flags);
        const uint64_t items = std::max<uint64_t>(n_walks, n_ids);
        const unsigned blocks = static_cast<unsigned>(
            std::max<uint64_t>(1, std::min<uint64_t>((items + 255) / 256, static_cast<uint64_t>(device_cu_count()) * 8)));
        hipLaunchKernelGGL(k_walk_lengths, dim3(blocks), dim3(256), 0, s, walk_off, ids, n_walks, n_ids, S, len,
                           flags);
        SIA_HIP(hipGetLastError());
        uint32_t h_flags = 0;
        SIA_HIP(hipMemcpyAsync(&h_flags, flags, sizeof(h_flags), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        SIA_REQUIRE(!(h_flags & 1u), SIA_EINVAL, "walk_off must be non-decreasing");
        SIA_REQUIRE(!(h_flags & 2u), SIA_EINVAL, "an id is outside [0, id_space)");

        std::vector<GreedyInput> in(1);
        GreedyInput &g = in[0];
        g.walk_off = walk_off;
        g.walk_len = len;
        g.ids = ids;
        g.id_space = S;
        g.n_walks = n_walks;
        g.n_ids = n_ids;
        g.k = k;
        g.cnt = reinterpret_cast<uint32_t *>(base + o_cnt);
        g.scratch = base + o_grd;
        g.selected = selected;
        g.gains = gains;
        g.out_on_device = true;
        GreedyResult res;
        run_greedy_jobs(in, base + o_job, s, false, &res);
    });
}
