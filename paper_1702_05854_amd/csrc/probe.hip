// Random-gather ceiling of the device: the rate at which 4-byte loads at
// uniformly random positions of a large array complete, each touching its own
// 128-byte line, either independent of each other (every lane streams loads)
// or as dependent chains (each lane's next address is the value it loaded,
// the access pattern of a walk).  A measuring stick for the sampler's line
// traffic; not part of the method.
#include "common.hpp"

#include <algorithm>

namespace sia {
namespace {

__device__ __forceinline__ uint32_t mix32(uint64_t x)
{
    // splitmix64 finaliser, folded to 32 bits
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return static_cast<uint32_t>(x ^ (x >> 32));
}

// a[i] = a pseudo-random position in [0, n) (the chains of the dependent probe)
__global__ void k_probe_fill(uint32_t *a, uint64_t n, uint64_t seed)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n; i += stride)
        gp(a)[i] = static_cast<uint32_t>((static_cast<uint64_t>(mix32(seed ^ (i * 0x2545F4914F6CDD1Dull))) * n) >> 32);
}

__global__ __launch_bounds__(256) void k_probe_independent(const uint32_t *a, uint64_t n, uint32_t loads,
                                                           uint64_t seed, uint32_t *sink)
{
    const uint64_t tid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    uint32_t acc = 0;
    constexpr int kBatch = 8;
    for (uint32_t i = 0; i < loads; i += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t h = mix32(seed + tid * 0x100000001B3ull + i + u);
            v[u] = gp(a)[(static_cast<uint64_t>(h) * n) >> 32];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) acc ^= v[u];
    }
    if (acc == 0x12345678u) gp(sink)[0] = acc;  // keeps the loads alive
}

__global__ __launch_bounds__(256) void k_probe_dependent(const uint32_t *a, uint64_t n, uint32_t loads,
                                                         uint64_t seed, uint32_t *sink)
{
    const uint64_t tid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    uint32_t x = static_cast<uint32_t>((static_cast<uint64_t>(mix32(seed ^ tid)) * n) >> 32);
    for (uint32_t i = 0; i < loads; ++i) x = gp(a)[x];
    if (x == 0xFFFFFFFFu) gp(sink)[0] = x;
}

}  // namespace
}  // namespace sia

using namespace sia;

extern "C" sia_status sia_probe_gather(uint64_t array_bytes, uint32_t loads_per_lane, int dependent,
                                       double *lines_per_s, double *ms, void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(lines_per_s != nullptr, SIA_EINVAL, "NULL argument");
        SIA_REQUIRE(array_bytes >= (uint64_t(1) << 20) && array_bytes <= (uint64_t(16) << 30), SIA_EINVAL,
                    "array_bytes must be in [1 MiB, 16 GiB]");
        SIA_REQUIRE(loads_per_lane >= 8 && loads_per_lane % 8 == 0 && loads_per_lane <= (1u << 20),
                    SIA_EINVAL, "loads_per_lane must be a multiple of 8 in [8, 2^20]");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const uint64_t n = array_bytes / 4;
        DevBuf arr, sink;
        arr.ensure(4 * n);
        sink.ensure(64);
        const int cus = device_cu_count();
        hipLaunchKernelGGL(k_probe_fill, dim3(cus * 64), dim3(256), 0, s, arr.as<uint32_t>(), n, 2017ull);
        SIA_HIP(hipGetLastError());
        int per_cu = 0;
        if (dependent)
            SIA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_probe_dependent, 256, 0));
        else
            SIA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_probe_independent, 256, 0));
        const unsigned blocks = static_cast<unsigned>(std::max(1, per_cu) * cus);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        SIA_HIP(hipEventCreate(&e0));
        SIA_HIP(hipEventCreate(&e1));
        float t = 0.f;
        for (int rep = 0; rep < 2; ++rep) {  // the first run warms up
            SIA_HIP(hipEventRecord(e0, s));
            if (dependent)
                hipLaunchKernelGGL(k_probe_dependent, dim3(blocks), dim3(256), 0, s, arr.as<uint32_t>(), n,
                                   loads_per_lane, 77ull + rep, sink.as<uint32_t>());
            else
                hipLaunchKernelGGL(k_probe_independent, dim3(blocks), dim3(256), 0, s, arr.as<uint32_t>(), n,
                                   loads_per_lane, 77ull + rep, sink.as<uint32_t>());
            SIA_HIP(hipGetLastError());
            SIA_HIP(hipEventRecord(e1, s));
            SIA_HIP(hipEventSynchronize(e1));
            SIA_HIP(hipEventElapsedTime(&t, e0, e1));
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        const double total = static_cast<double>(blocks) * 256.0 * loads_per_lane;
        *lines_per_s = total / (t * 1e-3);
        if (ms) *ms = t;
    });
}
