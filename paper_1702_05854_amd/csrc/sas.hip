// Stop-and-Stare driver: eSIA (Algorithm 6) / nSIA (Algorithm 9) with Check
// (Algorithm 5 / 8) over the single-query path.
//
// The HSAW stream R_1, R_2, ... is the kept walks in attempt-id order.  A
// walk is a function of (seed, attempt id), so the driver never stores or
// sorts walks: it probes attempt ranges, keeping only the attempt ids of the
// kept walks, finds by bisection the attempt bounds A (R_t = the kept walks
// of [0, A)) and A' (R'_t = those of [A, A')), and samples both ranges
// afresh: the greedy runs on R_t, and the coverage of its picks is counted
// on R'_t by a kernel.  The scalar steps of Check run on the host.
#include "common.hpp"

#include <chrono>
#include <cmath>
#include <limits>

namespace sia {
namespace {

constexpr int kWave = 64;

// n_out += #{i : att[i] < x}
__global__ __launch_bounds__(256) void k_count_below(const uint64_t *att, uint64_t n, uint64_t x,
                                                     unsigned long long *n_out)
{
    const GLOBAL uint64_t *a = gp(att);
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    uint32_t c = 0;
    for (; i < n; i += stride) c += a[i] < x ? 1u : 0u;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) c += __shfl_xor(c, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && c)
        __hip_atomic_fetch_add(gp(n_out), static_cast<unsigned long long>(c), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// set bit id of every selected id (bits cleared beforehand)
__global__ __launch_bounds__(256) void k_mark_selected(const int64_t *sel, int64_t k, uint32_t *bits)
{
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= k) return;
    const uint32_t x = static_cast<uint32_t>(gp(sel)[i]);
    __hip_atomic_fetch_or(gp(bits) + (x >> 5), 1u << (x & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// n_out += number of walks holding a marked id; one wave per walk
__global__ __launch_bounds__(256) void k_cover_walks(const uint64_t *walk_off, const uint32_t *walk_len,
                                                     const uint32_t *ids, uint64_t n_walks,
                                                     const uint32_t *bits, unsigned long long *n_out)
{
    const GLOBAL uint64_t *off = gp(walk_off);
    const GLOBAL uint32_t *len = gp(walk_len);
    const GLOBAL uint32_t *id = gp(ids);
    const GLOBAL uint32_t *b = gp(bits);
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    uint32_t covered = 0;
    for (uint64_t w = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave; w < n_walks;
         w += waves) {  // uniform per wave
        const uint64_t o = off[w];
        const uint32_t L = len[w];
        bool hit = false;
        for (uint32_t e = lane; e < L; e += kWave) {
            const uint32_t x = id[o + e];
            hit = hit || ((b[x >> 5] >> (x & 31)) & 1u);
        }
        if (__ballot(hit)) ++covered;
    }
    if (lane == 0 && covered)
        __hip_atomic_fetch_add(gp(n_out), static_cast<unsigned long long>(covered), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

unsigned grid_of(uint64_t items, unsigned block, unsigned cap)
{
    const uint64_t g = (items + block - 1) / block;
    return static_cast<unsigned>(std::max<uint64_t>(1, std::min<uint64_t>(g, cap)));
}

// Parameters of Algorithm 6 / 9 for id space S (m for edges, n for nodes).
struct SasParams {
    double lambda, lambda1, n_max;
    int t_max;
};

SasParams sas_params(double S, double k, double eps, double delta)
{
    const double c = 2.0 + 2.0 * eps / 3.0;
    const double ln_binom = std::lgamma(S + 1.0) - std::lgamma(k + 1.0) - std::lgamma(S - k + 1.0);
    const double g = 2.0 - 1.0 / M_E;
    SasParams P;
    P.n_max = g * g * c * S * (std::log(6.0 / delta) + ln_binom) / (k * eps * eps);  // "guard" / "nguard"
    // the iteration lemma: t_max = log2(2 N_max / Upsilon(eps, delta/3)),
    // Upsilon(eps, delta/3) = c ln(3/delta) / eps^2
    const double upsilon = c * std::log(3.0 / delta) / (eps * eps);
    P.t_max = std::max(1, static_cast<int>(std::ceil(std::log2(2.0 * P.n_max / upsilon))));
    const double L = c * std::log(3.0 * P.t_max / delta) / (eps * eps);
    P.lambda = L;                         // "lambda"
    P.lambda1 = 1.0 + (1.0 + eps) * L;    // "lambda_1"
    return P;
}

// Check (Algorithm 5 / 8): passes when eps_t <= eps; eps_t is NaN below Lambda_1.
bool sas_check(double cov_r, double cov_rp, double n_rp, int t, double eps, double lambda1, double *eps_t)
{
    *eps_t = std::numeric_limits<double>::quiet_NaN();
    if (cov_rp < lambda1) return false;
    const double e = 1.0 - 1.0 / M_E;
    const double scale = n_rp * (1.0 + eps) / (std::ldexp(1.0, t - 1) * cov_rp);
    const double e1 = cov_r / cov_rp - 1.0;
    const double e2 = eps * std::sqrt(scale);
    const double e3 = eps * std::sqrt(scale * (e - eps) / (1.0 + eps / 3.0));
    *eps_t = (e1 + e2 + e1 * e2) * (e - eps) + e * e3;
    return *eps_t <= eps;
}

// grow a device buffer keeping its first keep bytes
void grow_keep(DevBuf &b, size_t keep, size_t want, hipStream_t s)
{
    if (b.bytes >= want) return;
    DevBuf nb;
    nb.ensure(std::max(want, 2 * b.bytes));
    if (keep) SIA_HIP(hipMemcpyAsync(nb.ptr, b.ptr, keep, hipMemcpyDeviceToDevice, s));
    SIA_HIP(hipStreamSynchronize(s));
    b.swap(nb);
}

}  // namespace
}  // namespace sia

using namespace sia;

extern "C" {

sia_status sia_sas_solve(const sia_graph *cg, int mode, const int32_t *sources, int64_t n_sources,
                         int64_t k, double eps, double delta, uint64_t seed, uint64_t max_attempts,
                         int64_t *selected, uint64_t *gains, sia_sas_info *info, void *hip_stream)
{
    return guarded([&] {
        const auto t0 = std::chrono::steady_clock::now();
        SIA_REQUIRE(cg != nullptr && selected != nullptr && gains != nullptr && info != nullptr, SIA_EINVAL,
                    "NULL argument");
        SIA_REQUIRE(eps > 0.0 && eps < 1.0 - 1.0 / M_E, SIA_EINVAL, "eps must be in (0, 1 - 1/e)");
        SIA_REQUIRE(delta > 0.0 && delta < 1.0, SIA_EINVAL, "delta must be in (0, 1)");
        sia_graph *g = const_cast<sia_graph *>(cg);
        check_query(g->n, g->m, mode, sources, n_sources, k, max_attempts, 0);
        SIA_REQUIRE(k >= 1, SIA_EINVAL, "k must be >= 1");
        std::lock_guard<std::mutex> lock(g->mu);
        DeviceScope ds(g->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const int64_t S = mode == SIA_EDGES ? g->m : g->n;
        const SasParams P = sas_params(static_cast<double>(S), static_cast<double>(k), eps, delta);
        const SourceTables st = build_source_tables(g->n, sources, n_sources);

        sia_sas_info I{};
        I.lambda = P.lambda;
        I.lambda1 = P.lambda1;
        I.n_max = P.n_max;
        I.t_max = P.t_max;
        I.eps_t = std::numeric_limits<double>::quiet_NaN();

        DevBuf acc, scalar, bits, dsel;  // stream attempt ids, one counter, marks, picks
        scalar.ensure(sizeof(unsigned long long));
        bits.ensure(4 * ((static_cast<uint64_t>(S) + 31) / 32));
        dsel.ensure(sizeof(int64_t) * static_cast<uint64_t>(k));
        const unsigned cus = static_cast<unsigned>(device_cu_count());
        uint64_t end = 0, n_acc = 0, chunk = uint64_t(1) << 16;

        auto read_counter = [&]() {
            unsigned long long v = 0;
            SIA_HIP(hipMemcpyAsync(&v, scalar.ptr, sizeof(v), hipMemcpyDeviceToHost, s));
            SIA_HIP(hipStreamSynchronize(s));
            return static_cast<uint64_t>(v);
        };
        auto count_below = [&](uint64_t x) {
            SIA_HIP(hipMemsetAsync(scalar.ptr, 0, sizeof(unsigned long long), s));
            hipLaunchKernelGGL(k_count_below, dim3(grid_of(n_acc, 256, cus * 4)), dim3(256), 0, s,
                               acc.as<uint64_t>(), n_acc, x, scalar.as<unsigned long long>());
            SIA_HIP(hipGetLastError());
            return read_counter();
        };
        // smallest A with N stream walks among attempts [0, A)
        auto bound = [&](uint64_t N) {
            uint64_t lo = 0, hi = end;  // #below(lo) < N <= #below(hi)
            while (hi - lo > 1) {
                const uint64_t mid = lo + (hi - lo) / 2;
                if (count_below(mid) >= N) hi = mid;
                else lo = mid;
            }
            return hi;
        };

        for (int t = 1;; ++t) {
            const double nt_real = std::ceil(P.lambda * std::ldexp(1.0, t - 1));
            SIA_REQUIRE(nt_real < 9.0e15, SIA_EINVAL, "sample count out of range");
            const uint64_t n_t = static_cast<uint64_t>(nt_real);
            I.t = t;
            I.n_t = n_t;
            // probe until the stream holds 2 N_t walks
            while (n_acc < 2 * n_t && end < max_attempts) {
                const uint64_t c = std::min(chunk, max_attempts - end);
                const SampleResult r = run_sampler(g, mode, st, c, end, seed, s, false);
                grow_keep(acc, 8 * n_acc, 8 * (n_acc + r.walks), s);
                if (r.walks)
                    SIA_HIP(hipMemcpyAsync(acc.as<uint64_t>() + n_acc, g->ws.walk_attempt.ptr, 8 * r.walks,
                                           hipMemcpyDeviceToDevice, s));
                n_acc += r.walks;
                end += c;
                I.attempts_sampled += c;
                chunk = std::min<uint64_t>(2 * chunk, uint64_t(1) << 30);
            }
            if (n_acc < 2 * n_t) {
                I.status = -1;
                break;
            }
            const uint64_t a_r = bound(n_t), a_rp = bound(2 * n_t);
            // R_t: greedy
            std::vector<int64_t> sel(static_cast<size_t>(k));
            std::vector<uint64_t> gain(static_cast<size_t>(k));
            const SampleResult r1 = run_sampler(g, mode, st, a_r, 0, seed, s, false);
            I.attempts_sampled += a_r;
            SIA_REQUIRE(r1.walks == n_t, SIA_EDEVICE, "stream prefix does not hold N_t walks");
            run_greedy(g->ws, S, r1.walks, r1.ids, k, sel.data(), gain.data(), s, false);
            uint64_t cov_r = 0;
            for (uint64_t x : gain) cov_r += x;
            // R'_t: coverage of the picks
            const SampleResult r2 = run_sampler(g, mode, st, a_rp - a_r, a_r, seed, s, false);
            I.attempts_sampled += a_rp - a_r;
            SIA_REQUIRE(r2.walks == n_t, SIA_EDEVICE, "stream window does not hold N_t walks");
            SIA_HIP(hipMemsetAsync(bits.ptr, 0, bits.bytes, s));
            SIA_HIP(hipMemcpyAsync(dsel.ptr, sel.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
            SIA_HIP(hipMemsetAsync(scalar.ptr, 0, sizeof(unsigned long long), s));
            hipLaunchKernelGGL(k_mark_selected, dim3(grid_of(static_cast<uint64_t>(k), 256, 1u << 20)), dim3(256),
                               0, s, dsel.as<int64_t>(), k, bits.as<uint32_t>());
            hipLaunchKernelGGL(k_cover_walks, dim3(grid_of(r2.walks * kWave, 256, cus * 16)), dim3(256), 0, s,
                               g->ws.walk_off.as<uint64_t>(), g->ws.walk_len.as<uint32_t>(),
                               g->ws.ids.as<uint32_t>(), r2.walks, bits.as<uint32_t>(),
                               scalar.as<unsigned long long>());
            SIA_HIP(hipGetLastError());
            const uint64_t cov_rp = read_counter();
            double eps_t;
            const bool passed = sas_check(static_cast<double>(cov_r), static_cast<double>(cov_rp),
                                          static_cast<double>(n_t), t, eps, P.lambda1, &eps_t);
            if (passed || static_cast<double>(n_t) >= P.n_max) {
                I.status = passed ? 1 : 0;
                I.attempts_r = a_r;
                I.attempts_rp = a_rp;
                I.cov_r = cov_r;
                I.cov_rp = cov_rp;
                I.eps_t = eps_t;
                const double n_ns = static_cast<double>(g->n - n_sources);
                I.spread_est = static_cast<double>(n_sources) + n_ns * static_cast<double>(n_t) / a_r;
                I.suspension_est = n_ns * static_cast<double>(cov_r) / a_r;
                uint64_t in_x = 0;
                if (mode == SIA_NODES)
                    for (int64_t v : sel)
                        in_x += std::binary_search(st.sorted.begin(), st.sorted.end(), static_cast<int32_t>(v));
                I.suspension_nodes_est = I.suspension_est + static_cast<double>(in_x);
                std::copy(sel.begin(), sel.end(), selected);
                std::copy(gain.begin(), gain.end(), gains);
                break;
            }
        }
        I.ms_total = static_cast<float>(
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        *info = I;
    });
}

}  // extern "C"
