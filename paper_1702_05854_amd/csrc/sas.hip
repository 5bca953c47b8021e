// Stop-and-Stare driver: eSIA (Algorithm 6) / nSIA (Algorithm 9) with Check
// (Algorithm 5 / 8) over the single-query path.
//
// The HSAW stream R_1, R_2, ... is the kept walks in attempt-id order.  The
// driver samples attempt ranges [0, end) in chunks (sized from the hit rate
// seen so far) and appends each chunk's kept walks to a device store, in
// sampling order (unordered within a chunk).  A walk is a function of (seed,
// attempt id), so R_t is exactly the stored walks with attempt id below a
// bound A and R'_t those in [A, A'): the bounds are read off histograms of
// the stored attempt ids, R_t is compacted into the greedy's input, and the
// coverage of the picks is counted over the store's walks in [A, A').  The
// scalar steps of Check run on the host.  The driver reports no step counts,
// so its sampling ends cyclic walks as soon as a repeat is seen.
#include "common.hpp"

#include <chrono>
#include <cmath>
#include <limits>

namespace sia {
namespace {

constexpr int kWave = 64;

// h[(att[i] >> shift) - base] += 1 for the stored attempt ids with
// att[i] >> high == top (all of them when high >= 64), for indices below nbins
__global__ __launch_bounds__(256) void k_att_hist(const uint64_t *att, uint64_t n, uint32_t high, uint64_t top,
                                                  uint32_t shift, uint64_t base, uint32_t nbins, uint32_t *h)
{
    const GLOBAL uint64_t *a = gp(att);
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) {
        const uint64_t x = a[i];
        if (high < 64 && (x >> high) != top) continue;
        const uint64_t b = (x >> shift) - base;
        if (b < nbins) __hip_atomic_fetch_add(gp(h) + b, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// set bit id of every selected id (bits cleared beforehand)
__global__ __launch_bounds__(256) void k_mark_selected(const int64_t *sel, int64_t k, uint32_t *bits)
{
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= k) return;
    const uint32_t x = static_cast<uint32_t>(gp(sel)[i]);
    __hip_atomic_fetch_or(gp(bits) + (x >> 5), 1u << (x & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// n_out += number of walks with attempt id in [lo, hi) holding a marked id;
// one wave per walk
__global__ __launch_bounds__(256) void k_cover_walks(const uint64_t *walk_att, const uint64_t *walk_off,
                                                     const uint32_t *walk_len, const uint32_t *ids,
                                                     uint64_t n_walks, uint64_t lo, uint64_t hi,
                                                     const uint32_t *bits, unsigned long long *n_out)
{
    const GLOBAL uint64_t *att = gp(walk_att);
    const GLOBAL uint64_t *off = gp(walk_off);
    const GLOBAL uint32_t *len = gp(walk_len);
    const GLOBAL uint32_t *id = gp(ids);
    const GLOBAL uint32_t *b = gp(bits);
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    uint32_t covered = 0;
    for (uint64_t w = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kWave; w < n_walks;
         w += waves) {  // uniform per wave
        const uint64_t a = att[w];
        if (a < lo || a >= hi) continue;
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

// store offsets of an appended chunk: dst[i] = src[i] + base
__global__ __launch_bounds__(256) void k_add_base(uint64_t *dst, const uint64_t *src, uint64_t n, uint64_t base)
{
    uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) gp(dst)[i] = gp(src)[i] + base;
}

// ------------------------------------------------ compaction of a stream prefix
constexpr int kSelT = 1024;  // walks per compaction block

// exclusive scan of one value per thread over a kSelT-thread block (sh: kSelT/64 words)
__device__ __forceinline__ uint32_t sel_block_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(x, d, kWave);
        if (lane >= d) x += o;
    }
    if (lane == kWave - 1) sh[wid] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (int k = 0; k < kSelT / kWave; ++k) {
        if (k < wid) before += sh[k];
        total += sh[k];
    }
    __syncthreads();
    return before + x - v;
}

// per block of kSelT stored walks: how many have attempt id < bound, and their ids
__global__ __launch_bounds__(kSelT) void k_sel_count(const uint64_t *walk_att, const uint32_t *walk_len,
                                                   uint64_t n, uint64_t bound, uint32_t *blk)
{
    __shared__ uint32_t sh[kSelT / kWave];
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kSelT) + threadIdx.x;
    const bool sel = i < n && gp(walk_att)[i] < bound;
    uint32_t tw, ti;
    sel_block_scan(sel ? 1u : 0u, sh, tw);
    sel_block_scan(sel ? gp(walk_len)[i] : 0u, sh, ti);
    if (threadIdx.x == 0) {
        gp(blk)[2 * blockIdx.x] = tw;
        gp(blk)[2 * blockIdx.x + 1] = ti;
    }
}

// exclusive scan of the nb (walks, ids) pairs in place; totals at [2 nb], [2 nb + 1]
__global__ __launch_bounds__(kSelT) void k_sel_scan(uint32_t *blk, uint64_t nb)
{
    __shared__ uint32_t sh[kSelT / kWave];
    uint32_t cw = 0, ci = 0;
    for (uint64_t b0 = 0; b0 < nb; b0 += kSelT) {
        const uint64_t b = b0 + threadIdx.x;
        const uint32_t w = b < nb ? gp(blk)[2 * b] : 0u, d = b < nb ? gp(blk)[2 * b + 1] : 0u;
        uint32_t tw, ti;
        const uint32_t ew = sel_block_scan(w, sh, tw);
        const uint32_t ei = sel_block_scan(d, sh, ti);
        if (b < nb) {
            gp(blk)[2 * b] = cw + ew;
            gp(blk)[2 * b + 1] = ci + ei;
        }
        cw += tw;
        ci += ti;
    }
    if (threadIdx.x == 0) {
        gp(blk)[2 * nb] = cw;
        gp(blk)[2 * nb + 1] = ci;
    }
}

// write the selected walks (attempt id < bound) as a CSR set: offsets, lengths, ids
__global__ __launch_bounds__(kSelT) void k_sel_emit(const uint64_t *walk_att, const uint64_t *walk_off,
                                                  const uint32_t *walk_len, const uint32_t *ids, uint64_t n,
                                                  uint64_t bound, const uint32_t *blk, uint64_t *out_off,
                                                  uint32_t *out_len, uint32_t *out_ids)
{
    __shared__ uint32_t sh[kSelT / kWave];
    __shared__ uint64_t src[kSelT];
    __shared__ uint32_t dst[kSelT], cnt[kSelT];
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kSelT) + threadIdx.x;
    const bool sel = i < n && gp(walk_att)[i] < bound;
    const uint32_t L = sel ? gp(walk_len)[i] : 0u;
    uint32_t tw, ti;
    const uint32_t rw = sel_block_scan(sel ? 1u : 0u, sh, tw);
    const uint32_t ri = sel_block_scan(L, sh, ti);
    const uint32_t pw = gp(blk)[2 * blockIdx.x] + rw, pi = gp(blk)[2 * blockIdx.x + 1] + ri;
    if (sel) {
        gp(out_off)[pw] = pi;
        gp(out_len)[pw] = L;
        src[rw] = gp(walk_off)[i];
        dst[rw] = pi;
        cnt[rw] = L;
    }
    __syncthreads();
    // copy the ids, one wave per selected walk of the block
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (uint32_t w = wid; w < tw; w += kSelT / kWave)
        for (uint32_t e = lane; e < cnt[w]; e += kWave) gp(out_ids)[dst[w] + e] = gp(ids)[src[w] + e];
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

// Check (Algorithm 5 / 8): passes when eps_t <= eps.  terms[0..3] receive
// eps_1, eps_2, eps_3 and eps_t, all NaN below the Lambda_1 cut-off (where
// Check returns false without forming them).
bool sas_check(double cov_r, double cov_rp, double n_rp, int t, double eps, double lambda1, double terms[4])
{
    for (int i = 0; i < 4; ++i) terms[i] = std::numeric_limits<double>::quiet_NaN();
    if (cov_rp < lambda1) return false;
    const double e = 1.0 - 1.0 / M_E;
    const double scale = n_rp * (1.0 + eps) / (std::ldexp(1.0, t - 1) * cov_rp);
    const double e1 = cov_r / cov_rp - 1.0;
    const double e2 = eps * std::sqrt(scale);
    const double e3 = eps * std::sqrt(scale * (e - eps) / (1.0 + eps / 3.0));
    terms[0] = e1;
    terms[1] = e2;
    terms[2] = e3;
    terms[3] = (e1 + e2 + e1 * e2) * (e - eps) + e * e3;
    return terms[3] <= eps;
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

// The driver for the query whose sources (or suspects with probabilities) st
// holds; arguments checked by the callers.
static void sas_impl(sia_graph *g, int mode, const SourceTables &st, int64_t k, double eps, double delta,
                     uint64_t seed, uint64_t max_attempts, int64_t *selected, uint64_t *gains, sia_sas_info *info,
                     void *hip_stream)
{
    {
        const auto t0 = std::chrono::steady_clock::now();
        const int64_t n_sources = st.probabilistic ? 0 : static_cast<int64_t>(st.sorted.size());
        std::lock_guard<std::mutex> lock(g->mu);
        DeviceScope ds(g->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const int64_t S = mode == SIA_EDGES ? g->m : g->n;
        const SasParams P = sas_params(static_cast<double>(S), static_cast<double>(k), eps, delta);

        sia_sas_info I{};
        I.lambda = P.lambda;
        I.lambda1 = P.lambda1;
        I.n_max = P.n_max;
        I.t_max = P.t_max;
        I.eps_t = std::numeric_limits<double>::quiet_NaN();

        // the store: kept walks of attempts [0, end) in sampling order
        DevBuf s_att, s_off, s_len, s_ids;
        uint64_t s_n = 0, s_ni = 0;
        DevBuf scalar, bits, dsel, blk;  // one counter, marks, picks, compaction block sums
        scalar.ensure(sizeof(unsigned long long));
        bits.ensure(4 * ((static_cast<uint64_t>(S) + 31) / 32));
        dsel.ensure(sizeof(int64_t) * static_cast<uint64_t>(k));
        const unsigned cus = static_cast<unsigned>(device_cu_count());
        uint64_t end = 0, chunk = uint64_t(1) << 16;
        Workspace &ws = g->ws;

        auto read_counter = [&]() {
            unsigned long long v = 0;
            SIA_HIP(hipMemcpyAsync(&v, scalar.ptr, sizeof(v), hipMemcpyDeviceToHost, s));
            SIA_HIP(hipStreamSynchronize(s));
            return static_cast<uint64_t>(v);
        };
        // smallest A with N stream walks among attempts [0, A): the N-th
        // smallest stored attempt id plus one, by a two-level histogram of
        // the ids (high bits, then the low bits within the chosen bin)
        DevBuf hist;
        constexpr uint32_t kHistBits = 16;
        hist.ensure(sizeof(uint32_t) << kHistBits);
        std::vector<uint32_t> hh(size_t(1) << kHistBits);
        auto histogram = [&](uint32_t high, uint64_t top, uint32_t shift, uint64_t base, uint32_t nbins) {
            SIA_HIP(hipMemsetAsync(hist.ptr, 0, sizeof(uint32_t) * nbins, s));
            hipLaunchKernelGGL(k_att_hist, dim3(grid_of(s_n, 256, cus * 4)), dim3(256), 0, s, s_att.as<uint64_t>(),
                               s_n, high, top, shift, base, nbins, hist.as<uint32_t>());
            SIA_HIP(hipGetLastError());
            SIA_HIP(hipMemcpyAsync(hh.data(), hist.ptr, sizeof(uint32_t) * nbins, hipMemcpyDeviceToHost, s));
            SIA_HIP(hipStreamSynchronize(s));
        };
        auto bounds = [&](uint64_t N1, uint64_t N2, uint64_t *A1, uint64_t *A2) {
            uint32_t L = 0;  // attempt ids are below end <= 2^L
            while ((uint64_t(1) << L) < end) ++L;
            const uint32_t lo_bits = L > kHistBits ? L - kHistBits : 0;
            histogram(64, 0, lo_bits, 0, 1u << kHistBits);
            const std::vector<uint32_t> top = hh;
            for (int q = 0; q < 2; ++q) {
                const uint64_t N = q == 0 ? N1 : N2;
                uint64_t acc = 0, b = 0;
                while (acc + top[b] < N) acc += top[b++];  // bin of the N-th smallest
                uint64_t v = b << lo_bits;
                if (lo_bits) {
                    histogram(lo_bits, b, 0, b << lo_bits, 1u << lo_bits);
                    uint64_t r = 0;
                    while (acc + hh[r] < N) acc += hh[r++];
                    v += r;
                }
                *(q == 0 ? A1 : A2) = v + 1;
            }
        };

        for (int t = 1;; ++t) {
            const double nt_real = std::ceil(P.lambda * std::ldexp(1.0, t - 1));
            SIA_REQUIRE(nt_real < 9.0e15, SIA_EINVAL, "sample count out of range");
            const uint64_t n_t = static_cast<uint64_t>(nt_real);
            I.t = t;
            I.n_t = n_t;
            // sample until the store holds 2 N_t walks; after the first walks,
            // chunks aim at the walks still missing at the hit rate seen so far
            while (s_n < 2 * n_t && end < max_attempts) {
                uint64_t c = chunk;
                if (s_n > 0) {
                    const double rate = static_cast<double>(s_n) / static_cast<double>(end);
                    const double want = 1.05 * static_cast<double>(2 * n_t - s_n) / rate + 65536.0;
                    c = static_cast<uint64_t>(std::min(want, static_cast<double>(uint64_t(1) << 30)));
                }
                c = std::min(c, max_attempts - end);
                // (the driver reports no step counts: cyclic walks stop at detection)
                const SampleResult r = run_sampler(g, mode, st, c, end, seed, s, false, false);
                grow_keep(s_att, 8 * s_n, 8 * (s_n + r.walks), s);
                grow_keep(s_off, 8 * s_n, 8 * (s_n + r.walks), s);
                grow_keep(s_len, 4 * s_n, 4 * (s_n + r.walks), s);
                grow_keep(s_ids, 4 * s_ni, 4 * (s_ni + r.ids), s);
                if (r.walks) {
                    SIA_HIP(hipMemcpyAsync(s_att.as<uint64_t>() + s_n, ws.walk_attempt.ptr, 8 * r.walks,
                                           hipMemcpyDeviceToDevice, s));
                    SIA_HIP(hipMemcpyAsync(s_len.as<uint32_t>() + s_n, ws.walk_len.ptr, 4 * r.walks,
                                           hipMemcpyDeviceToDevice, s));
                    hipLaunchKernelGGL(k_add_base, dim3(grid_of(r.walks, 256, cus * 4)), dim3(256), 0, s,
                                       s_off.as<uint64_t>() + s_n, ws.walk_off.as<uint64_t>(), r.walks, s_ni);
                    SIA_HIP(hipGetLastError());
                }
                if (r.ids)
                    SIA_HIP(hipMemcpyAsync(s_ids.as<uint32_t>() + s_ni, ws.ids.ptr, 4 * r.ids,
                                           hipMemcpyDeviceToDevice, s));
                s_n += r.walks;
                s_ni += r.ids;
                end += c;
                chunk = std::min<uint64_t>(2 * chunk, uint64_t(1) << 30);
            }
            I.attempts_sampled = end;
            if (s_n < 2 * n_t) {
                I.status = -1;
                break;
            }
            SIA_REQUIRE(s_n < 0xFFFFFFFFull && s_ni < 0xFFFFFFFFull, SIA_EINVAL,
                        "the stream outgrew 32-bit walk and id positions");
            uint64_t a_r = 0, a_rp = 0;
            bounds(n_t, 2 * n_t, &a_r, &a_rp);
            // R_t: compact the store's walks below a_r into the greedy's input
            const uint64_t nb = (s_n + kSelT - 1) / kSelT;
            blk.ensure(4 * (2 * nb + 2));
            hipLaunchKernelGGL(k_sel_count, dim3(static_cast<unsigned>(nb)), dim3(kSelT), 0, s,
                               s_att.as<uint64_t>(), s_len.as<uint32_t>(), s_n, a_r, blk.as<uint32_t>());
            hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(kSelT), 0, s, blk.as<uint32_t>(), nb);
            SIA_HIP(hipGetLastError());
            uint32_t tot[2] = {0, 0};
            SIA_HIP(hipMemcpyAsync(tot, blk.as<uint32_t>() + 2 * nb, sizeof(tot), hipMemcpyDeviceToHost, s));
            SIA_HIP(hipStreamSynchronize(s));
            SIA_REQUIRE(tot[0] == n_t, SIA_EDEVICE, "stream prefix does not hold N_t walks");
            ws.walk_off.ensure(8 * std::max<uint64_t>(n_t, 1));
            ws.walk_len.ensure(4 * std::max<uint64_t>(n_t, 1));
            ws.ids.ensure(4 * std::max<uint64_t>(tot[1], 1));
            hipLaunchKernelGGL(k_sel_emit, dim3(static_cast<unsigned>(nb)), dim3(kSelT), 0, s,
                               s_att.as<uint64_t>(), s_off.as<uint64_t>(), s_len.as<uint32_t>(),
                               s_ids.as<uint32_t>(), s_n, a_r, blk.as<uint32_t>(), ws.walk_off.as<uint64_t>(),
                               ws.walk_len.as<uint32_t>(), ws.ids.as<uint32_t>());
            SIA_HIP(hipGetLastError());
            std::vector<int64_t> sel(static_cast<size_t>(k));
            std::vector<uint64_t> gain(static_cast<size_t>(k));
            run_greedy(ws, S, n_t, tot[1], k, sel.data(), gain.data(), s, false);
            uint64_t cov_r = 0;
            for (uint64_t x : gain) cov_r += x;
            // R'_t: coverage of the picks over the store's walks in [a_r, a_rp)
            SIA_HIP(hipMemsetAsync(bits.ptr, 0, bits.bytes, s));
            SIA_HIP(hipMemcpyAsync(dsel.ptr, sel.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
            SIA_HIP(hipMemsetAsync(scalar.ptr, 0, sizeof(unsigned long long), s));
            hipLaunchKernelGGL(k_mark_selected, dim3(grid_of(static_cast<uint64_t>(k), 256, 1u << 20)), dim3(256),
                               0, s, dsel.as<int64_t>(), k, bits.as<uint32_t>());
            hipLaunchKernelGGL(k_cover_walks, dim3(grid_of(s_n * kWave, 256, cus * 16)), dim3(256), 0, s,
                               s_att.as<uint64_t>(), s_off.as<uint64_t>(), s_len.as<uint32_t>(),
                               s_ids.as<uint32_t>(), s_n, a_r, a_rp, bits.as<uint32_t>(),
                               scalar.as<unsigned long long>());
            SIA_HIP(hipGetLastError());
            const uint64_t cov_rp = read_counter();
            double terms[4];
            const bool passed = sas_check(static_cast<double>(cov_r), static_cast<double>(cov_rp),
                                          static_cast<double>(n_t), t, eps, P.lambda1, terms);
            if (passed || static_cast<double>(n_t) >= P.n_max) {
                I.status = passed ? 1 : 0;
                I.attempts_r = a_r;
                I.attempts_rp = a_rp;
                I.cov_r = cov_r;
                I.cov_rp = cov_rp;
                I.eps_t = terms[3];
                const double n_ns = static_cast<double>(g->n - n_sources);
                I.spread_est = static_cast<double>(n_sources) + n_ns * static_cast<double>(n_t) / a_r;
                I.suspension_est = n_ns * static_cast<double>(cov_r) / a_r;
                uint64_t in_x = 0;
                if (mode == SIA_NODES && !st.probabilistic)  // (suspects: a seed's own walk is sampled)
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
    }
}

static void sas_check_args(const sia_graph *cg, int64_t *selected, uint64_t *gains, sia_sas_info *info,
                           double eps, double delta)
{
    SIA_REQUIRE(cg != nullptr && selected != nullptr && gains != nullptr && info != nullptr, SIA_EINVAL,
                "NULL argument");
    SIA_REQUIRE(eps > 0.0 && eps < 1.0 - 1.0 / M_E, SIA_EINVAL, "eps must be in (0, 1 - 1/e)");
    SIA_REQUIRE(delta > 0.0 && delta < 1.0, SIA_EINVAL, "delta must be in (0, 1)");
}

sia_status sia_sas_solve(const sia_graph *cg, int mode, const int32_t *sources, int64_t n_sources,
                         int64_t k, double eps, double delta, uint64_t seed, uint64_t max_attempts,
                         int64_t *selected, uint64_t *gains, sia_sas_info *info, void *hip_stream)
{
    return guarded([&] {
        sas_check_args(cg, selected, gains, info, eps, delta);
        sia_graph *g = const_cast<sia_graph *>(cg);
        check_query(g->n, g->m, mode, sources, n_sources, k, max_attempts, 0);
        SIA_REQUIRE(k >= 1, SIA_EINVAL, "k must be >= 1");
        sas_impl(g, mode, build_source_tables(g->n, sources, n_sources), k, eps, delta, seed, max_attempts,
                 selected, gains, info, hip_stream);
    });
}

sia_status sia_sas_solve_suspects(const sia_graph *cg, int mode, const int32_t *suspects, const float *p,
                                  int64_t n_suspects, int64_t k, double eps, double delta, uint64_t seed,
                                  uint64_t max_attempts, int64_t *selected, uint64_t *gains, sia_sas_info *info,
                                  void *hip_stream)
{
    return guarded([&] {
        sas_check_args(cg, selected, gains, info, eps, delta);
        sia_graph *g = const_cast<sia_graph *>(cg);
        const SourceTables st = build_suspect_tables(g->n, suspects, p, n_suspects);
        check_query(g->n, g->m, mode, st.sorted.data(), 1, k, max_attempts, 0);  // mode, k, attempts
        SIA_REQUIRE(k >= 1, SIA_EINVAL, "k must be >= 1");
        sas_impl(g, mode, st, k, eps, delta, seed, max_attempts, selected, gains, info, hip_stream);
    });
}

sia_status sia_evaluate(const sia_graph *cg, int mode, const int32_t *sources, int64_t n_sources,
                        const int64_t *selected, int64_t k, uint64_t n_attempts, uint64_t attempt_offset,
                        uint64_t seed, sia_stats *stats, void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(cg != nullptr && selected != nullptr && stats != nullptr, SIA_EINVAL, "NULL argument");
        sia_graph *g = const_cast<sia_graph *>(cg);
        check_query(g->n, g->m, mode, sources, n_sources, k, n_attempts, attempt_offset);
        SIA_REQUIRE(k >= 1, SIA_EINVAL, "k must be >= 1");
        const int64_t S = mode == SIA_EDGES ? g->m : g->n;
        for (int64_t i = 0; i < k; ++i)
            SIA_REQUIRE(selected[i] >= 0 && selected[i] < S, SIA_EINVAL, "a selected id is outside the id space");
        std::lock_guard<std::mutex> lock(g->mu);
        DeviceScope ds(g->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const SourceTables st = build_source_tables(g->n, sources, n_sources);
        const SampleResult r = run_sampler(g, mode, st, n_attempts, attempt_offset, seed, s, false);
        DevBuf scalar, bits, dsel;
        scalar.ensure(sizeof(unsigned long long));
        bits.ensure(4 * ((static_cast<uint64_t>(S) + 31) / 32));
        dsel.ensure(sizeof(int64_t) * static_cast<uint64_t>(k));
        SIA_HIP(hipMemsetAsync(bits.ptr, 0, bits.bytes, s));
        SIA_HIP(hipMemsetAsync(scalar.ptr, 0, sizeof(unsigned long long), s));
        SIA_HIP(hipMemcpyAsync(dsel.ptr, selected, sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
        const unsigned cus = static_cast<unsigned>(device_cu_count());
        hipLaunchKernelGGL(k_mark_selected, dim3(grid_of(static_cast<uint64_t>(k), 256, 1u << 20)), dim3(256), 0,
                           s, dsel.as<int64_t>(), k, bits.as<uint32_t>());
        hipLaunchKernelGGL(k_cover_walks, dim3(grid_of(r.walks * kWave, 256, cus * 16)), dim3(256), 0, s,
                           g->ws.walk_attempt.as<uint64_t>(), g->ws.walk_off.as<uint64_t>(),
                           g->ws.walk_len.as<uint32_t>(), g->ws.ids.as<uint32_t>(), r.walks, uint64_t(0),
                           ~uint64_t(0), bits.as<uint32_t>(), scalar.as<unsigned long long>());
        SIA_HIP(hipGetLastError());
        unsigned long long covered = 0;
        SIA_HIP(hipMemcpyAsync(&covered, scalar.ptr, sizeof(covered), hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));
        sia_stats R{};
        R.attempts = n_attempts;
        R.hits = r.hits;
        R.dead_ends = r.dead;
        R.cycles = r.cycles;
        R.steps = r.steps;
        R.evaluations = r.evals;
        R.walk_ids = r.ids;
        R.covered = covered;
        const double n_ns = static_cast<double>(g->n - n_sources);
        R.spread_est = static_cast<double>(n_sources) + n_ns * static_cast<double>(r.hits) / n_attempts;
        R.suspension_est = n_ns * static_cast<double>(covered) / n_attempts;
        uint64_t in_x = 0;
        if (mode == SIA_NODES)
            for (int64_t i = 0; i < k; ++i)
                in_x += std::binary_search(st.sorted.begin(), st.sorted.end(), static_cast<int32_t>(selected[i]));
        R.suspension_nodes_est = R.suspension_est + static_cast<double>(in_x);
        *stats = R;
    });
}

sia_status sia_sas_params(int64_t id_space, int64_t k, double eps, double delta, double *lambda,
                          double *lambda1, double *n_max, int32_t *t_max)
{
    return guarded([&] {
        SIA_REQUIRE(id_space >= 1 && k >= 1 && k <= id_space, SIA_EINVAL, "need 1 <= k <= id_space");
        SIA_REQUIRE(eps > 0.0 && eps < 1.0 - 1.0 / M_E, SIA_EINVAL, "eps must be in (0, 1 - 1/e)");
        SIA_REQUIRE(delta > 0.0 && delta < 1.0, SIA_EINVAL, "delta must be in (0, 1)");
        const SasParams P = sas_params(static_cast<double>(id_space), static_cast<double>(k), eps, delta);
        if (lambda) *lambda = P.lambda;
        if (lambda1) *lambda1 = P.lambda1;
        if (n_max) *n_max = P.n_max;
        if (t_max) *t_max = P.t_max;
    });
}

sia_status sia_sas_check(double cov_r, double cov_rp, double n_rp, int32_t t, double eps, double lambda1,
                         double *terms, int32_t *passed)
{
    return guarded([&] {
        SIA_REQUIRE(terms != nullptr && passed != nullptr, SIA_EINVAL, "NULL argument");
        SIA_REQUIRE(t >= 1 && t < 1024, SIA_EINVAL, "t must be in [1, 1024)");
        SIA_REQUIRE(cov_rp > 0.0 && n_rp > 0.0 && cov_r >= 0.0, SIA_EINVAL, "need cov_rp > 0, n_rp > 0, cov_r >= 0");
        SIA_REQUIRE(eps > 0.0 && eps < 1.0 - 1.0 / M_E, SIA_EINVAL, "eps must be in (0, 1 - 1/e)");
        *passed = sas_check(cov_r, cov_rp, n_rp, t, eps, lambda1, terms) ? 1 : 0;
    });
}

}  // extern "C"
