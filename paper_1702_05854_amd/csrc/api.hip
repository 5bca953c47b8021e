// C ABI entry points (declared in include/sia.h): argument checks, the
// host-side source tables, and orchestration of the device phases.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstddef>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>

namespace sia {

namespace {
thread_local std::string g_last_error;

constexpr uint32_t kMaxBuckets = 1u << 16;
}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

void finish_stats(sia_stats &S, const SourceTables &st, int mode, uint64_t n_attempts,
                  const int64_t *selected, const uint64_t *gains, int64_t k)
{
    uint64_t covered = 0;
    int64_t src_selected = 0;
    for (int64_t i = 0; i < k; ++i) {
        covered += gains[i];
        if (mode == SIA_NODES &&
            std::binary_search(st.sorted.begin(), st.sorted.end(), static_cast<int32_t>(selected[i])))
            ++src_selected;
    }
    S.attempts = n_attempts;
    S.covered = covered;
    const double n_ns = static_cast<double>(st.n_ns), N = static_cast<double>(n_attempts);
    if (st.probabilistic) {  // starts over all of V; a seed's own walk is among the kept ones
        S.spread_est = n_ns * static_cast<double>(S.hits) / N;
        S.suspension_est = n_ns * static_cast<double>(covered) / N;
        S.suspension_nodes_est = S.suspension_est;
        return;
    }
    S.spread_est = static_cast<double>(st.sorted.size()) + n_ns * static_cast<double>(S.hits) / N;
    S.suspension_est = n_ns * static_cast<double>(covered) / N;
    S.suspension_nodes_est = S.suspension_est + static_cast<double>(src_selected);
}
void clear_error() { g_last_error.clear(); }

namespace {
// Test hook: when nonzero, the allocation that brings it to zero fails.
std::atomic<uint32_t> g_fail_alloc{0};
}  // namespace

void DevBuf::ensure(size_t want)
{
    if (want == 0) want = 1;
    if (ptr && bytes >= want) return;
    release();
    uint32_t c = g_fail_alloc.load();
    while (c && !g_fail_alloc.compare_exchange_weak(c, c - 1)) {
    }
    if (c == 1) throw Error{SIA_ENOMEM, "device allocation failed (injected by sia_test_fail_alloc)"};
    if (hipMalloc(&ptr, want) != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        throw Error{SIA_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed"};
    }
    bytes = want;
}

void DevBuf::release()
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

void check_query(int64_t n, int64_t m, int mode, const int32_t *sources, int64_t n_sources,
                 int64_t k, uint64_t n_attempts, uint64_t attempt_offset)
{
    SIA_REQUIRE(n >= 2 && n < (int64_t(1) << 31), SIA_EINVAL, "n must be in [2, 2^31)");
    SIA_REQUIRE(m >= 0 && m < (int64_t(1) << 32), SIA_EINVAL, "m must be in [0, 2^32)");
    SIA_REQUIRE(mode == SIA_EDGES || mode == SIA_NODES, SIA_EINVAL, "mode must be SIA_EDGES or SIA_NODES");
    SIA_REQUIRE(sources != nullptr, SIA_EINVAL, "sources is NULL");
    SIA_REQUIRE(n_sources >= 1 && n_sources <= n - 1, SIA_EINVAL,
                "n_sources must be in [1, n-1]");
    const int64_t id_space = mode == SIA_EDGES ? m : n;
    SIA_REQUIRE(k >= 0 && k <= id_space, SIA_EINVAL,
                "k must be in [1, m] (edges) or [1, n] (nodes)");
    SIA_REQUIRE(n_attempts >= 1 && n_attempts < (uint64_t(1) << 32), SIA_EINVAL,
                "n_attempts must be in [1, 2^32)");
    SIA_REQUIRE(attempt_offset <= ~uint64_t(0) - n_attempts, SIA_EINVAL,
                "attempt_offset + n_attempts overflows");
    std::vector<int32_t> s(sources, sources + n_sources);
    std::sort(s.begin(), s.end());
    SIA_REQUIRE(s.front() >= 0 && s.back() < n, SIA_EINVAL, "a source is outside [0, n)");
    SIA_REQUIRE(std::adjacent_find(s.begin(), s.end()) == s.end(), SIA_EINVAL,
                "sources must be distinct");
}

SourceTables build_source_tables(int64_t n, const int32_t *sources, int64_t n_sources)
{
    SourceTables st;
    st.sorted.assign(sources, sources + n_sources);
    std::sort(st.sorted.begin(), st.sorted.end());
    st.t.resize(n_sources);
    for (int64_t i = 0; i < n_sources; ++i)
        st.t[i] = static_cast<uint32_t>(st.sorted[i] - i);  // non-sources below s_i
    st.n_ns = static_cast<uint64_t>(n - n_sources);
    uint32_t shift = 0;
    while (((st.n_ns + (uint64_t(1) << shift) - 1) >> shift) > kMaxBuckets) ++shift;
    st.shift = shift;
    const uint64_t nb = ((st.n_ns + (uint64_t(1) << shift) - 1) >> shift) + 1;
    // pairs (c_b, t_{c_b}): the count below the bucket and the next t at or
    // after its start (0xFFFFFFFF past the last source)
    st.bucket.resize(2 * nb);
    uint64_t c = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        const uint64_t lo = b << shift;
        while (c < static_cast<uint64_t>(n_sources) && st.t[c] < lo) ++c;
        st.bucket[2 * b] = static_cast<uint32_t>(c);
        st.bucket[2 * b + 1] = c < static_cast<uint64_t>(n_sources) ? st.t[c] : 0xFFFFFFFFu;
    }
    // whole 16-byte blocks: the sampler reads both tables a block at a time
    st.t.resize((st.t.size() + 3) & ~size_t(3), 0xFFFFFFFFu);
    st.bucket.resize((st.bucket.size() + 3) & ~size_t(3), static_cast<uint32_t>(n_sources));
    return st;
}

SourceTables build_suspect_tables(int64_t n, const int32_t *suspects, const float *p, int64_t n_suspects)
{
    SIA_REQUIRE(n >= 2 && n < (int64_t(1) << 31), SIA_EINVAL, "n must be in [2, 2^31)");
    SIA_REQUIRE(n_suspects >= 1 && n_suspects <= n, SIA_EINVAL, "need 1 <= n_suspects <= n");
    SIA_REQUIRE(suspects != nullptr && p != nullptr, SIA_EINVAL, "suspects / p is NULL");
    std::vector<std::pair<int32_t, uint32_t>> sp(static_cast<size_t>(n_suspects));
    for (int64_t i = 0; i < n_suspects; ++i) {
        SIA_REQUIRE(suspects[i] >= 0 && suspects[i] < n, SIA_EINVAL, "a suspect is outside [0, n)");
        const float x = p[i];
        SIA_REQUIRE(x >= 0.0f && x <= 1.0f, SIA_EINVAL, "a suspect probability is outside [0, 1] (or NaN)");
        // the weights' rounding rule: round-half-even(p 2^32), clamped below 2^32
        const uint64_t q = static_cast<uint64_t>(std::llrint(std::ldexp(static_cast<double>(x), 32)));
        sp[static_cast<size_t>(i)] = {suspects[i], static_cast<uint32_t>(std::min<uint64_t>(q, 0xFFFFFFFFull))};
    }
    std::sort(sp.begin(), sp.end());
    SourceTables st;
    st.probabilistic = true;
    st.n_ns = static_cast<uint64_t>(n);
    for (size_t i = 0; i < sp.size(); ++i) {
        SIA_REQUIRE(i == 0 || sp[i].first != sp[i - 1].first, SIA_EINVAL, "suspects must be distinct");
        st.sorted.push_back(sp[i].first);
        st.coin.push_back(sp[i].second);
    }
    st.t.assign(4, 0xFFFFFFFFu);  // unused (no rank among sources): one block
    st.bucket.assign(4, 0u);
    return st;
}

}  // namespace sia

using namespace sia;

extern "C" {

const char *sia_version(void) { return "sia 0.1 (gfx950)"; }

void sia_test_fail_alloc(uint32_t nth) { g_fail_alloc.store(nth); }

const char *sia_last_error(void) { return g_last_error.c_str(); }

sia_status sia_check_query(int64_t n, int64_t m, int mode, const int32_t *sources,
                           int64_t n_sources, int64_t k, uint64_t n_attempts,
                           uint64_t attempt_offset)
{
    return guarded([&] { check_query(n, m, mode, sources, n_sources, k, n_attempts, attempt_offset); });
}

sia_status sia_graph_create(int64_t n, int64_t m, const int64_t *col_off, const int32_t *row_idx,
                            const float *w, int inputs_on_device, void *hip_stream,
                            sia_graph **out)
{
    return guarded([&] {
        SIA_REQUIRE(out != nullptr, SIA_EINVAL, "out is NULL");
        *out = nullptr;
        SIA_REQUIRE(n >= 2 && n < (int64_t(1) << 31), SIA_EINVAL, "n must be in [2, 2^31)");
        SIA_REQUIRE(m >= 0 && m < (int64_t(1) << 32), SIA_EINVAL, "m must be in [0, 2^32)");
        SIA_REQUIRE(col_off != nullptr, SIA_EINVAL, "col_off is NULL");
        SIA_REQUIRE(m == 0 || (row_idx != nullptr && w != nullptr), SIA_EINVAL,
                    "row_idx / w is NULL");
        std::unique_ptr<sia_graph> g(new sia_graph);
        g->n = n;
        g->m = m;
        // host structure checks need no device; run them before touching HIP
        if (!inputs_on_device) host_check_structure(n, m, col_off, row_idx);
        SIA_HIP(hipGetDevice(&g->device));
        ingest_graph(g.get(), col_off, row_idx, w, inputs_on_device != 0,
                     static_cast<hipStream_t>(hip_stream));
        *out = g.release();
    });
}

sia_status sia_graph_destroy(sia_graph *g)
{
    return guarded([&] {
        if (!g) return;
        DeviceScope ds(g->device);
        delete g;
    });
}

sia_status sia_graph_info(const sia_graph *g, int64_t *n, int64_t *m)
{
    return guarded([&] {
        SIA_REQUIRE(g != nullptr, SIA_EINVAL, "graph is NULL");
        if (n) *n = g->n;
        if (m) *m = g->m;
    });
}

sia_status sia_graph_arc_bytes(const sia_graph *g, uint32_t *arc_bytes)
{
    return guarded([&] {
        SIA_REQUIRE(g != nullptr && arc_bytes != nullptr, SIA_EINVAL, "NULL argument");
        *arc_bytes = g->arc_bytes;
    });
}

sia_status sia_graph_thresholds(const sia_graph *g, uint32_t *thr_host, void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(g != nullptr && thr_host != nullptr, SIA_EINVAL, "NULL argument");
        DeviceScope ds(g->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        if (!g->m) return;
        if (g->arc_bytes == sizeof(ArcRec)) {
            // thr_hi of every arc: a strided copy straight into the caller's array
            SIA_HIP(hipMemcpy2DAsync(thr_host, sizeof(uint32_t), g->arcs.as<char>() + offsetof(ArcRec, thr_hi),
                                     sizeof(ArcRec), sizeof(uint32_t), static_cast<size_t>(g->m),
                                     hipMemcpyDeviceToHost, s));
        } else {  // compact records hold no thresholds: they follow from the in-degrees
            DevBuf tmp;
            tmp.ensure(sizeof(uint32_t) * static_cast<size_t>(g->m));
            compact_thresholds(g, tmp.as<uint32_t>(), s);
            SIA_HIP(hipMemcpyAsync(thr_host, tmp.ptr, sizeof(uint32_t) * g->m, hipMemcpyDeviceToHost, s));
            SIA_HIP(hipStreamSynchronize(s));
        }
        SIA_HIP(hipStreamSynchronize(s));
    });
}

sia_status sia_quantize(const float *w_dev, uint64_t *q_dev, uint64_t count, void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(count == 0 || (w_dev && q_dev), SIA_EINVAL, "NULL argument");
        quantize_device(w_dev, q_dev, count, static_cast<hipStream_t>(hip_stream));
    });
}

void sia_walks_free(sia_walks *w)
{
    if (!w) return;
    std::free(w->attempt);
    std::free(w->off);
    std::free(w->ids);
    w->attempt = nullptr;
    w->off = nullptr;
    w->ids = nullptr;
    w->n_walks = w->n_ids = 0;
}

static void sample_impl(sia_graph *g, int mode, const SourceTables &st, uint64_t n_attempts,
                        uint64_t attempt_offset, uint64_t seed, sia_walks *out, hipStream_t s)
{
    {
        const SampleResult r = run_sampler(g, mode, st, n_attempts, attempt_offset, seed, s, false);

        std::vector<uint64_t> att(r.walks), off(r.walks);
        std::vector<uint32_t> len(r.walks), ids(r.ids);
        if (r.walks) {
            SIA_HIP(hipMemcpyAsync(att.data(), g->ws.walk_attempt.ptr, 8 * r.walks, hipMemcpyDeviceToHost, s));
            SIA_HIP(hipMemcpyAsync(off.data(), g->ws.walk_off.ptr, 8 * r.walks, hipMemcpyDeviceToHost, s));
            SIA_HIP(hipMemcpyAsync(len.data(), g->ws.walk_len.ptr, 4 * r.walks, hipMemcpyDeviceToHost, s));
        }
        if (r.ids)
            SIA_HIP(hipMemcpyAsync(ids.data(), g->ws.ids.ptr, 4 * r.ids, hipMemcpyDeviceToHost, s));
        SIA_HIP(hipStreamSynchronize(s));

        std::vector<uint64_t> order(r.walks);
        std::iota(order.begin(), order.end(), uint64_t(0));
        std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) { return att[a] < att[b]; });
        out->attempt = static_cast<uint64_t *>(std::malloc(8 * std::max<uint64_t>(r.walks, 1)));
        out->off = static_cast<uint64_t *>(std::malloc(8 * (r.walks + 1)));
        out->ids = static_cast<uint32_t *>(std::malloc(4 * std::max<uint64_t>(r.ids, 1)));
        if (!out->attempt || !out->off || !out->ids) {
            sia_walks_free(out);
            throw std::bad_alloc();
        }
        uint64_t pos = 0;
        for (uint64_t i = 0; i < r.walks; ++i) {
            const uint64_t w = order[i];
            out->attempt[i] = att[w];
            out->off[i] = pos;
            std::memcpy(out->ids + pos, ids.data() + off[w], 4 * static_cast<size_t>(len[w]));
            pos += len[w];
        }
        out->off[r.walks] = pos;
        out->n_walks = r.walks;
        out->n_ids = pos;
        sia_stats &S = out->stats;
        S.attempts = n_attempts;
        S.hits = r.hits;
        S.dead_ends = r.dead;
        S.cycles = r.cycles;
        S.steps = r.steps;
        S.evaluations = r.evals;
        S.walk_ids = r.ids;
        const double n_ns = static_cast<double>(st.n_ns);
        S.spread_est = (st.probabilistic ? 0.0 : static_cast<double>(st.sorted.size())) +
                       n_ns * r.hits / static_cast<double>(n_attempts);
    }
}

sia_status sia_sample(const sia_graph *cg, int mode, const int32_t *sources, int64_t n_sources,
                      uint64_t n_attempts, uint64_t attempt_offset, uint64_t seed,
                      sia_walks *out, void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(cg != nullptr && out != nullptr, SIA_EINVAL, "NULL argument");
        std::memset(out, 0, sizeof(*out));
        sia_graph *g = const_cast<sia_graph *>(cg);
        check_query(g->n, g->m, mode, sources, n_sources, 0, n_attempts, attempt_offset);
        std::lock_guard<std::mutex> lock(g->mu);
        DeviceScope ds(g->device);
        sample_impl(g, mode, build_source_tables(g->n, sources, n_sources), n_attempts, attempt_offset, seed, out,
                    static_cast<hipStream_t>(hip_stream));
    });
}

sia_status sia_sample_suspects(const sia_graph *cg, int mode, const int32_t *suspects, const float *p,
                               int64_t n_suspects, uint64_t n_attempts, uint64_t attempt_offset, uint64_t seed,
                               sia_walks *out, void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(cg != nullptr && out != nullptr, SIA_EINVAL, "NULL argument");
        std::memset(out, 0, sizeof(*out));
        sia_graph *g = const_cast<sia_graph *>(cg);
        const SourceTables st = build_suspect_tables(g->n, suspects, p, n_suspects);
        check_query(g->n, g->m, mode, st.sorted.data(), 1, 0, n_attempts, attempt_offset);  // mode, attempts
        std::lock_guard<std::mutex> lock(g->mu);
        DeviceScope ds(g->device);
        sample_impl(g, mode, st, n_attempts, attempt_offset, seed, out, static_cast<hipStream_t>(hip_stream));
    });
}

sia_status sia_greedy(int64_t id_space, const uint64_t *walk_off, const uint32_t *ids,
                      uint64_t n_walks, int64_t k, int64_t *selected, uint64_t *gains,
                      void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(id_space >= 1 && id_space < (int64_t(1) << 32), SIA_EINVAL,
                    "id_space must be in [1, 2^32)");
        SIA_REQUIRE(k >= 1 && k <= id_space, SIA_EINVAL, "k must be in [1, id_space]");
        SIA_REQUIRE(walk_off != nullptr && selected != nullptr && gains != nullptr, SIA_EINVAL,
                    "NULL argument");
        const uint64_t n_ids = walk_off[n_walks];
        SIA_REQUIRE(walk_off[0] == 0, SIA_EINVAL, "walk_off[0] must be 0");
        SIA_REQUIRE(n_ids == 0 || ids != nullptr, SIA_EINVAL, "ids is NULL");
        std::vector<uint32_t> len(n_walks);
        for (uint64_t w = 0; w < n_walks; ++w) {
            SIA_REQUIRE(walk_off[w + 1] >= walk_off[w], SIA_EINVAL, "walk_off must be non-decreasing");
            len[w] = static_cast<uint32_t>(walk_off[w + 1] - walk_off[w]);
        }
        for (uint64_t e = 0; e < n_ids; ++e)
            SIA_REQUIRE(ids[e] < static_cast<uint64_t>(id_space), SIA_EINVAL, "an id is outside [0, id_space)");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        Workspace ws;
        ws.walk_off.ensure(8 * std::max<uint64_t>(n_walks, 1));
        ws.walk_len.ensure(4 * std::max<uint64_t>(n_walks, 1));
        ws.ids.ensure(4 * std::max<uint64_t>(n_ids, 1));
        if (n_walks) {
            SIA_HIP(hipMemcpyAsync(ws.walk_off.ptr, walk_off, 8 * n_walks, hipMemcpyHostToDevice, s));
            SIA_HIP(hipMemcpyAsync(ws.walk_len.ptr, len.data(), 4 * n_walks, hipMemcpyHostToDevice, s));
        }
        if (n_ids) SIA_HIP(hipMemcpyAsync(ws.ids.ptr, ids, 4 * n_ids, hipMemcpyHostToDevice, s));
        run_greedy(ws, id_space, n_walks, n_ids, k, selected, gains, s, false);
    });
}

// p != NULL: sources are suspects with these probabilities
static sia_status solve_impl(const sia_graph *cg, int mode, const int32_t *sources, const float *p,
                             int64_t n_sources, const int64_t *candidates, int64_t n_candidates, int64_t k,
                             uint64_t n_attempts, uint64_t attempt_offset, uint64_t seed,
                             int64_t *selected, uint64_t *gains, sia_stats *stats, int flags,
                             void *hip_stream)
{
    return guarded([&] {
        SIA_REQUIRE(cg != nullptr && selected != nullptr && gains != nullptr, SIA_EINVAL,
                    "NULL argument");
        SIA_REQUIRE((flags & ~(SIA_FLAG_TIMING | SIA_FLAG_NO_CYCLE_STEPS)) == 0, SIA_EINVAL, "unknown flag bits");
        const bool timing = (flags & SIA_FLAG_TIMING) != 0;
        const bool cycle_steps = (flags & SIA_FLAG_NO_CYCLE_STEPS) == 0;
        sia_graph *g = const_cast<sia_graph *>(cg);
        const SourceTables st = p ? build_suspect_tables(g->n, sources, p, n_sources)
                                  : (check_query(g->n, g->m, mode, sources, n_sources, k, n_attempts, attempt_offset),
                                     build_source_tables(g->n, sources, n_sources));
        if (p) check_query(g->n, g->m, mode, st.sorted.data(), 1, k, n_attempts, attempt_offset);
        SIA_REQUIRE(k >= 1, SIA_EINVAL, "k must be >= 1");
        const int64_t id_space_c = mode == SIA_EDGES ? cg->m : cg->n;
        std::vector<uint32_t> cand_bits;
        if (candidates) {
            SIA_REQUIRE(n_candidates >= k, SIA_EINVAL, "fewer candidates than k");
            cand_bits.assign(static_cast<size_t>((id_space_c + 31) / 32), 0u);
            for (int64_t i = 0; i < n_candidates; ++i) {
                const int64_t x = candidates[i];
                SIA_REQUIRE(x >= 0 && x < id_space_c, SIA_EINVAL, "a candidate is outside the id space");
                uint32_t &w = cand_bits[static_cast<size_t>(x >> 5)];
                SIA_REQUIRE(!((w >> (x & 31)) & 1u), SIA_EINVAL, "candidates must be distinct");
                w |= 1u << (x & 31);
            }
        }
        std::lock_guard<std::mutex> lock(g->mu);
        DeviceScope ds(g->device);
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            SIA_HIP(hipEventCreate(&e0));
            SIA_HIP(hipEventCreate(&e1));
            SIA_HIP(hipEventRecord(e0, s));
        }
        // counts are taken by the greedy's counting pass: atomics fused into the
        // sampler's emission cost it 15% on rmat24 (their random lines compete
        // with its gathers)
        const SampleResult r = run_sampler(g, mode, st, n_attempts, attempt_offset, seed, s, timing, cycle_steps);
        const int64_t id_space = mode == SIA_EDGES ? g->m : g->n;
        DevBuf d_cand;
        if (candidates) {
            d_cand.ensure(4 * cand_bits.size());
            SIA_HIP(hipMemcpyAsync(d_cand.ptr, cand_bits.data(), 4 * cand_bits.size(), hipMemcpyHostToDevice, s));
        }
        const GreedyResult gr = run_greedy(g->ws, id_space, r.walks, r.ids, k, selected, gains, s,
                                           timing, candidates ? d_cand.as<uint32_t>() : nullptr);
        float ms_total = 0.f;
        if (timing) {
            SIA_HIP(hipEventRecord(e1, s));
            SIA_HIP(hipEventSynchronize(e1));
            SIA_HIP(hipEventElapsedTime(&ms_total, e0, e1));
            SIA_HIP(hipEventDestroy(e0));
            SIA_HIP(hipEventDestroy(e1));
        }
        if (stats) {
            sia_stats S{};
            S.hits = r.hits;
            S.dead_ends = r.dead;
            S.cycles = r.cycles;
            S.steps = r.steps;
            S.evaluations = r.evals;
            S.walk_ids = r.ids;
            finish_stats(S, st, mode, n_attempts, selected, gains, k);
            S.ms_sample = r.ms;
            S.ms_count = gr.ms_count;
            S.ms_greedy = gr.ms_greedy;
            S.ms_total = ms_total;
            *stats = S;
        }
    });
}

sia_status sia_solve(const sia_graph *cg, int mode, const int32_t *sources, int64_t n_sources,
                     int64_t k, uint64_t n_attempts, uint64_t attempt_offset, uint64_t seed,
                     int64_t *selected, uint64_t *gains, sia_stats *stats, int flags,
                     void *hip_stream)
{
    return solve_impl(cg, mode, sources, nullptr, n_sources, nullptr, 0, k, n_attempts, attempt_offset, seed,
                      selected, gains, stats, flags, hip_stream);
}

sia_status sia_solve_suspects(const sia_graph *cg, int mode, const int32_t *suspects, const float *p,
                              int64_t n_suspects, int64_t k, uint64_t n_attempts, uint64_t attempt_offset,
                              uint64_t seed, int64_t *selected, uint64_t *gains, sia_stats *stats, int flags,
                              void *hip_stream)
{
    if (!p) {
        sia::set_error("p is NULL");
        return SIA_EINVAL;
    }
    return solve_impl(cg, mode, suspects, p, n_suspects, nullptr, 0, k, n_attempts, attempt_offset, seed,
                      selected, gains, stats, flags, hip_stream);
}

sia_status sia_solve_candidates(const sia_graph *cg, int mode, const int32_t *sources,
                                int64_t n_sources, const int64_t *candidates, int64_t n_candidates,
                                int64_t k, uint64_t n_attempts, uint64_t attempt_offset, uint64_t seed,
                                int64_t *selected, uint64_t *gains, sia_stats *stats, int flags,
                                void *hip_stream)
{
    if (!candidates) {
        sia::set_error("candidates is NULL");
        return SIA_EINVAL;
    }
    return solve_impl(cg, mode, sources, nullptr, n_sources, candidates, n_candidates, k, n_attempts,
                      attempt_offset, seed, selected, gains, stats, flags, hip_stream);
}

}  // extern "C"
