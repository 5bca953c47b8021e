// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sia.h"
#include "layout.hpp"

namespace sia {

// ------------------------------------------------------------ errors
void set_error(const std::string &msg);
void clear_error();

struct Error {
    sia_status status;
    std::string msg;
};

#define SIA_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::sia::Error{e_ == hipErrorOutOfMemory ? SIA_ENOMEM : SIA_EDEVICE,    \
                               std::string(#call) + ": " + hipGetErrorString(e_)};      \
    } while (0)

#define SIA_REQUIRE(cond, status, msg)                                                  \
    do {                                                                                \
        if (!(cond)) throw ::sia::Error{(status), (msg)};                               \
    } while (0)

// Run f(); turn failures into a status and the calling thread's message.
template <class F>
sia_status guarded(F &&f)
{
    try {
        clear_error();
        f();
        return SIA_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return SIA_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return SIA_EDEVICE;
    }
}

// Make a device current for the duration of a call.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        SIA_HIP(hipGetDevice(&prev));
        if (prev != dev) SIA_HIP(hipSetDevice(dev));
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
    DeviceScope(const DeviceScope &) = delete;
    DeviceScope &operator=(const DeviceScope &) = delete;
};

// ------------------------------------------------------------ device buffers
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    void ensure(size_t want);  // grow-only, contents not preserved
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
    void swap(DevBuf &o)
    {
        std::swap(ptr, o.ptr);
        std::swap(bytes, o.bytes);
    }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

struct Workspace {
    DevBuf walk_attempt, walk_off, walk_len, ids;  // sampler output
    DevBuf counters;                               // sampler / greedy scalars
    DevBuf src_sorted, src_t, bucket, bitmap;      // per-query source tables
    DevBuf cnt;                                    // coverage counts
    DevBuf greedy, jobs;                           // greedy scratch + job table
    DevBuf ring;                                   // the sampler's walk ring
    DevBuf coin_thr, coin_src;                     // suspects' coin thresholds: per node, per suspect
    uint64_t walk_cap = 0, id_cap = 0;
};

}  // namespace sia

struct sia_graph {
    int64_t n = 0, m = 0;
    int device = 0;
    sia::DevBuf nodes;  // NodeRec[n]
    sia::DevBuf arcs;   // ArcRec[m] or ArcRec16[m] (arc_bytes), in CSR order
    uint32_t arc_bytes = sizeof(sia::ArcRec);
    sia::Workspace ws;
    std::mutex mu;      // one query at a time per graph handle
    std::mutex tag_mu;  // guards tag_bits
    uint32_t tag_bits = 0;  // source-tag bits 0..30 held by batches
};

namespace sia {

// Per-query source tables, built on the host.
struct SourceTables {
    std::vector<int32_t> sorted;   // ascending sources
    std::vector<uint32_t> t;       // t_i = s_i - i (non-sources below s_i)
    std::vector<uint32_t> bucket;  // pairs: [2b] = #{i : t_i < b << shift}, [2b+1] = t at that count
    // (t and bucket are padded to whole 16-byte blocks: 0xFFFFFFFF, |X|)
    uint32_t shift = 0;
    uint64_t n_ns = 0;
    // probabilistic suspects (sorted holds them): the seed coin threshold of
    // each, min(round-half-even(p 2^32), 2^32 - 1); start over all of V
    bool probabilistic = false;
    std::vector<uint32_t> coin;
};
void check_query(int64_t n, int64_t m, int mode, const int32_t *sources, int64_t n_sources,
                 int64_t k, uint64_t n_attempts, uint64_t attempt_offset);
SourceTables build_source_tables(int64_t n, const int32_t *sources, int64_t n_sources);
// Suspects with probabilities (checked: distinct ids in [0,n), 1 <= count <= n,
// every p in [0,1]).
SourceTables build_suspect_tables(int64_t n, const int32_t *suspects, const float *p, int64_t n_suspects);
// Fill attempts, covered and the estimates of a finished query into S (whose
// counters are already set).
void finish_stats(sia_stats &S, const SourceTables &st, int mode, uint64_t n_attempts,
                  const int64_t *selected, const uint64_t *gains, int64_t k);

// One entry of a sampling wave: attempts [local_start, local_start + count)
// of the query in slot `slot` (index into the wave's SlotDev array).
struct WaveItem {
    uint32_t slot;
    uint64_t local_start;
    uint64_t count;
};

void fill_wave_table(WaveTable &t, const WaveItem *items, uint32_t n_items, uint32_t n_slots);

// Launch shape of the sampler: persistent workgroups per CU (0: as many as
// fit) and attempts a wave takes from the chunk counter per refill.
struct SamplerConfig {
    int blocks_per_cu = 0;
    uint32_t chunk = 256;
    int cus = 0;  // CUs the launch stream may use (0: all of the device)
};
int sampler_max_blocks_per_cu(const sia_graph *g);  // for the graph's record format

// Sample the wave described by d_table (device) over the n_slots SlotDev
// entries at d_slots (device).  Asynchronous on stream s.
void launch_wave(const sia_graph *g, const SlotDev *d_slots, uint32_t n_slots,
                 const WaveTable *d_table, const SamplerConfig &cfg, uint32_t *ring, hipStream_t s);
// Bytes of the walk ring a launch on g needs (the largest grid; device memory
// owned by the caller, contents need no clearing; one ring per concurrent launch).
size_t sampler_ring_bytes(const sia_graph *g);
// Set or clear the tag bit `mask` of the given sources (device array).
void tag_sources(const sia_graph *g, const int32_t *d_src, uint32_t n_src, uint32_t mask, bool set,
                 hipStream_t s);

struct SampleResult {
    uint64_t walks = 0, ids = 0, hits = 0, dead = 0, cycles = 0, steps = 0, evals = 0;
    float ms = 0.f;
};

// A single query (slot bit 31): upload sources, tag them, run one wave
// (rerunning with larger buffers if the output did not fit), untag.
// Results stay in g->ws; coverage counts are taken by the greedy.
// cycle_steps: search cyclic walks for their entry so that the steps counter
// is exact (false: such walks stop at detection and count no steps).
SampleResult run_sampler(sia_graph *g, int mode, const SourceTables &st, uint64_t n_attempts,
                         uint64_t attempt_offset, uint64_t seed, hipStream_t s, bool timing,
                         bool cycle_steps = true);

struct GreedyResult {
    float ms_count = 0.f, ms_greedy = 0.f;
};

// One greedy job: the kept walks of one query (device arrays) and where its
// answer goes.  scratch holds greedy_scratch_bytes(id_space, n_walks, n_ids,
// k) bytes of device memory owned by the caller.
struct GreedyInput {
    const uint64_t *walk_off = nullptr;
    const uint32_t *walk_len = nullptr;
    const uint32_t *ids = nullptr;
    uint64_t id_space = 0, n_walks = 0, n_ids = 0;
    int64_t k = 0;
    uint32_t *cnt = nullptr;    // id_space coverage counts (device), written here
    const uint32_t *cand = nullptr;  // candidate bitmap over [0, id_space) (device); NULL: every id
    void *scratch = nullptr;
    int64_t *selected = nullptr;  // k entries each; host memory (device memory
    uint64_t *gains = nullptr;    // when out_on_device: written in place)
    bool out_on_device = false;
    uint32_t rounds_seen = 0;     // progress bookkeeping
};
size_t greedy_scratch_bytes(uint64_t id_space, uint64_t n_walks, uint64_t n_ids, int64_t k);
size_t greedy_job_table_bytes(uint32_t n_jobs);  // job records + their states

// Inverted index + k greedy rounds for every job, concurrently (blockIdx.y /
// one workgroup per job).  d_job_table: greedy_job_table_bytes(jobs.size())
// bytes of device memory.  Synchronises s; writes each job's selected ids and
// gains to its host arrays.  Timing (if requested) covers all jobs.
// hist_base: histogram workgroups for a single job (0: one per CU).
void run_greedy_jobs(std::vector<GreedyInput> &jobs, void *d_job_table, hipStream_t s, bool timing,
                     GreedyResult *res, unsigned hist_base = 0);

// A single job over the walks held in ws (walk_off / walk_len / ids, n_walks
// walks, n_ids ids); the counts go to ws.cnt.  cand: candidate bitmap
// (device, NULL: every id); the caller guarantees at least k candidates.
GreedyResult run_greedy(Workspace &ws, int64_t id_space, uint64_t n_walks, uint64_t n_ids,
                        int64_t k, int64_t *selected, uint64_t *gains, hipStream_t s,
                        bool timing, const uint32_t *cand = nullptr);

// Ingest: host structure checks (no device needed) and the device kernels.
void host_check_structure(int64_t n, int64_t m, const int64_t *col_off, const int32_t *row_idx);
void ingest_graph(sia_graph *g, const int64_t *col_off, const int32_t *row_idx, const float *w,
                  bool on_device, hipStream_t s);
void quantize_device(const float *w, uint64_t *q, uint64_t count, hipStream_t s);
// Threshold table thr[m] (device) of a graph with compact records.
void compact_thresholds(const sia_graph *g, uint32_t *d_thr, hipStream_t s);

int device_cu_count();

}  // namespace sia
