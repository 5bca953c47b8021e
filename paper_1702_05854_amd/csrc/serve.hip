// Batched / served queries on one resident graph (an addition to the
// method: the paper runs one query per launch).
//
// Two host threads drive the device:
//  * the sampler thread admits queued queries into free slots (one source-tag
//    bit each), and runs sampling launches that give every admitted query a
//    share of its attempts.  Each slot's walk-reservation counters start at
//    the query's committed watermark, so a share whose kept walks outgrow the
//    slot's buffer is simply discarded and sampled again with a buffer of the
//    size the counters report.  Shares are deterministic functions of their
//    attempt ids, so a query's walks -- and its answer -- do not depend on
//    how it was cut into shares or what it shared launches with.
//  * a query whose attempts are all sampled waits for its greedy, which runs
//    with others in shared launches (one job each; coverage is counted there
//    from the kept walks).  By default (time-sliced) the sampler thread runs
//    them between sampling launches, once greedy_batch of them wait or
//    sampling cannot go on without them; in the concurrent mode the greedy
//    thread runs them on its own stream, overlapping the sampling launches.
//
// Walk memory: slot buffers grow on demand within the budget and are kept
// for the slot's next query; buffers of idle slots are released when a busy
// slot needs the room.  If every sampling query is stalled for memory and
// nothing else can free any, the most recently admitted one is restarted
// from its first attempt (eviction), so the oldest always progresses.
#include "common.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>

namespace sia {
namespace {

using Clock = std::chrono::steady_clock;

enum class TState { Pending, Sampling, Ready, Greedy, Done };

struct Ticket {
    uint64_t id = 0;
    int mode = SIA_EDGES;
    int64_t k = 0;
    uint64_t n_attempts = 0, offset = 0, seed = 0;
    bool cycle_steps = true;  // search cyclic walks for their entry (exact steps)
    SourceTables st;
    TState state = TState::Pending;
    sia_status status = SIA_OK;
    std::string error;
    bool cancel = false;
    int slot = -1;
    uint64_t admit_seq = 0;
    // sampling progress (sampler thread)
    uint64_t done = 0;         // attempts committed
    uint64_t retry_chunk = 0;  // size of a share that overflowed (0: none)
    uint64_t need_walks = 0, need_ids = 0;  // its exact needs beyond the watermarks
    uint64_t wm_walks = 0, wm_ids = 0;
    uint64_t hits = 0, dead = 0, cycles = 0, steps = 0, evals = 0;
    std::vector<int64_t> selected;
    std::vector<uint64_t> gains;
    sia_stats stats{};
    sia_ticket_info info{};
};
using TicketP = std::shared_ptr<Ticket>;

struct Slot {
    uint32_t tag_mask = 0;
    DevBuf src_sorted, src_t, bucket;
    DevBuf walk_attempt, walk_off, walk_len, ids;
    uint64_t walk_cap = 0, id_cap = 0;
    DevBuf cnt, greedy;
    TicketP t;  // occupant (guarded by the batch mutex)
};

constexpr uint64_t kBytesPerWalk = 8 + 8 + 4;  // attempt, offset, length
constexpr uint64_t kWalkSlack = 1024, kIdSlack = 16384;
constexpr double kHeadroom = 1.3;
constexpr double kGreedyMaxWait = 0.1;  // s a finished query waits at most for a greedy batch

uint64_t walk_bytes_of(uint64_t walks, uint64_t ids) { return walks * kBytesPerWalk + ids * 4; }

// Reallocate a device buffer to exactly `bytes`, keeping its first `keep`
// bytes (the copy runs on s and is waited for before the old buffer goes).
void realloc_keep(DevBuf &b, size_t bytes, size_t keep, hipStream_t s)
{
    if (b.ptr && b.bytes == bytes) return;
    void *p = nullptr;
    SIA_HIP(hipMalloc(&p, bytes ? bytes : 1));
    if (keep && b.ptr) {
        const hipError_t e = hipMemcpyAsync(p, b.ptr, keep, hipMemcpyDeviceToDevice, s);
        const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize(s) : e;
        if (e2 != hipSuccess) {
            (void)hipFree(p);
            SIA_HIP(e2);
        }
    }
    b.release();
    b.ptr = p;
    b.bytes = bytes;
}

}  // namespace
}  // namespace sia

using namespace sia;

struct sia_batch {
    sia_graph *g = nullptr;
    uint32_t n_slots = 0;
    uint32_t tag_bits = 0;
    uint64_t budget = 0;
    sia_batch_config cfg{};
    std::vector<Slot> slots;
    hipStream_t s_sample = nullptr, s_greedy = nullptr;
    WaveTable *h_table = nullptr;  // pinned staging of the launch inputs / outputs
    SlotDev *h_slots = nullptr;
    uint64_t *h_ctr_in = nullptr, *h_ctr_out = nullptr;
    DevBuf d_table, d_slots, d_ctr, d_jobs;
    DevBuf d_ring;  // the sampler's walk ring (one launch at a time)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    SamplerConfig exec_cfg{};
    int sampler_cus = 0;  // CUs of the sampling stream (0: all)

    std::mutex mu;
    std::condition_variable cv_sampler, cv_greedy, cv_done;
    std::deque<TicketP> pending, ready;
    std::map<uint64_t, TicketP> tickets;
    uint64_t next_id = 1, admit_seq = 0;
    uint64_t mem_epoch = 0;     // bumped whenever a slot frees up
    uint32_t spins = 0;         // stall resolutions in a row that changed nothing
    uint64_t greedy_running = 0;
    bool stop = false, tuning = false;
    sia_status fatal = SIA_OK;
    std::string fatal_msg;
    sia_batch_stats ctr{};      // counters (under mu)
    std::atomic<uint64_t> walk_bytes{0};
    // sampler-thread estimates of kept walks and ids per attempt, per mode
    double est_att[2] = {0, 0}, est_walks[2] = {0, 0}, est_ids[2] = {0, 0};
    Clock::time_point t0;
    std::thread th_sample, th_greedy;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    // ------------------------------------------------------------ helpers
    SamplerConfig sampler_config() const
    {
        SamplerConfig sc;
        sc.blocks_per_cu = cfg.sampler_blocks_per_cu;
        sc.chunk = cfg.refill_chunk;
        sc.cus = sampler_cus;
        return sc;
    }

    uint64_t slot_bytes(const Slot &s) const { return walk_bytes_of(s.walk_cap, s.id_cap); }

    // rates for sizing a share of ticket t (own rates once it has some, else the mode's)
    void rates(const Ticket &t, double &wpa, double &ipa) const
    {
        const int m = t.mode;
        if (t.done >= 65536) {
            wpa = static_cast<double>(t.wm_walks) / t.done;
            ipa = static_cast<double>(t.wm_ids) / t.done;
        } else if (est_att[m] > 0) {
            wpa = est_walks[m] / est_att[m];
            ipa = est_ids[m] / est_att[m];
        } else {
            wpa = 0.25;
            ipa = m == SIA_EDGES ? 2.0 : 2.5;
        }
    }

    void share_needs(const Ticket &t, uint64_t chunk, uint64_t &walks, uint64_t &ids) const
    {
        if (t.retry_chunk && chunk == t.retry_chunk) {
            walks = t.wm_walks + t.need_walks;
            ids = t.wm_ids + t.need_ids;
            return;
        }
        double wpa, ipa;
        rates(t, wpa, ipa);
        walks = t.wm_walks + std::min<uint64_t>(chunk, static_cast<uint64_t>(std::ceil(chunk * wpa * kHeadroom)) + kWalkSlack);
        ids = t.wm_ids + static_cast<uint64_t>(std::ceil(chunk * ipa * kHeadroom)) + kIdSlack;
    }

    // Budget bytes slot i may hold, given what the other slots hold.
    uint64_t room_of(const Slot &sl) const
    {
        const uint64_t others = walk_bytes.load() - slot_bytes(sl);
        return others < budget ? budget - others : 0;
    }

    // Resize slot i's walk buffers to exactly (w walks, d ids), both at or
    // above its watermarks, keeping the committed prefix.
    void resize(uint32_t i, uint64_t w, uint64_t d)
    {
        Slot &sl = slots[i];
        const Ticket &t = *sl.t;
        const uint64_t before = slot_bytes(sl);
        if (w != sl.walk_cap) {
            realloc_keep(sl.walk_attempt, 8 * w, 8 * t.wm_walks, s_sample);
            realloc_keep(sl.walk_off, 8 * w, 8 * t.wm_walks, s_sample);
            realloc_keep(sl.walk_len, 4 * w, 4 * t.wm_walks, s_sample);
            sl.walk_cap = w;
        }
        if (d != sl.id_cap) {
            realloc_keep(sl.ids, 4 * d, 4 * t.wm_ids, s_sample);
            sl.id_cap = d;
        }
        walk_bytes = walk_bytes.load() - before + slot_bytes(sl);
        std::lock_guard<std::mutex> lk(mu);
        ctr.walk_bytes_peak = std::max<uint64_t>(ctr.walk_bytes_peak, walk_bytes.load());
    }

    // Make slot i hold room for at least (walks, ids).  Prefers 1.5x growth
    // (fewer reallocations), then growth to the need, then exactly the need
    // (shrinking the part that is larger than needed).  False if the budget
    // does not allow it even after releasing idle slots' buffers.
    bool reserve(uint32_t i, uint64_t walks, uint64_t ids)
    {
        Slot &sl = slots[i];
        if (sl.walk_cap >= walks && sl.id_cap >= ids) return true;
        const uint64_t mw = std::max(walks, sl.walk_cap), mi = std::max(ids, sl.id_cap);
        if (walk_bytes_of(walks, ids) > room_of(sl)) release_idle();
        const uint64_t room = room_of(sl);
        const uint64_t gw = walks > sl.walk_cap ? std::max(walks, sl.walk_cap + sl.walk_cap / 2) : sl.walk_cap;
        const uint64_t gi = ids > sl.id_cap ? std::max(ids, sl.id_cap + sl.id_cap / 2) : sl.id_cap;
        if (walk_bytes_of(gw, gi) <= room) resize(i, gw, gi);
        else if (walk_bytes_of(mw, mi) <= room) resize(i, mw, mi);
        else if (walk_bytes_of(walks, ids) <= room) resize(i, walks, ids);
        else return false;
        return true;
    }

    // Give slot i all the room the budget has left, for a share of c
    // attempts: walk records for the walks the share is expected to keep
    // (at most c, at least one), the rest for ids.  False if that leaves no
    // room for one more walk and one more id.
    bool reserve_all(uint32_t i, uint64_t c)
    {
        Slot &sl = slots[i];
        const Ticket &t = *sl.t;
        release_idle();
        const uint64_t room = room_of(sl);
        const uint64_t base = walk_bytes_of(t.wm_walks, t.wm_ids);
        if (room < base + kBytesPerWalk + 4) return false;
        double wpa, ipa;
        rates(t, wpa, ipa);
        uint64_t extra_w = std::min<uint64_t>(c, static_cast<uint64_t>(std::ceil(c * wpa * kHeadroom)) + 64);
        extra_w = std::max<uint64_t>(1, std::min<uint64_t>(extra_w, (room - base - 4) / kBytesPerWalk));
        const uint64_t w = t.wm_walks + extra_w;
        const uint64_t d = (room - walk_bytes_of(w, 0)) / 4;
        resize(i, w, d);
        return true;
    }

    // Release the walk buffers of slots without a query.
    void release_idle()
    {
        std::vector<uint32_t> idle;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (uint32_t i = 0; i < n_slots; ++i)
                if (!slots[i].t && slots[i].walk_cap) idle.push_back(i);
        }
        for (uint32_t i : idle) release_walks(i);  // a slot only gets a query from this thread
    }

    void release_walks(uint32_t i)
    {
        Slot &sl = slots[i];
        walk_bytes -= slot_bytes(sl);
        sl.walk_attempt.release();
        sl.walk_off.release();
        sl.walk_len.release();
        sl.ids.release();
        sl.walk_cap = sl.id_cap = 0;
    }

    void upload_sources(uint32_t i)
    {
        Slot &sl = slots[i];
        const SourceTables &st = sl.t->st;
        const size_t ns = st.sorted.size();
        sl.src_sorted.ensure(4 * ns);
        sl.src_t.ensure(4 * st.t.size());
        sl.bucket.ensure(4 * st.bucket.size());
        SIA_HIP(hipMemcpyAsync(sl.src_sorted.ptr, st.sorted.data(), 4 * ns, hipMemcpyHostToDevice, s_sample));
        SIA_HIP(hipMemcpyAsync(sl.src_t.ptr, st.t.data(), 4 * st.t.size(), hipMemcpyHostToDevice, s_sample));
        SIA_HIP(hipMemcpyAsync(sl.bucket.ptr, st.bucket.data(), 4 * st.bucket.size(), hipMemcpyHostToDevice,
                               s_sample));
        tag_sources(g, sl.src_sorted.as<int32_t>(), static_cast<uint32_t>(ns), sl.tag_mask, true, s_sample);
        // the host tables must stay alive until the copies ran
        SIA_HIP(hipStreamSynchronize(s_sample));
    }

    void untag(uint32_t i) { untag_n(i, static_cast<uint32_t>(slots[i].t->st.sorted.size())); }

    // clear slot i's tag bit on its n_src uploaded sources (needs no ticket)
    void untag_n(uint32_t i, uint32_t n_src)
    {
        Slot &sl = slots[i];
        tag_sources(g, sl.src_sorted.as<int32_t>(), n_src, sl.tag_mask, false, s_sample);
    }

    SlotDev slot_dev(uint32_t i) const
    {
        const Slot &sl = slots[i];
        const Ticket &t = *sl.t;
        SlotDev S{};
        S.seed = t.seed;
        S.attempt_base = t.offset;
        S.n_ns = t.st.n_ns;
        S.src_t = sl.src_t.as<uint32_t>();
        S.bucket = sl.bucket.as<uint32_t>();
        S.n_src = static_cast<uint32_t>(t.st.sorted.size());
        S.bucket_shift = t.st.shift;
        S.tag_mask = sl.tag_mask;
        S.mode = static_cast<uint32_t>(t.mode);
        S.walk_attempt = sl.walk_attempt.as<uint64_t>();
        S.walk_off = sl.walk_off.as<uint64_t>();
        S.walk_len = sl.walk_len.as<uint32_t>();
        S.ids = sl.ids.as<uint32_t>();
        S.walk_cap = sl.walk_cap;
        S.id_cap = sl.id_cap;
        S.counters = d_ctr.as<uint64_t>() + static_cast<size_t>(i) * ST_COUNT;
        S.cycle_steps = t.cycle_steps ? 1u : 0u;
        return S;
    }

    void enqueue_wave(const SamplerConfig &sc)
    {
        const size_t cb = sizeof(uint64_t) * ST_COUNT * n_slots;
        SIA_HIP(hipMemcpyAsync(d_table.ptr, h_table, sizeof(WaveTable), hipMemcpyHostToDevice, s_sample));
        SIA_HIP(hipMemcpyAsync(d_slots.ptr, h_slots, sizeof(SlotDev) * n_slots, hipMemcpyHostToDevice, s_sample));
        SIA_HIP(hipMemcpyAsync(d_ctr.ptr, h_ctr_in, cb, hipMemcpyHostToDevice, s_sample));
        launch_wave(g, d_slots.as<SlotDev>(), n_slots, d_table.as<WaveTable>(), sc, d_ring.as<uint32_t>(),
                    s_sample);
        SIA_HIP(hipMemcpyAsync(h_ctr_out, d_ctr.ptr, cb, hipMemcpyDeviceToHost, s_sample));
    }

    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }

    // One sampling launch from the staged inputs; waits for it.  Returns true
    // if it was a graph replay.
    bool run_wave()
    {
        const SamplerConfig sc = sampler_config();
        bool replay = false;
        if (cfg.use_graph) {
            if (!exec || exec_cfg.blocks_per_cu != sc.blocks_per_cu || exec_cfg.chunk != sc.chunk) {
                drop_graph();
                SIA_HIP(hipStreamBeginCapture(s_sample, hipStreamCaptureModeRelaxed));
                try {
                    enqueue_wave(sc);
                } catch (...) {
                    hipGraph_t tmp = nullptr;
                    (void)hipStreamEndCapture(s_sample, &tmp);
                    if (tmp) (void)hipGraphDestroy(tmp);
                    throw;
                }
                SIA_HIP(hipStreamEndCapture(s_sample, &graph));
                SIA_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
                exec_cfg = sc;
            }
            SIA_HIP(hipGraphLaunch(exec, s_sample));
            replay = true;
        } else {
            enqueue_wave(sc);
        }
        SIA_HIP(hipStreamSynchronize(s_sample));
        return replay;
    }

    // finish a ticket (under mu); frees its slot
    void finish_locked(const TicketP &t, sia_status st, const std::string &msg)
    {
        t->state = TState::Done;
        t->status = st;
        t->error = msg;
        t->info.t_done = now();
        if (st == SIA_OK) ++ctr.completed;
        else if (st == SIA_ECANCELLED) ++ctr.cancelled;
        else ++ctr.failed;
        if (t->slot >= 0) {
            slots[t->slot].t.reset();
            ++mem_epoch;
        }
        cv_done.notify_all();
        cv_sampler.notify_all();
    }

    bool free_slot_locked() const
    {
        for (uint32_t i = 0; i < n_slots; ++i)
            if (!slots[i].t) return true;
        return false;
    }

    bool sampling_locked() const
    {
        for (uint32_t i = 0; i < n_slots; ++i)
            if (slots[i].t && slots[i].t->state == TState::Sampling) return true;
        return false;
    }

    // ------------------------------------------------------------ sampler thread
    void sampler_loop()
    {
        (void)hipSetDevice(g->device);
        uint64_t seen_epoch = ~uint64_t(0);
        bool stalled = false;
        for (;;) {
            std::vector<uint32_t> admitted, dropped, active;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_sampler.wait(lk, [&] {
                    if (stop) return true;
                    if (tuning) return false;
                    if (!concurrent() && !ready.empty()) return true;
                    if (stalled && mem_epoch == seen_epoch) return false;
                    return sampling_locked() || (!pending.empty() && free_slot_locked());
                });
                if (stop) return;
                stalled = false;
                seen_epoch = mem_epoch;
                for (uint32_t i = 0; i < n_slots; ++i) {
                    const TicketP &t = slots[i].t;
                    if (t && t->state == TState::Sampling && t->cancel) dropped.push_back(i);
                }
                while (!pending.empty()) {
                    int fs = -1;
                    for (uint32_t i = 0; i < n_slots && fs < 0; ++i)
                        if (!slots[i].t) fs = static_cast<int>(i);
                    if (fs < 0) break;
                    TicketP t = pending.front();
                    pending.pop_front();
                    slots[fs].t = t;
                    t->slot = fs;
                    t->state = TState::Sampling;
                    t->admit_seq = ++admit_seq;
                    t->info.t_admit = now();
                    admitted.push_back(static_cast<uint32_t>(fs));
                }
                for (uint32_t i = 0; i < n_slots; ++i) {
                    const TicketP &t = slots[i].t;
                    if (t && t->state == TState::Sampling && !t->cancel) active.push_back(i);
                }
                std::sort(active.begin(), active.end(), [&](uint32_t a, uint32_t b) {
                    return slots[a].t->admit_seq < slots[b].t->admit_seq;
                });
            }
            std::vector<uint32_t> in_wave;
            std::vector<uint64_t> chunk(n_slots, 0);
            try {
                for (uint32_t i : dropped) untag(i);
                for (uint32_t i : admitted) upload_sources(i);
                if (!dropped.empty()) {
                    SIA_HIP(hipStreamSynchronize(s_sample));
                    std::lock_guard<std::mutex> lk(mu);
                    for (uint32_t i : dropped) finish_locked(slots[i].t, SIA_ECANCELLED, "cancelled");
                }
                plan(active, in_wave, chunk);
                if (in_wave.empty()) {
                    // time-sliced: finished queries hold memory and slots; their
                    // greedy (on this thread) is what frees them
                    if (!concurrent() && run_greedy_if(true)) continue;
                    if (!active.empty()) resolve_stall(active, stalled);
                    continue;
                }
                std::vector<WaveItem> items;
                std::memset(h_ctr_in, 0, sizeof(uint64_t) * ST_COUNT * n_slots);
                for (uint32_t i : in_wave) {
                    const Ticket &t = *slots[i].t;
                    items.push_back(WaveItem{i, t.done, chunk[i]});
                    h_slots[i] = slot_dev(i);
                    h_ctr_in[i * ST_COUNT + ST_WALKS] = t.wm_walks;
                    h_ctr_in[i * ST_COUNT + ST_IDS] = t.wm_ids;
                }
                fill_wave_table(*h_table, items.data(), static_cast<uint32_t>(items.size()), n_slots);
                const auto w0 = Clock::now();
                const bool replay = run_wave();
                const double dt = std::chrono::duration<double>(Clock::now() - w0).count();
                {
                    std::lock_guard<std::mutex> lk(mu);
                    ctr.sample_busy_s += dt;
                }
                spins = 0;
                commit(in_wave, chunk, replay);
                if (!concurrent()) run_greedy_if(false);
            } catch (const Error &e) {
                fail_sampling(e.status, e.msg);
            } catch (const std::exception &e) {
                fail_sampling(SIA_EDEVICE, e.what());
            }
        }
    }

    bool concurrent() const { return cfg.greedy_mode != 0; }

    // Time-sliced mode: run the greedy of the finished queries between
    // sampling launches once enough of them wait (greedy_batch), or when
    // sampling cannot proceed without it: nothing left to sample, the oldest
    // has waited long, or (force) the launch planner found no share to run.
    // Queued queries may wait for the slots finished queries hold: sampling
    // throughput hardly depends on how many queries share a launch, while
    // the greedy's launch time is that of its slowest query.
    bool run_greedy_if(bool force)
    {
        std::vector<TicketP> batch;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (ready.empty()) return false;
            const bool due = force || ready.size() >= cfg.greedy_batch || !sampling_locked() ||
                             now() - ready.front()->info.t_sampled > kGreedyMaxWait;
            if (!due) return false;
            batch = take_ready_locked();
        }
        if (!batch.empty()) run_greedy_batch(batch);
        return true;
    }

    // Choose each active query's share and make its buffer room for it.
    // Oldest first; once an older query cannot get memory, younger ones may
    // only run shares that fit the room they already hold, so memory that
    // frees up goes to the oldest.
    void plan(const std::vector<uint32_t> &active, std::vector<uint32_t> &in_wave, std::vector<uint64_t> &chunk)
    {
        if (active.empty()) return;
        const uint64_t share = std::max<uint64_t>(cfg.min_share, cfg.wave_attempts / active.size());
        bool blocked = false;
        for (uint32_t i : active) {
            Ticket &t = *slots[i].t;
            const uint64_t left = t.n_attempts - t.done;
            auto room = [&](uint64_t c) {
                uint64_t w, d;
                share_needs(t, c, w, d);
                if (blocked) return slots[i].walk_cap >= w && slots[i].id_cap >= d;
                return reserve(i, w, d);
            };
            uint64_t c = t.retry_chunk ? t.retry_chunk : std::min(left, share);
            bool ok = room(c);
            if (!ok && !t.retry_chunk) {  // the largest share that still fits
                for (c = c / 2; c >= std::min<uint64_t>(left, 4096) && c > 0; c /= 2)
                    if ((ok = room(c))) break;
            }
            if (!ok && !t.retry_chunk && !blocked) {
                // estimates carry headroom: try the smallest share with all the
                // room there is; an overflow then reports the exact need
                c = std::min<uint64_t>(left, 4096);
                ok = reserve_all(i, c);
            }
            if (ok && c > 0) {
                chunk[i] = c;
                in_wave.push_back(i);
            } else {
                blocked = true;
            }
        }
    }

    // Every active query is stalled for walk memory.  If a greedy is pending
    // or running it will free a slot: wait.  Otherwise restart younger
    // queries (youngest first) until the oldest one's next share fits, or
    // fail the oldest if it cannot fit even alone.
    void resolve_stall(const std::vector<uint32_t> &active, bool &stalled)
    {
        std::unique_lock<std::mutex> lk(mu);
        if (greedy_running || !ready.empty()) {
            stalled = true;
            return;
        }
        lk.unlock();
        const uint32_t oldest = active.front();
        Slot &so = slots[oldest];
        const Ticket &t = *so.t;
        // the least room the oldest query's next share can run in: its exact
        // need after an overflow, else one more walk and one more id
        const uint64_t want = t.retry_chunk ? walk_bytes_of(t.wm_walks + t.need_walks, t.wm_ids + t.need_ids)
                                            : walk_bytes_of(t.wm_walks + 1, t.wm_ids + 1);
        auto fits = [&] { return walk_bytes.load() - slot_bytes(so) + want <= budget; };
        if (want <= budget) {
            release_idle();
            uint64_t evicted = 0;
            for (size_t j = active.size(); j-- > 1 && !fits();) {
                const uint32_t v = active[j];
                if (!slots[v].walk_cap) continue;
                Ticket &vt = *slots[v].t;
                vt.done = vt.wm_walks = vt.wm_ids = 0;
                vt.retry_chunk = vt.need_walks = vt.need_ids = 0;
                vt.hits = vt.dead = vt.cycles = vt.steps = vt.evals = 0;
                release_walks(v);
                ++evicted;
            }
            // (room freed by idle slots alone is progress too; a stall that
            // neither evicts nor frees anything repeatedly would be a
            // scheduler fault, reported instead of spinning)
            spins = evicted ? 0 : spins + 1;
            if (fits() && spins < 64) {
                lk.lock();
                ctr.evictions += evicted;
                return;
            }
        }
        // the query cannot fit the budget even alone
        untag(oldest);
        SIA_HIP(hipStreamSynchronize(s_sample));
        release_walks(oldest);
        lk.lock();
        finish_locked(slots[oldest].t, SIA_ENOMEM, "walk buffer budget too small for this query");
    }

    void commit(const std::vector<uint32_t> &in_wave, const std::vector<uint64_t> &chunk, bool replay)
    {
        std::vector<std::pair<uint32_t, uint32_t>> finished;  // slot, sources
        {
            std::lock_guard<std::mutex> lk(mu);
            ++ctr.waves;
            if (replay) ++ctr.graph_replays;
            for (uint32_t i : in_wave) {
                const TicketP &tp = slots[i].t;
                Ticket &t = *tp;
                const uint64_t *c = h_ctr_out + static_cast<size_t>(i) * ST_COUNT;
                ++t.info.waves;
                if (c[ST_FAULTS]) {
                    untag(i);
                    finish_locked(tp, SIA_EDEVICE, "sampler consistency check failed");
                    continue;
                }
                if (c[ST_OVERFLOW]) {
                    t.retry_chunk = chunk[i];
                    t.need_walks = c[ST_WALKS] - t.wm_walks;
                    t.need_ids = c[ST_IDS] - t.wm_ids;
                    ++t.info.reruns;
                    ++ctr.reruns;
                    continue;
                }
                est_att[t.mode] += chunk[i];
                est_walks[t.mode] += c[ST_WALKS] - t.wm_walks;
                est_ids[t.mode] += c[ST_IDS] - t.wm_ids;
                t.wm_walks = c[ST_WALKS];
                t.wm_ids = c[ST_IDS];
                t.done += chunk[i];
                t.retry_chunk = t.need_walks = t.need_ids = 0;
                t.hits += c[ST_HITS];
                t.dead += c[ST_DEAD];
                t.cycles += c[ST_CYCLE];
                t.steps += c[ST_STEPS];
                t.evals += c[ST_EVALS];
                if (t.done == t.n_attempts) {
                    t.state = TState::Ready;
                    t.info.t_sampled = now();
                    ready.push_back(tp);
                    finished.emplace_back(i, static_cast<uint32_t>(t.st.sorted.size()));
                }
            }
            if (!finished.empty()) cv_greedy.notify_all();
        }
        // the greedy may already own (or have released) these slots; the bits
        // are cleared on this stream before any later admission reuses them
        for (const auto &f : finished) untag_n(f.first, f.second);
    }

    void fail_sampling(sia_status st, const std::string &msg)
    {
        std::lock_guard<std::mutex> lk(mu);
        for (uint32_t i = 0; i < n_slots; ++i) {
            const TicketP t = slots[i].t;
            if (t && t->state == TState::Sampling) {
                try {
                    untag(i);
                } catch (...) {
                }
                finish_locked(t, st, msg);
            }
        }
        if (st == SIA_EDEVICE) {
            fatal = st;
            fatal_msg = msg;
            while (!pending.empty()) {
                finish_locked(pending.front(), st, msg);
                pending.pop_front();
            }
        }
    }

    // ------------------------------------------------------------ greedy thread
    // Concurrent mode: the greedy thread runs every finished query's greedy
    // on its own stream as soon as it is ready.
    void greedy_loop()
    {
        (void)hipSetDevice(g->device);
        for (;;) {
            std::vector<TicketP> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_greedy.wait(lk, [&] { return stop || (concurrent() && !ready.empty()); });
                if (stop) return;
                batch = take_ready_locked();
            }
            if (!batch.empty()) run_greedy_batch(batch);
        }
    }

    // Move the ready queries into the greedy (cancelled ones finish here).
    std::vector<TicketP> take_ready_locked()
    {
        std::vector<TicketP> batch;
        while (!ready.empty()) {
            TicketP t = ready.front();
            ready.pop_front();
            if (t->cancel) {
                finish_locked(t, SIA_ECANCELLED, "cancelled");
                continue;
            }
            t->state = TState::Greedy;
            batch.push_back(t);
        }
        greedy_running = batch.size();
        return batch;
    }

    // Index + greedy of a batch of queries in shared launches; finishes them.
    void run_greedy_batch(const std::vector<TicketP> &batch)
    {
        sia_status st = SIA_OK;
        std::string msg;
        try {
            std::vector<GreedyInput> in(batch.size());
            for (size_t q = 0; q < batch.size(); ++q) {
                Ticket &t = *batch[q];
                Slot &sl = slots[t.slot];
                const uint64_t S = t.mode == SIA_EDGES ? static_cast<uint64_t>(g->m) : static_cast<uint64_t>(g->n);
                sl.cnt.ensure(4 * S);
                sl.greedy.ensure(greedy_scratch_bytes(S, t.wm_walks, t.wm_ids, t.k));
                t.selected.assign(static_cast<size_t>(t.k), 0);
                t.gains.assign(static_cast<size_t>(t.k), 0);
                GreedyInput &gi = in[q];
                gi.walk_off = sl.walk_off.as<uint64_t>();
                gi.walk_len = sl.walk_len.as<uint32_t>();
                gi.ids = sl.ids.as<uint32_t>();
                gi.id_space = S;
                gi.n_walks = t.wm_walks;
                gi.n_ids = t.wm_ids;
                gi.k = t.k;
                gi.cnt = sl.cnt.as<uint32_t>();
                gi.scratch = sl.greedy.ptr;
                gi.selected = t.selected.data();
                gi.gains = t.gains.data();
            }
            GreedyResult res;
            const auto g0 = Clock::now();
            run_greedy_jobs(in, d_jobs.ptr, s_greedy, true, &res, cfg.hist_blocks);
            const double dt = std::chrono::duration<double>(Clock::now() - g0).count();
            std::lock_guard<std::mutex> lk(mu);
            ctr.greedy_busy_s += dt;
            ctr.greedy_index_s += res.ms_count * 1e-3;
        } catch (const Error &e) {
            st = e.status;
            msg = e.msg;
        } catch (const std::exception &e) {
            st = SIA_EDEVICE;
            msg = e.what();
        }
        std::lock_guard<std::mutex> lk(mu);
        ++ctr.greedy_launches;
        ctr.greedy_jobs += batch.size();
        greedy_running = 0;
        for (const TicketP &tp : batch) {
            Ticket &t = *tp;
            if (st == SIA_OK) {
                sia_stats S{};
                S.hits = t.hits;
                S.dead_ends = t.dead;
                S.cycles = t.cycles;
                S.steps = t.steps;
                S.evaluations = t.evals;
                S.walk_ids = t.wm_ids;
                finish_stats(S, t.st, t.mode, t.n_attempts, t.selected.data(), t.gains.data(), t.k);
                t.stats = S;
            }
            finish_locked(tp, st != SIA_OK ? st : (t.cancel ? SIA_ECANCELLED : SIA_OK),
                          st != SIA_OK ? msg : (t.cancel ? "cancelled" : ""));
        }
        if (st == SIA_EDEVICE) {
            fatal = st;
            fatal_msg = msg;
        }
    }

    // ------------------------------------------------------------ tuning
    sia_batch_config tune(const sia_query &q, double target_ms)
    {
        std::unique_lock<std::mutex> lk(mu);
        for (const auto &kv : tickets)
            SIA_REQUIRE(kv.second->state == TState::Done, SIA_EBUSY, "batch is not idle");
        SIA_REQUIRE(!tuning, SIA_EBUSY, "already tuning");
        for (uint32_t i = 0; i < n_slots; ++i) SIA_REQUIRE(!slots[i].t, SIA_EBUSY, "batch is not idle");
        tuning = true;
        lk.unlock();
        struct Reset {
            sia_batch *b;
            ~Reset()
            {
                std::lock_guard<std::mutex> l(b->mu);
                b->tuning = false;
                b->slots[0].t.reset();
                b->cv_sampler.notify_all();
            }
        } reset{this};

        auto t = std::make_shared<Ticket>();
        t->mode = q.mode;
        t->k = 0;
        t->n_attempts = q.n_attempts;
        t->offset = q.attempt_offset;
        t->seed = q.seed;
        t->cycle_steps = (q.flags & SIA_FLAG_NO_CYCLE_STEPS) == 0;  // measured as it will run
        t->st = build_source_tables(g->n, q.sources, q.n_sources);
        {
            std::lock_guard<std::mutex> l(mu);
            slots[0].t = t;
        }
        upload_sources(0);
        const int max_b = sampler_max_blocks_per_cu(g);
        std::vector<SamplerConfig> cands;
        for (int b = max_b; b >= std::max(1, max_b - 2); --b)
            for (uint32_t c : {64u, 128u, 256u, 512u}) cands.push_back(SamplerConfig{b, c});
        hipEvent_t e0 = nullptr, e1 = nullptr;
        SIA_HIP(hipEventCreate(&e0));
        SIA_HIP(hipEventCreate(&e1));
        float best_ms = 0.f;
        SamplerConfig best = cands.front();
        try {
            for (size_t ci = 0; ci < cands.size(); ++ci) {
                for (int rep = 0; rep < 3; ++rep) {
                    std::memset(h_ctr_in, 0, sizeof(uint64_t) * ST_COUNT * n_slots);
                    uint64_t w, d;
                    share_needs(*t, q.n_attempts, w, d);
                    SIA_REQUIRE(reserve(0, w, d), SIA_ENOMEM, "probe walks exceed the walk budget");
                    h_slots[0] = slot_dev(0);
                    const WaveItem item{0u, 0u, q.n_attempts};
                    fill_wave_table(*h_table, &item, 1, n_slots);
                    SIA_HIP(hipEventRecord(e0, s_sample));
                    enqueue_wave(cands[ci]);
                    SIA_HIP(hipEventRecord(e1, s_sample));
                    SIA_HIP(hipStreamSynchronize(s_sample));
                    const uint64_t *c = h_ctr_out;
                    SIA_REQUIRE(!c[ST_FAULTS], SIA_EDEVICE, "sampler consistency check failed");
                    if (c[ST_OVERFLOW]) {  // size exactly, then measure
                        t->retry_chunk = q.n_attempts;
                        t->need_walks = c[ST_WALKS];
                        t->need_ids = c[ST_IDS];
                        --rep;
                        continue;
                    }
                    if (rep == 0) continue;  // warm-up
                    float ms = 0.f;
                    SIA_HIP(hipEventElapsedTime(&ms, e0, e1));
                    // fewer workgroups per CU must win by 3%: on one probe query the
                    // shapes are close and run-to-run noise decided, while a mix of
                    // queries ran faster on the most workgroups (5 against 4: 3%)
                    const float need = cands[ci].blocks_per_cu < best.blocks_per_cu ? 0.97f : 1.0f;
                    if (best_ms == 0.f || ms < best_ms * need) {
                        best_ms = ms;
                        best = cands[ci];
                    }
                }
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            untag(0);
            (void)hipStreamSynchronize(s_sample);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        untag(0);
        SIA_HIP(hipStreamSynchronize(s_sample));

        // histogram tiling of the greedy, on the probe's walks (still in slot 0)
        const uint64_t n_walks = h_ctr_out[ST_WALKS], n_ids = h_ctr_out[ST_IDS];
        const uint64_t S = q.mode == SIA_EDGES ? static_cast<uint64_t>(g->m) : static_cast<uint64_t>(g->n);
        const int64_t kq = std::min<int64_t>(q.k > 0 ? q.k : 1000, static_cast<int64_t>(S));
        Slot &sl = slots[0];
        sl.cnt.ensure(4 * S);
        sl.greedy.ensure(greedy_scratch_bytes(S, n_walks, n_ids, kq));
        std::vector<int64_t> gsel(static_cast<size_t>(kq));
        std::vector<uint64_t> ggain(static_cast<size_t>(kq));
        const unsigned cus = static_cast<unsigned>(device_cu_count());
        unsigned best_h = 0;
        float best_gms = 0.f;
        for (unsigned hb : {cus / 8, cus / 4, cus / 2, cus}) {
            if (!hb) continue;
            for (int rep = 0; rep < 2; ++rep) {
                std::vector<GreedyInput> in(1);
                GreedyInput &gi = in[0];
                gi.walk_off = sl.walk_off.as<uint64_t>();
                gi.walk_len = sl.walk_len.as<uint32_t>();
                gi.ids = sl.ids.as<uint32_t>();
                gi.id_space = S;
                gi.n_walks = n_walks;
                gi.n_ids = n_ids;
                gi.k = kq;
                gi.cnt = sl.cnt.as<uint32_t>();
                gi.scratch = sl.greedy.ptr;
                gi.selected = gsel.data();
                gi.gains = ggain.data();
                GreedyResult res;
                run_greedy_jobs(in, d_jobs.ptr, s_greedy, true, &res, hb);
                const float ms = res.ms_count + res.ms_greedy;
                if (rep == 1 && (best_gms == 0.f || ms < best_gms)) {
                    best_gms = ms;
                    best_h = hb;
                }
            }
        }
        std::lock_guard<std::mutex> l(mu);
        cfg.sampler_blocks_per_cu = best.blocks_per_cu;
        cfg.refill_chunk = best.chunk;
        cfg.hist_blocks = best_h;
        if (target_ms > 0 && best_ms > 0) {
            const double rate = q.n_attempts / (best_ms * 1e-3);
            const double w = rate * target_ms * 1e-3;
            cfg.wave_attempts = static_cast<uint64_t>(std::min(std::max(w, 1048576.0), 1073741824.0));
        }
        return cfg;
    }
};

namespace {

sia_batch_config defaults(const sia_batch_config *c)
{
    sia_batch_config d{};
    if (c) d = *c;
    if (d.sampler_blocks_per_cu < 0) d.sampler_blocks_per_cu = 0;
    if (!d.refill_chunk) d.refill_chunk = 256;
    if (!d.wave_attempts) d.wave_attempts = uint64_t(1) << 23;
    if (!d.min_share) d.min_share = uint64_t(1) << 16;
    if (!d.greedy_batch) d.greedy_batch = 32;
    return d;
}

void destroy_batch(sia_batch *b)
{
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->stop = true;
    }
    b->cv_sampler.notify_all();
    b->cv_greedy.notify_all();
    b->cv_done.notify_all();
    if (b->th_sample.joinable()) b->th_sample.join();
    if (b->th_greedy.joinable()) b->th_greedy.join();
    // untag sources of queries still holding a slot
    for (uint32_t i = 0; i < b->n_slots; ++i) {
        if (b->slots[i].t && b->slots[i].t->state == TState::Sampling && b->slots[i].src_sorted.ptr) {
            try {
                b->untag(i);
            } catch (...) {
            }
        }
    }
    if (b->s_sample) (void)hipStreamSynchronize(b->s_sample);
    if (b->s_greedy) (void)hipStreamSynchronize(b->s_greedy);
    b->drop_graph();
    if (b->s_sample) (void)hipStreamDestroy(b->s_sample);
    if (b->s_greedy) (void)hipStreamDestroy(b->s_greedy);
    if (b->h_table) (void)hipHostFree(b->h_table);
    if (b->h_slots) (void)hipHostFree(b->h_slots);
    if (b->h_ctr_in) (void)hipHostFree(b->h_ctr_in);
    if (b->h_ctr_out) (void)hipHostFree(b->h_ctr_out);
    if (b->g) {
        std::lock_guard<std::mutex> lk(b->g->tag_mu);
        b->g->tag_bits &= ~b->tag_bits;
    }
    delete b;
}

// Copy a finished ticket's results out (under b->mu) and release it.
sia_status take_result(sia_batch *b, std::map<uint64_t, TicketP>::iterator it, int64_t *selected,
                       uint64_t *gains, sia_stats *stats, sia_ticket_info *info)
{
    const Ticket &t = *it->second;
    const sia_status st = t.status;
    if (st == SIA_OK) {
        if (selected) std::copy(t.selected.begin(), t.selected.end(), selected);
        if (gains) std::copy(t.gains.begin(), t.gains.end(), gains);
        if (stats) *stats = t.stats;
    } else {
        set_error(t.error);
    }
    if (info) *info = t.info;
    b->tickets.erase(it);
    return st;
}

}  // namespace

extern "C" {

sia_status sia_batch_create(const sia_graph *cg, uint64_t walk_budget_bytes, int32_t max_slots,
                            const sia_batch_config *config, sia_batch **out)
{
    return guarded([&] {
        SIA_REQUIRE(out != nullptr && cg != nullptr, SIA_EINVAL, "NULL argument");
        *out = nullptr;
        SIA_REQUIRE(max_slots >= 1 && max_slots <= static_cast<int32_t>(kMaxSlots), SIA_EINVAL,
                    "max_slots must be in [1, 31]");
        SIA_REQUIRE(walk_budget_bytes >= (uint64_t(1) << 20), SIA_EINVAL, "walk budget below 1 MiB");
        sia_graph *g = const_cast<sia_graph *>(cg);
        DeviceScope ds(g->device);
        std::unique_ptr<sia_batch> b(new sia_batch);
        b->cfg = defaults(config);
        SIA_REQUIRE(b->cfg.refill_chunk <= (1u << 20), SIA_EINVAL, "refill_chunk above 2^20");
        b->budget = walk_budget_bytes;
        b->n_slots = static_cast<uint32_t>(max_slots);
        b->slots = std::vector<Slot>(b->n_slots);
        {
            std::lock_guard<std::mutex> lk(g->tag_mu);
            uint32_t got = 0;
            std::vector<uint32_t> bits;
            for (uint32_t bit = 0; bit < kMaxSlots && bits.size() < b->n_slots; ++bit)
                if (!(g->tag_bits & (1u << bit))) bits.push_back(bit);
            SIA_REQUIRE(bits.size() == b->n_slots, SIA_EBUSY, "not enough free source-tag bits on this graph");
            for (uint32_t i = 0; i < b->n_slots; ++i) {
                b->slots[i].tag_mask = 1u << bits[i];
                got |= 1u << bits[i];
            }
            g->tag_bits |= got;
            b->tag_bits = got;
            b->g = g;
        }
        sia_batch *raw = b.get();
        struct Undo {
            std::unique_ptr<sia_batch> &b;
            ~Undo()
            {
                if (b) destroy_batch(b.release());
            }
        } undo{b};
        const int cus = device_cu_count();
        SIA_REQUIRE(raw->cfg.greedy_cus >= 0 && raw->cfg.greedy_cus < cus, SIA_EINVAL,
                    "greedy_cus must be in [0, number of CUs)");
        SIA_REQUIRE(raw->cfg.greedy_mode == 0 || raw->cfg.greedy_mode == 1, SIA_EINVAL,
                    "greedy_mode must be 0 or 1");
        SIA_REQUIRE(raw->cfg.greedy_cus == 0 || raw->cfg.greedy_mode == 1, SIA_EINVAL,
                    "greedy_cus needs greedy_mode 1");
        if (raw->cfg.greedy_cus > 0) {
            // disjoint CU sets: the sampler keeps the first CUs, the greedy the last
            const uint32_t words = static_cast<uint32_t>((cus + 31) / 32);
            std::vector<uint32_t> ms(words, 0), mg(words, 0);
            const int split = cus - raw->cfg.greedy_cus;
            for (int c = 0; c < cus; ++c) (c < split ? ms : mg)[c / 32] |= 1u << (c % 32);
            SIA_HIP(hipExtStreamCreateWithCUMask(&raw->s_sample, words, ms.data()));
            SIA_HIP(hipExtStreamCreateWithCUMask(&raw->s_greedy, words, mg.data()));
            raw->sampler_cus = split;
        } else {
            SIA_HIP(hipStreamCreateWithFlags(&raw->s_sample, hipStreamNonBlocking));
            SIA_HIP(hipStreamCreateWithFlags(&raw->s_greedy, hipStreamNonBlocking));
        }
        SIA_HIP(hipHostMalloc(reinterpret_cast<void **>(&raw->h_table), sizeof(WaveTable), hipHostMallocDefault));
        SIA_HIP(hipHostMalloc(reinterpret_cast<void **>(&raw->h_slots), sizeof(SlotDev) * raw->n_slots,
                              hipHostMallocDefault));
        const size_t cb = sizeof(uint64_t) * ST_COUNT * raw->n_slots;
        SIA_HIP(hipHostMalloc(reinterpret_cast<void **>(&raw->h_ctr_in), cb, hipHostMallocDefault));
        SIA_HIP(hipHostMalloc(reinterpret_cast<void **>(&raw->h_ctr_out), cb, hipHostMallocDefault));
        std::memset(raw->h_slots, 0, sizeof(SlotDev) * raw->n_slots);
        std::memset(raw->h_ctr_in, 0, cb);
        raw->d_table.ensure(sizeof(WaveTable));
        raw->d_slots.ensure(sizeof(SlotDev) * raw->n_slots);
        raw->d_ctr.ensure(cb);
        raw->d_jobs.ensure(greedy_job_table_bytes(raw->n_slots));
        raw->d_ring.ensure(sampler_ring_bytes(g));
        (void)sampler_max_blocks_per_cu(g);  // occupancy query before any capture
        raw->ctr.walk_budget = walk_budget_bytes;
        raw->ctr.slots = raw->n_slots;
        raw->t0 = Clock::now();
        raw->th_sample = std::thread([raw] { raw->sampler_loop(); });
        raw->th_greedy = std::thread([raw] { raw->greedy_loop(); });
        *out = b.release();
    });
}

sia_status sia_batch_destroy(sia_batch *b)
{
    return guarded([&] {
        if (!b) return;
        DeviceScope ds(b->g->device);
        destroy_batch(b);
    });
}

sia_status sia_batch_submit(sia_batch *b, const sia_query *q, uint64_t *ticket)
{
    return guarded([&] {
        SIA_REQUIRE(b != nullptr && q != nullptr && ticket != nullptr, SIA_EINVAL, "NULL argument");
        check_query(b->g->n, b->g->m, q->mode, q->sources, q->n_sources, q->k, q->n_attempts,
                    q->attempt_offset);
        SIA_REQUIRE(q->k >= 1, SIA_EINVAL, "k must be >= 1");
        SIA_REQUIRE((q->flags & ~SIA_FLAG_NO_CYCLE_STEPS) == 0, SIA_EINVAL, "unknown flag bits");
        auto t = std::make_shared<Ticket>();
        t->cycle_steps = (q->flags & SIA_FLAG_NO_CYCLE_STEPS) == 0;
        t->mode = q->mode;
        t->k = q->k;
        t->n_attempts = q->n_attempts;
        t->offset = q->attempt_offset;
        t->seed = q->seed;
        t->st = build_source_tables(b->g->n, q->sources, q->n_sources);
        std::lock_guard<std::mutex> lk(b->mu);
        SIA_REQUIRE(b->fatal == SIA_OK, b->fatal, "batch stopped after an error: " + b->fatal_msg);
        t->id = b->next_id++;
        t->info.t_submit = b->now();
        b->tickets[t->id] = t;
        b->pending.push_back(t);
        ++b->ctr.submitted;
        *ticket = t->id;
        b->cv_sampler.notify_all();
    });
}

sia_status sia_batch_poll(sia_batch *b, uint64_t ticket, int64_t *selected, uint64_t *gains,
                          sia_stats *stats, sia_ticket_info *info)
{
    sia_status result = SIA_OK;
    const sia_status st = guarded([&] {
        SIA_REQUIRE(b != nullptr, SIA_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(b->mu);
        auto it = b->tickets.find(ticket);
        SIA_REQUIRE(it != b->tickets.end(), SIA_EINVAL, "unknown ticket");
        if (it->second->state != TState::Done) {
            result = SIA_ENOTREADY;
            return;
        }
        result = take_result(b, it, selected, gains, stats, info);
    });
    return st != SIA_OK ? st : result;
}

sia_status sia_batch_wait(sia_batch *b, uint64_t ticket, int64_t timeout_ms, int64_t *selected,
                          uint64_t *gains, sia_stats *stats, sia_ticket_info *info)
{
    sia_status result = SIA_OK;
    const sia_status st = guarded([&] {
        SIA_REQUIRE(b != nullptr, SIA_EINVAL, "NULL argument");
        std::unique_lock<std::mutex> lk(b->mu);
        auto it = b->tickets.find(ticket);
        SIA_REQUIRE(it != b->tickets.end(), SIA_EINVAL, "unknown ticket");
        TicketP t = it->second;
        auto done = [&] { return t->state == TState::Done || b->stop; };
        if (timeout_ms < 0) b->cv_done.wait(lk, done);
        else b->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
        if (t->state != TState::Done) {
            result = SIA_ENOTREADY;
            return;
        }
        it = b->tickets.find(ticket);
        SIA_REQUIRE(it != b->tickets.end(), SIA_EINVAL, "ticket released by another caller");
        result = take_result(b, it, selected, gains, stats, info);
    });
    return st != SIA_OK ? st : result;
}

sia_status sia_batch_cancel(sia_batch *b, uint64_t ticket)
{
    return guarded([&] {
        SIA_REQUIRE(b != nullptr, SIA_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(b->mu);
        auto it = b->tickets.find(ticket);
        SIA_REQUIRE(it != b->tickets.end(), SIA_EINVAL, "unknown ticket");
        const TicketP t = it->second;
        SIA_REQUIRE(t->state != TState::Done, SIA_EINVAL, "ticket already finished");
        t->cancel = true;
        ++b->mem_epoch;  // wakes a sampler that waits for memory
        if (t->state == TState::Pending) {
            b->pending.erase(std::find(b->pending.begin(), b->pending.end(), t));
            b->finish_locked(t, SIA_ECANCELLED, "cancelled");
        }
        b->cv_sampler.notify_all();
    });
}

sia_status sia_batch_stats_get(sia_batch *b, sia_batch_stats *out)
{
    return guarded([&] {
        SIA_REQUIRE(b != nullptr && out != nullptr, SIA_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(b->mu);
        sia_batch_stats s = b->ctr;
        s.walk_bytes = b->walk_bytes.load();
        s.walk_bytes_peak = std::max(s.walk_bytes_peak, s.walk_bytes);
        s.busy_slots = 0;
        for (uint32_t i = 0; i < b->n_slots; ++i)
            if (b->slots[i].t) ++s.busy_slots;
        s.pending = static_cast<uint32_t>(b->pending.size());
        s.config = b->cfg;
        *out = s;
    });
}

sia_status sia_batch_tune(sia_batch *b, const sia_query *probe, double target_ms,
                          sia_batch_config *chosen)
{
    return guarded([&] {
        SIA_REQUIRE(b != nullptr && probe != nullptr, SIA_EINVAL, "NULL argument");
        check_query(b->g->n, b->g->m, probe->mode, probe->sources, probe->n_sources, 0,
                    probe->n_attempts, probe->attempt_offset);
        SIA_REQUIRE((probe->flags & ~SIA_FLAG_NO_CYCLE_STEPS) == 0, SIA_EINVAL, "unknown flag bits");
        DeviceScope ds(b->g->device);
        const sia_batch_config c = b->tune(*probe, target_ms);
        if (chosen) *chosen = c;
    });
}

}  // extern "C"
