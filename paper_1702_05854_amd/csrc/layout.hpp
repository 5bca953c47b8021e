// Device-side records shared by the host code and the sampling kernel: the
// graph's node and edge records, a query slot as the sampler sees it, the
// work table of one sampling launch and the per-query counters.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sia {

// Global-address-space view of a pointer.  Pointers that reach a kernel
// inside a record loaded from memory are generic, and the compiler would
// access them with flat instructions, whose completion every LDS wait (and so
// every barrier) must also await; explicit global pointers avoid that.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T *gp(T *p)
{
    return (GLOBAL T *)p;
}

// One 16-byte record per node: where its in-edges start, how many, the last
// cumulative threshold (so the dead-end test needs no extra load), and the
// source tag: bit b is set exactly when the node is a source of the query
// holding slot bit b.  Bit 31 belongs to single-query calls, bits 0..30 to
// batches.  The tag is kept in step with the copies in the node's in-edge
// records (ArcRec.head_tag).
struct NodeRec {
    uint32_t off;
    uint32_t deg;
    uint32_t thr_last;
    uint32_t tag;
};
static_assert(sizeof(NodeRec) == 16, "NodeRec layout");

// One 32-byte record per in-edge j of head x (CSR position j, line-aligned,
// four to a 128-byte line): the interval [thr_lo, thr_hi) of draws that make
// j the live in-edge of x (thr_lo is the cumulative threshold of the previous
// in-edge, 0 for the first), the tail u, a copy of x's source tag, and a copy
// of u's node record (off, deg, thr_last).  A live-edge evaluation of x reads
// one record: it certifies the choice, says whether x is a source, and holds
// all the next evaluation, of u, needs -- one random line per step.
struct ArcRec {
    uint32_t thr_lo;
    uint32_t thr_hi;
    uint32_t row;       // tail u
    uint32_t head_tag;  // = NodeRec.tag of the head x
    uint32_t u_off;     // = NodeRec.off of u
    uint32_t u_deg;     // = NodeRec.deg of u
    uint32_t u_thr;     // = NodeRec.thr_last of u
    uint32_t pad;
};
static_assert(sizeof(ArcRec) == 32, "ArcRec layout");

// Compact 16-byte record for graphs whose every column has the weights
// w = 1/d_in of the node (the paper's setting), checked exactly at ingest:
// all in-edges of a node with in-degree d then carry the same quantised weight
// q(d) = inv_indeg_quantum(d), the live in-edge for draw r is floor(r / q(d))
// and the node's last threshold is min(d * q(d), 2^32 - 1), so a record needs
// no thresholds: the tail u, a copy of the head's source tag and u's offset and
// degree -- one 16-byte load per step.
struct ArcRec16 {
    uint32_t row;       // tail u
    uint32_t head_tag;  // = NodeRec.tag of the head x
    uint32_t u_off;     // = NodeRec.off of u
    uint32_t u_deg;     // = NodeRec.deg of u
};
static_assert(sizeof(ArcRec16) == 16, "ArcRec16 layout");

// Live-edge threshold unit of a weight x in [0,1]: round-half-even(x * 2^32).
// (double)x is exact and so is the scaling by 2^32; rint rounds half to even.
__device__ __forceinline__ uint64_t quantize_weight(float x)
{
    return static_cast<uint64_t>(rint(static_cast<double>(x) * 4294967296.0));
}

// Quantised weight of every in-edge of a node with in-degree d >= 1 under
// w = 1/d in fp32 (correctly rounded division).
__device__ __forceinline__ uint64_t inv_indeg_quantum(uint32_t d)
{
    return quantize_weight(1.0f / static_cast<float>(d));
}

// Walk ring of the sampler: per wave, kRingRows rows of 64 lanes x 4 bytes;
// a lane's walk position t (the chosen in-edge position for edges, the node
// evaluated for nodes) sits in row (it0 + t) mod kRingRows of its column.
constexpr uint32_t kRingRows = 1024;

// Per-query counters written by the sampler.
enum StatSlot {
    ST_WALKS = 0, ST_IDS = 1, ST_HITS = 2, ST_DEAD = 3, ST_CYCLE = 4, ST_STEPS = 5,
    ST_EVALS = 6, ST_OVERFLOW = 7, ST_FAULTS = 8, ST_COUNT = 16
};

constexpr uint32_t kSoloBit = 31;   // source-tag bit of single-query calls
constexpr uint32_t kMaxSlots = 31;  // source-tag bits 0..30 for batches

// Device-side state of one query while it samples (read by the sampler).
struct SlotDev {
    uint64_t seed;
    uint64_t attempt_base;   // attempt id of the query's local attempt 0
    uint64_t n_ns;           // non-sources
    const uint32_t *src_t;   // t_i = s_i - i over the sorted sources
    const uint32_t *bucket;  // pairs: [2b] = #{i : t_i < b << bucket_shift}, [2b+1] = t at that count
    uint32_t n_src;
    uint32_t bucket_shift;
    uint32_t tag_mask;       // source-tag bit of this query
    uint32_t mode;           // SIA_EDGES / SIA_NODES
    uint64_t *walk_attempt;  // kept walks: attempt id, offset, length
    uint64_t *walk_off;
    uint32_t *walk_len;
    uint32_t *ids;
    uint64_t walk_cap;
    uint64_t id_cap;
    uint64_t *counters;      // StatSlot entries
    const uint32_t *coin_thr; // probabilistic suspects: per node, the seed coin's
                              // threshold (read for tagged nodes only); NULL:
                              // the tagged nodes are sources, start over V\X
    uint32_t cycle_steps;     // 1: search each cyclic walk for its cycle entry so
                              // its draws count exactly in the steps counter;
                              // 0: stop it at detection (its outcome is the same)
    uint32_t pad;
};

// The work table a sampling launch reads from device memory: the wave's
// items laid end to end and the chunk counter the persistent lanes draw
// from.  Host code fills it (fill_wave_table) and copies it to the device
// before each launch, so a captured launch can be replayed with new contents.
constexpr uint32_t kMaxItems = 32;
struct WaveTable {
    uint64_t next[8];                // next[0]: wave-global chunk counter (own 64-B line)
    uint64_t prefix[kMaxItems + 1];  // wave-global index of each item's first attempt
    uint64_t local[kMaxItems];       // local attempt index of each item's first attempt
    uint32_t slot[kMaxItems];
    uint32_t n_items;
    uint32_t pad;
};

}  // namespace sia
