// Internal layout shared by the host runtime and the HIP kernels of libgsim.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsim {

constexpr int kMaxPins = 4;
constexpr uint8_t kX = 2;
constexpr int64_t kInf = INT64_MAX;
constexpr int64_t kTimeLimit = int64_t(1) << 62;  // times live in [0, 2^62)

// Device transitions are packed into one 64-bit word: time << 2 | value.
// Times are below 2^62, so the word is unsigned-ordered by time first; no two
// transitions of one waveform share a time. kNoKey sorts after every
// transition.
constexpr uint64_t kNoKey = ~uint64_t(0);
__host__ __device__ constexpr uint64_t pack_key(int64_t t, uint32_t v) {
    return ((uint64_t)t << 2) | (uint64_t)v;
}
__host__ __device__ constexpr int64_t key_time(uint64_t k) { return (int64_t)(k >> 2); }
__host__ __device__ constexpr uint32_t key_value(uint64_t k) { return (uint32_t)(k & 3); }

// Wavefront evaluate kernel: input transitions in flight per round (over all
// pins of the gate), and the delay classes it serves. A tentative output
// transition appears after the round's horizon H and at most the gate's
// largest pin delay after it, and tentative appearance times are distinct
// integers, so a gate whose largest pin delay is at most the class's window
// never holds more tentative transitions than that.
constexpr int kRoundSlots = 512;
constexpr int kWindowSmall = 64;
constexpr int kWindowLarge = 256;
// Gates handled per sizing block.
constexpr int kSizeBlock = 256;

// Evaluate work lists (one each per step): the wavefront kernel for each
// variant -- delay window (small, large) times delay model (output value
// only; input edge and output value) -- and pin count (1-4), then the lane
// kernel.
constexpr int kVariants = 4;
constexpr int kNumLists = kVariants * 4 + 1;
constexpr int kListLane = kVariants * 4;
__host__ __device__ constexpr int wave_variant(int large_window, int edge_model) {
    return edge_model * 2 + large_window;
}
__host__ __device__ constexpr int wave_list(int variant, int pins) {
    return variant * 4 + pins - 1;
}
// Dispatch order of the wavefront lists: each gate gets a segment by its
// estimated cost (half-octave buckets of w_g times a per-pin-count weight,
// costliest first, then pin count), a counting sort by segment gives one
// sorted list per delay window, and the evaluate launch takes it in order
// (longest jobs first, so the short ones fill the tail of the level).
constexpr int kCostBuckets = 32;
constexpr int kSegments = kCostBuckets * 4;  // per variant
// Per-step counters: list lengths, then the segment sizes of every variant.
constexpr int kSegCountAt = kNumLists;
constexpr int kCountWords = kSegCountAt + kVariants * kSegments;
// A pin's delay entry for an unrelated output (the paper's inf).
constexpr int32_t kNoRelation = INT32_MAX;

// One gate, 64 bytes, in level order. Nets are internal ids: sources keep
// their id, the gate at internal position i drives net S + i.
struct alignas(64) GateRec {
    int32_t net[kMaxPins];   // unused pins: 0
    int32_t rise[kMaxPins];
    int32_t fall[kMaxPins];
    uint8_t type;
    uint8_t k;               // pin count
    uint8_t window;          // wavefront kernels: 0 the small delay window, 1 the large one
    uint8_t pad0;
    int32_t dmax;            // largest rise/fall delay over the pins
    int32_t user_gate;       // the caller's gate index
    int32_t pad1;
};
static_assert(sizeof(GateRec) == 64, "GateRec must be 64 bytes");

// Per-job device state.
struct DevState {
    int64_t arena_top;       // first free transition slot
    int64_t capacity;        // arena size in transitions
    int64_t pin_reads;       // sum of reserved bounds = sum over pins of read lengths
    int64_t n_out;           // output transitions (filled by the final reduction)
    int32_t overflow;        // arena exhausted: later levels are skipped
    int32_t check_error;     // an internal consistency check failed (never expected); 3: the
                             // dependency-driven schedule made no progress for too long;
                             // 4: a gate's round took no input and finalised nothing (an
                             // input waveform out of order)
};

// One job's share of a step: the gates of its current level.
struct JobDesc {
    const GateRec *rec;      // the job's netlist, level order
    int64_t S;
    int64_t *off;            // [S+G] arena offset of each net
    int64_t *len;            // [S+G] transitions of each net
    uint64_t *K;             // arena of packed transitions
    DevState *state;
    int64_t lvl_begin;       // first gate of the level
    int64_t n_gates;         // gates of the level
    int64_t sblock_begin;    // first sizing block of this job in the step
    int32_t lane_threshold;  // gates reading fewer input transitions go to the lane kernel
    int32_t pad;
    const uint8_t *lut;      // [types][256] gate value by packed pin values (built-in + user tables)
    const int32_t *edly;     // [G][4 pins][2 edges][2 outputs] delays by input edge, or null
};
static_assert(sizeof(JobDesc) == 96, "JobDesc layout");

// A step: one level of each of n_jobs jobs.
struct StepArgs {
    const JobDesc *jobs;
    int32_t n_jobs;
    int32_t pad;
    int64_t n_sblocks;       // sizing blocks over all jobs
    int64_t *blocksum;       // [n_sblocks]: block totals, then absolute arena bases
    uint64_t *list[kNumLists];  // work lists: job << 32 | gate
    uint64_t *key[kListLane];   // per wavefront-list entry: segment << 32 | rank in segment
    uint64_t *sorted[kVariants];  // per variant: the wavefront entries in dispatch order
    uint32_t *count;         // [kCountWords] counters of this step (see kSegCountAt)
    uint32_t *next_count;    // [kCountWords] counters of the next step (cleared here)
};

// Dependency-driven schedule: one job per launch, no level barrier. A gate
// becomes ready when the last of its fan-in gates has finished; ready gates
// enter `queue` in that order and persistent wavefronts take them in turn.
struct DfCtl {
    uint32_t head;   // next queue slot to hand out
    uint32_t tail;   // next queue slot to fill
    uint32_t pad[2];
};

struct DfArgs {
    JobDesc job;            // netlist and storage of the job (level fields unused)
    const int64_t *fo_off;  // [G+1] consumers of each gate's output net, one per reading pin
    const int32_t *fo;
    int32_t *pend;          // [G] fan-in pins whose gate has not finished
    int32_t *queue;         // [G] gates in the order they became ready; -1: not yet
    DfCtl *ctl;
    const uint8_t *lut;     // [12][256]
    int64_t G;
    int64_t n_first;        // gates reading sources only (the first level): ready at the start
    int64_t chunk;          // arena reservation granule per wavefront, in transitions
    uint32_t tickets;       // queue slots a wavefront claims per atomic (1..4)
};

// Level-barrier schedule: one persistent launch per job; its wavefronts take
// the gates of each level in turn and meet at a device-wide barrier before
// the next level. Barrier storage: 128-byte lines of 32 words, the top
// arrival counter, one arrival counter per group of kLsGroup wavefronts, then
// one release flag per group (zeroed per launch).
constexpr uint32_t kLsGroup = 64;
constexpr int64_t kLsMaxWaves = 64 * 64;
constexpr int kLsLineWords = 32;
constexpr int kLsLineTop = 0, kLsLineGroups = 1, kLsLineFlags = 1 + 64;
constexpr int64_t kLsSyncWords = (int64_t)kLsLineWords * (1 + 2 * 64);
struct LsArgs {
    JobDesc job;               // netlist and storage of the job (level fields unused)
    const int64_t *level_off;  // [n_levels + 1] first gate of each level (internal order)
    uint32_t *sync;            // [kLsSyncWords] barrier counters and flags
    int64_t chunk;             // arena reservation granule per wavefront, in transitions
    int32_t n_levels;
    int32_t pad;
};

// Kernel launchers (kernels.hip). All are asynchronous on `s`.
hipError_t launch_init_sources(const int64_t *d_src_off, const int64_t *d_t, const uint8_t *d_v,
                               int64_t S, int64_t n_in, int64_t *off, int64_t *len, uint64_t *K,
                               DevState *state, int64_t capacity, hipStream_t s);
// size + classify (grid: n_sblocks), then per-job scan (grid: n_jobs)
hipError_t launch_size(const StepArgs &a, hipStream_t s);
// evaluate the work list of class `cls`; `max_items` bounds the list length
// Wavefront kernel over the four pin-count lists of one delay window
// (max_items[k-1]: upper bound of the k-pin list's length).
// form: kFormSegmented (eval_gate_seg) or kFormMerged (eval_gate).
constexpr int kFormSegmented = 0, kFormMerged = 1;
hipError_t launch_eval_wave(const StepArgs &a, int variant, const int64_t *max_items, int form,
                            hipStream_t s);
// Per job of the step: its level's arena bases (exclusive scan of the sizing
// blocks' totals, arena top bumped, overflow flagged); then the counting-sort
// scatter of the wavefront lists into one sorted list per variant
// (max_items[c]: upper bound of list c's length, c < kListLane).
hipError_t launch_sort_lists(const StepArgs &a, const int64_t *max_items, hipStream_t s);
hipError_t launch_eval_lane(const StepArgs &a, int64_t max_items, hipStream_t s);
// Dependency-driven schedule: reset the counters and queue, then run every
// gate of the job with n_waves persistent wavefronts.
hipError_t launch_df_init(const DfArgs &a, const int32_t *pend0, hipStream_t s);
hipError_t launch_dataflow(const DfArgs &a, int64_t n_waves, hipStream_t s);
// Level-barrier schedule: clear the barrier counter, then run every level of
// the job with n_waves persistent wavefronts in a cooperative launch (every
// one resident; at most levelsync_max_waves and kLsMaxWaves).
hipError_t launch_levelsync(const LsArgs &a, int64_t n_waves, hipStream_t s);
// Wavefronts of the level-barrier kernel that fit the device at once.
hipError_t levelsync_max_waves(int n_cu, int64_t *out);
hipError_t launch_count_out(const int64_t *len, int64_t S, int64_t G, int64_t *partial,
                            int64_t n_partial, DevState *state, hipStream_t s);
hipError_t launch_gather(const int64_t *src_off, const int64_t *n_items, const int64_t *dst_off,
                         int64_t n_nets, const uint64_t *K, int64_t *out_t, uint8_t *out_v,
                         hipStream_t s);
hipError_t launch_clear_u32(uint32_t *p, int64_t n, hipStream_t s);
// per-net fingerprints (see hash_kernel) and off/len of a list of nets
hipError_t launch_hash(const int64_t *nets_off, const int64_t *nets_len, int64_t n_nets,
                       const uint64_t *K, uint64_t *out, hipStream_t s);
hipError_t launch_gather_meta(const int64_t *net, int64_t n, const int64_t *off, const int64_t *len,
                              int64_t *out_off, int64_t *out_len, hipStream_t s);

// No-allocation run (sim_run_device_noalloc): a static device array of
// kNoAllocScratchBytes per GPU holds every step buffer of the level schedule.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
// Look up `device`'s copy of the array (with that device current); once per
// device, at context creation.
hipError_t noalloc_scratch_setup(int device);
// Its device address, or null before the set-up succeeded on that device.
void *noalloc_scratch(int device);
// Step descriptors of up to kDescBatch levels, written to dst[0, n) by one launch.
constexpr int kDescBatch = 32;
struct DescBatch {
    JobDesc d[kDescBatch];
    JobDesc *dst;
    int32_t n;
    int32_t pad;
};
hipError_t launch_write_descs(const DescBatch &b, hipStream_t s);
// out[0..3] = n_out, overflow flag, check code, arena transitions used
hipError_t launch_run_result(const DevState *st, int64_t *out, hipStream_t s);

}  // namespace gsim
