// Host runtime of libgsim: validation, levelizer, netlist upload, device
// memory pool, the job executor (admission by HBM budget, one step per level
// covering every active job), and waveform fetch. Exposes the C ABI declared
// in include/gsim.h.
#include "gsim.h"
#include "gsim_internal.h"

#include <algorithm>
#include <atomic>
#include <exception>
#include <new>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace gsim;

namespace {

// ---------------------------------------------------------------------------
// Errors.

std::mutex g_err_mu;
std::string g_err;  // last error of a context-free call

struct Failure {
    gsim_status st;
    std::string msg;
};

Failure fail(gsim_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return Failure{st, buf};
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(GSIM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));      \
    } while (0)

const Failure kOk{GSIM_OK, ""};

// ---------------------------------------------------------------------------
// Gate functions for the device look-up table.
//
// A 4-value signal is held as the pair (can be 0, can be 1): 0 = (1,0),
// 1 = (0,1), X and Z = (1,1) -- X may be either level and Z is read as X
// (Section 2.2). AND can be 1 only if every input can be 1 and can be 0 if any
// can; OR is the dual; XOR is unknown if any input is, else the parity;
// NOT swaps the pair; MUX2 can take a level if a select level that is possible
// leads to a data input that can take it.
struct Pair {
    bool c0, c1;
};
Pair pair_of(int v) { return v == 0 ? Pair{true, false} : v == 1 ? Pair{false, true} : Pair{true, true}; }
uint8_t value_of(Pair p) { return (p.c0 && p.c1) ? kX : (p.c1 ? 1 : 0); }

const int kArity[GSIM_NUM_TYPES] = {1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 4, 4};

uint8_t gate_value(int type, const int *in) {
    Pair a[kMaxPins];
    for (int i = 0; i < kArity[type]; i++) a[i] = pair_of(in[i]);
    auto all1 = [&](int k) { bool r = true; for (int i = 0; i < k; i++) r = r && a[i].c1; return r; };
    auto any1 = [&](int k) { bool r = false; for (int i = 0; i < k; i++) r = r || a[i].c1; return r; };
    auto all0 = [&](int k) { bool r = true; for (int i = 0; i < k; i++) r = r && a[i].c0; return r; };
    auto any0 = [&](int k) { bool r = false; for (int i = 0; i < k; i++) r = r || a[i].c0; return r; };
    auto neg = [](Pair p) { return Pair{p.c1, p.c0}; };
    auto parity = [&](int k) {
        bool unknown = false;
        int ones = 0;
        for (int i = 0; i < k; i++) {
            unknown = unknown || (a[i].c0 && a[i].c1);
            ones += a[i].c1 ? 1 : 0;
        }
        if (unknown) return Pair{true, true};
        return (ones & 1) ? Pair{false, true} : Pair{true, false};
    };
    Pair r{true, true};
    switch (type) {
    case GSIM_BUF: r = a[0]; break;
    case GSIM_NOT: r = neg(a[0]); break;
    case GSIM_AND2: r = Pair{any0(2), all1(2)}; break;
    case GSIM_OR2: r = Pair{all0(2), any1(2)}; break;
    case GSIM_NAND2: r = neg(Pair{any0(2), all1(2)}); break;
    case GSIM_NOR2: r = neg(Pair{all0(2), any1(2)}); break;
    case GSIM_XOR2: r = parity(2); break;
    case GSIM_XNOR2: r = neg(parity(2)); break;
    case GSIM_AND3: r = Pair{any0(3), all1(3)}; break;
    case GSIM_AND4: r = Pair{any0(4), all1(4)}; break;
    case GSIM_OR4: r = Pair{all0(4), any1(4)}; break;
    case GSIM_MUX2: {
        const Pair d0 = a[0], d1 = a[1], s = a[2];
        r = Pair{(s.c0 && d0.c0) || (s.c1 && d1.c0), (s.c0 && d0.c1) || (s.c1 && d1.c1)};
        break;
    }
    }
    return value_of(r);
}

// [type][packed] with pin i's value in bits 2i..2i+1; bits of absent pins are ignored.
std::vector<uint8_t> build_lut() {
    std::vector<uint8_t> lut(GSIM_NUM_TYPES * 256);
    for (int t = 0; t < GSIM_NUM_TYPES; t++)
        for (int packed = 0; packed < 256; packed++) {
            int in[kMaxPins];
            for (int i = 0; i < kMaxPins; i++) in[i] = (packed >> (2 * i)) & 3;
            lut[t * 256 + packed] = gate_value(t, in);
        }
    return lut;
}

// ---------------------------------------------------------------------------
// Netlist validation and levelization (host).

struct Levelized {
    std::vector<int32_t> level;  // [G], >= 1
    int32_t n_levels = 0;
    int32_t max_delay = 0;
    int64_t max_path_delay = 0;
};

// n_udp: user-defined gate types 12 .. 11 + n_udp are allowed (any 1-4 pins).
Failure levelize(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                 const int64_t *pin_net, const int32_t *rise, const int32_t *fall, Levelized *out,
                 int n_udp = 0) {
    if (S < 0 || G < 0) return fail(GSIM_E_ARG, "S and G must be >= 0 (S=%lld G=%lld)", (long long)S, (long long)G);
    if (S + G > INT32_MAX) return fail(GSIM_E_ARG, "S + G exceeds 2^31-1 nets");
    if (G > 0 && (!type || !pin_off || !pin_net || !rise || !fall))
        return fail(GSIM_E_ARG, "null netlist array");
    if (G > 0 && pin_off[0] != 0) return fail(GSIM_E_ARG, "pin_off[0] must be 0");
    for (int64_t g = 0; g < G; g++) {
        const int64_t k = pin_off[g + 1] - pin_off[g];
        if (type[g] >= GSIM_NUM_TYPES && type[g] < GSIM_NUM_TYPES + n_udp) {
            if (k < 1 || k > kMaxPins)
                return fail(GSIM_E_ARG, "gate %lld: user-defined type with %lld pins (1-4 allowed)",
                            (long long)g, (long long)k);
            continue;
        }
        if (type[g] >= GSIM_NUM_TYPES) return fail(GSIM_E_ARG, "gate %lld: unknown type %d", (long long)g, type[g]);
        if (k != kArity[type[g]])
            return fail(GSIM_E_ARG, "gate %lld: %lld pins, type %d needs %d", (long long)g, (long long)k,
                        type[g], kArity[type[g]]);
    }
    const int64_t P = G > 0 ? pin_off[G] : 0;
    int32_t max_delay = 0;
    for (int64_t g = 0; g < G; g++)
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++) {
            const int64_t n = pin_net[p];
            if (n < 0 || n >= S + G) return fail(GSIM_E_ARG, "pin %lld: net %lld out of range", (long long)p, (long long)n);
            if (n == S + g) return fail(GSIM_E_CYCLE, "gate %lld reads its own output", (long long)g);
            if (rise[p] < 0 || fall[p] < 0) return fail(GSIM_E_ARG, "pin %lld: negative delay", (long long)p);
            max_delay = std::max(max_delay, std::max(rise[p], fall[p]));
        }
    // Kahn's algorithm over gate-to-gate edges.
    std::vector<int64_t> indeg(G, 0), fo_start(G + 1, 0);
    for (int64_t p = 0; p < P; p++)
        if (pin_net[p] >= S) fo_start[pin_net[p] - S + 1]++;
    for (int64_t g = 0; g < G; g++) fo_start[g + 1] += fo_start[g];
    std::vector<int64_t> fo(fo_start[G]);
    {
        std::vector<int64_t> fill(fo_start.begin(), fo_start.end() - 1);
        for (int64_t g = 0; g < G; g++)
            for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
                if (pin_net[p] >= S) {
                    indeg[g]++;
                    fo[fill[pin_net[p] - S]++] = g;
                }
    }
    out->level.assign(G, 1);
    std::vector<int64_t> path(G, 0);  // longest sum of per-gate max delays ending at g
    std::vector<int64_t> queue;
    queue.reserve(G);
    for (int64_t g = 0; g < G; g++)
        if (indeg[g] == 0) queue.push_back(g);
    int32_t nl = 0;
    int64_t mpd = 0;
    for (size_t h = 0; h < queue.size(); h++) {
        const int64_t g = queue[h];
        int32_t dm = 0;
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++) dm = std::max(dm, std::max(rise[p], fall[p]));
        path[g] += dm;
        nl = std::max(nl, out->level[g]);
        mpd = std::max(mpd, path[g]);
        for (int64_t e = fo_start[g]; e < fo_start[g + 1]; e++) {
            const int64_t c = fo[e];
            out->level[c] = std::max(out->level[c], out->level[g] + 1);
            path[c] = std::max(path[c], path[g]);
            if (--indeg[c] == 0) queue.push_back(c);
        }
    }
    if ((int64_t)queue.size() != G)
        return fail(GSIM_E_CYCLE, "netlist has a cycle (%lld of %lld gates ordered)", (long long)queue.size(), (long long)G);
    out->n_levels = nl;
    out->max_delay = max_delay;
    out->max_path_delay = mpd;
    return kOk;
}

// Sources [s0, s1) of a host stimulus (see validate_stimulus).
Failure validate_sources(int64_t s0, int64_t s1, const int64_t *src_off, const int64_t *t, const uint8_t *v,
                         int64_t max_path_delay) {
    const int64_t limit = kTimeLimit - max_path_delay;
    for (int64_t s = s0; s < s1; s++) {
        const int64_t a = src_off[s], b = src_off[s + 1];
        if (b < a) return fail(GSIM_E_WAVEFORM, "source %lld: negative length", (long long)s);
        if (b > a && (!t || !v)) return fail(GSIM_E_ARG, "null t or v");
        uint8_t prev = kX;
        for (int64_t i = a; i < b; i++) {
            if (v[i] > 3) return fail(GSIM_E_WAVEFORM, "source %lld: value %d at index %lld", (long long)s, v[i], (long long)i);
            if (v[i] == prev)
                return fail(GSIM_E_WAVEFORM, "source %lld: value %d repeats the previous one (or a leading X) at index %lld",
                            (long long)s, v[i], (long long)i);
            if (t[i] < 0) return fail(GSIM_E_WAVEFORM, "source %lld: negative time", (long long)s);
            if (i > a && t[i] <= t[i - 1])
                return fail(GSIM_E_WAVEFORM, "source %lld: times not strictly increasing at index %lld", (long long)s, (long long)i);
            if (t[i] >= limit)
                return fail(GSIM_E_OVERFLOW, "source %lld: time %lld plus the longest path delay %lld leaves [0, 2^62)",
                            (long long)s, (long long)t[i], (long long)max_path_delay);
            prev = v[i];
        }
    }
    return kOk;
}

Failure validate_stimulus(int64_t S, const int64_t *src_off, const int64_t *t, const uint8_t *v,
                          int64_t max_path_delay) {
    if (!src_off) return fail(GSIM_E_ARG, "null src_off");
    if (src_off[0] != 0) return fail(GSIM_E_WAVEFORM, "src_off[0] must be 0");
    return validate_sources(0, S, src_off, t, v, max_path_delay);
}

// ---------------------------------------------------------------------------
// Device memory: the context reserves its whole HBM budget as one slab on
// first use and carves every buffer out of it (best fit, free neighbours
// merged on release). After that no call reaches hipMalloc/hipFree, whose cost
// for multi-GB job arenas would dominate short jobs.

class Pool {
  public:
    explicit Pool(uint64_t budget) : budget_(budget & ~uint64_t(kAlign - 1)) {}
    ~Pool() {
        if (slab_) (void)hipFree(slab_);
    }

    void *get(size_t bytes) {
        if (!slab_ && !reserve()) return nullptr;
        bytes = (bytes + kAlign - 1) & ~size_t(kAlign - 1);
        if (bytes == 0) bytes = kAlign;
        auto it = by_size_.lower_bound(bytes);  // best fit
        if (it == by_size_.end()) return nullptr;
        const uint64_t off = it->second, sz = it->first;
        by_size_.erase(it);
        by_off_.erase(off);
        if (sz > bytes) insert_free(off + bytes, sz - bytes);
        used_[off] = bytes;
        live_ += bytes;
        return slab_ + off;
    }
    void put(void *p) {
        if (!p) return;
        const uint64_t off = (uint64_t)((char *)p - slab_);
        auto it = used_.find(off);
        if (it == used_.end()) return;
        uint64_t start = off, size = it->second;
        live_ -= size;
        used_.erase(it);
        auto next = by_off_.find(start + size);  // merge with the free range after
        if (next != by_off_.end()) {
            erase_free(next->first, next->second);
            size += next->second;
        }
        auto prev = by_off_.lower_bound(start);  // and with the one before
        if (prev != by_off_.begin()) {
            --prev;
            if (prev->first + prev->second == start) {
                start = prev->first;
                size += prev->second;
                erase_free(prev->first, prev->second);
            }
        }
        insert_free(start, size);
    }
    uint64_t budget() const { return budget_; }
    uint64_t live() const { return live_; }
    // Largest block that can still be allocated.
    uint64_t largest_free() const {
        if (!slab_) return budget_;
        return by_size_.empty() ? 0 : by_size_.rbegin()->first;
    }

  private:
    static constexpr uint64_t kAlign = 4096;
    bool reserve() {
        // take the budget, or as much of it as the device gives
        uint64_t want = budget_;
        while (want >= (uint64_t(64) << 20)) {
            void *p = nullptr;
            if (hipMalloc(&p, want) == hipSuccess) {
                slab_ = (char *)p;
                budget_ = want;
                insert_free(0, want);
                return true;
            }
            (void)hipGetLastError();
            want = (want / 10 * 9) & ~uint64_t(kAlign - 1);
        }
        return false;
    }
    void insert_free(uint64_t off, uint64_t size) {
        by_off_[off] = size;
        by_size_.emplace(size, off);
    }
    void erase_free(uint64_t off, uint64_t size) {
        by_off_.erase(off);
        auto range = by_size_.equal_range(size);
        for (auto i = range.first; i != range.second; ++i)
            if (i->second == off) {
                by_size_.erase(i);
                break;
            }
    }
    uint64_t budget_, live_ = 0;
    char *slab_ = nullptr;
    std::map<uint64_t, uint64_t> by_off_;        // free ranges: offset -> size
    std::multimap<uint64_t, uint64_t> by_size_;  // free ranges: size -> offset
    std::unordered_map<uint64_t, uint64_t> used_;
};

// Pinned host buffers, kept for reuse by power-of-two size class (pinning and
// unpinning multi-MB buffers per job is slow).
class PinnedCache {
  public:
    ~PinnedCache() {
        for (auto &kv : free_) (void)hipHostFree(kv.second);
    }
    void *get(size_t bytes) {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        auto it = free_.find(c);
        if (it != free_.end()) {
            void *p = it->second;
            free_.erase(it);
            size_[p] = c;
            return p;
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        size_[p] = c;
        return p;
    }
    void put(void *p) {
        if (!p) return;
        auto it = size_.find(p);
        if (it == size_.end()) return;
        free_.emplace(it->second, p);
        size_.erase(it);
    }

  private:
    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> size_;
};

// ---------------------------------------------------------------------------

// Gates of one level in consecutive groups, one per work list: by largest
// pin delay (<= kWindowSmall, <= kWindowLarge; the small window only when
// its gates are not fewer than the large window's) and pin count for the
// wavefront kernels, then the gates whose delays need the lane kernel. The
// group sizes bound the wavefront work lists of a step (the lane list may
// take any gate).
struct LevelRange {
    int64_t begin, n;
    int64_t n_list[kNumLists];
};

struct Netlist {
    int64_t S = 0, G = 0, P = 0;
    int32_t n_levels = 0, max_delay = 0;
    int64_t max_path_delay = 0;
    int64_t lane_gates = 0;  // gates whose largest delay needs the lane kernel
    std::vector<LevelRange> levels;
    std::vector<int64_t> internal_of_user;  // [G]
    GateRec *d_rec = nullptr;
    uint8_t *d_lut = nullptr;       // netlist's own gate tables (built-in + user-defined), or null
    int32_t *d_edly = nullptr;      // [G][4][2][2] delays by input edge and output value, or null
    // dependency-driven schedule: consumers of each gate's net (one entry per
    // reading pin), each gate's count of pins that read gate nets, and the
    // number of gates that read sources only (they come first in level order)
    int64_t *d_fo_off = nullptr;
    int32_t *d_fo = nullptr;
    int32_t *d_pend0 = nullptr;
    int64_t n_first = 0;
    // level-barrier schedule: first gate of each level, then G ([n_levels + 1])
    int64_t *d_level_off = nullptr;
    int64_t active_jobs = 0;
    int64_t max_level_n = 0;        // gates of the largest level
    int32_t lane_threshold = -1;    // -1: the context's GSIM_OPT_LANE_THRESHOLD
    int32_t schedule = -1;          // -1: the context's GSIM_OPT_SCHEDULE
    int32_t form = -1;              // -1: the context's GSIM_OPT_EVAL_FORM
    int32_t df_tickets = -1;        // -1: the context's GSIM_OPT_DF_TICKETS
    double arena_per_input = 0.0;   // largest arena use per input transition seen so far
};

// Device time of one step's evaluate launches (with GSIM_OPT_KERNEL_TIMING).
struct StepTiming {
    hipEvent_t a = nullptr, b = nullptr;
    ~StepTiming() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct Executor;

enum JobPhase { kQueued, kActive, kEnqueued };

struct Job {
    int64_t id = 0, nl_id = 0;
    Netlist *nl = nullptr;
    Executor *ex = nullptr;
    JobPhase phase = kQueued;
    int32_t next_level = 0;
    int64_t n_in = 0, capacity = 0, capacity_request = 0;
    int64_t *d_off = nullptr, *d_len = nullptr, *d_partial = nullptr;
    int64_t *d_src_off = nullptr;    // host submissions: device copy of the offsets
    // host submissions: pinned copies of the caller's stimuli, uploaded into
    // the job's arena at admission (a queued job holds no device memory)
    int64_t *h_src_off = nullptr, *h_t = nullptr;
    uint8_t *h_v = nullptr;
    // device submissions: the caller's arrays, used in place
    const int64_t *dev_src_off = nullptr, *dev_t = nullptr;
    const uint8_t *dev_v = nullptr;
    uint64_t *d_K = nullptr;      // arena of packed transitions
    DevState *d_state = nullptr;
    DevState *h_state = nullptr;  // pinned
    hipEvent_t ev_start = nullptr, ev_end = nullptr, ev_done = nullptr;
    std::vector<std::shared_ptr<StepTiming>> timing;
    int64_t n_partial = 0;
    bool dataflow = false;        // dependency-driven schedule (one launch for every gate)
    bool levelsync = false;       // level-barrier schedule (one launch, a device-wide barrier per level)
    // the job's step descriptor of every level, for steps it has alone
    // (uploaded once at admission instead of once per step)
    JobDesc *h_desc = nullptr;    // pinned
    JobDesc *d_desc = nullptr;
    int32_t *d_pend = nullptr, *d_queue = nullptr;
    DfCtl *d_ctl = nullptr;
    uint32_t *d_sync = nullptr;   // level-barrier schedule: barrier counters and flags
    int32_t retries = 0;          // automatic re-runs after an arena overflow
    bool waited = false, failed = false;
};

constexpr int kMaxJobsPerStep = 256;
constexpr int64_t kStage = int64_t(8) << 20;       // fetch staging buffer, transitions
constexpr int64_t kStageBatch = int64_t(1) << 16;  // nets per gather batch
constexpr int kRing = 32;  // steps whose descriptors may be in flight

// One executor per stream: its jobs advance one level per step, all active
// jobs in the same launches.
struct Executor {
    hipStream_t stream = nullptr;
    uint32_t *d_counts = nullptr;  // 2 x kCountWords step counters (this step / next step)
    int parity = 0;
    JobDesc *d_jobs = nullptr;
    int64_t jobs_cap = 0;
    int64_t *d_blocksum = nullptr;
    int64_t blocksum_cap = 0;
    uint64_t *d_list = nullptr;    // kNumLists lists of list_cap entries
    uint64_t *d_keys = nullptr;    // kListLane key arrays of list_cap entries
    uint64_t *d_sorted = nullptr;  // kVariants sorted lists of list_cap entries
    int64_t list_cap = 0;
    JobDesc *h_ring = nullptr;     // pinned [kRing][kMaxJobsPerStep]
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int64_t steps = 0;
    std::vector<Job *> active;     // admitted, levels left to enqueue
    std::deque<Job *> queue;       // submitted, waiting for memory
};

}  // namespace

struct gsim_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::unique_ptr<Pool> pool;
    PinnedCache pinned;
    uint8_t *d_lut = nullptr;
    std::string err;
    int64_t next_id = 1;
    std::map<int64_t, std::unique_ptr<Netlist>> netlists;
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    std::map<hipStream_t, std::unique_ptr<Executor>> executors;
    int64_t arenas_held = 0;  // jobs that hold an output arena (admitted, not yet released)
    int64_t *d_stage_t = nullptr;  // fetch staging buffers, 2 x kStage transitions
    uint8_t *d_stage_v = nullptr;
    int64_t *d_stage_meta = nullptr;
    int64_t opt_arena = 0;
    int opt_kernel = 0;
    int opt_timing = 0;
    int opt_schedule = 0;
    int opt_form = kFormMerged;
    int opt_df_tickets = 0;
    int64_t n_waves_resident = 0;  // persistent wavefronts of the dependency-driven schedule
    int64_t n_waves_levelsync = 0; // level-barrier kernel's wavefronts that fit the device at once
    // the last level-barrier launch of this context: the next one, from any
    // executor's stream, waits for it, so that two such grids never share the
    // device (each needs every wavefront resident)
    hipEvent_t ls_event = nullptr;
    int32_t opt_lane_threshold = 0;
};

namespace {

gsim_status record(gsim_ctx ctx, const Failure &f) {
    if (f.st != GSIM_OK) {
        if (ctx) {
            ctx->err = f.msg;
        } else {
            std::lock_guard<std::mutex> lk(g_err_mu);
            g_err = f.msg;
        }
    }
    return f.st;
}

Failure set_device(gsim_ctx ctx) {
    HIP_TRY(hipSetDevice(ctx->device));
    return kOk;
}

template <class T>
T *pool_get(Pool &pool, int64_t n) {
    return (T *)pool.get(sizeof(T) * (size_t)std::max<int64_t>(n, 1));
}

// ---- netlists ---------------------------------------------------------------

void put_netlist(gsim_ctx ctx, Netlist *nl) {
    ctx->pool->put(nl->d_rec);
    ctx->pool->put(nl->d_fo_off);
    ctx->pool->put(nl->d_fo);
    ctx->pool->put(nl->d_pend0);
    ctx->pool->put(nl->d_lut);
    ctx->pool->put(nl->d_edly);
    ctx->pool->put(nl->d_level_off);
    nl->d_rec = nullptr;
    nl->d_fo_off = nullptr;
    nl->d_fo = nullptr;
    nl->d_pend0 = nullptr;
    nl->d_lut = nullptr;
    nl->d_edly = nullptr;
    nl->d_level_off = nullptr;
}

// dly (optional): per pin [2 edges][2 outputs] delays of the extended model;
// then rise/fall are ignored. udp (optional): n_udp tables of 256 values.
Failure load_netlist(gsim_ctx ctx, int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                     const int64_t *pin_net, const int32_t *rise, const int32_t *fall, gsim_netlist *out,
                     const int32_t *dly = nullptr, int n_udp = 0, const uint8_t *udp = nullptr) {
    if (!out) return fail(GSIM_E_ARG, "null output handle");
    if (n_udp < 0 || n_udp > 256 - GSIM_NUM_TYPES) return fail(GSIM_E_ARG, "n_udp must be in [0, %d]", 256 - GSIM_NUM_TYPES);
    if (n_udp > 0 && !udp) return fail(GSIM_E_ARG, "null user-defined gate tables");
    for (int64_t i = 0; i < (int64_t)n_udp * 256; i++)
        if (udp[i] > 2) return fail(GSIM_E_ARG, "user-defined table %lld: entry %lld is %d (0, 1 or X allowed)",
                                    (long long)(i / 256), (long long)(i % 256), udp[i]);
    std::vector<int32_t> erise, efall;  // extended model: each pin's largest finite delay
    if (dly) {
        const int64_t P = G > 0 && pin_off ? pin_off[G] : 0;
        erise.assign(std::max<int64_t>(P, 1), 0);
        for (int64_t p = 0; p < P; p++)
            for (int e = 0; e < 4; e++) {
                const int32_t x = dly[4 * p + e];
                if (x < 0) return fail(GSIM_E_ARG, "pin %lld: negative delay", (long long)p);
                if (x != kNoRelation) erise[p] = std::max(erise[p], x);
            }
        efall = erise;
        rise = erise.data();
        fall = efall.data();
    }
    Levelized lv;
    Failure f = levelize(S, G, type, pin_off, pin_net, rise, fall, &lv, n_udp);
    if (f.st != GSIM_OK) return f;
    auto nl = std::make_unique<Netlist>();
    nl->S = S;
    nl->G = G;
    nl->P = G > 0 ? pin_off[G] : 0;
    nl->n_levels = lv.n_levels;
    nl->max_delay = lv.max_delay;
    nl->max_path_delay = lv.max_path_delay;

    // Gate order: by level; inside a level by delay group (see LevelRange),
    // each group in the caller's order.
    auto gate_dmax = [&](int64_t g) {
        int32_t d = 0;
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++) d = std::max(d, std::max(rise[p], fall[p]));
        return d;
    };
    const int edge_model = dly ? 1 : 0;
    std::vector<int32_t> dmax_of(G);
    int64_t n_small = 0, n_large = 0;
    for (int64_t g = 0; g < G; g++) {
        dmax_of[g] = gate_dmax(g);
        n_small += dmax_of[g] <= kWindowSmall;
        n_large += dmax_of[g] > kWindowSmall && dmax_of[g] <= kWindowLarge;
    }
    // The small window's kernel runs more wavefronts per SIMD, but a launch of
    // its own per level only pays while it has a real share of the gates:
    // when they are fewer than the large window's, they join those (the
    // large window is exact for them too).
    const bool small_window = n_small >= n_large;
    auto window_of = [&](int64_t g) { return small_window && dmax_of[g] <= kWindowSmall ? 0 : 1; };
    auto group_of = [&](int64_t g) {
        if (ctx->opt_kernel == 1) return kListLane;  // every gate on the lane kernel
        const int k = (int)(pin_off[g + 1] - pin_off[g]);
        return dmax_of[g] <= kWindowLarge ? wave_list(wave_variant(window_of(g), edge_model), k) : kListLane;
    };
    const int32_t L = lv.n_levels;
    constexpr size_t NL = kNumLists;
    std::vector<int64_t> cnt(NL * ((size_t)L + 1), 0);
    std::vector<int> grp(G);
    for (int64_t g = 0; g < G; g++) {
        grp[g] = group_of(g);
        cnt[NL * (size_t)lv.level[g] + grp[g]]++;
    }
    std::vector<int64_t> start(cnt.size() + 1, 0);
    for (size_t i = 0; i < cnt.size(); i++) start[i + 1] = start[i] + cnt[i];
    nl->levels.resize(L);
    for (int32_t l = 1; l <= L; l++) {
        LevelRange &r = nl->levels[l - 1];
        r.begin = start[NL * (size_t)l];
        r.n = 0;
        for (int c = 0; c < kNumLists; c++) {
            r.n_list[c] = cnt[NL * (size_t)l + c];
            r.n += r.n_list[c];
        }
        nl->lane_gates += r.n_list[kListLane];
        nl->max_level_n = std::max(nl->max_level_n, r.n);
    }
    nl->internal_of_user.resize(G);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t g = 0; g < G; g++) nl->internal_of_user[g] = fill[NL * (size_t)lv.level[g] + grp[g]]++;
    }
    std::vector<GateRec> recs(G);
    for (int64_t g = 0; g < G; g++) {
        GateRec r;
        std::memset(&r, 0, sizeof r);
        r.type = type[g];
        r.k = (uint8_t)(pin_off[g + 1] - pin_off[g]);
        for (int i = 0; i < r.k; i++) {
            const int64_t p = pin_off[g] + i;
            const int64_t n = pin_net[p];
            r.net[i] = (int32_t)(n < S ? n : S + nl->internal_of_user[n - S]);
            r.rise[i] = rise[p];
            r.fall[i] = fall[p];
        }
        // the lane-kernel option routes every gate to the lane kernel
        r.dmax = ctx->opt_kernel == 1 ? INT32_MAX : dmax_of[g];
        r.window = (uint8_t)window_of(g);
        r.user_gate = (int32_t)g;
        recs[nl->internal_of_user[g]] = r;
    }
    // consumers of each gate, in internal ids, for the dependency-driven schedule
    std::vector<int64_t> fo_off(G + 1, 0);
    std::vector<int32_t> pend0(G, 0);
    for (int64_t c = 0; c < G; c++)
        for (int i = 0; i < recs[c].k; i++)
            if (recs[c].net[i] >= S) {
                fo_off[recs[c].net[i] - S + 1]++;
                pend0[c]++;
            }
    for (int64_t g = 0; g < G; g++) fo_off[g + 1] += fo_off[g];
    std::vector<int32_t> fo(std::max<int64_t>(fo_off[G], 1));
    {
        std::vector<int64_t> fill(fo_off.begin(), fo_off.end() - 1);
        for (int64_t c = 0; c < G; c++)
            for (int i = 0; i < recs[c].k; i++)
                if (recs[c].net[i] >= S) fo[fill[recs[c].net[i] - S]++] = (int32_t)c;
    }
    while (nl->n_first < G && pend0[nl->n_first] == 0) nl->n_first++;
    f = set_device(ctx);
    if (f.st != GSIM_OK) return f;
    if (G > 0) {
        nl->d_fo_off = pool_get<int64_t>(*ctx->pool, G + 1);
        nl->d_fo = pool_get<int32_t>(*ctx->pool, (int64_t)fo.size());
        nl->d_pend0 = pool_get<int32_t>(*ctx->pool, G);
        if (!nl->d_fo_off || !nl->d_fo || !nl->d_pend0 ||
            hipMemcpy(nl->d_fo_off, fo_off.data(), sizeof(int64_t) * (size_t)(G + 1), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(nl->d_fo, fo.data(), sizeof(int32_t) * fo.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(nl->d_pend0, pend0.data(), sizeof(int32_t) * (size_t)G, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            ctx->pool->put(nl->d_fo_off);
            ctx->pool->put(nl->d_fo);
            ctx->pool->put(nl->d_pend0);
            return fail(GSIM_E_OOM, "no device memory for the fanout table of %lld gates", (long long)G);
        }
        nl->d_rec = (GateRec *)ctx->pool->get(sizeof(GateRec) * (size_t)G);
        if (!nl->d_rec) {
            ctx->pool->put(nl->d_fo_off);
            ctx->pool->put(nl->d_fo);
            ctx->pool->put(nl->d_pend0);
            return fail(GSIM_E_OOM, "no device memory for %lld gate records", (long long)G);
        }
        hipError_t e = hipMemcpy(nl->d_rec, recs.data(), sizeof(GateRec) * (size_t)G, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            ctx->pool->put(nl->d_rec);
            ctx->pool->put(nl->d_fo_off);
            ctx->pool->put(nl->d_fo);
            ctx->pool->put(nl->d_pend0);
            return fail(GSIM_E_DEVICE, "netlist upload: %s", hipGetErrorString(e));
        }
    }
    if (n_udp > 0) {
        std::vector<uint8_t> lut = build_lut();
        lut.resize((size_t)(GSIM_NUM_TYPES + n_udp) * 256);
        std::memcpy(lut.data() + (size_t)GSIM_NUM_TYPES * 256, udp, (size_t)n_udp * 256);
        nl->d_lut = (uint8_t *)ctx->pool->get(lut.size());
        if (!nl->d_lut || hipMemcpy(nl->d_lut, lut.data(), lut.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            put_netlist(ctx, nl.get());
            return fail(GSIM_E_OOM, "no device memory for the user-defined gate tables");
        }
    }
    if (dly && G > 0) {
        std::vector<int32_t> ed((size_t)G * 16, kNoRelation);
        for (int64_t g = 0; g < G; g++) {
            const int64_t ig = nl->internal_of_user[g];
            for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
                for (int e = 0; e < 4; e++) ed[(size_t)ig * 16 + (p - pin_off[g]) * 4 + e] = dly[4 * p + e];
        }
        nl->d_edly = pool_get<int32_t>(*ctx->pool, G * 16);
        if (!nl->d_edly ||
            hipMemcpy(nl->d_edly, ed.data(), sizeof(int32_t) * ed.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            put_netlist(ctx, nl.get());
            return fail(GSIM_E_OOM, "no device memory for the edge delay table");
        }
    }
    if (nl->n_levels > 0) {
        std::vector<int64_t> lo((size_t)nl->n_levels + 1);
        for (int32_t l = 0; l < nl->n_levels; l++) lo[l] = nl->levels[l].begin;
        lo[nl->n_levels] = G;
        nl->d_level_off = pool_get<int64_t>(*ctx->pool, nl->n_levels + 1);
        if (!nl->d_level_off ||
            hipMemcpy(nl->d_level_off, lo.data(), sizeof(int64_t) * lo.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            put_netlist(ctx, nl.get());
            return fail(GSIM_E_OOM, "no device memory for the level table");
        }
    }
    const int64_t id = ctx->next_id++;
    ctx->netlists[id] = std::move(nl);
    *out = id;
    return kOk;
}

// ---- executors ----------------------------------------------------------------

Failure get_executor(gsim_ctx ctx, hipStream_t stream, Executor **out) {
    if (!stream) stream = ctx->stream;
    auto it = ctx->executors.find(stream);
    if (it != ctx->executors.end()) {
        *out = it->second.get();
        return kOk;
    }
    auto ex = std::make_unique<Executor>();
    ex->stream = stream;
    ex->d_counts = pool_get<uint32_t>(*ctx->pool, 2 * kCountWords);
    if (!ex->d_counts) return fail(GSIM_E_OOM, "no device memory for the executor");
    HIP_TRY(hipHostMalloc((void **)&ex->h_ring, sizeof(JobDesc) * kRing * kMaxJobsPerStep, hipHostMallocDefault));
    for (int i = 0; i < kRing; i++) HIP_TRY(hipEventCreateWithFlags(&ex->ring_ev[i], hipEventDisableTiming));
    HIP_TRY(launch_clear_u32(ex->d_counts, 2 * kCountWords, stream));
    *out = ex.get();
    ctx->executors[stream] = std::move(ex);
    return kOk;
}

void destroy_executor(gsim_ctx ctx, Executor *ex) {
    (void)hipStreamSynchronize(ex->stream);
    Pool &pool = *ctx->pool;
    pool.put(ex->d_counts);
    pool.put(ex->d_jobs);
    pool.put(ex->d_blocksum);
    pool.put(ex->d_list);
    pool.put(ex->d_keys);
    pool.put(ex->d_sorted);
    if (ex->h_ring) (void)hipHostFree(ex->h_ring);
    for (int i = 0; i < kRing; i++)
        if (ex->ring_ev[i]) (void)hipEventDestroy(ex->ring_ev[i]);
}

// Grow a step scratch buffer (the old one is kept if the new allocation fails).
template <class T>
Failure ensure_cap(gsim_ctx ctx, Executor *ex, T *&buf, int64_t &cap, int64_t need) {
    if (need <= cap) return kOk;
    const int64_t ncap = std::max<int64_t>(need, std::max<int64_t>(2 * cap, 1024));
    T *nbuf = pool_get<T>(*ctx->pool, ncap);
    if (!nbuf) return fail(GSIM_E_OOM, "no device memory for step scratch (%lld entries)", (long long)ncap);
    HIP_TRY(hipStreamSynchronize(ex->stream));  // queued steps may still read the old buffer
    ctx->pool->put(buf);
    buf = nbuf;
    cap = ncap;
    return kOk;
}

// Work lists, their keys and the two sorted lists, for `items` gates per step.
Failure ensure_lists(gsim_ctx ctx, Executor *ex, int64_t items) {
    if (items <= ex->list_cap) return kOk;
    const int64_t L = std::max<int64_t>(items, std::max<int64_t>(2 * ex->list_cap, 1024));
    Pool &pool = *ctx->pool;
    uint64_t *nlist = pool_get<uint64_t>(pool, kNumLists * L);
    uint64_t *nkeys = pool_get<uint64_t>(pool, kListLane * L);
    uint64_t *nsorted = pool_get<uint64_t>(pool, kVariants * L);
    if (!nlist || !nkeys || !nsorted) {
        pool.put(nlist);
        pool.put(nkeys);
        pool.put(nsorted);
        return fail(GSIM_E_OOM, "no device memory for step work lists (%lld entries)", (long long)L);
    }
    HIP_TRY(hipStreamSynchronize(ex->stream));  // queued steps may still read the old lists
    pool.put(ex->d_list);
    pool.put(ex->d_keys);
    pool.put(ex->d_sorted);
    ex->d_list = nlist;
    ex->d_keys = nkeys;
    ex->d_sorted = nsorted;
    ex->list_cap = L;
    return kOk;
}

// ---- jobs ----------------------------------------------------------------------

void free_job_buffers(gsim_ctx ctx, Job *j) {
    Pool &pool = *ctx->pool;
    if (j->d_K) ctx->arenas_held--;
    pool.put(j->d_off);
    pool.put(j->d_len);
    pool.put(j->d_partial);
    pool.put(j->d_src_off);
    pool.put(j->d_K);
    pool.put(j->d_state);
    pool.put(j->d_pend);
    pool.put(j->d_queue);
    pool.put(j->d_ctl);
    pool.put(j->d_sync);
    pool.put(j->d_desc);
    j->d_desc = nullptr;
    j->d_off = j->d_len = j->d_partial = j->d_src_off = nullptr;
    j->d_K = nullptr;
    j->d_state = nullptr;
    j->d_pend = j->d_queue = nullptr;
    j->d_ctl = nullptr;
    j->d_sync = nullptr;
}

void destroy_job(gsim_ctx ctx, Job *j) {
    if (j->phase != kQueued && j->ev_done) (void)hipEventSynchronize(j->ev_done);
    if (j->ex) {
        auto &act = j->ex->active;
        act.erase(std::remove(act.begin(), act.end(), j), act.end());
        auto &q = j->ex->queue;
        q.erase(std::remove(q.begin(), q.end(), j), q.end());
        if (j->phase == kActive) (void)hipStreamSynchronize(j->ex->stream);
    }
    if (j->nl) j->nl->active_jobs--;
    free_job_buffers(ctx, j);
    ctx->pinned.put(j->h_state);
    ctx->pinned.put(j->h_desc);
    j->h_desc = nullptr;
    ctx->pinned.put(j->h_src_off);
    ctx->pinned.put(j->h_t);
    ctx->pinned.put(j->h_v);
    j->h_src_off = j->h_t = nullptr;
    j->h_v = nullptr;
    if (j->ev_start) (void)hipEventDestroy(j->ev_start);
    if (j->ev_end) (void)hipEventDestroy(j->ev_end);
    if (j->ev_done) (void)hipEventDestroy(j->ev_done);
    j->timing.clear();
    j->h_state = nullptr;
    j->ev_start = j->ev_end = j->ev_done = nullptr;
}

int64_t default_capacity(const Netlist &nl, int64_t n_in) {
    double est;
    if (nl.arena_per_input > 0.0) {
        // 1.5x the largest arena use per input transition seen on this netlist
        est = 1.5 * nl.arena_per_input * (double)n_in + 4096.0;
    } else {
        // twice the pin-read volume of a circuit whose every net is as long as
        // the mean source waveform, plus the sources (in transitions)
        const double mean = nl.S > 0 ? (double)n_in / (double)nl.S : 0.0;
        est = (double)n_in + 2.0 * (double)nl.P * mean + 1024.0;
    }
    return (int64_t)std::min(est, 9.0e18);
}

// Create a queued job: host stimuli are staged on the device now (the caller's
// arrays may go away when the call returns); device stimuli are used in place.
// Automatic schedule (GSIM_OPT_SCHEDULE = 2): the dependency-driven launch
// wins on small netlists, where the level chain is launch-bound, and on
// uneven source activity (measured on MI355X: the 1M-gate mid netlist is
// faster level by level up to WCV 2 and dependency-driven from WCV 3; uniform
// jobs switch between 30k and 100k gates at 60 levels). src_off: the host
// copy of the source offsets, or null when they live on the device.
bool prefer_dependency_driven(const Netlist &nl, const int64_t *src_off) {
    if (nl.G < int64_t(800) * std::max<int64_t>(nl.n_levels, 1)) return true;
    if (!src_off || nl.S == 0) return false;
    double sum = 0.0, sq = 0.0;
    for (int64_t s = 0; s < nl.S; s++) {
        const double n = (double)(src_off[s + 1] - src_off[s]);
        sum += n;
        sq += n * n;
    }
    const double mean = sum / (double)nl.S;
    if (mean <= 0.0) return false;
    const double var = sq / (double)nl.S - mean * mean;
    return std::sqrt(var > 0.0 ? var : 0.0) / mean >= 2.5;
}

// Host stimuli of one job copied into pinned staging.
struct HostStim {
    int64_t *src_off = nullptr, *t = nullptr;
    uint8_t *v = nullptr;
    int64_t n_in = 0;
};

void stage_free(gsim_ctx ctx, HostStim *hs) {
    ctx->pinned.put(hs->src_off);
    ctx->pinned.put(hs->t);
    ctx->pinned.put(hs->v);
    *hs = HostStim{};
}

// Pinned staging for S sources and n_in transitions (the pinned cache is not
// shared across threads: call from the caller's thread).
Failure stage_alloc(gsim_ctx ctx, int64_t S, int64_t n_in, HostStim *hs) {
    hs->n_in = n_in;
    hs->src_off = (int64_t *)ctx->pinned.get(sizeof(int64_t) * ((size_t)S + 1));
    hs->t = (int64_t *)ctx->pinned.get(sizeof(int64_t) * (size_t)std::max<int64_t>(n_in, 1));
    hs->v = (uint8_t *)ctx->pinned.get((size_t)std::max<int64_t>(n_in, 1));
    if (!hs->src_off || !hs->t || !hs->v) {
        stage_free(ctx, hs);
        return fail(GSIM_E_OOM, "no pinned host memory to hold the stimuli");
    }
    return kOk;
}

void parallel_copy(void *dst, const void *src, size_t bytes);

// threads: whether the copies may use host threads of their own
void stage_copy(int64_t S, const int64_t *src_off, const int64_t *t, const uint8_t *v, HostStim *hs,
                bool threads) {
    std::memcpy(hs->src_off, src_off, sizeof(int64_t) * ((size_t)S + 1));
    if (hs->n_in > 0) {
        auto copy = threads ? parallel_copy : [](void *d, const void *s, size_t n) { std::memcpy(d, s, n); };
        copy(hs->t, t, sizeof(int64_t) * (size_t)hs->n_in);
        copy(hs->v, v, (size_t)hs->n_in);
    }
}

// fn(i) for i in [0, n) on up to 16 host threads (fewer if none can start).
template <typename Fn>
void parallel_for(int64_t n, Fn fn) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t nt = std::min<int64_t>({16, (int64_t)hw, n});
    std::atomic<int64_t> next{0};
    auto work = [&] {
        for (int64_t i = next++; i < n; i = next++) fn(i);
    };
    std::vector<std::thread> pool;
    try {
        for (int64_t k = 1; k < nt; k++) pool.emplace_back(work);
    } catch (...) {  // no more threads: fewer helpers
    }
    work();
    for (auto &th : pool) th.join();
}

// validate_stimulus over ranges of sources on host threads, for large
// stimuli; the first failing source is reported, as by the serial check
// (which also handles offsets that are not increasing).
Failure validate_stimulus_mt(int64_t S, const int64_t *src_off, const int64_t *t, const uint8_t *v,
                             int64_t max_path_delay) {
    constexpr int64_t kMinParallel = int64_t(1) << 20;  // transitions
    if (!src_off || src_off[0] != 0 || S < 64 || src_off[S] < kMinParallel)
        return validate_stimulus(S, src_off, t, v, max_path_delay);
    for (int64_t s = 0; s < S; s++)
        if (src_off[s + 1] < src_off[s]) return validate_stimulus(S, src_off, t, v, max_path_delay);
    constexpr int64_t kParts = 64;
    std::vector<Failure> part((size_t)kParts, kOk);
    parallel_for(kParts, [&](int64_t c) {
        part[c] = validate_sources(S * c / kParts, S * (c + 1) / kParts, src_off, t, v, max_path_delay);
    });
    for (const Failure &f : part)
        if (f.st != GSIM_OK) return f;
    return kOk;
}

// A job over staged host stimuli (hs, taken over by the job) or over device
// arrays, queued on the executor.
Failure queue_job(gsim_ctx ctx, gsim_netlist nlh, Netlist &nl, Executor *ex, HostStim *hs,
                  const int64_t *dev_src_off, const int64_t *dev_t, const uint8_t *dev_v, int64_t n_in,
                  Job **out) {
    auto j = std::make_unique<Job>();
    j->nl_id = nlh;
    j->nl = &nl;
    j->ex = ex;
    j->n_in = n_in;
    j->capacity_request = ctx->opt_arena;
    const int schedule = nl.schedule >= 0 ? nl.schedule : ctx->opt_schedule;
    j->dataflow = schedule == 1 || (schedule == 2 && prefer_dependency_driven(nl, hs ? hs->src_off : nullptr));
    j->levelsync = schedule == 3;
    if (hs) {
        j->h_src_off = hs->src_off;
        j->h_t = hs->t;
        j->h_v = hs->v;
        *hs = HostStim{};
    } else {
        j->dev_src_off = dev_src_off;
        j->dev_t = dev_t;
        j->dev_v = dev_v;
    }
    j->id = ctx->next_id++;
    nl.active_jobs++;
    Job *raw = j.get();
    ctx->jobs[j->id] = std::move(j);
    ex->queue.push_back(raw);
    *out = raw;
    return kOk;
}

Failure submit(gsim_ctx ctx, gsim_netlist nlh, const int64_t *src_off, const int64_t *t, const uint8_t *v,
               bool device_arrays, int64_t n_in_device, int validate, hipStream_t stream, Job **out) {
    if (!src_off) return fail(GSIM_E_ARG, "null src_off");
    auto it = ctx->netlists.find(nlh);
    if (it == ctx->netlists.end()) return fail(GSIM_E_HANDLE, "unknown netlist handle %lld", (long long)nlh);
    Netlist &nl = *it->second;
    Failure f = set_device(ctx);
    if (f.st != GSIM_OK) return f;
    Executor *ex = nullptr;
    f = get_executor(ctx, stream, &ex);
    if (f.st != GSIM_OK) return f;
    int64_t n_in = 0;
    if (!device_arrays) {
        f = validate_stimulus_mt(nl.S, src_off, t, v, nl.max_path_delay);
        if (f.st != GSIM_OK) return f;
        n_in = src_off[nl.S];
    } else {
        n_in = n_in_device;
        if (n_in < 0 || (n_in > 0 && (!t || !v))) return fail(GSIM_E_ARG, "bad device stimulus");
        if (validate) {
            std::vector<int64_t> so(nl.S + 1), tt(n_in);
            std::vector<uint8_t> vv(n_in);
            HIP_TRY(hipStreamSynchronize(ex->stream));
            HIP_TRY(hipMemcpy(so.data(), src_off, sizeof(int64_t) * (size_t)(nl.S + 1), hipMemcpyDeviceToHost));
            if (so[nl.S] != n_in)
                return fail(GSIM_E_ARG, "src_off[S] = %lld but n_in = %lld", (long long)so[nl.S], (long long)n_in);
            if (n_in > 0) {
                HIP_TRY(hipMemcpy(tt.data(), t, sizeof(int64_t) * (size_t)n_in, hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(vv.data(), v, (size_t)n_in, hipMemcpyDeviceToHost));
            }
            f = validate_stimulus(nl.S, so.data(), tt.data(), vv.data(), nl.max_path_delay);
            if (f.st != GSIM_OK) return f;
        }
    }
    if (device_arrays) return queue_job(ctx, nlh, nl, ex, nullptr, src_off, t, v, n_in, out);
    HostStim hs;
    f = stage_alloc(ctx, nl.S, n_in, &hs);
    if (f.st != GSIM_OK) return f;
    stage_copy(nl.S, src_off, t, v, &hs, true);
    return queue_job(ctx, nlh, nl, ex, &hs, nullptr, nullptr, nullptr, n_in, out);
}

// Emit the work that closes a job after its last level.
Failure finish_job(Job *j, hipStream_t s) {
    HIP_TRY(hipEventRecord(j->ev_end, s));
    HIP_TRY(launch_count_out(j->d_len, j->nl->S, j->nl->G, j->d_partial, j->n_partial, j->d_state, s));
    HIP_TRY(hipMemcpyAsync(j->h_state, j->d_state, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(j->ev_done, s));
    j->phase = kEnqueued;
    return kOk;
}

// A job's step descriptor for one level, its sizing blocks starting at sblock_begin.
void fill_desc(gsim_ctx ctx, Job *j, int32_t level, int64_t sblock_begin, JobDesc &d) {
    const LevelRange &r = j->nl->levels[level];
    d.rec = j->nl->d_rec;
    d.S = j->nl->S;
    d.off = j->d_off;
    d.len = j->d_len;
    d.K = j->d_K;
    d.state = j->d_state;
    d.lvl_begin = r.begin;
    d.n_gates = r.n;
    d.sblock_begin = sblock_begin;
    d.lane_threshold = j->nl->lane_threshold >= 0 ? j->nl->lane_threshold : ctx->opt_lane_threshold;
    d.pad = 0;
    d.lut = j->nl->d_lut ? j->nl->d_lut : ctx->d_lut;
    d.edly = j->nl->d_edly;
}

// Every gate of an admitted job in one dependency-driven launch.
Failure enqueue_dataflow(gsim_ctx ctx, Job *j, hipStream_t s) {
    Netlist &nl = *j->nl;
    DfArgs a;
    std::memset(&a, 0, sizeof a);
    a.job.rec = nl.d_rec;
    a.job.S = nl.S;
    a.job.off = j->d_off;
    a.job.len = j->d_len;
    a.job.K = j->d_K;
    a.job.state = j->d_state;
    a.job.lut = nl.d_lut ? nl.d_lut : ctx->d_lut;
    a.job.edly = nl.d_edly;
    a.fo_off = nl.d_fo_off;
    a.fo = nl.d_fo;
    a.pend = j->d_pend;
    a.queue = j->d_queue;
    a.ctl = j->d_ctl;
    a.G = nl.G;
    a.n_first = nl.n_first;
    const int64_t n_waves = std::min<int64_t>(nl.G, ctx->n_waves_resident);
    // reservation granule: at most 1/16 of the arena left idle over all wavefronts
    a.chunk = std::min<int64_t>(int64_t(1) << 15, (j->capacity - j->n_in) / (16 * std::max<int64_t>(n_waves, 1)));
    // small jobs are latency-bound: one ticket per claim keeps every ready gate
    // on a wavefront of its own; large ones are bound by the claim counter and
    // by the fences, which a batch of ready gates shares
    a.tickets = nl.df_tickets > 0 ? (uint32_t)nl.df_tickets
                : ctx->opt_df_tickets > 0 ? (uint32_t)ctx->opt_df_tickets
                : nl.G < 16 * ctx->n_waves_resident ? 1u : 2u;
    HIP_TRY(launch_df_init(a, nl.d_pend0, s));
    std::shared_ptr<StepTiming> tm;
    if (ctx->opt_timing) {
        tm = std::make_shared<StepTiming>();
        HIP_TRY(hipEventCreate(&tm->a));
        HIP_TRY(hipEventCreate(&tm->b));
        HIP_TRY(hipEventRecord(tm->a, s));
    }
    HIP_TRY(launch_dataflow(a, n_waves, s));
    if (tm) {
        HIP_TRY(hipEventRecord(tm->b, s));
        j->timing.push_back(tm);
    }
    j->next_level = nl.n_levels;
    return finish_job(j, s);
}

// Every level of an admitted job in one launch with a device-wide barrier
// between levels. The grid is no larger than what is resident at once nor
// than the widest level, and the launch waits for the context's previous one
// (on whatever stream it ran).
Failure enqueue_levelsync(gsim_ctx ctx, Job *j, hipStream_t s) {
    Netlist &nl = *j->nl;
    LsArgs a;
    std::memset(&a, 0, sizeof a);
    a.job.rec = nl.d_rec;
    a.job.S = nl.S;
    a.job.off = j->d_off;
    a.job.len = j->d_len;
    a.job.K = j->d_K;
    a.job.state = j->d_state;
    a.job.lut = nl.d_lut ? nl.d_lut : ctx->d_lut;
    a.job.edly = nl.d_edly;
    a.level_off = nl.d_level_off;
    a.sync = j->d_sync;
    a.n_levels = nl.n_levels;
    const int64_t n_waves =
        std::max<int64_t>(1, std::min({ctx->n_waves_levelsync, nl.max_level_n, kLsMaxWaves}));
    a.chunk = std::min<int64_t>(int64_t(1) << 15, (j->capacity - j->n_in) / (16 * n_waves));
    if (!ctx->ls_event) HIP_TRY(hipEventCreateWithFlags(&ctx->ls_event, hipEventDisableTiming));
    else HIP_TRY(hipStreamWaitEvent(s, ctx->ls_event, 0));
    std::shared_ptr<StepTiming> tm;
    if (ctx->opt_timing) {
        tm = std::make_shared<StepTiming>();
        HIP_TRY(hipEventCreate(&tm->a));
        HIP_TRY(hipEventCreate(&tm->b));
        HIP_TRY(hipEventRecord(tm->a, s));
    }
    HIP_TRY(launch_levelsync(a, n_waves, s));
    HIP_TRY(hipEventRecord(ctx->ls_event, s));
    if (tm) {
        HIP_TRY(hipEventRecord(tm->b, s));
        j->timing.push_back(tm);
    }
    j->next_level = nl.n_levels;
    return finish_job(j, s);
}

// Allocate a queued job's device storage and pack its sources into the arena.
// Returns GSIM_E_OOM (and leaves the job queued) if the budget has no room.
Failure admit(gsim_ctx ctx, Executor *ex, Job *j) {
    Netlist &nl = *j->nl;
    Pool &pool = *ctx->pool;
    const int64_t N = nl.S + nl.G;
    {
        // step scratch for the active set with this job, before its arena
        int64_t sblocks = 0, items = 0;
        for (Job *a : ex->active) {
            sblocks += (a->nl->max_level_n + kSizeBlock - 1) / kSizeBlock;
            items += a->nl->max_level_n;
        }
        sblocks += (nl.max_level_n + kSizeBlock - 1) / kSizeBlock;
        items += nl.max_level_n;
        Failure f = ensure_cap(ctx, ex, ex->d_jobs, ex->jobs_cap, (int64_t)ex->active.size() + 1);
        if (f.st == GSIM_OK) f = ensure_cap(ctx, ex, ex->d_blocksum, ex->blocksum_cap, sblocks);
        if (f.st == GSIM_OK) f = ensure_lists(ctx, ex, items);
        if (f.st != GSIM_OK) return f;
    }
    j->n_partial = std::max<int64_t>(1, std::min<int64_t>(1024, (nl.G + 255) / 256));
    // host stimuli are uploaded into the arena itself: times over the first
    // n_in slots (packed in place), values as bytes in its last slots
    const int64_t staged = j->h_t ? j->n_in + (j->n_in + 7) / 8 + 1 : j->n_in;
    int64_t cap = j->capacity_request > 0 ? j->capacity_request : default_capacity(nl, j->n_in);
    cap = std::max(cap, staged);
    if (j->capacity_request <= 0) {
        // An automatic estimate that does not fit what the budget leaves waits
        // for memory; only when no other job holds an arena is a job started
        // with what is left (an overflow then re-runs it larger).
        const uint64_t room = pool.largest_free();
        const int64_t fit = (int64_t)(room / sizeof(uint64_t) * 90 / 100) - (int64_t)(N * 2 + 4096);
        if (cap > fit) {
            if (ctx->arenas_held > 0) return fail(GSIM_E_OOM, "waiting for device memory");
            cap = std::max(staged, fit);
        }
    }
    j->capacity = cap;
    j->d_off = pool_get<int64_t>(pool, N);
    j->d_len = pool_get<int64_t>(pool, N);
    j->d_partial = pool_get<int64_t>(pool, j->n_partial);
    j->d_state = pool_get<DevState>(pool, 1);
    j->d_K = pool_get<uint64_t>(pool, cap);
    if (j->h_t) j->d_src_off = pool_get<int64_t>(pool, nl.S + 1);
    if (j->dataflow) {
        j->d_pend = pool_get<int32_t>(pool, std::max<int64_t>(nl.G, 1));
        j->d_queue = pool_get<int32_t>(pool, std::max<int64_t>(nl.G, 1));
    }
    if (j->dataflow) j->d_ctl = pool_get<DfCtl>(pool, 1);
    if (j->levelsync) j->d_sync = pool_get<uint32_t>(pool, kLsSyncWords);
    if (!j->d_off || !j->d_len || !j->d_partial || !j->d_state || !j->d_K || (j->h_t && !j->d_src_off) ||
        (j->dataflow && (!j->d_pend || !j->d_queue || !j->d_ctl)) || (j->levelsync && !j->d_sync)) {
        pool.put(j->d_off); pool.put(j->d_len); pool.put(j->d_partial); pool.put(j->d_state); pool.put(j->d_K);
        pool.put(j->d_src_off);
        pool.put(j->d_pend); pool.put(j->d_queue); pool.put(j->d_ctl); pool.put(j->d_sync);
        j->d_off = j->d_len = j->d_partial = j->d_src_off = nullptr;
        j->d_pend = j->d_queue = nullptr;
        j->d_ctl = nullptr;
        j->d_sync = nullptr;
        j->d_state = nullptr;
        j->d_K = nullptr;
        return fail(GSIM_E_OOM, "no device memory for a job of %lld transitions of output storage", (long long)cap);
    }
    ctx->arenas_held++;
    if (!j->h_state) {
        j->h_state = (DevState *)ctx->pinned.get(sizeof(DevState));
        if (!j->h_state || hipEventCreate(&j->ev_start) != hipSuccess || hipEventCreate(&j->ev_end) != hipSuccess ||
            hipEventCreateWithFlags(&j->ev_done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GSIM_E_DEVICE, "event or pinned-memory creation failed");
        }
    }
    hipStream_t s = ex->stream;
    HIP_TRY(hipEventRecord(j->ev_start, s));
    const int64_t *src_off = j->dev_src_off, *src_t = j->dev_t;
    const uint8_t *src_v = j->dev_v;
    if (j->h_t) {
        uint8_t *vbytes = (uint8_t *)(j->d_K + (cap - (j->n_in + 7) / 8 - 1));
        HIP_TRY(hipMemcpyAsync(j->d_src_off, j->h_src_off, sizeof(int64_t) * (size_t)(nl.S + 1),
                               hipMemcpyHostToDevice, s));
        if (j->n_in > 0) {
            HIP_TRY(hipMemcpyAsync(j->d_K, j->h_t, sizeof(int64_t) * (size_t)j->n_in, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(vbytes, j->h_v, (size_t)j->n_in, hipMemcpyHostToDevice, s));
        }
        src_off = j->d_src_off;
        src_t = (const int64_t *)j->d_K;
        src_v = vbytes;
    }
    HIP_TRY(launch_init_sources(src_off, src_t, src_v, nl.S, j->n_in, j->d_off, j->d_len, j->d_K,
                                j->d_state, j->capacity, s));
    j->phase = kActive;
    j->next_level = 0;
    if (nl.n_levels == 0) return finish_job(j, s);
    if (j->dataflow) return enqueue_dataflow(ctx, j, s);
    if (j->levelsync) return enqueue_levelsync(ctx, j, s);
    // descriptors for the steps this job has alone (optional: skipped if no memory)
    const size_t desc_bytes = sizeof(JobDesc) * (size_t)nl.n_levels;
    if (!j->h_desc) j->h_desc = (JobDesc *)ctx->pinned.get(desc_bytes);
    j->d_desc = j->h_desc ? pool_get<JobDesc>(pool, nl.n_levels) : nullptr;
    if (j->d_desc) {
        for (int32_t l = 0; l < nl.n_levels; l++) {
            JobDesc &d = j->h_desc[l];
            std::memset(&d, 0, sizeof d);
            fill_desc(ctx, j, l, 0, d);
        }
        HIP_TRY(hipMemcpyAsync(j->d_desc, j->h_desc, desc_bytes, hipMemcpyHostToDevice, s));
    }
    ex->active.push_back(j);
    return kOk;
}

// Admit queued jobs that fit, first fit in submission order: a job that does
// not fit now does not hold back smaller ones behind it.
Failure admit_queued(gsim_ctx ctx, Executor *ex) {
    for (auto it = ex->queue.begin(); it != ex->queue.end() && (int)ex->active.size() < kMaxJobsPerStep;) {
        Job *j = *it;
        Failure f = admit(ctx, ex, j);
        if (f.st == GSIM_E_OOM) {
            ++it;
            continue;
        }
        it = ex->queue.erase(it);
        if (f.st != GSIM_OK) {
            j->failed = true;
            return f;
        }
    }
    return kOk;
}

// Enqueue one step: the next level of every active job.
Failure enqueue_step(gsim_ctx ctx, Executor *ex) {
    std::vector<Job *> &act = ex->active;
    if (act.empty()) return kOk;
    const int slot = (int)(ex->steps % kRing);
    if (ex->ring_used[slot]) HIP_TRY(hipEventSynchronize(ex->ring_ev[slot]));
    JobDesc *desc = ex->h_ring + (size_t)slot * kMaxJobsPerStep;
    const int n = (int)act.size();
    int64_t n_sblocks = 0, n_items = 0, n_lane = 0;
    int64_t n_list[kNumLists] = {};
    for (int i = 0; i < n; i++) {
        Job *j = act[i];
        const LevelRange &r = j->nl->levels[j->next_level];
        JobDesc &d = desc[i];
        fill_desc(ctx, j, j->next_level, n_sblocks, d);
        n_sblocks += (r.n + kSizeBlock - 1) / kSizeBlock;
        n_items += r.n;
        for (int c = 0; c < kNumLists; c++) n_list[c] += r.n_list[c];
        // the lane list takes the gates whose delays need it, plus any gate that
        // reads fewer than lane_threshold transitions
        n_lane += d.lane_threshold > 0 ? r.n : r.n_list[kListLane];
    }
    Failure f = ensure_cap(ctx, ex, ex->d_jobs, ex->jobs_cap, n);
    if (f.st == GSIM_OK) f = ensure_cap(ctx, ex, ex->d_blocksum, ex->blocksum_cap, n_sblocks);
    if (f.st == GSIM_OK) f = ensure_lists(ctx, ex, n_items);
    if (f.st != GSIM_OK) return f;
    hipStream_t s = ex->stream;
    // a job alone in the step uses its descriptor table from admission (the
    // lane threshold is the one in force at admission)
    const JobDesc *step_jobs = ex->d_jobs;
    if (n == 1 && act[0]->d_desc) {
        step_jobs = act[0]->d_desc + act[0]->next_level;
    } else {
        HIP_TRY(hipMemcpyAsync(ex->d_jobs, desc, sizeof(JobDesc) * (size_t)n, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipEventRecord(ex->ring_ev[slot], s));
    ex->ring_used[slot] = true;
    StepArgs a;
    a.jobs = step_jobs;
    a.n_jobs = n;
    a.pad = 0;
    a.n_sblocks = n_sblocks;
    a.blocksum = ex->d_blocksum;
    for (int c = 0; c < kNumLists; c++) a.list[c] = ex->d_list + (size_t)c * ex->list_cap;
    for (int c = 0; c < kListLane; c++) a.key[c] = ex->d_keys + (size_t)c * ex->list_cap;
    for (int w = 0; w < kVariants; w++) a.sorted[w] = ex->d_sorted + (size_t)w * ex->list_cap;
    a.count = ex->d_counts + ex->parity * kCountWords;
    a.next_count = ex->d_counts + (1 - ex->parity) * kCountWords;
    HIP_TRY(launch_size(a, s));
    HIP_TRY(launch_sort_lists(a, n_list, s));
    std::shared_ptr<StepTiming> tm;
    if (ctx->opt_timing) {
        tm = std::make_shared<StepTiming>();
        HIP_TRY(hipEventCreate(&tm->a));
        HIP_TRY(hipEventCreate(&tm->b));
        HIP_TRY(hipEventRecord(tm->a, s));
    }
    // the step's jobs share its launches: the first job's netlist sets the form
    const int form = act[0]->nl->form >= 0 ? act[0]->nl->form : ctx->opt_form;
    for (int v = 0; v < kVariants; v++) HIP_TRY(launch_eval_wave(a, v, n_list + wave_list(v, 1), form, s));
    HIP_TRY(launch_eval_lane(a, n_lane, s));
    if (tm) HIP_TRY(hipEventRecord(tm->b, s));
    ex->parity ^= 1;
    ex->steps++;
    std::vector<Job *> still;
    still.reserve(n);
    for (Job *j : act) {
        if (tm) j->timing.push_back(tm);
        j->next_level++;
        if (j->next_level == j->nl->n_levels) {
            f = finish_job(j, s);
            if (f.st != GSIM_OK) return f;
        } else {
            still.push_back(j);
        }
    }
    act.swap(still);
    return kOk;
}

// One scheduling pass: admit what fits, enqueue one step, then block until at
// most `max_ahead` steps are unfinished on the device (0: no bound).
Failure drive(gsim_ctx ctx, Executor *ex, int max_ahead) {
    Failure f = admit_queued(ctx, ex);
    if (f.st != GSIM_OK) return f;
    f = enqueue_step(ctx, ex);
    if (f.st != GSIM_OK) return f;
    if (max_ahead > 0 && ex->steps > max_ahead) {
        const int64_t older = ex->steps - 1 - max_ahead;
        HIP_TRY(hipEventSynchronize(ex->ring_ev[older % kRing]));
    }
    return kOk;
}

// Drive until every level of `j` is enqueued.
Failure drive_until_enqueued(gsim_ctx ctx, Job *j) {
    Executor *ex = j->ex;
    while (j->phase != kEnqueued && !j->failed) {
        const int64_t before = ex->steps;
        const size_t queued = ex->queue.size();
        Failure f = drive(ctx, ex, 0);
        if (f.st != GSIM_OK) return f;
        if (ex->steps == before && ex->queue.size() == queued && j->phase == kQueued)
            return fail(GSIM_E_OOM, "job %lld cannot be admitted: the HBM budget is held by unreleased jobs",
                        (long long)j->id);
    }
    return kOk;
}

Failure find_job(gsim_ctx ctx, gsim_job id, Job **out) {
    auto it = ctx->jobs.find(id);
    if (it == ctx->jobs.end()) return fail(GSIM_E_HANDLE, "unknown job handle %lld", (long long)id);
    *out = it->second.get();
    return kOk;
}

// A job a failed call created: freed, and the caller's handle cleared, so the
// failure leaves nothing behind (a job that could not be admitted would
// otherwise stay queued).
void discard_job(gsim_ctx ctx, gsim_job *out) {
    auto it = ctx->jobs.find(*out);
    if (it != ctx->jobs.end()) {
        destroy_job(ctx, it->second.get());
        ctx->jobs.erase(it);
    }
    *out = 0;
}

constexpr int kMaxRetries = 6;

// A finished job whose automatically sized arena overflowed goes back to the
// front of its executor's queue with twice the storage; returns true if so.
bool requeue_if_overflowed(gsim_ctx ctx, Job *j) {
    if (!j->h_state->overflow || ctx == nullptr) return false;
    if (j->capacity_request > 0 && j->retries == 0) return false;  // caller-sized: report it
    if (j->retries >= kMaxRetries) return false;
    j->retries++;
    j->capacity_request = 2 * j->capacity;
    // every device buffer of the run goes back to the pool: admission
    // allocates them all again (sources, descriptors, dependency-driven state)
    free_job_buffers(ctx, j);
    j->timing.clear();
    j->phase = kQueued;
    j->ex->queue.push_front(j);
    return true;
}

// Record what a finished job taught about arena use on its netlist.
void learn(Job *j) {
    if (!j->h_state->overflow && j->n_in > 0)
        j->nl->arena_per_input = std::max(j->nl->arena_per_input,
                                          (double)j->h_state->arena_top / (double)j->n_in);
}

Failure wait_job(gsim_ctx ctx, Job *j) {
    while (!j->waited && !j->failed) {
        Failure f = set_device(ctx);
        if (f.st != GSIM_OK) return f;
        f = drive_until_enqueued(ctx, j);
        if (f.st != GSIM_OK) return f;
        HIP_TRY(hipEventSynchronize(j->ev_done));
        if (requeue_if_overflowed(ctx, j)) continue;
        j->waited = true;
        learn(j);
        if (j->h_state->overflow) {
            j->failed = true;
            free_job_buffers(ctx, j);
        }
    }
    if (j->failed)
        return fail(GSIM_E_OOM, "output arena of %lld transitions overflowed or could not be allocated "
                    "(after %d automatic retries); set GSIM_OPT_ARENA_TRANSITIONS larger",
                    (long long)j->capacity, (int)j->retries);
    if (j->h_state->check_error == 3)
        return fail(GSIM_E_DEVICE, j->levelsync ? "the level-barrier schedule's barrier wait timed out"
                                                : "the dependency-driven schedule made no progress and stopped");
    if (j->h_state->check_error == 4)
        return fail(GSIM_E_DEVICE, "a gate's evaluation made no progress (an input waveform out of order)");
    if (j->h_state->check_error)
        return fail(GSIM_E_DEVICE, "internal consistency check failed (code %d)", j->h_state->check_error);
    return kOk;
}

// ---- the no-allocation run ---------------------------------------------------------

// Where each step buffer of a level-by-level run of `nl` sits in the static
// scratch array (byte offsets): the job state, the two step-counter halves,
// the partial sums of the output count, one descriptor per level, the sizing
// block sums, and the work lists, keys and sorted lists, each sized for the
// largest level (the lane list for every gate of a level when a lane
// threshold may move gates there).
struct NoAllocLayout {
    size_t state = 0, counts = 0, partial = 0, desc = 0, blocksum = 0;
    size_t list[kNumLists] = {}, key[kListLane] = {}, sorted[kVariants] = {};
    size_t total = 0;
    int64_t n_partial = 0;
};

NoAllocLayout noalloc_layout(const Netlist &nl, int32_t lane_threshold) {
    int64_t cap[kNumLists] = {}, scap[kVariants] = {};
    for (const LevelRange &r : nl.levels) {
        for (int c = 0; c < kNumLists; c++) cap[c] = std::max(cap[c], r.n_list[c]);
        for (int v = 0; v < kVariants; v++) {
            int64_t n = 0;
            for (int k = 1; k <= 4; k++) n += r.n_list[wave_list(v, k)];
            scap[v] = std::max(scap[v], n);
        }
    }
    if (lane_threshold > 0) cap[kListLane] = nl.max_level_n;
    NoAllocLayout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at += (bytes + 255) / 256 * 256;
        return here;
    };
    L.n_partial = std::max<int64_t>(1, std::min<int64_t>(1024, (nl.G + 255) / 256));
    L.state = take(sizeof(DevState));
    L.counts = take(sizeof(uint32_t) * 2 * kCountWords);
    L.partial = take(sizeof(int64_t) * (size_t)L.n_partial);
    L.desc = take(sizeof(JobDesc) * (size_t)nl.n_levels);
    L.blocksum = take(sizeof(int64_t) * (size_t)((nl.max_level_n + kSizeBlock - 1) / kSizeBlock));
    for (int c = 0; c < kNumLists; c++) L.list[c] = take(sizeof(uint64_t) * (size_t)cap[c]);
    for (int c = 0; c < kListLane; c++) L.key[c] = take(sizeof(uint64_t) * (size_t)cap[c]);
    for (int v = 0; v < kVariants; v++) L.sorted[v] = take(sizeof(uint64_t) * (size_t)scap[v]);
    L.total = at;
    return L;
}

// Every level of `nl` over the caller's buffers and the scratch array, on
// stream `s`, in the launches of the level schedule. Allocates nothing.
Failure run_noalloc(gsim_ctx ctx, const Netlist &nl, const int64_t *d_src_off, const int64_t *d_t,
                    const uint8_t *d_v, int64_t n_in, int64_t *d_off, int64_t *d_len, uint64_t *d_arena,
                    int64_t arena_cap, int64_t *d_result, hipStream_t s) {
    uint8_t *base = (uint8_t *)noalloc_scratch(ctx->device);
    if (!base) return fail(GSIM_E_DEVICE, "the no-allocation scratch of device %d was not set up", ctx->device);
    const int32_t thr = nl.lane_threshold >= 0 ? nl.lane_threshold : ctx->opt_lane_threshold;
    const NoAllocLayout L = noalloc_layout(nl, thr);
    if (L.total > kNoAllocScratchBytes)
        return fail(GSIM_E_ARG,
                    "the netlist needs %llu bytes of step scratch (largest level %lld gates, %d levels); "
                    "the no-allocation entry point holds %llu: use sim_run_device",
                    (unsigned long long)L.total, (long long)nl.max_level_n, (int)nl.n_levels,
                    (unsigned long long)kNoAllocScratchBytes);
    DevState *state = (DevState *)(base + L.state);
    uint32_t *counts = (uint32_t *)(base + L.counts);
    JobDesc *desc = (JobDesc *)(base + L.desc);
    HIP_TRY(launch_clear_u32(counts, 2 * kCountWords, s));
    HIP_TRY(launch_init_sources(d_src_off, d_t, d_v, nl.S, n_in, d_off, d_len, d_arena, state, arena_cap, s));
    for (int32_t l0 = 0; l0 < nl.n_levels; l0 += kDescBatch) {
        DescBatch b;
        std::memset(&b, 0, sizeof b);
        b.n = std::min<int32_t>(kDescBatch, nl.n_levels - l0);
        b.dst = desc + l0;
        for (int32_t i = 0; i < b.n; i++) {
            const LevelRange &r = nl.levels[l0 + i];
            JobDesc &d = b.d[i];
            d.rec = nl.d_rec;
            d.S = nl.S;
            d.off = d_off;
            d.len = d_len;
            d.K = d_arena;
            d.state = state;
            d.lvl_begin = r.begin;
            d.n_gates = r.n;
            d.sblock_begin = 0;
            d.lane_threshold = thr;
            d.lut = nl.d_lut ? nl.d_lut : ctx->d_lut;
            d.edly = nl.d_edly;
        }
        HIP_TRY(launch_write_descs(b, s));
    }
    for (int32_t l = 0; l < nl.n_levels; l++) {
        const LevelRange &r = nl.levels[l];
        StepArgs a;
        std::memset(&a, 0, sizeof a);
        a.jobs = desc + l;
        a.n_jobs = 1;
        a.n_sblocks = (r.n + kSizeBlock - 1) / kSizeBlock;
        a.blocksum = (int64_t *)(base + L.blocksum);
        for (int c = 0; c < kNumLists; c++) a.list[c] = (uint64_t *)(base + L.list[c]);
        for (int c = 0; c < kListLane; c++) a.key[c] = (uint64_t *)(base + L.key[c]);
        for (int v = 0; v < kVariants; v++) a.sorted[v] = (uint64_t *)(base + L.sorted[v]);
        a.count = counts + (l & 1) * kCountWords;
        a.next_count = counts + (1 - (l & 1)) * kCountWords;
        const int64_t n_lane = thr > 0 ? r.n : r.n_list[kListLane];
        HIP_TRY(launch_size(a, s));
        HIP_TRY(launch_sort_lists(a, r.n_list, s));
        for (int v = 0; v < kVariants; v++)
            HIP_TRY(launch_eval_wave(a, v, r.n_list + wave_list(v, 1), nl.form >= 0 ? nl.form : ctx->opt_form, s));
        HIP_TRY(launch_eval_lane(a, n_lane, s));
    }
    HIP_TRY(launch_count_out(d_len, nl.S, nl.G, (int64_t *)(base + L.partial), L.n_partial, state, s));
    HIP_TRY(launch_run_result(state, d_result, s));
    return kOk;
}

// Internal ids of the requested nets (all nets in id order when nets is null).
Failure internal_ids(const Netlist &nl, const int64_t *nets, int64_t n, std::vector<int64_t> &ids) {
    const int64_t N = nl.S + nl.G;
    ids.resize(n);
    for (int64_t i = 0; i < n; i++) {
        const int64_t u = nets ? nets[i] : i;
        if (u < 0 || u >= N) return fail(GSIM_E_ARG, "net %lld out of range", (long long)u);
        ids[i] = u < nl.S ? u : nl.S + nl.internal_of_user[u - nl.S];
    }
    return kOk;
}

// Arena offset and length of each requested net, gathered on the device in
// batches of kStageBatch (one small copy each way per batch).
Failure net_meta(gsim_ctx ctx, Job *j, const std::vector<int64_t> &ids, std::vector<int64_t> &off,
                 std::vector<int64_t> &len) {
    const int64_t n = (int64_t)ids.size();
    off.resize(n);
    len.resize(n);
    hipStream_t s = ctx->stream;
    int64_t *d_ids = ctx->d_stage_meta, *d_off = d_ids + kStageBatch, *d_len = d_off + kStageBatch;
    for (int64_t i0 = 0; i0 < n; i0 += kStageBatch) {
        const int64_t m = std::min<int64_t>(kStageBatch, n - i0);
        HIP_TRY(hipMemcpyAsync(d_ids, ids.data() + i0, sizeof(int64_t) * (size_t)m, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_gather_meta(d_ids, m, j->d_off, j->d_len, d_off, d_len, s));
        HIP_TRY(hipMemcpyAsync(off.data() + i0, d_off, sizeof(int64_t) * (size_t)m, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(len.data() + i0, d_len, sizeof(int64_t) * (size_t)m, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return kOk;
}

// True for memory from hipHostMalloc (or registered with HIP); pageable
// memory reads as unregistered (or the query fails, and its error is cleared).
bool is_pinned_host(const void *ptr) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeHost;
}

// memcpy split over up to 16 threads for large copies out of pinned staging.
void parallel_copy(void *dst, const void *src, size_t bytes) {
    constexpr size_t kMinPerThread = size_t(4) << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({16, hw, std::max<size_t>(1, bytes / kMinPerThread)});
    if (nt <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t part = (bytes + nt - 1) / nt;
    std::vector<std::thread> pool;
    size_t started = 1;  // parts [1, started) have a thread; the rest are copied here
    try {
        pool.reserve(nt - 1);
        for (size_t k = 1; k < nt; k++, started++) {
            const size_t a = k * part, e = std::min(bytes, a + part);
            if (a >= e) break;
            pool.emplace_back([=] { std::memcpy((char *)dst + a, (const char *)src + a, e - a); });
        }
    } catch (...) {  // no more threads: fewer helpers
    }
    std::memcpy(dst, src, std::min(bytes, part));
    for (size_t k = started; k < nt; k++) {
        const size_t a = k * part, e = std::min(bytes, a + part);
        if (a < e) std::memcpy((char *)dst + a, (const char *)src + a, e - a);
    }
    for (auto &t : pool) t.join();
}

// Pinned host staging (two batches) and the events of one fetch call.
struct FetchStaging {
    gsim_ctx ctx;
    int64_t *h_t[2] = {nullptr, nullptr};
    uint8_t *h_v[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool good = true;
    FetchStaging(gsim_ctx c, bool direct) : ctx(c) {
        for (int p = 0; p < 2; p++) {
            if (hipEventCreateWithFlags(&ev[p], hipEventDisableTiming) != hipSuccess) {
                ev[p] = nullptr;
                good = false;
            }
            if (direct) continue;
            h_t[p] = (int64_t *)ctx->pinned.get(sizeof(int64_t) * (size_t)kStage);
            h_v[p] = (uint8_t *)ctx->pinned.get((size_t)kStage);
            if (!h_t[p] || !h_v[p]) good = false;
        }
    }
    ~FetchStaging() {
        // the stream may still copy into the staging buffers after an error
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        for (int p = 0; p < 2; p++) {
            ctx->pinned.put(h_t[p]);
            ctx->pinned.put(h_v[p]);
            if (ev[p]) (void)hipEventDestroy(ev[p]);
        }
    }
    bool ok() const { return good; }
};

Failure fetch(gsim_ctx ctx, Job *j, const int64_t *nets, int64_t n, int64_t *out_off, int64_t *out_t,
              uint8_t *out_v, int64_t cap) {
    Failure f = wait_job(ctx, j);
    if (f.st != GSIM_OK) return f;
    Netlist &nl = *j->nl;
    if (!nets) n = nl.S + nl.G;
    if (n < 0 || !out_off) return fail(GSIM_E_ARG, "bad net list");
    std::vector<int64_t> ids, off, len;
    f = internal_ids(nl, nets, n, ids);
    if (f.st == GSIM_OK) f = net_meta(ctx, j, ids, off, len);
    if (f.st != GSIM_OK) return f;
    out_off[0] = 0;
    for (int64_t i = 0; i < n; i++) out_off[i + 1] = out_off[i] + len[i];
    if (!out_t) return kOk;
    if (!out_v) return fail(GSIM_E_ARG, "null out_v");
    if (cap < out_off[n]) return fail(GSIM_E_ARG, "capacity %lld < %lld transitions", (long long)cap, (long long)out_off[n]);
    // Gather in batches through two device staging buffers; a net that does
    // not fit in what is left of a batch is split across batches. Batch b is
    // gathered and copied to the host while the host copies batch b-1 out of
    // its pinned staging buffer into the caller's memory (several threads);
    // if the caller's buffers are pinned themselves, they are copied to
    // directly.
    const bool direct = is_pinned_host(out_t) && is_pinned_host(out_v);
    FetchStaging fs(ctx, direct);
    if (!fs.ok()) return fail(GSIM_E_OOM, "no pinned host memory for the fetch staging buffers");
    const int64_t stage = kStage, max_batch = kStageBatch;
    hipStream_t s = ctx->stream;
    std::vector<int64_t> meta[2] = {std::vector<int64_t>(3 * max_batch), std::vector<int64_t>(3 * max_batch)};
    int64_t pend_dst[2] = {0, 0}, pend_n[2] = {0, 0};
    bool pending[2] = {false, false};
    auto drain = [&](int p) -> Failure {
        if (!pending[p]) return kOk;
        pending[p] = false;
        HIP_TRY(hipEventSynchronize(fs.ev[p]));
        if (!direct && pend_n[p] > 0) {
            parallel_copy(out_t + pend_dst[p], fs.h_t[p], sizeof(int64_t) * (size_t)pend_n[p]);
            parallel_copy(out_v + pend_dst[p], fs.h_v[p], (size_t)pend_n[p]);
        }
        return kOk;
    };
    int64_t i = 0, done_in_net = 0;  // next net, transitions of it already copied
    for (int b = 0; i < n; b++) {
        const int p = b & 1;
        int64_t nb = 0, acc = 0;
        const int64_t dst0 = out_off[i] + done_in_net;
        int64_t *m = meta[p].data();
        while (i < n && nb < max_batch && acc < stage) {
            const int64_t li = len[i] - done_in_net;
            const int64_t take = std::min(li, stage - acc);
            m[nb] = off[i] + done_in_net;
            m[max_batch + nb] = take;
            m[2 * max_batch + nb] = acc;
            nb++;
            acc += take;
            if (take == li) {
                i++;
                done_in_net = 0;
            } else {
                done_in_net += take;
            }
        }
        int64_t *d_meta = ctx->d_stage_meta + p * 3 * max_batch;
        int64_t *d_st = ctx->d_stage_t + p * stage;
        uint8_t *d_sv = ctx->d_stage_v + p * stage;
        HIP_TRY(hipMemcpyAsync(d_meta, m, sizeof(int64_t) * 3 * (size_t)max_batch, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_gather(d_meta, d_meta + max_batch, d_meta + 2 * max_batch, nb, j->d_K, d_st, d_sv, s));
        if (acc > 0) {
            HIP_TRY(hipMemcpyAsync(direct ? (void *)(out_t + dst0) : (void *)fs.h_t[p], d_st,
                                   sizeof(int64_t) * (size_t)acc, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(direct ? (void *)(out_v + dst0) : (void *)fs.h_v[p], d_sv, (size_t)acc,
                                   hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipEventRecord(fs.ev[p], s));
        pend_dst[p] = dst0;
        pend_n[p] = acc;
        pending[p] = true;
        f = drain(p ^ 1);  // the previous batch, while this one is copied
        if (f.st != GSIM_OK) return f;
    }
    f = drain(0);
    if (f.st == GSIM_OK) f = drain(1);
    return f;
}

Failure fetch_hashes(gsim_ctx ctx, Job *j, const int64_t *nets, int64_t n, uint64_t *out) {
    Failure f = wait_job(ctx, j);
    if (f.st != GSIM_OK) return f;
    Netlist &nl = *j->nl;
    if (!nets) n = nl.S + nl.G;
    if (n < 0 || (n > 0 && !out)) return fail(GSIM_E_ARG, "bad net list");
    std::vector<int64_t> ids;
    f = internal_ids(nl, nets, n, ids);
    if (f.st != GSIM_OK) return f;
    hipStream_t s = ctx->stream;
    int64_t *d_ids = ctx->d_stage_meta, *d_off = d_ids + kStageBatch, *d_len = d_off + kStageBatch;
    uint64_t *d_h = (uint64_t *)ctx->d_stage_t;
    for (int64_t i0 = 0; i0 < n; i0 += kStageBatch) {
        const int64_t m = std::min<int64_t>(kStageBatch, n - i0);
        HIP_TRY(hipMemcpyAsync(d_ids, ids.data() + i0, sizeof(int64_t) * (size_t)m, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_gather_meta(d_ids, m, j->d_off, j->d_len, d_off, d_len, s));
        HIP_TRY(launch_hash(d_off, d_len, m, j->d_K, d_h, s));
        HIP_TRY(hipMemcpyAsync(out + i0, d_h, sizeof(uint64_t) * (size_t)m, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return kOk;
}

}  // namespace
// ===========================================================================
// C ABI.

namespace {
// The C entry points never throw: an exception from the host runtime (out of
// host memory, a thread that could not start) becomes a status, recorded on
// the context when there is one.
gsim_status exception_status(gsim_ctx ctx) noexcept {
    gsim_status st = GSIM_E_DEVICE;
    const char *what = "unexpected host error";
    try {
        throw;
    } catch (const std::bad_alloc &) {
        st = GSIM_E_OOM;
        what = "host memory exhausted";
    } catch (const std::exception &e) {
        what = e.what();
    } catch (...) {
    }
    try {
        return record(ctx, fail(st, "%s", what));
    } catch (...) {
        return st;
    }
}
}  // namespace

extern "C" {

const char *sim_version(void) { return "gsim 0.2 (gfx950)"; }

const char *sim_last_error(gsim_ctx ctx) {
    if (ctx) return ctx->err.c_str();
    std::lock_guard<std::mutex> lk(g_err_mu);
    static thread_local std::string copy;
    copy = g_err;
    return copy.c_str();
}

gsim_status sim_create(int device, uint64_t hbm_budget_bytes, gsim_ctx *out) try {
    if (!out) return record(nullptr, fail(GSIM_E_ARG, "null output"));
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return record(nullptr, fail(GSIM_E_DEVICE, "no HIP device"));
    }
    if (device < 0 || device >= n) return record(nullptr, fail(GSIM_E_ARG, "device %d of %d", device, n));
    auto ctx = std::make_unique<gsim_ctx_s>();
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) return record(nullptr, fail(GSIM_E_DEVICE, "hipSetDevice failed"));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return record(nullptr, fail(GSIM_E_DEVICE, "hipMemGetInfo failed"));
    const uint64_t budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(free_b / 10 * 9);
    ctx->pool = std::make_unique<Pool>(budget);
    {
        // persistent wavefronts of the dependency-driven schedule: four per SIMD
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess)
            return record(nullptr, fail(GSIM_E_DEVICE, "hipGetDeviceProperties failed"));
        ctx->n_waves_resident = (int64_t)prop.multiProcessorCount * 16;
        if (levelsync_max_waves(prop.multiProcessorCount, &ctx->n_waves_levelsync) != hipSuccess)
            return record(nullptr, fail(GSIM_E_DEVICE, "occupancy query failed"));
    }
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess)
        return record(nullptr, fail(GSIM_E_DEVICE, "stream creation failed"));
    // from here a failure also destroys the stream (the pool frees its slab itself)
    auto give_up = [&](gsim_status st, const char *msg) {
        (void)hipStreamDestroy(ctx->stream);
        return record(nullptr, fail(st, "%s", msg));
    };
    ctx->d_stage_t = (int64_t *)ctx->pool->get(sizeof(int64_t) * 2 * kStage);
    ctx->d_stage_v = (uint8_t *)ctx->pool->get(2 * kStage);
    ctx->d_stage_meta = (int64_t *)ctx->pool->get(sizeof(int64_t) * 2 * 3 * kStageBatch);
    if (!ctx->d_stage_t || !ctx->d_stage_v || !ctx->d_stage_meta)
        return give_up(GSIM_E_OOM, "no device memory for the fetch staging buffers");
    std::vector<uint8_t> lut = build_lut();
    ctx->d_lut = (uint8_t *)ctx->pool->get(lut.size());
    if (!ctx->d_lut) return give_up(GSIM_E_OOM, "no device memory for the gate table");
    if (hipMemcpy(ctx->d_lut, lut.data(), lut.size(), hipMemcpyHostToDevice) != hipSuccess)
        return give_up(GSIM_E_DEVICE, "gate table upload failed");
    // the no-allocation entry point's scratch on this device: its address is
    // looked up once here (sim_run_device_noalloc reports a failure)
    if (noalloc_scratch_setup(device) != hipSuccess) (void)hipGetLastError();
    *out = ctx.release();
    return GSIM_OK;
} catch (...) {
    return exception_status(nullptr);
}

gsim_status sim_destroy(gsim_ctx ctx) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    (void)hipSetDevice(ctx->device);
    for (auto &kv : ctx->jobs) destroy_job(ctx, kv.second.get());
    ctx->jobs.clear();
    for (auto &kv : ctx->executors) destroy_executor(ctx, kv.second.get());
    ctx->executors.clear();
    for (auto &kv : ctx->netlists) {
        put_netlist(ctx, kv.second.get());
    }
    ctx->netlists.clear();
    ctx->pool->put(ctx->d_lut);
    ctx->pool->put(ctx->d_stage_t);
    ctx->pool->put(ctx->d_stage_v);
    ctx->pool->put(ctx->d_stage_meta);
    ctx->pool.reset();
    if (ctx->ls_event) (void)hipEventDestroy(ctx->ls_event);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_set_option(gsim_ctx ctx, int option, int64_t value) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    switch (option) {
    case GSIM_OPT_ARENA_TRANSITIONS:
        if (value < 0) return record(ctx, fail(GSIM_E_ARG, "arena size must be >= 0"));
        ctx->opt_arena = value;
        return GSIM_OK;
    case GSIM_OPT_KERNEL:
        if (value < 0 || value > 1) return record(ctx, fail(GSIM_E_ARG, "kernel option must be 0 or 1"));
        ctx->opt_kernel = (int)value;
        return GSIM_OK;
    case GSIM_OPT_KERNEL_TIMING:
        if (value < 0 || value > 1) return record(ctx, fail(GSIM_E_ARG, "timing option must be 0 or 1"));
        ctx->opt_timing = (int)value;
        return GSIM_OK;
    case GSIM_OPT_LANE_THRESHOLD:
        if (value < 0 || value > INT32_MAX) return record(ctx, fail(GSIM_E_ARG, "lane threshold out of range"));
        ctx->opt_lane_threshold = (int32_t)value;
        return GSIM_OK;
    case GSIM_OPT_SCHEDULE:
        if (value < 0 || value > 3) return record(ctx, fail(GSIM_E_ARG, "schedule option must be 0, 1, 2 or 3"));
        ctx->opt_schedule = (int)value;
        return GSIM_OK;
    case GSIM_OPT_EVAL_FORM:
        if (value < 0 || value > 1) return record(ctx, fail(GSIM_E_ARG, "evaluation form must be 0 or 1"));
        ctx->opt_form = (int)value;
        return GSIM_OK;
    case GSIM_OPT_DF_TICKETS:
        if (value < 0 || value > 16) return record(ctx, fail(GSIM_E_ARG, "tickets per claim must be in [0, 16]"));
        ctx->opt_df_tickets = (int)value;
        return GSIM_OK;
    }
    return record(ctx, fail(GSIM_E_ARG, "unknown option %d", option));
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_load_netlist(gsim_ctx ctx, int64_t S, int64_t G, const uint8_t *type,
                             const int64_t *pin_off, const int64_t *pin_net,
                             const int32_t *rise_ps, const int32_t *fall_ps, gsim_netlist *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    return record(ctx, load_netlist(ctx, S, G, type, pin_off, pin_net, rise_ps, fall_ps, out));
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_load_netlist_ext(gsim_ctx ctx, int64_t S, int64_t G, const uint8_t *type,
                                 const int64_t *pin_off, const int64_t *pin_net, const int32_t *dly,
                                 int32_t n_udp, const uint8_t *udp, gsim_netlist *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (G > 0 && !dly) return record(ctx, fail(GSIM_E_ARG, "null delay table"));
    return record(ctx, load_netlist(ctx, S, G, type, pin_off, pin_net, nullptr, nullptr, out,
                                    G > 0 ? dly : nullptr, n_udp, udp));
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_unload_netlist(gsim_ctx ctx, gsim_netlist nl) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    auto it = ctx->netlists.find(nl);
    if (it == ctx->netlists.end()) return record(ctx, fail(GSIM_E_HANDLE, "unknown netlist handle %lld", (long long)nl));
    if (it->second->active_jobs > 0)
        return record(ctx, fail(GSIM_E_ARG, "netlist %lld still has %lld unreleased jobs", (long long)nl,
                                (long long)it->second->active_jobs));
    put_netlist(ctx, it->second.get());
    ctx->netlists.erase(it);
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_set_netlist_option(gsim_ctx ctx, gsim_netlist nl, int option, int64_t value) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    auto it = ctx->netlists.find(nl);
    if (it == ctx->netlists.end()) return record(ctx, fail(GSIM_E_HANDLE, "unknown netlist handle %lld", (long long)nl));
    Netlist &n = *it->second;
    switch (option) {
    case GSIM_OPT_LANE_THRESHOLD:
        if (value < -1 || value > INT32_MAX) return record(ctx, fail(GSIM_E_ARG, "lane threshold out of range"));
        n.lane_threshold = (int32_t)value;
        return GSIM_OK;
    case GSIM_OPT_SCHEDULE:
        if (value < -1 || value > 3) return record(ctx, fail(GSIM_E_ARG, "schedule must be -1, 0, 1, 2 or 3"));
        n.schedule = (int32_t)value;
        return GSIM_OK;
    case GSIM_OPT_EVAL_FORM:
        if (value < -1 || value > 1) return record(ctx, fail(GSIM_E_ARG, "evaluation form must be -1, 0 or 1"));
        n.form = (int32_t)value;
        return GSIM_OK;
    case GSIM_OPT_DF_TICKETS:
        if (value < -1 || value > 16) return record(ctx, fail(GSIM_E_ARG, "tickets per claim must be in [-1, 16]"));
        n.df_tickets = (int32_t)value <= 0 ? -1 : (int32_t)value;
        return GSIM_OK;
    }
    return record(ctx, fail(GSIM_E_ARG, "option %d is not per netlist", option));
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_netlist_info(gsim_ctx ctx, gsim_netlist nl, gsim_netlist_info *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    auto it = ctx->netlists.find(nl);
    if (it == ctx->netlists.end()) return record(ctx, fail(GSIM_E_HANDLE, "unknown netlist handle %lld", (long long)nl));
    if (!out) return record(ctx, fail(GSIM_E_ARG, "null output"));
    const Netlist &n = *it->second;
    out->S = n.S;
    out->G = n.G;
    out->P = n.P;
    out->levels = n.n_levels;
    out->max_delay_ps = n.max_delay;
    out->max_path_delay = n.max_path_delay;
    out->lane_gates = n.lane_gates;
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_memory_info(gsim_ctx ctx, gsim_memory_info *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (!out) return record(ctx, fail(GSIM_E_ARG, "null output"));
    out->budget_bytes = ctx->pool->budget();
    out->live_bytes = ctx->pool->live();
    out->largest_free_bytes = ctx->pool->largest_free();
    out->jobs_holding_storage = ctx->arenas_held;
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_submit(gsim_ctx ctx, gsim_netlist nl, const int64_t *src_off, const int64_t *t,
                       const uint8_t *v, void *hip_stream, gsim_job *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (!out) return record(ctx, fail(GSIM_E_ARG, "null output"));
    Job *j = nullptr;
    Failure f = submit(ctx, nl, src_off, t, v, false, 0, 0, (hipStream_t)hip_stream, &j);
    if (f.st == GSIM_OK) *out = j->id;
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_submit_device(gsim_ctx ctx, gsim_netlist nl, const int64_t *d_src_off, const int64_t *d_t,
                              const uint8_t *d_v, int64_t n_in, int validate, void *hip_stream,
                              gsim_job *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (!out) return record(ctx, fail(GSIM_E_ARG, "null output"));
    Job *j = nullptr;
    Failure f = submit(ctx, nl, d_src_off, d_t, d_v, true, n_in, validate, (hipStream_t)hip_stream, &j);
    if (f.st == GSIM_OK) *out = j->id;
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_run(gsim_ctx ctx, gsim_netlist nl, const int64_t *src_off, const int64_t *t,
                    const uint8_t *v, void *hip_stream, gsim_job *out) try {
    gsim_status st = sim_submit(ctx, nl, src_off, t, v, hip_stream, out);
    if (st != GSIM_OK) return st;
    Job *j = nullptr;
    Failure f = find_job(ctx, *out, &j);
    if (f.st == GSIM_OK) f = drive_until_enqueued(ctx, j);
    if (f.st != GSIM_OK) discard_job(ctx, out);
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_run_device(gsim_ctx ctx, gsim_netlist nl, const int64_t *d_src_off,
                           const int64_t *d_t, const uint8_t *d_v, int64_t n_in, int validate,
                           void *hip_stream, gsim_job *out) try {
    gsim_status st = sim_submit_device(ctx, nl, d_src_off, d_t, d_v, n_in, validate, hip_stream, out);
    if (st != GSIM_OK) return st;
    Job *j = nullptr;
    Failure f = find_job(ctx, *out, &j);
    if (f.st == GSIM_OK) f = drive_until_enqueued(ctx, j);
    if (f.st != GSIM_OK) discard_job(ctx, out);
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_run_device_noalloc(gsim_ctx ctx, gsim_netlist nl, const int64_t *d_src_off,
                                   const int64_t *d_t, const uint8_t *d_v, int64_t n_in, int64_t *d_off,
                                   int64_t *d_len, uint64_t *d_arena, int64_t arena_cap, int64_t *d_result,
                                   void *hip_stream) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    auto it = ctx->netlists.find(nl);
    if (it == ctx->netlists.end()) return record(ctx, fail(GSIM_E_HANDLE, "unknown netlist handle %lld", (long long)nl));
    const Netlist &n = *it->second;
    if (!d_src_off || !d_off || !d_len || !d_arena || !d_result || (n_in > 0 && (!d_t || !d_v)))
        return record(ctx, fail(GSIM_E_ARG, "null device buffer"));
    if (n_in < 0 || arena_cap < n_in)
        return record(ctx, fail(GSIM_E_ARG, "n_in = %lld with arena_cap = %lld (need 0 <= n_in <= arena_cap)",
                                (long long)n_in, (long long)arena_cap));
    Failure f = set_device(ctx);
    if (f.st == GSIM_OK)
        f = run_noalloc(ctx, n, d_src_off, d_t, d_v, n_in, d_off, d_len, d_arena, arena_cap, d_result,
                        hip_stream ? (hipStream_t)hip_stream : ctx->stream);
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_netlist_net_order(gsim_ctx ctx, gsim_netlist nl, int64_t *net_index) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    auto it = ctx->netlists.find(nl);
    if (it == ctx->netlists.end()) return record(ctx, fail(GSIM_E_HANDLE, "unknown netlist handle %lld", (long long)nl));
    if (!net_index) return record(ctx, fail(GSIM_E_ARG, "null output"));
    const Netlist &n = *it->second;
    for (int64_t i = 0; i < n.S; i++) net_index[i] = i;
    for (int64_t g = 0; g < n.G; g++) net_index[n.S + g] = n.S + n.internal_of_user[g];
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_run_batch(gsim_ctx ctx, gsim_netlist nl, int32_t n_sets, const int64_t *const *src_off,
                          const int64_t *const *t, const uint8_t *const *v, void *hip_stream,
                          gsim_job *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (n_sets < 0 || (n_sets > 0 && (!src_off || !t || !v || !out)))
        return record(ctx, fail(GSIM_E_ARG, "bad batch arguments"));
    std::vector<Job *> made;
    if (n_sets > 0) {
        // every set is checked and copied into pinned staging on host threads
        // (submit's work, in parallel), then queued in order
        auto it = ctx->netlists.find(nl);
        if (it == ctx->netlists.end()) return record(ctx, fail(GSIM_E_HANDLE, "unknown netlist handle %lld", (long long)nl));
        Netlist &net = *it->second;
        Failure f = set_device(ctx);
        Executor *ex = nullptr;
        if (f.st == GSIM_OK) f = get_executor(ctx, (hipStream_t)hip_stream, &ex);
        if (f.st != GSIM_OK) return record(ctx, f);
        for (int32_t i = 0; i < n_sets; i++)
            if (!src_off[i]) return record(ctx, fail(GSIM_E_ARG, "set %d: null src_off", i));
        std::vector<Failure> checked((size_t)n_sets, kOk);
        parallel_for(n_sets, [&](int64_t i) {
            checked[i] = validate_stimulus(net.S, src_off[i], t[i], v[i], net.max_path_delay);
        });
        for (int32_t i = 0; i < n_sets; i++)
            if (checked[i].st != GSIM_OK) return record(ctx, checked[i]);
        std::vector<HostStim> staged((size_t)n_sets);
        for (int32_t i = 0; i < n_sets && f.st == GSIM_OK; i++) f = stage_alloc(ctx, net.S, src_off[i][net.S], &staged[i]);
        if (f.st != GSIM_OK) {
            for (HostStim &hs : staged) stage_free(ctx, &hs);
            return record(ctx, f);
        }
        parallel_for(n_sets, [&](int64_t i) { stage_copy(net.S, src_off[i], t[i], v[i], &staged[i], false); });
        for (int32_t i = 0; i < n_sets; i++) {
            Job *j = nullptr;
            (void)queue_job(ctx, nl, net, ex, &staged[i], nullptr, nullptr, nullptr, staged[i].n_in, &j);
            made.push_back(j);
            out[i] = j->id;
        }
    }
    // drive while jobs can be admitted or have levels left; jobs that do not
    // fit yet are admitted by later calls as released jobs free memory
    if (!made.empty()) {
        Executor *ex = made.front()->ex;
        for (;;) {
            const int64_t before = ex->steps;
            Failure f = drive(ctx, ex, 0);
            if (f.st != GSIM_OK) return record(ctx, f);
            if (ex->steps == before) break;
        }
    }
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_drive(gsim_ctx ctx, void *hip_stream, int32_t max_ahead, int32_t *n_active,
                      int32_t *n_queued) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (max_ahead < 0 || max_ahead >= kRing) return record(ctx, fail(GSIM_E_ARG, "max_ahead must be in [0, %d)", kRing));
    Failure f = set_device(ctx);
    Executor *ex = nullptr;
    if (f.st == GSIM_OK) f = get_executor(ctx, (hipStream_t)hip_stream, &ex);
    if (f.st == GSIM_OK) f = drive(ctx, ex, max_ahead);
    if (f.st == GSIM_OK) {
        if (n_active) *n_active = (int32_t)ex->active.size();
        if (n_queued) *n_queued = (int32_t)ex->queue.size();
    }
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_job_done(gsim_ctx ctx, gsim_job job, int32_t *done) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (!done) return record(ctx, fail(GSIM_E_ARG, "null output"));
    Job *j = nullptr;
    Failure f = find_job(ctx, job, &j);
    if (f.st != GSIM_OK) return record(ctx, f);
    *done = 0;
    if (j->failed || j->waited) {
        *done = 1;
    } else if (j->phase == kEnqueued) {
        const hipError_t e = hipEventQuery(j->ev_done);
        if (e == hipSuccess) {
            if (!requeue_if_overflowed(ctx, j)) *done = 1;
        } else if (e != hipErrorNotReady) {
            return record(ctx, fail(GSIM_E_DEVICE, "event query: %s", hipGetErrorString(e)));
        }
    }
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_wait(gsim_ctx ctx, gsim_job job) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    Job *j = nullptr;
    Failure f = find_job(ctx, job, &j);
    if (f.st == GSIM_OK) f = wait_job(ctx, j);
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_job_stats(gsim_ctx ctx, gsim_job job, gsim_job_stats *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    if (!out) return record(ctx, fail(GSIM_E_ARG, "null output"));
    Job *j = nullptr;
    Failure f = find_job(ctx, job, &j);
    if (f.st == GSIM_OK) f = wait_job(ctx, j);
    if (f.st != GSIM_OK) return record(ctx, f);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, j->ev_start, j->ev_end) != hipSuccess)
        return record(ctx, fail(GSIM_E_DEVICE, "event timing failed"));
    out->n_in = j->n_in;
    out->n_out = j->h_state->n_out;
    out->pin_reads = j->h_state->pin_reads;
    out->arena_used = j->h_state->arena_top;
    out->arena_capacity = j->capacity;
    out->device_ms = ms;
    out->eval_ms = 0.0;
    out->eval_launches = 0;
    out->retries = j->retries;
    out->schedule = j->dataflow ? 1 : j->levelsync ? 3 : 0;
    for (const auto &tm : j->timing) {
        float e = 0.f;
        if (hipEventElapsedTime(&e, tm->a, tm->b) != hipSuccess)
            return record(ctx, fail(GSIM_E_DEVICE, "event timing failed"));
        out->eval_ms += e;
        out->eval_launches++;
    }
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_fetch_waveforms(gsim_ctx ctx, gsim_job job, const int64_t *nets, int64_t n,
                                int64_t *out_off, int64_t *out_t, uint8_t *out_v, int64_t cap) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    Job *j = nullptr;
    Failure f = find_job(ctx, job, &j);
    if (f.st == GSIM_OK) f = set_device(ctx);
    if (f.st == GSIM_OK) f = fetch(ctx, j, nets, n, out_off, out_t, out_v, cap);
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_fetch_hashes(gsim_ctx ctx, gsim_job job, const int64_t *nets, int64_t n, uint64_t *out) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    Job *j = nullptr;
    Failure f = find_job(ctx, job, &j);
    if (f.st == GSIM_OK) f = set_device(ctx);
    if (f.st == GSIM_OK) f = fetch_hashes(ctx, j, nets, n, out);
    return record(ctx, f);
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_release_job(gsim_ctx ctx, gsim_job job) try {
    if (!ctx) return record(nullptr, fail(GSIM_E_HANDLE, "null context"));
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end()) return record(ctx, fail(GSIM_E_HANDLE, "unknown job handle %lld", (long long)job));
    (void)hipSetDevice(ctx->device);
    destroy_job(ctx, it->second.get());
    ctx->jobs.erase(it);
    return GSIM_OK;
} catch (...) {
    return exception_status(ctx);
}

gsim_status sim_levelize(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                         const int64_t *pin_net, const int32_t *rise_ps, const int32_t *fall_ps,
                         int32_t *level_out, int32_t *n_levels_out) try {
    Levelized lv;
    Failure f = levelize(S, G, type, pin_off, pin_net, rise_ps, fall_ps, &lv);
    if (f.st != GSIM_OK) return record(nullptr, f);
    if (level_out) std::copy(lv.level.begin(), lv.level.end(), level_out);
    if (n_levels_out) *n_levels_out = lv.n_levels;
    return GSIM_OK;
} catch (...) {
    return exception_status(nullptr);
}

gsim_status sim_validate_stimulus(int64_t S, const int64_t *src_off, const int64_t *t,
                                  const uint8_t *v, int64_t max_path_delay) try {
    if (S < 0 || max_path_delay < 0) return record(nullptr, fail(GSIM_E_ARG, "negative S or path delay"));
    return record(nullptr, validate_stimulus(S, src_off, t, v, max_path_delay));
} catch (...) {
    return exception_status(nullptr);
}

}  // extern "C"
