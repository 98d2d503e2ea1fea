// HIP kernels of libgsim for gfx950 (CDNA4, wave64).
//
// One job = one pass over the levels of the netlist, all enqueued on one
// stream with no host synchronisation (the one-round-trip idea of Section 3).
// Per level:
//   size   : w_g = sum of the lengths of gate g's input waveforms. A gate's
//            output has at most as many transitions as it has distinct input
//            times (each merged time yields at most one candidate), which is
//            at most w_g -- Eq. 2 applied to one gate -- so w_g slots are
//            reserved for it. Block-local exclusive scan.
//   scan   : one block turns the block totals into absolute arena bases and
//            advances the arena top (a device bump allocator).
//   eval   : the output waveform of every gate of the level (Algorithm 2 with
//            the Eq. 1 denial and the Fig. 3 drop), written at its base.
// Transitions live in the arena packed as time << 2 | value (8 bytes).
#include "eval_core.h"

#include <mutex>

namespace gsim {

namespace {

// -------------------------------------------------------------------------
// Sources: packed into the arena at [0, n_in); their offsets and lengths; the
// job state.
// `t` may be the arena itself (each element is read, then overwritten by the
// same thread), so no restrict on t and K.
__global__ void init_sources_kernel(const int64_t *__restrict__ src_off, const int64_t *t,
                                    const uint8_t *__restrict__ v, int64_t S, int64_t n_in,
                                    int64_t *__restrict__ off, int64_t *__restrict__ len,
                                    uint64_t *K, DevState *state, int64_t capacity) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < n_in; i += stride) K[i] = pack_key(t[i], v[i]);
    for (int64_t i = i0; i < S; i += stride) {
        const int64_t a = src_off[i];
        off[i] = a;
        len[i] = src_off[i + 1] - a;
    }
    if (i0 == 0) {
        state->arena_top = n_in;
        state->capacity = capacity;
        state->pin_reads = 0;
        state->n_out = 0;
        state->overflow = 0;
        state->check_error = 0;
    }
}

// -------------------------------------------------------------------------
// A step covers the current level of several jobs; sizing blocks are laid out
// job after job. The job of a block (or of a work-list entry) is looked up in
// the step's job table.
__device__ __forceinline__ int job_of_block(const JobDesc *jobs, int n_jobs, int64_t b) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].sblock_begin <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Segment of a wavefront gate in the dispatch order: half-octave bucket of
// its estimated cost w_g * weight (relative cost per input transition by
// pin count, from the rounds' fill and length), costliest first, then pin
// count from four down.
__device__ __forceinline__ uint32_t cost_segment(int64_t w, int k) {
    const uint64_t weight = k == 1 ? 2 : k == 2 ? 3 : k == 3 ? 5 : 4;
    const uint64_t est = (uint64_t)(w > 0 ? w : 1) * weight;
    const int lg = 63 - __clzll((long long)est);
    const int half = lg > 0 ? (int)((est >> (lg - 1)) & 1u) : 0;
    int bucket = 2 * lg + half - 16;
    bucket = bucket < 0 ? 0 : bucket > kCostBuckets - 1 ? kCostBuckets - 1 : bucket;
    return (uint32_t)((kCostBuckets - 1 - bucket) * 4 + (4 - k));
}

// Per-level sizing and binning: w_g (the sum of the gate's input lengths, an
// upper bound of its output length), its block-local exclusive scan, and the
// gate's work list -- lane kernel if its largest delay exceeds the large
// window or it reads fewer than lane_threshold transitions, else the
// wavefront kernel of its delay window and pin count -- appended to that list,
// with its segment in the dispatch order and its rank in that segment.
__global__ __launch_bounds__(kSizeBlock) void size_kernel(StepArgs A) {
    constexpr int kAllSegs = kVariants * kSegments;
    static_assert(kAllSegs % kSizeBlock == 0, "segments per thread");
    __shared__ int64_t wsum[kSizeBlock / 64];
    __shared__ uint32_t l_cnt[kNumLists], l_base[kNumLists];
    __shared__ uint32_t s_cnt[kAllSegs], s_base[kAllSegs];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x;
    for (int q = t; q < kAllSegs; q += kSizeBlock) s_cnt[q] = 0;
    if (t < kNumLists) l_cnt[t] = 0;
    const int j = job_of_block(A.jobs, A.n_jobs, b);
    const JobDesc &J = A.jobs[j];
    const int64_t i = (b - J.sblock_begin) * kSizeBlock + t;
    const int64_t g = J.lvl_begin + i;
    int64_t w = 0;
    int cls = -1;
    uint32_t seg_key = 0;  // variant * kSegments + segment, for wavefront gates
    if (i < J.n_gates) {
        const GateRec &r = J.rec[g];
        const int k = r.k;
#pragma unroll
        for (int p = 0; p < kMaxPins; p++)
            if (p < k) w += J.len[r.net[p]];
        cls = (r.dmax > kWindowLarge || w < J.lane_threshold)
                  ? kListLane
                  : wave_list(wave_variant(r.window, J.edly ? 1 : 0), k);
        if (cls != kListLane) seg_key = (uint32_t)(cls / 4) * kSegments + cost_segment(w, k);
    }
    const int lane = lane_id(), wv = t >> 6;
    int64_t x = w;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const int lo = __shfl_up((int)(uint32_t)x, s, 64);
        const int hi = __shfl_up((int)(uint32_t)((uint64_t)x >> 32), s, 64);
        const int64_t o = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        if (lane >= s) x += o;
    }
    if (lane == 63) wsum[wv] = x;
    if (b == 0)
        for (int q = t; q < kCountWords; q += kSizeBlock) A.next_count[q] = 0;
    __syncthreads();
    // list positions and segment ranks: block-local (LDS atomics), then one
    // global atomic per list and per segment the block touches
    const bool wave_gate = cls >= 0 && cls != kListLane;
    uint32_t lpos = 0, spos = 0;
    if (cls >= 0) lpos = atomicAdd(&l_cnt[cls], 1u);
    if (wave_gate) spos = atomicAdd(&s_cnt[seg_key], 1u);
    __syncthreads();
    if (t < kNumLists && l_cnt[t]) l_base[t] = atomicAdd(&A.count[t], l_cnt[t]);
    for (int q = t; q < kAllSegs; q += kSizeBlock)
        if (s_cnt[q]) s_base[q] = atomicAdd(&A.count[kSegCountAt + q], s_cnt[q]);
    __syncthreads();
    if (cls >= 0) {
        const uint32_t pos = l_base[cls] + lpos;
        A.list[cls][pos] = ((uint64_t)(uint32_t)j << 32) | (uint64_t)g;
        if (wave_gate)
            A.key[cls][pos] = ((uint64_t)(seg_key % kSegments) << 32) | (uint64_t)(s_base[seg_key] + spos);
    }
    int64_t before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kSizeBlock / 64; q++) {
        if (q < wv) before += wsum[q];
        total += wsum[q];
    }
    if (i < J.n_gates) J.off[J.S + g] = before + x - w;
    if (t == 0) A.blocksum[b] = total;
}

// One block per job (any block size up to 1024): the job's block totals ->
// absolute arena bases; bump the job's arena top (a device bump allocator);
// flag overflow.
__device__ void job_scan(const StepArgs &A, int job) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry_s;
    const JobDesc &J = A.jobs[job];
    DevState *state = J.state;
    int64_t *blocksum = A.blocksum + J.sblock_begin;
    const int64_t nb = (J.n_gates + kSizeBlock - 1) / kSizeBlock;
    const int lane = lane_id(), wv = threadIdx.x >> 6, n_waves = (int)blockDim.x >> 6;
    if (threadIdx.x == 0) carry_s = state->arena_top;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += blockDim.x) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t w = i < nb ? blocksum[i] : 0;
        int64_t x = w;
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const int lo = __shfl_up((int)(uint32_t)x, s, 64);
            const int hi = __shfl_up((int)(uint32_t)((uint64_t)x >> 32), s, 64);
            const int64_t o = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
            if (lane >= s) x += o;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int64_t before = 0, total = 0;
        for (int q = 0; q < n_waves; q++) {
            if (q < wv) before += wsum[q];
            total += wsum[q];
        }
        const int64_t base = carry_s;
        if (i < nb) blocksum[i] = base + before + x - w;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = base + total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t top = carry_s;
        const int64_t used = top - state->arena_top;
        if (top > state->capacity || state->overflow) {
            state->overflow = 1;
        } else {
            state->pin_reads += used;
            state->arena_top = top;
        }
    }
}

// -------------------------------------------------------------------------
// Counting-sort scatter of the wavefront lists: entry (c, pos) goes to
// sorted[variant][base of its segment + its rank]. The segment bases are an
// exclusive scan of the segment sizes per variant, redone by every block.
struct ListBounds {
    int64_t cum[kListLane + 1];  // cumulative upper bounds of the list lengths
};

__global__ __launch_bounds__(kVariants * kSegments) void sort_lists_kernel(StepArgs A, ListBounds lb) {
    static_assert(kSegments == 128, "two waves per variant");
    __shared__ uint32_t seg_base[kVariants * kSegments];
    __shared__ uint32_t wave_tot[2 * kVariants];
    // the first n_jobs blocks also place their job's level in the arena
    if ((int)blockIdx.x < A.n_jobs) job_scan(A, (int)blockIdx.x);
    const int t = threadIdx.x, lane = lane_id(), wv = t >> 6;
    const uint32_t cnt = A.count[kSegCountAt + t];
    uint32_t x = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)x, d, 64);
        if (lane >= d) x += o;
    }
    if (lane == 63) wave_tot[wv] = x;
    __syncthreads();
    // variant v: waves 2v and 2v + 1
    seg_base[t] = x - cnt + ((wv & 1) ? wave_tot[wv - 1] : 0u);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + t;
    int c = 0;
#pragma unroll
    for (int q = 1; q < kListLane; q++)
        if (i >= lb.cum[q]) c = q;
    const int64_t p = i - lb.cum[c];
    if (i < lb.cum[kListLane] && p < (int64_t)A.count[c]) {
        const uint64_t key = A.key[c][p];
        const int var = c / 4;
        A.sorted[var][seg_base[var * kSegments + (int)(key >> 32)] + (uint32_t)key] = A.list[c][p];
    }
}

// Every gate of the step in one variant (largest delay at most W; delay model
// EDGE), in one launch, one wavefront per entry of the variant's sorted list
// (costliest first). Occupancy: six wavefronts per SIMD for the 64 ps window
// (6 KB of LDS each; a seventh would need 168 KB of the CU's 160 KB), five
// for 256 (6.75 KB each). Six cost a few spilled registers and measured 3 %
// faster than five.
template <int W, bool EDGE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W == 64 ? 6 : 5))) void eval_wave_kernel(StepArgs A,
                                                                                              int var) {
    __shared__ WaveLds<W> L;
    const int lane = lane_id();
    const int64_t item = blockIdx.x;
    const int list0 = var * 4;
    const int64_t total = (int64_t)A.count[list0] + A.count[list0 + 1] + A.count[list0 + 2] +
                          A.count[list0 + 3];
    if (item >= total) return;
    const uint64_t e = A.sorted[var][item];
    const JobDesc &J = A.jobs[(int)(e >> 32)];
    const int64_t gate = (int64_t)(uint32_t)e;
    const GateRec R = J.rec[gate];
    if (J.state->overflow) {
        if (lane == 0) { J.len[J.S + gate] = 0; J.off[J.S + gate] = 0; }
        return;
    }
    reinterpret_cast<uint32_t *>(L.lut)[lane] =
        reinterpret_cast<const uint32_t *>(J.lut + (int)R.type * 256)[lane];
    const int64_t ob = A.blocksum[J.sblock_begin + (gate - J.lvl_begin) / kSizeBlock] + J.off[J.S + gate];
    switch (R.k) {
    // every pin count prefetches its next tiles during the round
    case 1: eval_gate<1, W, EDGE, true, true, false>(J, ob, R, gate, L); break;
    case 2: eval_gate<2, W, EDGE, true, true, false>(J, ob, R, gate, L); break;
    case 3: eval_gate<3, W, EDGE, true, true, false>(J, ob, R, gate, L); break;
    default: eval_gate<4, W, EDGE, true, true, false>(J, ob, R, gate, L); break;
    }
}

// The same lists with the segmented form (eval_gate_seg): five wavefronts per
// SIMD (the LDS limit: 6.9 KB per wavefront for the 64 ps window, 7.7 KB for
// 256).
template <int W, bool EDGE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void eval_seg_kernel(StepArgs A,
                                                                                             int var) {
    __shared__ SegLds<W> L;
    const int lane = lane_id();
    const int64_t item = blockIdx.x;
    const int list0 = var * 4;
    const int64_t total = (int64_t)A.count[list0] + A.count[list0 + 1] + A.count[list0 + 2] +
                          A.count[list0 + 3];
    if (item >= total) return;
    const uint64_t e = A.sorted[var][item];
    const JobDesc &J = A.jobs[(int)(e >> 32)];
    const int64_t gate = (int64_t)(uint32_t)e;
    const GateRec R = J.rec[gate];
    if (J.state->overflow) {
        if (lane == 0) { J.len[J.S + gate] = 0; J.off[J.S + gate] = 0; }
        return;
    }
    reinterpret_cast<uint32_t *>(L.lut)[lane] =
        reinterpret_cast<const uint32_t *>(J.lut + (int)R.type * 256)[lane];
    const int64_t ob = A.blocksum[J.sblock_begin + (gate - J.lvl_begin) / kSizeBlock] + J.off[J.S + gate];
    switch (R.k) {
    case 1: eval_gate_seg<1, W, EDGE, true, false>(J, ob, R, gate, L); break;
    case 2: eval_gate_seg<2, W, EDGE, true, false>(J, ob, R, gate, L); break;
    case 3: eval_gate_seg<3, W, EDGE, true, false>(J, ob, R, gate, L); break;
    default: eval_gate_seg<4, W, EDGE, true, false>(J, ob, R, gate, L); break;
    }
}

__global__ __launch_bounds__(64) void eval_lane_kernel(StepArgs A) {
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= (int64_t)A.count[kListLane]) return;
    const uint64_t e = A.list[kListLane][item];
    const JobDesc &J = A.jobs[(int)(e >> 32)];
    const int64_t gate = (int64_t)(uint32_t)e;
    if (J.state->overflow) {
        J.len[J.S + gate] = 0;
        J.off[J.S + gate] = 0;
        return;
    }
    const GateRec R = J.rec[gate];
    const int64_t ob = A.blocksum[J.sblock_begin + (gate - J.lvl_begin) / kSizeBlock] + J.off[J.S + gate];
    eval_seq<false>(J, R, gate, ob, J.lut + (int)R.type * 256);
}

// -------------------------------------------------------------------------
// Dependency-driven schedule (the non-partitioned, dependency-triggered task
// control of Section 3.3, Algorithm 1): no level barrier. Each wavefront
// takes the next queue slot (a ticket), waits until a gate has been put
// there, evaluates it into a region it reserves from the arena with one
// atomic add (the bounded reservation w_g of Eq. 2), then decrements the
// pending count of every consumer and queues those that reach zero. Every
// gate enters the queue exactly once, so the G tickets are all filled and a
// wavefront leaves when its ticket is past the end. Ordering across the
// XCDs' L2 caches: outputs are published with an agent-scope release fence
// before the decrements; the wavefront that takes a gate reads its pending
// count (0) and then takes an agent-scope acquire fence, which orders every
// producer's outputs before its reads (see df_acquire_inputs).
// Safety exit: a wavefront that sees no new queue entry for kDfSpinLimit
// polls (each after a sleep of about 2k cycles: tens of seconds in all) flags
// the job (check_error = 3) and leaves, and so does every wavefront that sees
// the flag.
constexpr uint32_t kDfSpinLimit = 1u << 24;

__global__ void df_init_kernel(DfArgs A, const int32_t *__restrict__ pend0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < A.G) {
        A.pend[i] = pend0[i];
        A.queue[i] = i < A.n_first ? (int32_t)i : -1;
    }
    if (i == 0) {
        A.ctl->head = 0;
        A.ctl->tail = (uint32_t)A.n_first;
    }
}

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until queue slot t holds a gate; -1 if the job was flagged meanwhile.
__device__ int32_t df_wait_slot(const DfArgs &A, uint32_t t, DevState *st) {
    const int lane = lane_id();
    uint32_t spins = 0, seen_tail = 0;
    for (;;) {
        uint32_t q = 0;
        if (lane == 0) q = load_agent(reinterpret_cast<const uint32_t *>(A.queue + t));
        q = (uint32_t)__builtin_amdgcn_readfirstlane((int)q);
        if ((int32_t)q >= 0) return (int32_t)q;
        if ((++spins & 31u) == 0) {  // now and then: an error elsewhere, or no progress
            uint32_t err = 0, tl = 0;
            if (lane == 0) {
                err = load_agent(reinterpret_cast<const uint32_t *>(&st->check_error));
                tl = load_agent(&A.ctl->tail);
            }
            err = (uint32_t)__builtin_amdgcn_readfirstlane((int)err);
            tl = (uint32_t)__builtin_amdgcn_readfirstlane((int)tl);
            if (err) return -1;
            if (tl != seen_tail) {
                seen_tail = tl;
                spins = 0;
            } else if (spins > kDfSpinLimit) {
                if (lane == 0) atomicMax(&st->check_error, 3);
                return -1;
            }
        }
        __builtin_amdgcn_s_sleep(32);
    }
}

// Before it reads the inputs of the gates it took from the queue, a
// wavefront synchronises with every producer of those gates. Each producer
// decrements a consumer's pending count after its agent-scope release fence;
// the decrements form one release sequence on that count, so a relaxed read
// of the count's final value 0 followed by an agent-scope acquire fence
// synchronises with every producer's fence (fence-to-fence synchronisation
// through the count). The queue slot only says which gate to take. The read
// finds 0 at once in practice (the count reached 0 before the slot was
// written); the loop waits for it rather than assume cross-location order.
__device__ __forceinline__ void df_acquire_inputs(const DfArgs &A, int32_t g_lane, int nb) {
    const int lane = lane_id();
    for (;;) {
        uint32_t pend = 0;
        if (lane < nb) pend = load_agent(reinterpret_cast<const uint32_t *>(A.pend + g_lane));
        if (__ballot(pend != 0) == 0) break;
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Queue the n gates listed at list[0, n) (LDS) with one atomic on the tail.
constexpr int kDfReadyList = 512;
static_assert(kDfReadyList <= kWindowLarge + kRoundSlots + 32, "the ready list fits the survivor area");
__device__ __forceinline__ void df_push(const DfArgs &A, const uint32_t *list, int n) {
    const int lane = lane_id();
    __syncthreads();  // the list's entries, written by every lane
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&A.ctl->tail, (uint32_t)n);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
    for (int i = lane; i < n; i += 64)
        __hip_atomic_store(A.queue + base + i, (int32_t)list[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();  // before the list is written again
}

// A wavefront takes A.tickets (1..kDfMaxTickets) consecutive tickets per
// atomic and works through them in order; the gates of those tickets whose
// slots are already filled run as one batch between one acquire and one
// release fence. Queue slots are allocated in the
// order gates become ready, so while a wavefront waits on its next slot no
// later slot holds a ready gate that only it could run (the deadlock-freedom
// argument is unchanged). More tickets per atomic relieve the one contended
// counter; fewer keep gates near the critical path on wavefronts of their own.
constexpr uint32_t kDfMaxTickets = 16;
// Arena space is reserved per wavefront in chunks of A.chunk transitions (or
// one gate's bound if larger), so the arena top takes one atomic per chunk.

template <bool EDGE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void dataflow_kernel(DfArgs A) {
    __shared__ WaveLds<kWindowLarge> L;
    // the batch, one gate per entry: record, read bound w_g, fanout range
    __shared__ GateRec brec[kDfMaxTickets];
    __shared__ int64_t bw[kDfMaxTickets], bfo[kDfMaxTickets], bpre[kDfMaxTickets], bfst[kDfMaxTickets];
    const int lane = lane_id();
    const JobDesc &J = A.job;
    DevState *st = J.state;
    int64_t chunk_at = 0, chunk_end = 0;  // this wavefront's unused arena space
    int64_t reads = 0;                    // sum of w_g over this wavefront's gates
    bool stop = false;
    while (!stop) {
        const uint32_t n_t = A.tickets < 1u ? 1u : A.tickets > kDfMaxTickets ? kDfMaxTickets : A.tickets;
        uint32_t t0 = 0;
        if (lane == 0) t0 = atomicAdd(&A.ctl->head, n_t);
        t0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)t0);
        if ((int64_t)t0 >= A.G) break;
        const uint32_t t1 = (uint32_t)min64((int64_t)t0 + n_t, A.G);
        uint32_t t = t0;
        while (t < t1) {
            // the next gate, and the following tickets whose slots are already
            // filled: all run between one acquire and one release fence
            const int32_t g0 = df_wait_slot(A, t, st);
            if (g0 < 0) {
                stop = true;
                break;
            }
            // lane b holds the gate of ticket t + b (b < nb)
            int32_t g_lane = lane == 0 ? g0 : -1;
            if (lane > 0 && t + (uint32_t)lane < t1)
                g_lane = (int32_t)load_agent(reinterpret_cast<const uint32_t *>(A.queue + t + lane));
            const uint64_t filled = __ballot(g_lane >= 0);
            const int nb = (~filled) == 0 ? 64 : __builtin_ctzll(~filled);  // leading filled slots
            df_acquire_inputs(A, g_lane, nb);
            // the batch's gate records, read bounds and fanout sizes, loaded
            // together (lane b: ticket t + b) and kept in LDS
            if (lane < nb) {
                const GateRec Rl = J.rec[g_lane];
                int64_t w = 0;
#pragma unroll
                for (int p = 0; p < kMaxPins; p++)
                    if (p < Rl.k) w += J.len[Rl.net[p]];
                brec[lane] = Rl;
                bw[lane] = w;
                bfst[lane] = A.fo_off[g_lane];
                bfo[lane] = A.fo_off[g_lane + 1] - bfst[lane];
            }
            const bool halted = load_agent(reinterpret_cast<const uint32_t *>(&st->overflow)) != 0;
            __syncthreads();
            for (int b = 0; b < nb; b++) {
                const int32_t g = __builtin_amdgcn_readlane(g_lane, b);
                GateRec R;
                {
                    const int32_t *src = reinterpret_cast<const int32_t *>(&brec[b]);
                    int32_t *dst = reinterpret_cast<int32_t *>(&R);
#pragma unroll
                    for (int d = 0; d < 16; d++) dst[d] = __builtin_amdgcn_readfirstlane(src[d]);
                }
                const int64_t w = uniform64(bw[b]);
                reads += w;
                if (chunk_end - chunk_at < w) {
                    const int64_t want = w > A.chunk ? w : A.chunk;
                    int64_t at = 0;
                    if (lane == 0)
                        at = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&st->arena_top),
                                                (unsigned long long)want);
                    chunk_at = (int64_t)readlane_u64((uint64_t)at, 0);
                    chunk_end = chunk_at + want;
                }
                const int64_t ob = chunk_at;
                chunk_at += w;
                const bool full = ob + w > st->capacity;
                if (full || halted) {
                    if (lane == 0) {
                        if (full) atomicOr(&st->overflow, 1);
                        put<true>(J.len + J.S + g, (int64_t)0);
                        put<true>(J.off + J.S + g, (int64_t)0);
                    }
                } else if (R.dmax > kWindowLarge) {
                    if (lane == 0) eval_seq<true>(J, R, g, ob, J.lut + (int)R.type * 256);
                } else {
                    reinterpret_cast<uint32_t *>(L.lut)[lane] =
                        reinterpret_cast<const uint32_t *>(J.lut + (int)R.type * 256)[lane];
                    switch (R.k) {
                    case 1: eval_gate<1, kWindowLarge, EDGE, !EDGE, false, true>(J, ob, R, g, L); break;
                    case 2: eval_gate<2, kWindowLarge, EDGE, !EDGE, false, true>(J, ob, R, g, L); break;
                    case 3: eval_gate<3, kWindowLarge, EDGE, !EDGE, false, true>(J, ob, R, g, L); break;
                    default: eval_gate<4, kWindowLarge, EDGE, !EDGE, false, true>(J, ob, R, g, L); break;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            // consumers whose last pending pin this was: listed in LDS (the
            // evaluation's survivor area, free between gates) and queued with
            // one tail atomic for the whole batch. The batch's fanout entries
            // (one per reading pin) are decremented 64 at a time across its
            // gates. (A consumer synchronises with every producer through its
            // pending count: df_acquire_inputs.)
            int n_ready = 0;
            {
                int64_t total = 0;
                for (int b = 0; b < nb; b++) {
                    if (lane == 0) bpre[b] = total;
                    total += uniform64(bfo[b]);
                }
                __syncthreads();
                for (int64_t i0 = 0; i0 < total; i0 += 64) {
                    const int64_t i = i0 + lane;
                    int32_t c = -1;
                    if (i < total) {
                        int b = nb - 1;
                        while (b > 0 && i < bpre[b]) b--;
                        c = A.fo[bfst[b] + (i - bpre[b])];
                    }
                    const bool ready = c >= 0 && atomicSub(&A.pend[c], 1) == 1;
                    const uint64_t mask = __ballot(ready);
                    if (mask == 0) continue;
                    if (ready) L.seq[n_ready + lanes_below(mask)] = (uint32_t)c;
                    n_ready += __popcll(mask);
                    if (n_ready > kDfReadyList - 64) {
                        df_push(A, L.seq, n_ready);
                        n_ready = 0;
                    }
                }
            }
            if (n_ready > 0) df_push(A, L.seq, n_ready);
            t += nb;
        }
    }
    if (lane == 0 && reads > 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(&st->pin_reads), (unsigned long long)reads);
}

// -------------------------------------------------------------------------
// Level-barrier schedule: the level chain of one job in a single launch. The
// persistent wavefronts take the gates of each level in strides of the grid,
// reserve each gate's region from a per-wave arena chunk, evaluate it as the
// level kernel does, and meet at a device-wide barrier before the next level.
//
// The barrier is a combining tree with one release flag per group of 64
// wavefronts, each counter and flag on a cache line of its own, so that no
// address is polled by more than 64 wavefronts: a wavefront's agent-scope
// release fence (its level's plain stores become visible), one relaxed
// increment of its group's arrival counter; the group's last arrival
// (acquire-release fence) increments the top counter; the last of those
// (acquire-release fence) sets every group's flag to the barrier's
// generation; a waiting wavefront polls its group's flag, then takes an
// agent-scope acquire fence (fence-to-fence synchronisation at each step).
// Counters only grow: generation g has completed when a group counter reaches
// g times the group's size. Every wavefront of the grid is resident (a
// cooperative launch), so the wait ends; as a safety exit, a wait longer than
// kLsSpinLimit polls flags the job (check_error = 3), and a flagged job stops
// every wavefront at its next barrier.
constexpr uint32_t kLsSpinLimit = 1u << 22;

__device__ __forceinline__ uint32_t *ls_line(const LsArgs &A, int i) { return A.sync + (size_t)i * kLsLineWords; }

__device__ bool ls_barrier(const LsArgs &A, uint32_t gen, DevState *st) {
    const int lane = lane_id();
    const uint32_t nw = gridDim.x, m = blockIdx.x / kLsGroup, M = (nw + kLsGroup - 1) / kLsGroup;
    const uint32_t gs = m + 1 < M ? kLsGroup : nw - kLsGroup * m;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    uint32_t old = 0;
    if (lane == 0)
        old = __hip_atomic_fetch_add(ls_line(A, kLsLineGroups + m), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = (uint32_t)__builtin_amdgcn_readfirstlane((int)old);
    if (old + 1 == gs * gen) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        uint32_t top = 0;
        if (lane == 0)
            top = __hip_atomic_fetch_add(ls_line(A, kLsLineTop), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        top = (uint32_t)__builtin_amdgcn_readfirstlane((int)top);
        if (top + 1 == M * gen) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            if ((uint32_t)lane < M)
                __hip_atomic_store(ls_line(A, kLsLineFlags + lane), gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    const uint32_t *flag = ls_line(A, kLsLineFlags + m);
    for (uint32_t spins = 0;; spins++) {
        uint32_t seen = 0;
        if (lane == 0) seen = load_agent(flag);
        seen = (uint32_t)__builtin_amdgcn_readfirstlane((int)seen);
        if (seen >= gen) break;
        if ((spins & 255u) == 255u) {
            uint32_t err = 0;
            if (lane == 0) err = load_agent(reinterpret_cast<const uint32_t *>(&st->check_error));
            if (__builtin_amdgcn_readfirstlane((int)err)) return false;
            if (spins > kLsSpinLimit) {
                if (lane == 0) atomicMax(&st->check_error, 3);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

template <bool EDGE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void levelsync_kernel(LsArgs A) {
    __shared__ WaveLds<kWindowLarge> L;
    const int lane = lane_id();
    const JobDesc &J = A.job;
    DevState *st = J.state;
    const int64_t nw = gridDim.x, capacity = st->capacity;
    int64_t chunk_at = 0, chunk_end = 0;  // this wavefront's unused arena space
    int64_t reads = 0;                    // sum of w_g over this wavefront's gates
    for (int32_t l = 0; l < A.n_levels; l++) {
        const int64_t g1 = A.level_off[l + 1];
        const bool halted = load_agent(reinterpret_cast<const uint32_t *>(&st->overflow)) != 0;
        for (int64_t g = A.level_off[l] + blockIdx.x; g < g1; g += nw) {
            const GateRec R = J.rec[g];
            int64_t w = 0;
#pragma unroll
            for (int p = 0; p < kMaxPins; p++)
                if (p < R.k) w += J.len[R.net[p]];
            reads += w;
            if (chunk_end - chunk_at < w) {
                const int64_t want = w > A.chunk ? w : A.chunk;
                int64_t at = 0;
                if (lane == 0)
                    at = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&st->arena_top),
                                            (unsigned long long)want);
                chunk_at = (int64_t)readlane_u64((uint64_t)at, 0);
                chunk_end = chunk_at + want;
            }
            const int64_t ob = chunk_at;
            chunk_at += w;
            const bool full = ob + w > capacity;
            if (full || halted) {
                if (lane == 0) {
                    if (full) atomicOr(&st->overflow, 1);
                    J.len[J.S + g] = 0;
                    J.off[J.S + g] = 0;
                }
            } else if (R.dmax > kWindowLarge) {
                if (lane == 0) eval_seq<false>(J, R, g, ob, J.lut + (int)R.type * 256);
            } else {
                reinterpret_cast<uint32_t *>(L.lut)[lane] =
                    reinterpret_cast<const uint32_t *>(J.lut + (int)R.type * 256)[lane];
                switch (R.k) {
                case 1: eval_gate<1, kWindowLarge, EDGE, true, true, false>(J, ob, R, g, L); break;
                case 2: eval_gate<2, kWindowLarge, EDGE, true, true, false>(J, ob, R, g, L); break;
                case 3: eval_gate<3, kWindowLarge, EDGE, true, true, false>(J, ob, R, g, L); break;
                default: eval_gate<4, kWindowLarge, EDGE, true, true, false>(J, ob, R, g, L); break;
                }
            }
        }
        if (l + 1 < A.n_levels && !ls_barrier(A, (uint32_t)(l + 1), st)) break;
    }
    if (lane == 0 && reads > 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(&st->pin_reads), (unsigned long long)reads);
}

// -------------------------------------------------------------------------
// Per-net fingerprint: mix(n) + sum over transitions i of mix(key_i ^ mix(i))
// (mod 2^64), key_i = time << 2 | value, mix = the SplitMix64 finaliser. The
// index inside mix binds each transition to its position, so reordering is
// detected; the sum lets a wavefront reduce one net's transitions in parallel.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ __launch_bounds__(256) void hash_kernel(const int64_t *__restrict__ nets_off,
                                                   const int64_t *__restrict__ nets_len,
                                                   int64_t n_nets, const uint64_t *__restrict__ K,
                                                   uint64_t *__restrict__ out) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * 256) >> 6;
    for (int64_t i = wave; i < n_nets; i += n_waves) {
        const int64_t a = nets_off[i], n = nets_len[i];
        uint64_t acc = 0;
        for (int64_t j = lane; j < n; j += 64) acc += mix64(K[a + j] ^ mix64((uint64_t)j));
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) acc += shfl_down_u64(acc, s);
        if (lane == 0) out[i] = acc + mix64((uint64_t)n);
    }
}

// off/len of requested nets: out_off[i] = off[net[i]], out_len[i] = len[net[i]]
__global__ void gather_meta_kernel(const int64_t *__restrict__ net, int64_t n,
                                   const int64_t *__restrict__ off, const int64_t *__restrict__ len,
                                   int64_t *__restrict__ out_off, int64_t *__restrict__ out_len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out_off[i] = off[net[i]];
        out_len[i] = len[net[i]];
    }
}

__global__ void clear_u32_kernel(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// -------------------------------------------------------------------------
// Sum of the gate output lengths (two stages: partial sums, then one block).
__global__ __launch_bounds__(256) void count_partial_kernel(const int64_t *__restrict__ len,
                                                            int64_t S, int64_t G,
                                                            int64_t *__restrict__ partial) {
    __shared__ int64_t ws[4];
    int64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < G; i += (int64_t)gridDim.x * 256)
        acc += len[S + i];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) acc += shfl_down64(acc, s);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(64) void count_final_kernel(const int64_t *__restrict__ partial,
                                                         int64_t n, DevState *state) {
    int64_t acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += 64) acc += partial[i];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) acc += shfl_down64(acc, s);
    if (threadIdx.x == 0) state->n_out = acc;
}

// -------------------------------------------------------------------------
// Gather: net i's n_items[i] transitions from the arena at src_off[i],
// unpacked into the staging buffers at dst_off[i]. One block per net.
__global__ __launch_bounds__(256) void gather_kernel(const int64_t *__restrict__ src_off,
                                                     const int64_t *__restrict__ n_items,
                                                     const int64_t *__restrict__ dst_off,
                                                     int64_t n_nets,
                                                     const uint64_t *__restrict__ K,
                                                     int64_t *__restrict__ out_t,
                                                     uint8_t *__restrict__ out_v) {
    for (int64_t i = blockIdx.x; i < n_nets; i += gridDim.x) {
        const int64_t a = src_off[i], n = n_items[i], d = dst_off[i];
        for (int64_t j = threadIdx.x; j < n; j += 256) {
            const uint64_t k = K[a + j];
            out_t[d + j] = key_time(k);
            out_v[d + j] = (uint8_t)key_value(k);
        }
    }
}

// -------------------------------------------------------------------------
// No-allocation run: the step descriptors of a batch of levels, written from
// the kernel argument into the scratch table; the job's outcome copied to
// the caller's result words.
__global__ void write_descs_kernel(DescBatch b) {
    const int i = threadIdx.x;
    if (i < b.n) b.dst[i] = b.d[i];
}

__global__ void run_result_kernel(const DevState *__restrict__ st, int64_t *__restrict__ out) {
    if (threadIdx.x == 0) {
        out[0] = st->n_out;
        out[1] = st->overflow;
        out[2] = st->check_error;
        out[3] = st->arena_top;
    }
}

}  // namespace

// -------------------------------------------------------------------------
// Device scratch of the no-allocation entry point: one array per GPU, held
// until the process ends, shared by every call on that GPU. The host-side
// name `scratch` is not a device address and is never passed to a kernel:
// set-up looks up each device's address once (noalloc_scratch_setup, with
// that device current) and launches use that address.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_at[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_at[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_at[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_at[device];
}

// -------------------------------------------------------------------------
// Launchers.

hipError_t launch_init_sources(const int64_t *d_src_off, const int64_t *d_t, const uint8_t *d_v,
                               int64_t S, int64_t n_in, int64_t *off, int64_t *len, uint64_t *K,
                               DevState *state, int64_t capacity, hipStream_t s) {
    const int64_t work = n_in > S ? n_in : S;
    int64_t nb = (work + 255) / 256;
    nb = nb < 1 ? 1 : nb > 8192 ? 8192 : nb;
    init_sources_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(d_src_off, d_t, d_v, S, n_in,
                                                                off, len, K, state, capacity);
    return hipGetLastError();
}

hipError_t launch_size(const StepArgs &a, hipStream_t s) {
    if (a.n_sblocks == 0) return hipSuccess;
    size_kernel<<<dim3((unsigned)a.n_sblocks), dim3(kSizeBlock), 0, s>>>(a);
    return hipGetLastError();
}


hipError_t launch_eval_wave(const StepArgs &a, int variant, const int64_t *max_items, int form,
                            hipStream_t s) {
    const int64_t total = max_items[0] + max_items[1] + max_items[2] + max_items[3];
    if (total <= 0) return hipSuccess;
    const dim3 grid((unsigned)total), block(64);
    if (form == kFormSegmented) {
        switch (variant) {
        case wave_variant(0, 0): eval_seg_kernel<kWindowSmall, false><<<grid, block, 0, s>>>(a, variant); break;
        case wave_variant(1, 0): eval_seg_kernel<kWindowLarge, false><<<grid, block, 0, s>>>(a, variant); break;
        case wave_variant(0, 1): eval_seg_kernel<kWindowSmall, true><<<grid, block, 0, s>>>(a, variant); break;
        default: eval_seg_kernel<kWindowLarge, true><<<grid, block, 0, s>>>(a, variant); break;
        }
        return hipGetLastError();
    }
    switch (variant) {
    case wave_variant(0, 0): eval_wave_kernel<kWindowSmall, false><<<grid, block, 0, s>>>(a, variant); break;
    case wave_variant(1, 0): eval_wave_kernel<kWindowLarge, false><<<grid, block, 0, s>>>(a, variant); break;
    case wave_variant(0, 1): eval_wave_kernel<kWindowSmall, true><<<grid, block, 0, s>>>(a, variant); break;
    default: eval_wave_kernel<kWindowLarge, true><<<grid, block, 0, s>>>(a, variant); break;
    }
    return hipGetLastError();
}

hipError_t launch_sort_lists(const StepArgs &a, const int64_t *max_items, hipStream_t s) {
    ListBounds lb;
    lb.cum[0] = 0;
    for (int c = 0; c < kListLane; c++) lb.cum[c + 1] = lb.cum[c] + max_items[c];
    if (lb.cum[kListLane] <= 0 && a.n_jobs <= 0) return hipSuccess;
    constexpr int kThreads = kVariants * kSegments;
    int64_t blocks = (lb.cum[kListLane] + kThreads - 1) / kThreads;
    blocks = blocks > a.n_jobs ? blocks : a.n_jobs;
    sort_lists_kernel<<<dim3((unsigned)blocks), dim3(kThreads), 0, s>>>(a, lb);
    return hipGetLastError();
}

hipError_t launch_eval_lane(const StepArgs &a, int64_t max_items, hipStream_t s) {
    if (max_items <= 0) return hipSuccess;
    eval_lane_kernel<<<dim3((unsigned)((max_items + 63) / 64)), dim3(64), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_df_init(const DfArgs &a, const int32_t *pend0, hipStream_t s) {
    const int64_t n = a.G > 1 ? a.G : 1;
    df_init_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(a, pend0);
    return hipGetLastError();
}

hipError_t launch_dataflow(const DfArgs &a, int64_t n_waves, hipStream_t s) {
    if (a.G <= 0 || n_waves <= 0) return hipSuccess;
    const dim3 grid((unsigned)n_waves), block(64);
    if (a.job.edly) dataflow_kernel<true><<<grid, block, 0, s>>>(a);
    else dataflow_kernel<false><<<grid, block, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t levelsync_max_waves(int n_cu, int64_t *out) {
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, levelsync_kernel<false>, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, levelsync_kernel<true>, 64, 0);
    if (e != hipSuccess) return e;
    *out = (int64_t)n_cu * (a < b ? a : b);
    return hipSuccess;
}

// A cooperative launch: the runtime starts it only with every wavefront
// resident at once, which the barrier needs.
hipError_t launch_levelsync(const LsArgs &a, int64_t n_waves, hipStream_t s) {
    if (a.n_levels <= 0 || n_waves <= 0) return hipSuccess;
    if (n_waves > kLsMaxWaves) return hipErrorInvalidValue;
    hipError_t e = launch_clear_u32(a.sync, kLsSyncWords, s);
    if (e != hipSuccess) return e;
    LsArgs arg = a;
    void *params[] = {&arg};
    const dim3 grid((unsigned)n_waves), block(64);
    if (a.job.edly) return hipLaunchCooperativeKernel(levelsync_kernel<true>, grid, block, params, 0, s);
    return hipLaunchCooperativeKernel(levelsync_kernel<false>, grid, block, params, 0, s);
}

hipError_t launch_hash(const int64_t *nets_off, const int64_t *nets_len, int64_t n_nets,
                       const uint64_t *K, uint64_t *out, hipStream_t s) {
    if (n_nets <= 0) return hipSuccess;
    const int64_t waves = n_nets < (1 << 16) ? n_nets : (1 << 16);
    hash_kernel<<<dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s>>>(nets_off, nets_len, n_nets, K, out);
    return hipGetLastError();
}

hipError_t launch_gather_meta(const int64_t *net, int64_t n, const int64_t *off, const int64_t *len,
                              int64_t *out_off, int64_t *out_len, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    gather_meta_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(net, n, off, len, out_off,
                                                                              out_len);
    return hipGetLastError();
}

hipError_t launch_clear_u32(uint32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    clear_u32_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_count_out(const int64_t *len, int64_t S, int64_t G, int64_t *partial,
                            int64_t n_partial, DevState *state, hipStream_t s) {
    count_partial_kernel<<<dim3((unsigned)n_partial), dim3(256), 0, s>>>(len, S, G, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    count_final_kernel<<<dim3(1), dim3(64), 0, s>>>(partial, n_partial, state);
    return hipGetLastError();
}

hipError_t launch_gather(const int64_t *src_off, const int64_t *n_items, const int64_t *dst_off,
                         int64_t n_nets, const uint64_t *K, int64_t *out_t, uint8_t *out_v,
                         hipStream_t s) {
    if (n_nets == 0) return hipSuccess;
    const int64_t nb = n_nets < 65536 ? n_nets : 65536;
    gather_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(src_off, n_items, dst_off, n_nets, K,
                                                          out_t, out_v);
    return hipGetLastError();
}

hipError_t launch_write_descs(const DescBatch &b, hipStream_t s) {
    if (b.n <= 0) return hipSuccess;
    write_descs_kernel<<<dim3(1), dim3(kDescBatch), 0, s>>>(b);
    return hipGetLastError();
}

hipError_t launch_run_result(const DevState *st, int64_t *out, hipStream_t s) {
    run_result_kernel<<<dim3(1), dim3(64), 0, s>>>(st, out);
    return hipGetLastError();
}

}  // namespace gsim
