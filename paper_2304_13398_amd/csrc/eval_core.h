// Device code of the per-gate evaluation shared by the level and the
// dependency-driven kernels: wave-wide primitives, the wavefront-per-gate
// procedure (eval_gate) and the lane-per-gate one (eval_seq).
#pragma once

#include "gsim_internal.h"

// Qualifier of pointers into device global memory (the emulator of tests/emu
// defines it empty).
#ifndef gsim_global
#define gsim_global __attribute__((address_space(1)))
#endif

namespace gsim {

namespace {

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_down_u64(uint64_t x, int d) {
    const uint32_t lo = (uint32_t)__shfl_down((int)(uint32_t)x, d, 64);
    const uint32_t hi = (uint32_t)__shfl_down((int)(uint32_t)(x >> 32), d, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int64_t shfl_down64(int64_t x, int d) {
    return (int64_t)shfl_down_u64((uint64_t)x, d);
}

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

// A value every lane holds alike, moved to scalar registers, so that what is
// computed from it (and branches on it) stays off the vector unit.
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// Delay of one pin for a new output value: 1 -> rise, 0 -> fall, X -> the
// smaller of the two.
__device__ __forceinline__ int32_t pin_delay(int32_t rise, int32_t fall, uint32_t v) {
    return v == 1 ? rise : v == 0 ? fall : (rise < fall ? rise : fall);
}

// -------------------------------------------------------------------------
// Wave-wide scans with DPP (GFX9 row shifts and row broadcasts): inclusive,
// in lane order, 12 VALU operations and no LDS traffic.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowShl1 = 0x101, kDppRowShl2 = 0x102, kDppRowShl4 = 0x104, kDppRowShl8 = 0x108;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t identity, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)x, CTRL, ROW_MASK, 0xf, false);
}

// The same move with every row and bank enabled and out-of-range source lanes
// reading 0: every lane is written, so no register is set up for `old`.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32_zero(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
}

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }


__device__ __forceinline__ uint32_t wave_prefix_sum(uint32_t x) {
    x += dpp_u32<kDppRowShr1>(0u, x);
    x += dpp_u32<kDppRowShr2>(0u, x);
    x += dpp_u32<kDppRowShr4>(0u, x);
    x += dpp_u32<kDppRowShr8>(0u, x);
    x += dpp_u32<kDppRowBcast15, 0xa>(0u, x);
    x += dpp_u32<kDppRowBcast31, 0xc>(0u, x);
    return x;
}

// The value of the previous lane (identity on lane 0).
__device__ __forceinline__ uint32_t wave_shift_up(uint32_t identity, uint32_t x) {
    return dpp_u32<kDppWaveShr1>(identity, x);
}

// The value of the next lane (identity on lane 63).
__device__ __forceinline__ uint32_t wave_shift_down(uint32_t identity, uint32_t x) {
    return dpp_u32<kDppWaveShl1>(identity, x);
}

// -------------------------------------------------------------------------
// Wavefront-per-gate evaluation.
//
// The per-gate procedure (Algorithm 2 with Eq. 1 and the Fig. 3 drop) is
// computed in the following equivalent data-parallel form. Let the distinct
// merged input times be t_1 < t_2 < ... and e_i the gate value once every
// input transition at or before t_i is applied (e_0 = X). A candidate is an
// i with e_i != e_{i-1}; it appears at r_i = t_i + the minimum delay over the
// pins with a transition at t_i. Appending candidates in order while denying
// every earlier one with an appearance time >= r_i (Eq. 1) keeps exactly the
// candidates j with r_j < r_k for every later candidate k (survivors); and
// dropping a transition equal to the output's current value (Fig. 3) is the
// same as keeping, among the survivors, those whose value differs from the
// previous survivor's (X before the first).
//
// The wave walks the inputs in rounds of up to 512 transitions. Each pin
// loads a tile of its next transitions (512 for one pin; 384, 256 and 192
// each for two, three and four pins: more than a round takes, so that one
// pin whose tile ends early does not cut the round short). The round's
// horizon H is the smallest last-loaded time over pins that have more
// transitions beyond their tile, capped so the round spans less than 2^28
// ps, and lowered to just before the time of the 513th merged transition
// (four pins: of the 257th of either pairwise merge) when there are more;
// every input transition at or before H is in the round. In-round inputs are
// 32-bit keys offset << 4 | value << 2 | pin (offset from the round's base),
// so the merged order of the round is plain key order (by time; the order
// inside a time group does not matter). The merge is done per lane: lane l
// owns merged positions [8l, 8l + 8), finds where they start in the two
// sorted lists it merges by a merge-path search, and takes the 8 smallest of
// the next 8 of each list with a bitonic network (three pins: the first 512
// of the first two through LDS, then with the third; four pins: the first
// 256 of each pair through LDS, then one more merge). Tiles are held as the
// low 32 bits of the packed transitions; a tile keeps only transitions whose
// high word equals its first one's (the rest wait for a later round), so
// one uniform word completes every key of the tile. Each lane applies its
// transitions to the pin values before its first position: with one pin the
// previous lane's last key gives them, with two the key before the
// merge-path split in each pin's tile, with three or four a wave scan of "set
// pin p to v" updates. A transition ends a time group when the next one has
// another time; the group's candidate takes its delay from a per-gate table
// indexed by new value and the set of pins in the group, and is kept if the
// gate value differs from the one after the previous group (decided after
// the pass for a group that began in the previous lane). Candidates appear
// at 32-bit offsets (offset << 2 | value). Survivors come from a suffix minimum over
// the round (DPP scans). A survivor with r <= H is final (later candidates
// appear after H); the others stay tentative in LDS and are re-tested
// against the next rounds -- at most W of them exist for gates whose largest
// pin delay is at most W (see kWindowSmall). The next round's tiles are
// prefetched into registers while the current one runs.
constexpr int kMergePad = 8;                       // INF keys after each sorted list
// pairwise-merge outputs with guards: two of 256 (four pins) or one of 512 (three)
constexpr int kMergeBuf = 2 * (256 + kMergePad + 1);
static_assert(kMergeBuf >= 512 + kMergePad + 1, "the three-pin merge buffer fits");

constexpr int kTileWords = 4 * (192 + 1 + kMergePad);  // the largest of the K x tile layouts
static_assert(kTileWords >= 512 + 1 + kMergePad && kTileWords >= 2 * (384 + 1 + kMergePad) &&
                  kTileWords >= 3 * (256 + 1 + kMergePad),
              "every pin count's tiles fit");

template <int W>
struct WaveLds {
    uint32_t seq[W + kRoundSlots + 32];  // tentative survivors [0, nq), then this round's;
                                         // the pairwise-merge buffers alias seq[W, W + kMergeBuf)
    uint32_t tile[kTileWords];           // K x [guard, T keys, 8 INF]
    uint32_t dtab[48];                   // by (new value e, set of changed pins): the smallest
                                         // delay d over those pins, as d << 2 | e
    uint32_t etab[12];                   // edge model: per (pin, edge class) the delays to
                                         // 0, 1 and X in 10-bit fields (kEdgeNone = unrelated)
    uint8_t lut[256];
};
static_assert(kMergeBuf <= kRoundSlots + 32, "merge buffers must fit the survivor area");

template <int K>
struct Tiling {
    // transitions loaded per pin; tile p of LDS is [guard, T keys, 8 INF]
    static constexpr int T = K == 1 ? 512 : K == 2 ? 384 : K == 3 ? 256 : 192;
    static constexpr int E = T / 64;  // per lane
    static constexpr int OFF(int p) { return p * (T + 1 + kMergePad); }
    static constexpr int WORDS = K * (T + 1 + kMergePad);
};
static_assert(kRoundSlots == 512, "tiling assumes 512-transition rounds");

constexpr uint32_t kNoKey32 = 0xFFFFFFFFu;
constexpr uint32_t kNoTime28 = kNoKey32 >> 4;
// Largest in-round time offset: input keys offset << 4 | value << 2 | pin stay
// below kNoKey32, and candidate offsets (<= kSpan + kWindowLarge) stay below
// 2^30, so candidate keys offset << 2 | value never reach kNoKey32 either.
constexpr int64_t kSpan = (int64_t(1) << 28) - 2;

__device__ __forceinline__ void cswap(uint32_t &a, uint32_t &b) {
    const uint32_t lo = umin32(a, b);
    b = a < b ? b : a;
    a = lo;
}

// Merged positions [d, d + 8) of the sorted lists A[0, a) and B[0, b) (keys
// distinct, each list followed by kMergePad kNoKey32, B preceded by a zero
// guard word); positions past a + b come out as kNoKey32. NIT search steps
// cover split ranges up to 2^NIT - 1. Once the search has converged, its
// test is false by itself (A's pad or B's guard decides it), so the steps
// need no check that the range is still open; CHECKED keeps that check (the
// dependency-driven kernel: without it, its register allocation spills).
template <int NIT, bool CHECKED>
__device__ __forceinline__ int merge8(const uint32_t *A, int a, const uint32_t *B, int b, int d,
                                      uint32_t (&c)[8]) {
    d = d < a + b ? d : a + b;
    int lo = d - b > 0 ? d - b : 0;
    int hi = d < a ? d : a;
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const int mid = (lo + hi) >> 1;
        const bool less = A[mid] < B[d - 1 - mid];
        const bool go = !CHECKED || lo < hi;
        lo = go && less ? mid + 1 : lo;
        hi = go && !less ? mid : hi;
    }
    const uint32_t *pa = A + lo, *pb = B + (d - lo);
#pragma unroll
    for (int k = 0; k < 8; k++) c[k] = umin32(pa[k], pb[7 - k]);  // the 8 smallest, bitonic
    cswap(c[0], c[4]); cswap(c[1], c[5]); cswap(c[2], c[6]); cswap(c[3], c[7]);
    cswap(c[0], c[2]); cswap(c[1], c[3]); cswap(c[4], c[6]); cswap(c[5], c[7]);
    cswap(c[0], c[1]); cswap(c[2], c[3]); cswap(c[4], c[5]); cswap(c[6], c[7]);
    return lo;  // keys of A among the first min(d, a + b) merged
}

// Pin-state updates: bits [2p, 2p+2) hold pin p's new value, bits [8+2p,
// 8+2p+2) mark pin p as set. compose(earlier, later) applies both in order.
__device__ __forceinline__ uint32_t compose_upd(uint32_t e, uint32_t l) {
    return (e & ~((l >> 8) & 0xFFu)) | l;
}

__device__ __forceinline__ uint32_t wave_prefix_compose(uint32_t x) {
    // (0 is the identity update)
    x = compose_upd(dpp_u32_zero<kDppRowShr1>(x), x);
    x = compose_upd(dpp_u32_zero<kDppRowShr2>(x), x);
    x = compose_upd(dpp_u32_zero<kDppRowShr4>(x), x);
    x = compose_upd(dpp_u32_zero<kDppRowShr8>(x), x);
    x = compose_upd(dpp_u32<kDppRowBcast15, 0xa>(0u, x), x);
    x = compose_upd(dpp_u32<kDppRowBcast31, 0xc>(0u, x), x);
    return x;
}

// Inclusive minimum over this lane and every higher lane.
__device__ __forceinline__ uint32_t wave_suffix_min(uint32_t x) {
    x = umin32(x, dpp_u32<kDppRowShl1>(~0u, x));
    x = umin32(x, dpp_u32<kDppRowShl2>(~0u, x));
    x = umin32(x, dpp_u32<kDppRowShl4>(~0u, x));
    x = umin32(x, dpp_u32<kDppRowShl8>(~0u, x));
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 16);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 32);
    const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
    const uint32_t s2 = r3, s1 = umin32(r2, r3), s0 = umin32(r1, s1);
    const int row = lane_id() >> 4;
    const uint32_t later_rows = row == 0 ? s0 : row == 1 ? s1 : row == 2 ? s2 : kNoKey32;
    return umin32(x, later_rows);
}

// Edge class of a pin change (extended delay model): 0 rise (new value 1, or
// 0 -> X/Z), 1 fall (new value 0, or 1 -> X/Z), 2 both (X <-> Z).
__device__ __forceinline__ uint32_t edge_class(uint32_t old_v, uint32_t new_v) {
    return (new_v == 1u || (old_v == 0u && new_v >= 2u)) ? 0u
           : (new_v == 0u || (old_v == 1u && new_v >= 2u)) ? 1u : 2u;
}
constexpr uint32_t kEdgeNone = 1023u;  // a 10-bit delay field of an unrelated pin

// A store of a gate's results. AGENT (dependency-driven kernel): agent scope,
// written through to memory, because every gate there ends with a release
// fence whose cost is the write-back of the cache lines left dirty (measured
// on MI355X: 1M release fences after 4 KB of plain stores each take 21.6 ms,
// after agent-scope stores 8.0 ms, alone 0.03 ms). Plain elsewhere.
template <bool AGENT, typename T>
__device__ __forceinline__ void put(T *p, T v) {
    if constexpr (AGENT) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

// One pin's tile: the low words of up to T of its next packed transitions
// (one per lane and register); lane 0 of aux holds the high word of the
// first, lane 1 that of the last (LEAN: lane 2 the low word of the last).
template <int T>
struct PinTile {
    uint32_t lo[T / 64];
    uint32_t aux;
    int n;  // transitions loaded
};

// Start loading the tile at src (r transitions left there); nothing waits.
template <int T, bool LEAN>
__device__ __forceinline__ void tile_fetch(const uint64_t *src, int64_t r, PinTile<T> &t) {
    const int lane = lane_id();
    t.n = (int)min64(r, (int64_t)T);
    if constexpr (LEAN) {
        // straight-line loads from one scalar base; lanes past the tile load
        // its last transition again (entries past n are never used)
        if (t.n > 0) {
            const uint64_t a = (uint64_t)src;
            const uint32_t a_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
            const uint32_t a_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
            // a global-memory pointer, so that the loads take the scalar base and
            // a 32-bit lane offset (a generic pointer costs a 64-bit address per lane)
            const gsim_global uint32_t *s32 =
                (const gsim_global uint32_t *)reinterpret_cast<const uint32_t *>(((uint64_t)a_hi << 32) | a_lo);
            const int last = t.n - 1;
#pragma unroll
            for (int e = 0; e < T / 64; e++) {
                const int i = lane + 64 * e < last ? lane + 64 * e : last;
                t.lo[e] = s32[2 * i];  // low word first
            }
            t.aux = s32[lane == 0 ? 1 : lane == 1 ? 2 * last + 1 : 2 * last];
        } else {
            // nothing is loaded; the tile's words are never read (its count is 0)
            const uint32_t z = 0u;
#pragma unroll
            for (int e = 0; e < T / 64; e++) t.lo[e] = __builtin_nondeterministic_value(z);
            t.aux = __builtin_nondeterministic_value(z);
        }
    } else {
        const uint32_t *s32 = reinterpret_cast<const uint32_t *>(src);  // low word first
#pragma unroll
        for (int e = 0; e < T / 64; e++) t.lo[e] = lane + 64 * e < t.n ? s32[2 * (lane + 64 * e)] : 0u;
        t.aux = lane < 2 && t.n > 0 ? s32[lane == 0 ? 1 : 2 * (t.n - 1) + 1] : 0u;
    }
}

// A loaded tile as the round uses it: the transitions [0, lim) that share the
// first one's high word hi; the time of its first transition; and the pin's
// horizon hp -- every transition of the pin up to hp is in [0, lim) (kInf if
// the tile holds all r that are left).
template <int T, bool LEAN>
__device__ __forceinline__ void tile_settle(const uint64_t *src, int64_t r, const PinTile<T> &t, int &lim,
                                            uint32_t &hi, int64_t &t0, int64_t &hp) {
    lim = t.n;
    hi = 0xFFFFFFFFu;
    t0 = kInf;
    hp = kInf;
    if (t.n == 0) return;
    hi = (uint32_t)__builtin_amdgcn_readlane((int)t.aux, 0);
    const uint32_t hi_last = (uint32_t)__builtin_amdgcn_readlane((int)t.aux, 1);
    const uint32_t lo_first = (uint32_t)__builtin_amdgcn_readlane((int)t.lo[0], 0);
    t0 = key_time(((uint64_t)hi << 32) | lo_first);
    if (r > t.n) {
        uint32_t lo_last;
        if constexpr (LEAN) {
            lo_last = (uint32_t)__builtin_amdgcn_readlane((int)t.aux, 2);
        } else {
            const int e_last = (t.n - 1) >> 6;
            uint32_t v = t.lo[0];
#pragma unroll
            for (int e = 1; e < T / 64; e++) v = e == e_last ? t.lo[e] : v;
            lo_last = (uint32_t)__builtin_amdgcn_readlane((int)v, (t.n - 1) & 63);
        }
        hp = key_time(((uint64_t)hi_last << 32) | lo_last);
    }
    if (hi_last != hi) {
        // rare: the tile reaches a later high word; keep the transitions before
        // it (a prefix, the tile being sorted)
        const uint32_t *s32 = reinterpret_cast<const uint32_t *>(src);
        const int lane = lane_id();
        int c = 0;
#pragma unroll
        for (int e = 0; e < T / 64; e++) {
            const int i = lane + 64 * e;
            c += __popcll(__ballot(i < t.n && s32[2 * i + 1] == hi));
        }
        lim = c;
        hp = (((int64_t)hi + 1) << 30) - 1;  // the last time with high word hi
    }
}

// PREFETCH: the next round's tiles load while the round runs (more
// registers); otherwise at the end of the round. LEAN (level kernel): the
// last loaded transition comes from an extra lane of the tile's auxiliary
// register, and the lane's trailing time group is looked for among its last
// K positions only (at most one transition per pin shares a time). The
// dependency-driven kernel keeps the longer form of both. One of its runs
// with the shorter form once did not finish; the cause found since was in
// that kernel's publication order (fixed), and the shorter form gives the
// oracle's result on every gate under the CPU wave emulator, but it has not
// run in that kernel on the device since.
template <int K, int W, bool EDGE, bool PREFETCH, bool LEAN, bool AGENT>
__device__ __forceinline__ void eval_gate(const JobDesc &J, int64_t ob, const GateRec &R,
                                          int64_t gate, WaveLds<W> &L) {
    using Tl = Tiling<K>;
    constexpr int TT = Tl::T;
    constexpr int E = Tl::E;
    const int lane = lane_id();
    const int64_t S = J.S;
    int64_t *len = J.len;
    int64_t *off = J.off;
    uint64_t *Kar = J.K;

    int64_t pb[K], pl[K], cur[K];
    int64_t reserved = 0;  // slots sized for this gate: the sum of its input lengths
#pragma unroll
    for (int p = 0; p < K; p++) {
        pb[p] = off[R.net[p]];
        pl[p] = len[R.net[p]];
        cur[p] = 0;
        reserved += pl[p];
    }
    uint32_t state0 = 0;  // pin values before the round, 2 bits per pin
#pragma unroll
    for (int p = 0; p < K; p++) state0 |= (uint32_t)kX << (2 * p);

    PinTile<TT> tl[K];  // this round's tiles
#pragma unroll
    for (int p = 0; p < K; p++) tile_fetch<TT, LEAN>(Kar + pb[p], pl[p], tl[p]);
    // INF keys after each tile, a zero guard before it (merge8); the delay table
#pragma unroll
    for (int p = 0; p < K; p++) {
        if (lane < kMergePad) L.tile[Tl::OFF(p) + 1 + TT + lane] = kNoKey32;
        if (!AGENT && lane == kMergePad) L.tile[Tl::OFF(p)] = 0u;  // (the checked search needs none)
    }
    if (EDGE) {
        // per (pin, edge class): delays to 0, 1 and X; finite ones are <= W
        if (lane < 3 * K) {
            const int pin = lane / 3, c = lane % 3;
            const int32_t *d = J.edly + (size_t)gate * 16 + pin * 4;  // [edge][out]
            uint32_t f[3];
#pragma unroll
            for (int o = 0; o < 2; o++) {
                const int32_t a = c == 1 ? kNoRelation : d[o], b = c == 0 ? kNoRelation : d[2 + o];
                const int32_t m = a < b ? a : b;
                f[o] = m == kNoRelation ? kEdgeNone : (uint32_t)m;
            }
            f[2] = f[0] < f[1] ? f[0] : f[1];
            L.etab[lane] = f[0] | f[1] << 10 | f[2] << 20;
        }
    } else if (lane < 48) {
        const uint32_t ev = (uint32_t)lane >> 4, mask = (uint32_t)lane & 15u;
        int32_t d = INT32_MAX;
#pragma unroll
        for (int q = 0; q < K; q++)
            if (mask & (1u << q)) {
                const int32_t dq = pin_delay(R.rise[q], R.fall[q], ev);
                d = dq < d ? dq : d;
            }
        L.dtab[lane] = (uint32_t)d << 2 | ev;  // (the empty set, d = INT32_MAX, is never read)
    }

    uint32_t last_val = kX;  // value of the last final survivor
    bool first_round = true; // the gate's previous value is X until its first input change
    int nq = 0;              // tentative survivors in L.seq[0, nq), offsets from base_prev
    int64_t base_prev = 0;
    int64_t out_n = 0;
    uint32_t *const AB = L.seq + W + 1;                    // pairwise merges (K >= 3)
    uint32_t *const CD = AB + 256 + kMergePad + 1;         // (K == 4)

    bool stalled = false;  // the last round made no progress (see below)
    for (;;) {
        // the loop-carried counts are the same on every lane; restating that
        // here lets the compiler keep the loop's control and the pins'
        // bookkeeping on the scalar unit (otherwise it treats the loop as
        // divergent and carries them in vector registers)
        nq = __builtin_amdgcn_readfirstlane(nq);
#pragma unroll
        for (int p = 0; p < K; p++) cur[p] = uniform64(cur[p]);
        int64_t rem[K];
        bool more = nq > 0 && !stalled;
#pragma unroll
        for (int p = 0; p < K; p++) {
            rem[p] = pl[p] - cur[p];
            more |= rem[p] > 0 && !stalled;
        }
        if (!more) break;

        // ---- base (earliest pending time), horizon from the tiles
        int lim[K];
        uint32_t thi[K];
        int64_t H = kInf, base = kInf;
#pragma unroll
        for (int p = 0; p < K; p++) {
            int64_t t0, hp;
            tile_settle<TT, LEAN>(Kar + pb[p] + cur[p], rem[p], tl[p], lim[p], thi[p], t0, hp);
            H = min64(H, hp);
            base = min64(base, t0);
        }
        if (nq > 0) {
            // every lane takes lane 0's read (in scalar registers) before
            // lane 0 rewrites that word just below
            const uint32_t q0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)L.seq[0]);
            base = min64(base, base_prev + (int64_t)(q0 >> 2));
            const uint32_t shift = (uint32_t)(base - base_prev) << 2;
            for (int c = lane; c < nq; c += 64) L.seq[c] -= shift;
        }
        H = min64(H, base + kSpan);
        const uint64_t hkey = H < kTimeLimit ? pack_key(H, 3u) : ~uint64_t(0);  // last key of the round
        const uint32_t base4 = (uint32_t)pack_key(base, 0u);  // low word of base << 2
        const uint32_t hk_hi = (uint32_t)(hkey >> 32);
        int m[K];
#pragma unroll
        for (int p = 0; p < K; p++) {
            // a tile key is at or before H by its (uniform) high word, else by
            // its low word. Both bounds go through scalar registers, so each
            // test below is one compare, and the count is the AND of two
            // ballots (a ballot of the conjunction would cost two vector
            // instructions more per key)
            const uint32_t lo_max =
                (uint32_t)__builtin_amdgcn_readfirstlane((int)(thi[p] < hk_hi ? 0xFFFFFFFFu : (uint32_t)hkey));
            const int lim_in = __builtin_amdgcn_readfirstlane(thi[p] > hk_hi ? 0 : lim[p]);
            m[p] = 0;
#pragma unroll
            for (int e = 0; e < E; e++) {
                const uint32_t lo = tl[p].lo[e];
                const bool in_lane = lane + 64 * e < lim_in, in_time = lo <= lo_max;
                const bool in = in_lane && in_time;
                m[p] += __popcll(__ballot(in_lane) & __ballot(in_time));
                // (t - base) << 2 | v < 2^30 equals the low word of key - (base << 2)
                L.tile[Tl::OFF(p) + 1 + 64 * e + lane] = in ? ((lo - base4) << 2) | (uint32_t)p : kNoKey32;
            }
        }
        __syncthreads();

        // ---- merged positions [8 lane, 8 lane + 8) of the round; the time
        // of a merged key past the round's 512 (pairs: 256) slots
        uint32_t mk[8];
        uint32_t cut = kNoTime28;
        int split = 0, merged = 0;  // two pins: keys of pin 0 before this lane's first position; keys merged
        if constexpr (K == 1) {
#pragma unroll
            for (int k = 0; k < 8; k++) mk[k] = L.tile[1 + 8 * lane + k];
        } else if constexpr (K == 2) {
            split = merge8<9, AGENT>(L.tile + Tl::OFF(0) + 1, m[0], L.tile + Tl::OFF(1) + 1, m[1], 8 * lane, mk);
            merged = m[0] + m[1];
            if (m[0] + m[1] > 512) cut = (uint32_t)__builtin_amdgcn_readlane((int)mk[7], 63) >> 4;
        } else if constexpr (K == 3) {
            // the first 512 of pins 0 and 1 into AB, then AB with pin 2's tile
            {
                uint32_t h[8];
                merge8<9, AGENT>(L.tile + Tl::OFF(0) + 1, m[0], L.tile + Tl::OFF(1) + 1, m[1], 8 * lane, h);
#pragma unroll
                for (int k = 0; k < 8; k++) AB[8 * lane + k] = h[k];
                if (lane < kMergePad) AB[512 + lane] = kNoKey32;
            }
            __syncthreads();
            const int ab = m[0] + m[1] < 512 ? m[0] + m[1] : 512;
            merge8<9, AGENT>(AB, ab, L.tile + Tl::OFF(2) + 1, m[2], 8 * lane, mk);
            if (m[0] + m[1] + m[2] > 512) cut = (uint32_t)__builtin_amdgcn_readlane((int)mk[7], 63) >> 4;
        } else {
            // the first 256 of one pair of pins (lanes 0-31) and of the other
            // (lanes 32-63). A pair ends the round at its 257th key, so the
            // pins are paired to make the larger pair's in-round count as
            // small as possible (the keys carry their pin; any pairing gives
            // the same merged order)
            int q1 = 1, q2 = 2, q3 = 3;  // pairs (0, q1) and (q2, q3)
            {
                const int a01 = m[0] + m[1], a23 = m[2] + m[K - 1], a02 = m[0] + m[2],
                          a13 = m[1] + m[K - 1], a03 = m[0] + m[K - 1], a12 = m[1] + m[2];
                const int s01 = a01 > a23 ? a01 : a23, s02 = a02 > a13 ? a02 : a13,
                          s03 = a03 > a12 ? a03 : a12;
                if (s02 < s01 && s02 <= s03) { q1 = 2; q2 = 1; }
                else if (s03 < s01 && s03 < s02) { q1 = 3; q2 = 1; q3 = 2; }
            }
            const int m_q1 = q1 == 1 ? m[1] : q1 == 2 ? m[2] : m[K - 1];
            const int m_q2 = q2 == 1 ? m[1] : m[2];
            const int m_q3 = q3 == 2 ? m[2] : m[K - 1];
            const int n_ab = m[0] + m_q1, n_cd = m_q2 + m_q3;
            const bool hi_half = lane >= 32;
            const uint32_t *A = L.tile + (hi_half ? q2 * (TT + 1 + kMergePad) : Tl::OFF(0)) + 1;
            const uint32_t *B = L.tile + (hi_half ? q3 : q1) * (TT + 1 + kMergePad) + 1;
            const int a = hi_half ? m_q2 : m[0];
            const int b = hi_half ? m_q3 : m_q1;
            uint32_t h[8];
            merge8<8, AGENT>(A, a, B, b, 8 * (lane & 31), h);
            uint32_t *dst = (hi_half ? CD : AB) + 8 * (lane & 31);
#pragma unroll
            for (int k = 0; k < 8; k++) dst[k] = h[k];
            if (lane < 2 * kMergePad) (lane < kMergePad ? AB : CD)[256 + (lane % kMergePad)] = kNoKey32;
            if (!AGENT && lane == 2 * kMergePad) CD[-1] = 0u;  // the second list's guard (after AB's pads)
            const uint32_t c_ab = (uint32_t)__builtin_amdgcn_readlane((int)h[7], 31) >> 4;
            const uint32_t c_cd = (uint32_t)__builtin_amdgcn_readlane((int)h[7], 63) >> 4;
            if (n_ab > 256) cut = c_ab;
            if (n_cd > 256) cut = umin32(cut, c_cd);
            __syncthreads();
            merge8<9, AGENT>(AB, n_ab < 256 ? n_ab : 256, CD, n_cd < 256 ? n_cd : 256, 8 * lane, mk);
        }
        if (cut != kNoTime28 && (int64_t)cut - 1 < H - base) {
            // the round ends before the cut key's time: fewer keys of each pin are in
            H = base + (int64_t)cut - 1;
            const uint32_t hoff = cut - 1;
            const uint32_t hk32 = hoff << 4 | 15u;
#pragma unroll
            for (int k = 0; k < 8; k++) mk[k] = mk[k] <= hk32 ? mk[k] : kNoKey32;
            // in-round keys per pin: a prefix of its sorted LDS tile (the rest
            // of the tile and its pads hold kNoKey32). Lane j tests the last
            // key of block [8j, 8j + 8); the full blocks counted, lanes 0-7
            // test the keys of the next block.
#pragma unroll
            for (int p = 0; p < K; p++) {
                const uint32_t *tp = L.tile + Tl::OFF(p) + 1;
                constexpr int kBlocks = TT / 8;
                const uint32_t k1 = tp[lane < kBlocks ? 8 * lane + 7 : TT - 1];
                const int c1 = __popcll(__ballot(lane < kBlocks && k1 <= hk32));
                const uint32_t k2 = tp[8 * c1 + (lane & 7)];  // < TT + 8: inside the tile and its pads
                m[p] = 8 * c1 + __popcll(__ballot(lane < 8 && k2 <= hk32));
            }
        }
        bool all_in = true;
#pragma unroll
        for (int p = 0; p < K; p++) all_in = all_in && m[p] == rem[p];
        // split horizon: with every remaining input in this round, all survivors are final
        const uint32_t hsplit = all_in ? kNoKey32 : (uint32_t)(H - base) << 2 | 3u;
        constexpr bool kPrefetch = PREFETCH;

        // ---- pin values before this lane's first position (st) and after
        // the round (st_round); the pins of this lane's trailing time group
        uint32_t st, st_round, trail_mask = 0;
        const uint32_t t_last = mk[7] >> 4;
        if constexpr (K <= 2) {
            // each pin's value is that of its last key before the lane's first
            // position: with one pin the previous lane's last key; with two
            // the key before the merge-path split in each pin's tile (the
            // split is exact for every lane that still holds a key of the
            // round after a cut)
            if constexpr (K == 1) {
                const uint32_t prev = dpp_u32_zero<kDppWaveShr1>(mk[7]);
                st = lane == 0 ? state0 : (prev >> 2) & 3u;
            } else {
                const int d = 8 * lane < merged ? 8 * lane : merged;
                const int na = split, nb = d - split;
                const uint32_t ka = L.tile[Tl::OFF(0) + na];  // key na - 1 of pin 0 (the guard if na = 0)
                const uint32_t kb = L.tile[Tl::OFF(1) + nb];
                st = (na > 0 ? (ka >> 2) & 3u : state0 & 3u) | (nb > 0 ? (kb >> 2) & 3u : (state0 >> 2) & 3u) << 2;
            }
            st_round = state0;
#pragma unroll
            for (int p = 0; p < K; p++)
                if (m[p] > 0) {
                    const uint32_t kl = (uint32_t)__builtin_amdgcn_readfirstlane((int)L.tile[Tl::OFF(p) + m[p]]);
                    st_round = (st_round & ~(3u << (2 * p))) | (((kl >> 2) & 3u) << (2 * p));
                }
#pragma unroll
            for (int k = LEAN ? 8 - K : 0; k < 8; k++) {
                const uint32_t sh = K == 1 ? 0u : (mk[k] & 3u) * 2u;
                trail_mask |= (mk[k] >> 4) == t_last ? 1u << (sh >> 1) : 0u;
            }
        } else {
            // this lane's composed update, scanned over the wave
            uint32_t upd = 0;
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const uint32_t sh = (mk[k] & 3u) * 2u;
                const bool valid = mk[k] != kNoKey32;
                const uint32_t nu = (upd & ~(0x303u << sh)) | ((((mk[k] >> 2) & 3u) | 0x300u) << sh);
                upd = valid ? nu : upd;
                if (!LEAN) trail_mask |= (mk[k] >> 4) == t_last ? 1u << (sh >> 1) : 0u;
            }
            if constexpr (LEAN) {
#pragma unroll
                for (int k = 8 - K; k < 8; k++) {
                    const uint32_t sh = (mk[k] & 3u) * 2u;
                    trail_mask |= (mk[k] >> 4) == t_last ? 1u << (sh >> 1) : 0u;
                }
            }
            const uint32_t upd_incl = wave_prefix_compose(upd);
            const uint32_t upd_excl = dpp_u32_zero<kDppWaveShr1>(upd_incl);
            const uint32_t upd_all = (uint32_t)__builtin_amdgcn_readlane((int)upd_incl, 63);
            st = (state0 & ~(upd_excl >> 8) & 0xFFu) | (upd_excl & 0xFFu);
            st_round = (state0 & ~(upd_all >> 8) & 0xFFu) | (upd_all & 0xFFu);
        }
        const uint32_t next_first = wave_shift_down(kNoTime28, mk[0] >> 4);
        const uint32_t prev_trail = wave_shift_up(kNoKey32, t_last << 4 | trail_mask);

        // ---- gate value after each transition, time-group ends and candidates
        uint32_t sk[8];
        if constexpr (!EDGE) {
            // One pass. A group's candidate is kept if its value differs from
            // the value after the previous group. For the lane's first group
            // that is the gate value at the lane's start, unless the group
            // began in the previous lane (a straddling group): then its
            // candidate is kept here and decided after the pass, against the
            // previous lane's value.
            const uint32_t e_start = lane == 0 && first_round ? kX : __builtin_amdgcn_ubfe(L.lut[st], 0, 2);
            uint32_t run_t = prev_trail >> 4, run_m = prev_trail & 15u;
            const bool straddle = mk[0] != kNoKey32 && (mk[0] >> 4) == run_t;
            bool open = straddle;  // the straddling group has not ended yet
            uint32_t e_prev = e_start;
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const uint32_t sh = K == 1 ? 0u : (mk[k] & 3u) * 2u;
                st = (st & ~(3u << sh)) | (((mk[k] >> 2) & 3u) << sh);
                // table entries are 0, 1 or X (2); the 2-bit extract replaces the
                // byte mask the compiler adds after each byte load
                const uint32_t ek = __builtin_amdgcn_ubfe(L.lut[st], 0, 2);
                const uint32_t tk = mk[k] >> 4;
                const uint32_t tn = k < 7 ? mk[k + 1] >> 4 : next_first;
                const bool end = mk[k] != kNoKey32 && tk != tn;
                const uint32_t pbit = K == 1 ? 1u : 1u << (mk[k] & 3u);
                run_m = tk == run_t ? run_m | pbit : pbit;
                run_t = tk;
                sk[k] = end && (open || ek != e_prev) ? (tk << 2) + L.dtab[ek * 16 + run_m] : kNoKey32;
                e_prev = end ? ek : e_prev;
                open = open && !end;
            }
            // the value after the previous lane's last group
            const uint32_t e0 = first_round ? kX : L.lut[state0];
            const uint32_t e_from_prev = wave_shift_up(e0, e_prev);
            if (straddle) {
                // its first candidate (the first key present) is dropped if
                // the gate value did not change
                bool seen = false;
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const bool here = !seen && sk[k] != kNoKey32;
                    if (here && (sk[k] & 3u) == e_from_prev) sk[k] = kNoKey32;
                    seen = seen || here;
                }
            }
        } else {
            uint32_t evs = 0;    // gate value after each transition, 2 bits each
            uint32_t edges = 0;  // edge class of each transition, 2 bits each
            uint32_t ge = 0, e_lastge = 0;
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const uint32_t sh = K == 1 ? 0u : (mk[k] & 3u) * 2u;
                const uint32_t nv = (mk[k] >> 2) & 3u;
                edges |= edge_class((st >> sh) & 3u, nv) << (2 * k);
                st = (st & ~(3u << sh)) | (nv << sh);
                const uint32_t ek = __builtin_amdgcn_ubfe(L.lut[st], 0, 2);
                evs |= ek << (2 * k);
                const uint32_t tn = k < 7 ? mk[k + 1] >> 4 : next_first;
                const bool end = mk[k] != kNoKey32 && (mk[k] >> 4) != tn;
                ge |= end ? 1u << k : 0u;
                e_lastge = end ? ek : e_lastge;
            }
            const uint32_t e0 = first_round ? kX : L.lut[state0];
            const uint32_t e_from_prev = wave_shift_up(e0, e_lastge);
            // this lane's trailing time group, delays to 0/1/X (10-bit fields)
            uint32_t prev_trail_d;
            {
                uint32_t d0 = kEdgeNone, d1 = kEdgeNone, dx = kEdgeNone;
#pragma unroll
                for (int k = LEAN ? 8 - K : 0; k < 8; k++) {
                    if ((mk[k] >> 4) != t_last || mk[k] == kNoKey32) continue;
                    const uint32_t ent = L.etab[(mk[k] & 3u) * 3 + ((edges >> (2 * k)) & 3u)];
                    d0 = umin32(d0, ent & 1023u);
                    d1 = umin32(d1, (ent >> 10) & 1023u);
                    dx = umin32(dx, ent >> 20);
                }
                prev_trail_d = wave_shift_up(kEdgeNone | kEdgeNone << 10 | kEdgeNone << 20,
                                             d0 | d1 << 10 | dx << 20);
            }
            // candidates at group ends
            uint32_t run_t = prev_trail >> 4;
            uint32_t r0 = prev_trail_d & 1023u, r1 = (prev_trail_d >> 10) & 1023u, rx = prev_trail_d >> 20;
            uint32_t e_prev = e_from_prev;
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const uint32_t tk = mk[k] >> 4;
                const bool cont = tk == run_t;
                const uint32_t ent = L.etab[(mk[k] & 3u) * 3 + ((edges >> (2 * k)) & 3u)];
                r0 = cont ? umin32(r0, ent & 1023u) : ent & 1023u;
                r1 = cont ? umin32(r1, (ent >> 10) & 1023u) : (ent >> 10) & 1023u;
                rx = cont ? umin32(rx, ent >> 20) : ent >> 20;
                run_t = tk;
                sk[k] = kNoKey32;
                if ((ge >> k) & 1u) {
                    const uint32_t ek = (evs >> (2 * k)) & 3u;
                    if (ek != e_prev) {
                        const uint32_t d = ek == 0u ? r0 : ek == 1u ? r1 : rx;
                        // no related pin changed: the candidate never appears
                        if (d != kEdgeNone) sk[k] = ((tk + d) << 2) | ek;
                    }
                    e_prev = ek;
                }
            }
        }
        first_round = false;
        state0 = st_round;

        // the next round's tiles load while the survivors are found
        PinTile<TT> nx[K];
        if constexpr (kPrefetch) {
#pragma unroll
            for (int p = 0; p < K; p++) tile_fetch<TT, LEAN>(Kar + pb[p] + cur[p] + m[p], rem[p] - m[p], nx[p]);
        }

        // ---- survivors among this round's candidates
        uint32_t lmin = kNoKey32;
#pragma unroll
        for (int k = 0; k < 8; k++) lmin = umin32(lmin, sk[k]);
        const uint32_t suf = wave_suffix_min(lmin);
        const uint32_t round_min = (uint32_t)__builtin_amdgcn_readlane((int)suf, 0);
        uint32_t later = wave_shift_down(kNoKey32, suf);
        uint32_t keepmask = 0;
#pragma unroll
        for (int k = 7; k >= 0; k--) {
            // appears before every later candidate (a missing one, kNoKey32,
            // is never below a key with its value bits cleared)
            const bool keep = sk[k] < (later & ~3u);
            later = umin32(later, sk[k]);
            keepmask |= keep ? (1u << k) : 0u;
        }
        const int nkeep = __popc(keepmask);
        // tentative survivors of earlier rounds outlive this round iff they
        // appear before every candidate of this round (they are increasing)
        int ncs = 0;
        for (int c0 = 0; c0 < nq; c0 += 64) {
            const int c = c0 + lane;
            ncs += __popcll(__ballot(c < nq && (L.seq[c] >> 2) < (round_min >> 2)));
        }
        const uint32_t incl_cnt = wave_prefix_sum((uint32_t)nkeep);
        const int nsurv = __builtin_amdgcn_readlane((int)incl_cnt, 63);
        __syncthreads();  // the merge buffers are read before survivors overwrite them
        {
            int pos = ncs + (int)incl_cnt - nkeep;
#pragma unroll
            for (int k = 0; k < 8; k++)
                if (keepmask & (1u << k)) L.seq[pos++] = sk[k];
        }
        const int nseq = ncs + nsurv;
        __syncthreads();

        // ---- final survivors (r <= H): drop repeats, append to the output
        int nf = 0;
        for (int c0 = 0; c0 < nseq; c0 += 64) {
            const int c = c0 + lane;
            nf += __popcll(__ballot(c < nseq && L.seq[c] <= hsplit));
        }
        // every round takes an input transition (the pin whose next one is at
        // the base is in) or makes a survivor final (one at the base); neither
        // means an input waveform is out of order: stop the gate with an error
        // instead of looping
        {
            int taken = 0;
#pragma unroll
            for (int p = 0; p < K; p++) taken += m[p];
            stalled = taken == 0 && nf == 0;
            if (stalled && lane == 0) J.state->check_error = 4;
        }
        for (int c0 = 0; c0 < nf; c0 += 64) {
            const int j = c0 + lane;
            const bool in = j < nf;
            const uint32_t kj = in ? L.seq[j] : 0u;
            const uint32_t v = kj & 3u;
            const uint32_t vp = j == 0 ? last_val : (in ? (L.seq[j - 1] & 3u) : 0u);
            const bool keep = in && v != vp;
            const uint64_t mask = __ballot(keep);
            const int64_t at = out_n + lanes_below(mask);
            if (keep && at < reserved) put<AGENT>(Kar + ob + at, pack_key(base + (int64_t)(kj >> 2), v));
            out_n += __popcll(mask);
        }
        if (nf > 0) last_val = L.seq[nf - 1] & 3u;

        // ---- keep the tentative ones at the front for the next round
        int ntent = nseq - nf;
        if (ntent > W) {  // cannot happen when dmax <= W
            if (lane == 0) J.state->check_error = 1;
            ntent = W;
        }
        if (nf > 0 && ntent > 0) {
            uint32_t rr[W / 64];
#pragma unroll
            for (int c = 0; c < W / 64; c++) {
                const int j = c * 64 + lane;
                if (j < ntent) rr[c] = L.seq[nf + j];
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < W / 64; c++) {
                const int j = c * 64 + lane;
                if (j < ntent) L.seq[j] = rr[c];
            }
        }
        nq = ntent;
        base_prev = base;

#pragma unroll
        for (int p = 0; p < K; p++) {
            cur[p] += m[p];
            if constexpr (kPrefetch) tl[p] = nx[p];
            else tile_fetch<TT, LEAN>(Kar + pb[p] + cur[p], rem[p] - m[p], tl[p]);
        }
        __syncthreads();
    }
    if (out_n > reserved) {  // cannot happen: at most one output per distinct input time
        if (lane == 0) J.state->check_error = 2;
        out_n = reserved;
    }
    if (lane == 0) {
        put<AGENT>(len + S + gate, out_n);
        put<AGENT>(off + S + gate, ob);
    }
}

// -------------------------------------------------------------------------
// Segmented wavefront-per-gate evaluation.
//
// The same per-gate procedure in a second data-parallel form, with lanes in
// time order instead of merged positions. Each round's input transitions (as
// in eval_gate: every transition at or before the horizon H, tiles of 512,
// 384, 256 or 192 per pin) are cut into 64 consecutive time segments, one per
// lane, at equal-count points of the pin with the most transitions in the
// round. Each lane finds where its segment starts in the other pins' tiles (a
// binary search), takes each pin's last value before it, and then runs
// Algorithm 2 itself over its segment: it merges its share of the tiles in
// time, applies each time group, evaluates the gate, and keeps its candidates
// on a stack, a new candidate first removing those that appear no earlier
// than it (Eq. 1). Candidates of a later lane deny too: of a lane's stack only
// the entries appearing before the earliest candidate of every later lane
// survive (a suffix minimum over the lanes; a stack's bottom is its lane's
// earliest candidate), and of the tentative survivors of earlier rounds those
// appearing before the round's earliest candidate. Survivors are increasing
// in appearance time; those at or before H are final (later rounds'
// candidates appear after H), and the Fig. 3 drop keeps a final survivor
// whose value differs from the previous survivor's, the previous lane's last
// one carried by a wave scan. The rest stay tentative for the next round.
// A lane's stack lives in LDS from its segment's first merged index, so the
// stacks never overlap.
template <int K>
struct SegTiling {
    static constexpr int T = K == 1 ? 512 : K == 2 ? 384 : K == 3 ? 256 : 192;
    static constexpr int E = T / 64;
    static constexpr int OFF(int p) { return p * T; }  // key 0 of pin p
    static constexpr int KEYS = K * T;
};
constexpr int kSegKeys = 768;  // the largest round: K x T
static_assert(SegTiling<1>::KEYS <= kSegKeys && SegTiling<2>::KEYS <= kSegKeys &&
                  SegTiling<3>::KEYS <= kSegKeys && SegTiling<4>::KEYS <= kSegKeys,
              "every pin count's tiles fit");

template <int W>
struct SegLds {
    uint32_t tile[kSegKeys];   // K x T in-round keys; after the segments, the output staging
    uint32_t stack[kSegKeys];  // lane stacks, each from its segment's first merged index
    uint32_t seq[W];           // tentative survivors of earlier rounds
    uint32_t dtab[48];         // min delay by (new value, set of changed pins)
    uint32_t etab[12];         // edge model: per (pin, edge class) delays to 0, 1, X (10-bit fields)
    uint8_t lut[256];
};

// The gate's delay tables in LDS: output-value model dtab[value * 16 + set of
// changed pins] = the smallest delay over those pins; edge model etab[pin * 3
// + edge class] = the pin's delays to 0, 1 and X for that input edge.
template <int K, bool EDGE>
__device__ __forceinline__ void delay_tables(const JobDesc &J, const GateRec &R, int64_t gate,
                                             uint32_t *dtab, uint32_t *etab) {
    const int lane = lane_id();
    if (EDGE) {
        if (lane < 3 * K) {
            const int pin = lane / 3, c = lane % 3;
            const int32_t *d = J.edly + (size_t)gate * 16 + pin * 4;  // [edge][out]
            uint32_t f[3];
#pragma unroll
            for (int o = 0; o < 2; o++) {
                const int32_t a = c == 1 ? kNoRelation : d[o], b = c == 0 ? kNoRelation : d[2 + o];
                const int32_t m = a < b ? a : b;
                f[o] = m == kNoRelation ? kEdgeNone : (uint32_t)m;
            }
            f[2] = f[0] < f[1] ? f[0] : f[1];
            etab[lane] = f[0] | f[1] << 10 | f[2] << 20;
        }
    } else if (lane < 48) {
        const uint32_t ev = (uint32_t)lane >> 4, mask = (uint32_t)lane & 15u;
        int32_t d = INT32_MAX;
#pragma unroll
        for (int q = 0; q < K; q++)
            if (mask & (1u << q)) {
                const int32_t dq = pin_delay(R.rise[q], R.fall[q], ev);
                d = dq < d ? dq : d;
            }
        dtab[lane] = (uint32_t)d;
    }
}

// Index of the first of the n keys at t[0, n) whose time is >= s (keys sorted).
template <int T>
__device__ __forceinline__ int seg_lower_bound(const uint32_t *t, int n, uint32_t s) {
    int idx = 0;
#pragma unroll
    for (int step = 512; step >= 1; step >>= 1) {
        if (step > T) continue;
        const int j = idx + step;
        const int at = (j < n ? j : n) - 1;
        const uint32_t k = t[at > 0 ? at : 0];
        idx = j <= n && (k >> 4) < s ? j : idx;
    }
    return idx;
}

// PREFETCH: the next round's tiles load into registers while the round runs
// (the level kernel); otherwise after it (the dependency-driven kernel, whose
// persistent loop leaves fewer registers).
template <int K, int W, bool EDGE, bool PREFETCH, bool AGENT>
__device__ __forceinline__ void eval_gate_seg(const JobDesc &J, int64_t ob, const GateRec &R,
                                              int64_t gate, SegLds<W> &L) {
    using Tl = SegTiling<K>;
    constexpr int TT = Tl::T;
    constexpr int E = Tl::E;
    const int lane = lane_id();
    const int64_t S = J.S;
    int64_t *len = J.len;
    int64_t *off = J.off;
    uint64_t *Kar = J.K;

    int64_t pb[K], pl[K], cur[K];
    int64_t reserved = 0;  // slots sized for this gate: the sum of its input lengths
#pragma unroll
    for (int p = 0; p < K; p++) {
        pb[p] = off[R.net[p]];
        pl[p] = len[R.net[p]];
        cur[p] = 0;
        reserved += pl[p];
    }
    uint32_t state0 = 0;  // pin values before the round, 2 bits per pin
#pragma unroll
    for (int p = 0; p < K; p++) state0 |= (uint32_t)kX << (2 * p);

    PinTile<TT> tl[K];
#pragma unroll
    for (int p = 0; p < K; p++) tile_fetch<TT, true>(Kar + pb[p], pl[p], tl[p]);
    delay_tables<K, EDGE>(J, R, gate, L.dtab, L.etab);
    // one and two pins: the gate table (16 values of 2 bits) and the delay
    // table (per new value, 10-bit fields for changed-pin sets 1, 2, 3) in
    // scalar registers, so the step reads neither from LDS
    uint32_t lut_reg = 0, dly_reg[3] = {0u, 0u, 0u};
    if (K <= 2) {
        __syncthreads();  // the caller's gate table copy
        const uint32_t part = lane < 16 ? (uint32_t)(L.lut[lane] & 3u) << (2 * lane) : 0u;
        lut_reg = (uint32_t)__builtin_amdgcn_readlane((int)wave_prefix_sum(part), 15);
        if (!EDGE) {
#pragma unroll
            for (int ev = 0; ev < 3; ev++) {
                uint32_t w = 0;
#pragma unroll
                for (int mset = 1; mset < 4; mset++) {
                    int32_t d = INT32_MAX;
#pragma unroll
                    for (int q = 0; q < K; q++)
                        if (mset & (1 << q)) {
                            const int32_t dq = pin_delay(R.rise[q], R.fall[q], (uint32_t)ev);
                            d = dq < d ? dq : d;
                        }
                    w |= (d == INT32_MAX ? 0u : (uint32_t)d) << (10 * (mset - 1));
                }
                dly_reg[ev] = (uint32_t)__builtin_amdgcn_readfirstlane((int)w);
            }
        }
    }

    uint32_t last_val = kX;  // value of the last final survivor
    bool first_round = true;
    int nq = 0;              // tentative survivors in L.seq[0, nq), offsets from base_prev
    int64_t base_prev = 0;
    int64_t out_n = 0;
    bool stalled = false;
    for (;;) {
        nq = __builtin_amdgcn_readfirstlane(nq);
#pragma unroll
        for (int p = 0; p < K; p++) cur[p] = uniform64(cur[p]);
        int64_t rem[K];
        bool more = nq > 0 && !stalled;
#pragma unroll
        for (int p = 0; p < K; p++) {
            rem[p] = pl[p] - cur[p];
            more |= rem[p] > 0 && !stalled;
        }
        if (!more) break;

        // ---- base (earliest pending time) and horizon, as in eval_gate
        int lim[K];
        uint32_t thi[K];
        int64_t H = kInf, base = kInf;
#pragma unroll
        for (int p = 0; p < K; p++) {
            int64_t t0, hp;
            tile_settle<TT, true>(Kar + pb[p] + cur[p], rem[p], tl[p], lim[p], thi[p], t0, hp);
            H = min64(H, hp);
            base = min64(base, t0);
        }
        if (nq > 0) {
            const uint32_t q0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)L.seq[0]);
            base = min64(base, base_prev + (int64_t)(q0 >> 2));
            const uint32_t shift = (uint32_t)(base - base_prev) << 2;
            for (int c = lane; c < nq; c += 64) L.seq[c] -= shift;
        }
        H = min64(H, base + kSpan);
        const uint64_t hkey = H < kTimeLimit ? pack_key(H, 3u) : ~uint64_t(0);
        const uint32_t base4 = (uint32_t)pack_key(base, 0u);
        const uint32_t hk_hi = (uint32_t)(hkey >> 32);
        int m[K];
#pragma unroll
        for (int p = 0; p < K; p++) {
            const uint32_t lo_max =
                (uint32_t)__builtin_amdgcn_readfirstlane((int)(thi[p] < hk_hi ? 0xFFFFFFFFu : (uint32_t)hkey));
            const int lim_in = __builtin_amdgcn_readfirstlane(thi[p] > hk_hi ? 0 : lim[p]);
            m[p] = 0;
#pragma unroll
            for (int e = 0; e < E; e++) {
                const uint32_t lo = tl[p].lo[e];
                const bool in_lane = lane + 64 * e < lim_in, in_time = lo <= lo_max;
                m[p] += __popcll(__ballot(in_lane) & __ballot(in_time));
                L.tile[Tl::OFF(p) + 64 * e + lane] =
                    in_lane && in_time ? ((lo - base4) << 2) | (uint32_t)p : kNoKey32;
            }
        }
        bool all_in = true;
#pragma unroll
        for (int p = 0; p < K; p++) all_in = all_in && m[p] == rem[p];
        const uint32_t hsplit = all_in ? kNoKey32 : (uint32_t)(H - base) << 2 | 3u;
        PinTile<TT> nx[K];
        if constexpr (PREFETCH) {
#pragma unroll
            for (int p = 0; p < K; p++) tile_fetch<TT, true>(Kar + pb[p] + cur[p] + m[p], rem[p] - m[p], nx[p]);
        }
        __syncthreads();

        // ---- this lane's segment: [s, next lane's s) in time. With one pin, an
        // equal share of its keys; otherwise equal shares of the merged keys of
        // the two pins with the most (a merge-path search), moved back to the
        // start of the time group they fall in, and the other pins' keys from
        // that time on (binary searches).
        int ip[K], endi[K];
        uint32_t s;
        if constexpr (K == 1) {
            ip[0] = (lane * m[0]) >> 6;
            s = lane == 0 ? 0u : L.tile[ip[0]] >> 4;
        } else {
            int pa = 0, pb2 = 1;
            if (m[1] > m[0]) {
                pa = 1;
                pb2 = 0;
            }
#pragma unroll
            for (int p = 2; p < K; p++) {
                if (m[p] > m[pa]) {
                    pb2 = pa;
                    pa = p;
                } else if (m[p] > m[pb2]) {
                    pb2 = p;
                }
            }
            const uint32_t *A = L.tile + pa * TT;
            const uint32_t *B = L.tile + pb2 * TT;
            const int ma = m[pa], mb = m[pb2];
            const int d = (lane * (ma + mb)) >> 6;
            int lo = d - mb > 0 ? d - mb : 0, hi = d < ma ? d : ma;
#pragma unroll
            for (int it = 0; it < 10; it++) {
                const int mid = (lo + hi) >> 1;
                const int jb = d - 1 - mid;
                const uint32_t ka = A[mid < TT ? mid : TT - 1];
                const uint32_t kb = B[jb < 0 ? 0 : jb < TT ? jb : TT - 1];
                const bool go = lo < hi;
                const bool less = ka < kb;
                lo = go && less ? mid + 1 : lo;
                hi = go && !less ? mid : hi;
            }
            int ia = lo, ib = d - lo;
            const uint32_t na = ia < ma ? A[ia] : kNoKey32;
            const uint32_t nb = ib < mb ? B[ib] : kNoKey32;
            s = lane == 0 ? 0u : umin32(na, nb) >> 4;
            const uint32_t pa_t = A[ia > 0 ? ia - 1 : 0] >> 4, pb_t = B[ib > 0 ? ib - 1 : 0] >> 4;
            ia -= ia > 0 && pa_t == s ? 1 : 0;
            ib -= ib > 0 && pb_t == s ? 1 : 0;
            if (lane == 0) ia = ib = 0;
#pragma unroll
            for (int p = 0; p < K; p++)
                ip[p] = p == pa ? ia : p == pb2 ? ib : seg_lower_bound<TT>(L.tile + Tl::OFF(p), m[p], s);
        }
        int sb = 0;  // merged index of the segment's first transition
#pragma unroll
        for (int p = 0; p < K; p++) {
            endi[p] = (int)wave_shift_down((uint32_t)m[p], (uint32_t)ip[p]);
            sb += ip[p];
        }
        // pin values before the segment; the gate's value there (X before any input change)
        uint32_t st = state0;
#pragma unroll
        for (int p = 0; p < K; p++)
            if (ip[p] > 0) {
                const uint32_t k = L.tile[Tl::OFF(p) + ip[p] - 1];
                st = (st & ~(3u << (2 * p))) | (((k >> 2) & 3u) << (2 * p));
            }
        uint32_t e_prev = first_round && sb == 0 ? (uint32_t)kX : __builtin_amdgcn_ubfe(L.lut[st], 0, 2);
        // pin values after the round (for the next one)
        uint32_t state_next = state0;
#pragma unroll
        for (int p = 0; p < K; p++)
            if (m[p] > 0) {
                const uint32_t k = (uint32_t)__builtin_amdgcn_readfirstlane((int)L.tile[Tl::OFF(p) + m[p] - 1]);
                state_next = (state_next & ~(3u << (2 * p))) | (((k >> 2) & 3u) << (2 * p));
            }

        // ---- Algorithm 2 over the segment; candidates on the lane's stack (Eq. 1).
        // Branch-free per pin: the pin's head and the key after it are held in
        // registers, so the LDS read of a pin's next key has a whole step to land.
        uint32_t head[K], after[K];  // after: the key at idx + 1 as read (bounds checked at use)
        int idx[K];
#pragma unroll
        for (int p = 0; p < K; p++) {
            idx[p] = ip[p];
            const int j = idx[p] + 1;
            const uint32_t k0 = L.tile[Tl::OFF(p) + (idx[p] < TT ? idx[p] : TT - 1)];
            head[p] = idx[p] < endi[p] ? k0 : kNoKey32;
            after[p] = L.tile[Tl::OFF(p) + (j < TT ? j : TT - 1)];
        }
        int n = 0;         // the stack: L.stack[sb, sb + n)
        uint32_t top = 0;  // L.stack[sb + n - 1] when n > 0
        for (;;) {
            uint32_t mn = head[0];
#pragma unroll
            for (int p = 1; p < K; p++) mn = umin32(mn, head[p]);
            const bool act = mn != kNoKey32;
            if (__ballot(act) == 0) break;
            if (act) {
                const uint32_t t = mn >> 4;
                const uint32_t t_end = (t + 1) << 4;  // keys of time t are below this
                uint32_t mask = 0;
                uint32_t r0 = kEdgeNone, r1 = kEdgeNone, rx = kEdgeNone;
#pragma unroll
                for (int p = 0; p < K; p++) {
                    const bool c = head[p] < t_end;
                    const uint32_t nv = (head[p] >> 2) & 3u;
                    if (EDGE) {
                        const uint32_t ent = L.etab[p * 3 + edge_class((st >> (2 * p)) & 3u, nv)];
                        r0 = c ? umin32(r0, ent & 1023u) : r0;
                        r1 = c ? umin32(r1, (ent >> 10) & 1023u) : r1;
                        rx = c ? umin32(rx, ent >> 20) : rx;
                    }
                    const uint32_t nst = (st & ~(3u << (2 * p))) | (nv << (2 * p));
                    st = c ? nst : st;
                    mask |= c ? 1u << p : 0u;
                    idx[p] += c ? 1 : 0;
                    const uint32_t hn = idx[p] < endi[p] ? after[p] : kNoKey32;
                    head[p] = c ? hn : head[p];
                    const int j = idx[p] + 1;
                    after[p] = L.tile[Tl::OFF(p) + (j < TT ? j : TT - 1)];
                }
                const uint32_t e = K <= 2 ? __builtin_amdgcn_ubfe(lut_reg, 2 * st, 2)
                                          : __builtin_amdgcn_ubfe(L.lut[st], 0, 2);
                if (e != e_prev) {
                    uint32_t d;
                    if (EDGE) d = e == 0u ? r0 : e == 1u ? r1 : rx;
                    else if (K <= 2) d = __builtin_amdgcn_ubfe(e == 0u ? dly_reg[0] : e == 1u ? dly_reg[1] : dly_reg[2],
                                                               10 * (mask - 1), 10);
                    else d = L.dtab[e * 16 + mask];
                    // (edge model: no related pin changed, the candidate never appears)
                    if (!EDGE || d != kEdgeNone) {
                        const uint32_t key = ((t + d) << 2) | e;
                        while (n > 0 && (top >> 2) >= (key >> 2)) {
                            n--;
                            top = n > 0 ? L.stack[sb + n - 1] : 0u;
                        }
                        L.stack[sb + n] = key;
                        n++;
                        top = key;
                    }
                    e_prev = e;
                }
            }
        }

        // ---- survivors: before every later lane's earliest candidate
        const uint32_t bottom = n > 0 ? L.stack[sb] : kNoKey32;
        const uint32_t suf = wave_suffix_min(bottom);
        const uint32_t round_min = (uint32_t)__builtin_amdgcn_readlane((int)suf, 0);
        const uint32_t later = wave_shift_down(kNoKey32, suf);
        while (n > 0 && (top >> 2) >= (later >> 2)) {
            n--;
            top = n > 0 ? L.stack[sb + n - 1] : 0u;
        }
        // tentative survivors of earlier rounds outlive this round iff they
        // appear before every candidate of this round (they are increasing)
        int ncs = 0;
        for (int c0 = 0; c0 < nq; c0 += 64) {
            const int c = c0 + lane;
            ncs += __popcll(__ballot(c < nq && (L.seq[c] >> 2) < (round_min >> 2)));
        }
        // final: appearing at or before H (a prefix of every ordered list)
        int nft = 0;
        for (int c0 = 0; c0 < ncs; c0 += 64) {
            const int c = c0 + lane;
            nft += __popcll(__ballot(c < ncs && L.seq[c] <= hsplit));
        }
        int f = n;
        {
            uint32_t tp = top;
            while (f > 0 && tp > hsplit) {
                f--;
                tp = f > 0 ? L.stack[sb + f - 1] : 0u;
            }
        }
        // the value before this lane's first survivor: the previous lane's last
        // one, else the last surviving tentative, else the last final value
        const uint32_t mark = n > 0 ? 0x300u | (top & 3u) : 0u;
        const uint32_t carried = wave_shift_up(0u, wave_prefix_compose(mark));
        const uint32_t tent_last =
            ncs > 0 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)L.seq[ncs - 1]) & 3u : last_val;
        const uint32_t vprev0 = (carried & 0x300u) ? (carried & 3u) : tent_last;

        // ---- final survivors whose value differs from the previous one: the
        // tentative ones first, then the lanes' in lane order
        int kt = 0;
        for (int c0 = 0; c0 < nft; c0 += 64) {
            const int c = c0 + lane;
            const bool in = c < nft;
            const uint32_t kc = in ? L.seq[c] : 0u;
            const uint32_t vp = c == 0 ? last_val : (in ? (L.seq[c - 1] & 3u) : 0u);
            const bool keep = in && (kc & 3u) != vp;
            const uint64_t mask = __ballot(keep);
            const int64_t at = out_n + kt + lanes_below(mask);
            if (keep && at < reserved) put<AGENT>(Kar + ob + at, pack_key(base + (int64_t)(kc >> 2), kc & 3u));
            kt += __popcll(mask);
        }
        int kl = 0;
        {
            uint32_t vp = vprev0;
            for (int j = 0; j < f; j++) {
                const uint32_t k = L.stack[sb + j];
                kl += (k & 3u) != vp ? 1 : 0;
                vp = k & 3u;
            }
        }
        const uint32_t kincl = wave_prefix_sum((uint32_t)kl);
        const int ktot = __builtin_amdgcn_readlane((int)kincl, 63);
        {
            uint32_t vp = vprev0;
            int at = (int)kincl - kl;
            for (int j = 0; j < f; j++) {
                const uint32_t k = L.stack[sb + j];
                if ((k & 3u) != vp) L.tile[at++] = k;  // the tiles are read no more this round
                vp = k & 3u;
            }
        }
        __syncthreads();
        for (int j0 = 0; j0 < ktot; j0 += 64) {
            const int j = j0 + lane;
            const int64_t at = out_n + kt + j;
            if (j < ktot && at < reserved) {
                const uint32_t k = L.tile[j];
                put<AGENT>(Kar + ob + at, pack_key(base + (int64_t)(k >> 2), k & 3u));
            }
        }
        out_n += kt + ktot;
        {
            // the value of the last final survivor
            const uint32_t fmark = f > 0 ? 0x300u | (L.stack[sb + f - 1] & 3u) : 0u;
            const uint32_t flast = (uint32_t)__builtin_amdgcn_readlane((int)wave_prefix_compose(fmark), 63);
            if (flast & 0x300u) last_val = flast & 3u;
            else if (nft > 0) last_val = (uint32_t)__builtin_amdgcn_readfirstlane((int)L.seq[nft - 1]) & 3u;
        }
        // every round takes an input transition or makes a survivor final;
        // neither means an input waveform is out of order: stop with an error
        {
            int taken = 0;
#pragma unroll
            for (int p = 0; p < K; p++) taken += m[p];
            stalled = taken == 0 && nft == 0 && __ballot(f > 0) == 0;
            if (stalled && lane == 0) J.state->check_error = 4;
        }

        // ---- the tentative ones, in order, at the front of L.seq
        const int keep_old = ncs - nft;
        const int tn = n - f;
        const uint32_t tincl = wave_prefix_sum((uint32_t)tn);
        int ntent = keep_old + __builtin_amdgcn_readlane((int)tincl, 63);
        if (ntent > W) {  // cannot happen when dmax <= W
            if (lane == 0) J.state->check_error = 1;
            ntent = W;
        }
        {
            uint32_t rr[W / 64];
#pragma unroll
            for (int c = 0; c < W / 64; c++) {
                const int j = c * 64 + lane;
                if (j < keep_old) rr[c] = L.seq[nft + j];
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < W / 64; c++) {
                const int j = c * 64 + lane;
                if (j < keep_old) L.seq[j] = rr[c];
            }
            const int d0 = keep_old + (int)tincl - tn;
            for (int i = 0; i < tn; i++)
                if (d0 + i < W) L.seq[d0 + i] = L.stack[sb + f + i];
        }
        nq = ntent;
        base_prev = base;
        first_round = false;
        state0 = state_next;
#pragma unroll
        for (int p = 0; p < K; p++) {
            if constexpr (PREFETCH) tl[p] = nx[p];
            else tile_fetch<TT, true>(Kar + pb[p] + cur[p] + m[p], rem[p] - m[p], tl[p]);
            cur[p] += m[p];
        }
        __syncthreads();
    }
    if (out_n > reserved) {  // cannot happen: at most one output per distinct input time
        if (lane == 0) J.state->check_error = 2;
        out_n = reserved;
    }
    if (lane == 0) {
        put<AGENT>(len + S + gate, out_n);
        put<AGENT>(off + S + gate, ob);
    }
}

// -------------------------------------------------------------------------
// Lane-per-gate evaluation: the sequential procedure on one lane, with the
// gate's reserved output region used directly as the list of scheduled
// transitions (denials pop its tail). Exact for any delay.
template <bool AGENT>
__device__ void eval_seq(const JobDesc &J, const GateRec &R, int64_t gate, int64_t ob,
                         const uint8_t *lut) {
    const int64_t S = J.S;
    const int k = R.k;
    int64_t pb[kMaxPins], pl[kMaxPins], idx[kMaxPins];
    uint32_t cv[kMaxPins];
    int64_t reserved = 0;
#pragma unroll
    for (int p = 0; p < kMaxPins; p++) {
        pb[p] = 0; pl[p] = 0; idx[p] = 0; cv[p] = kX;
        if (p < k) { pb[p] = J.off[R.net[p]]; pl[p] = J.len[R.net[p]]; reserved += pl[p]; }
    }
    uint64_t *Kar = J.K;
    uint32_t prev = kX;
    int64_t n = 0;
    for (;;) {
        int64_t te = kInf;
#pragma unroll
        for (int p = 0; p < kMaxPins; p++)
            if (idx[p] < pl[p]) te = min64(te, key_time(Kar[pb[p] + idx[p]]));
        if (te == kInf) break;
        int changed = 0;
        int pack = 0;
        uint32_t edge_of_pin = 0;  // extended model: edge class of each changed pin
#pragma unroll
        for (int p = 0; p < kMaxPins; p++) {
            if (idx[p] < pl[p]) {
                const uint64_t kp = Kar[pb[p] + idx[p]];
                if (key_time(kp) == te) {
                    edge_of_pin |= edge_class(cv[p], key_value(kp)) << (2 * p);
                    cv[p] = key_value(kp);
                    idx[p]++;
                    changed |= 1 << p;
                }
            }
            if (p < k) pack |= (int)cv[p] << (2 * p);
        }
        const uint32_t e = lut[pack];
        if (e != prev) {
            int64_t d = kInf;
#pragma unroll
            for (int p = 0; p < kMaxPins; p++) {
                if (!(changed & (1 << p))) continue;
                if (J.edly) {
                    // extended model: this pin's delay for its edge and the new value
                    const int32_t *dp = J.edly + (size_t)gate * 16 + p * 4;
                    const uint32_t c = (uint32_t)(edge_of_pin >> (2 * p)) & 3u;
#pragma unroll
                    for (int ed = 0; ed < 2; ed++)
#pragma unroll
                        for (int o = 0; o < 2; o++) {
                            const int32_t x = dp[ed * 2 + o];
                            if ((c == 2u || c == (uint32_t)ed) && (e == kX || e == (uint32_t)o) && x != kNoRelation)
                                d = min64(d, x);
                        }
                } else {
                    d = min64(d, pin_delay(R.rise[p], R.fall[p], e));
                }
            }
            if (d == kInf) {  // no related pin changed: the candidate never appears
                prev = e;
                continue;
            }
            const int64_t tr = te + d;
            while (n > 0 && key_time(Kar[ob + n - 1]) >= tr) n--;
            const uint32_t cur = n > 0 ? key_value(Kar[ob + n - 1]) : kX;
            if (e != cur) {
                if (n >= reserved) {  // cannot happen: at most one output per distinct input time
                    J.state->check_error = 2;
                    break;
                }
                put<AGENT>(Kar + ob + n, pack_key(tr, e));
                n++;
            }
        }
        prev = e;
    }
    put<AGENT>(J.len + S + gate, n);
    put<AGENT>(J.off + S + gate, ob);
}

}  // namespace

}  // namespace gsim
