// A wave64 emulator for running the kernels' per-gate evaluation code on the
// CPU (test infrastructure).
//
// Each of the 64 lanes of a wavefront runs the unchanged device code as a
// coroutine on its own stack. A cross-lane operation (ballot, readlane, DPP,
// shuffles, the workgroup barrier) is a rendezvous: every lane deposits its
// operand and switches back to the scheduler; once all 64 lanes have arrived
// at the same operation, each one resumes and computes its result from the
// deposited operands -- what the hardware does in one instruction. The
// scheduler checks that all lanes reach every cross-lane operation together
// (the device code must never execute one under divergent control flow),
// optionally that values passed to readfirstlane are the same on every lane,
// and stops a gate that runs more operations than a given limit.
#pragma once

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <climits>
#include <cstdint>

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#else
#define EMU_ASAN 0
#endif

namespace emu {

constexpr int kLanes = 64;
constexpr size_t kStackBytes = size_t(1) << 18;

enum Op : int { kOpBarrier = 1, kOpBallot, kOpReadlane, kOpReadfirst, kOpDpp, kOpShflUp, kOpShflDown, kOpBpermute };

struct Dim3 {
    unsigned x, y, z;
};

struct Wave {
    int lane = 0;                // lane now running
    void *sched_sp = nullptr;    // scheduler's saved stack pointer
    void *lane_sp[kLanes];
    char *stack[kLanes];
    int status[kLanes];          // 0 runnable, 1 at a cross-lane op, 2 returned, 3 failed
    uint64_t ops[kLanes];        // cross-lane operations passed
    int kind[kLanes];            // operation waited at
    uint64_t slot[2][kLanes];    // operands of the last two operations
    bool failed = false;
    char msg[512];
    uint64_t max_ops = 0;        // 0: no limit
    bool strict_uniform = true;  // readfirstlane operands must agree
    void (*body)(void *) = nullptr;
    void *arg = nullptr;
#if EMU_ASAN
    void *fake = nullptr;
    const void *sched_bottom = nullptr;
    size_t sched_size = 0;
#endif
};

Wave &wave();
void run(void (*body)(void *), void *arg);  // all 64 lanes to completion or failure
void yield_lane();                            // back to the scheduler
[[noreturn]] void fail(const char *fmt, ...);

inline int lane() { return wave().lane; }

// Deposit this lane's operand for the next cross-lane operation; returns the
// index of the slot row holding every lane's operand once all have arrived.
inline int exchange(int kind, uint64_t mine) {
    Wave &w = wave();
    const int l = w.lane;
    const uint64_t n = w.ops[l];
    w.slot[n & 1][l] = mine;
    w.kind[l] = kind;
    w.status[l] = 1;
    w.ops[l] = n + 1;
    yield_lane();
    return (int)(n & 1);
}

inline void syncthreads() { exchange(kOpBarrier, 0); }

inline uint64_t ballot(bool p) {
    const int r = exchange(kOpBallot, p ? 1 : 0);
    uint64_t m = 0;
    for (int i = 0; i < kLanes; i++) m |= (wave().slot[r][i] & 1ull) << i;
    return m;
}

inline int readlane(int x, int src) {
    const int r = exchange(kOpReadlane, (uint32_t)x);
    if (src < 0 || src >= kLanes) fail("readlane of lane %d", src);
    return (int)(uint32_t)wave().slot[r][src];
}

inline int readfirstlane(int x) {
    const int r = exchange(kOpReadfirst, (uint32_t)x);
    Wave &w = wave();
    if (w.strict_uniform)
        for (int i = 1; i < kLanes; i++)
            if (w.slot[r][i] != w.slot[r][0])
                fail("readfirstlane of a value that differs across lanes (lane 0: %u, lane %d: %u)",
                     (unsigned)w.slot[r][0], i, (unsigned)w.slot[r][i]);
    return (int)(uint32_t)w.slot[r][0];
}

// GFX9 DPP move (update_dpp): the source lane of each destination lane by
// the control word; a lane whose row or bank is masked off, or whose source
// is out of range (with bound_ctrl off), keeps `old`.
inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    const int r = exchange(kOpDpp, (uint32_t)src);
    const int i = lane();
    const int row = i >> 4, in_row = i & 15, bank = in_row >> 2;
    if (!((row_mask >> row) & 1) || !((bank_mask >> bank) & 1)) return old;
    int s = -1;
    if (ctrl >= 0x101 && ctrl <= 0x10F) {  // row_shl
        const int n = ctrl - 0x100;
        s = in_row + n < 16 ? i + n : -1;
    } else if (ctrl >= 0x111 && ctrl <= 0x11F) {  // row_shr
        const int n = ctrl - 0x110;
        s = in_row >= n ? i - n : -1;
    } else if (ctrl == 0x130) {  // wave_shl:1
        s = i < 63 ? i + 1 : -1;
    } else if (ctrl == 0x138) {  // wave_shr:1
        s = i > 0 ? i - 1 : -1;
    } else if (ctrl == 0x142) {  // row_bcast:15
        s = row >= 1 ? 16 * row - 1 : -1;
    } else if (ctrl == 0x143) {  // row_bcast:31
        s = row >= 2 ? 31 : -1;
    } else {
        fail("DPP control 0x%x not emulated", ctrl);
    }
    if (s < 0) return bound_ctrl ? 0 : old;
    return (int)(uint32_t)wave().slot[r][s];
}

// DPP move without an `old` operand: defined only when every lane is written
// (all rows and banks enabled, out-of-range sources reading 0).
inline int mov_dpp(int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    if (row_mask != 0xf || bank_mask != 0xf || !bound_ctrl)
        fail("mov_dpp leaves lanes unwritten (row mask 0x%x, bank mask 0x%x, bound_ctrl %d)",
             row_mask, bank_mask, (int)bound_ctrl);
    return update_dpp(0, src, ctrl, row_mask, bank_mask, bound_ctrl);
}

inline int shfl_up(int x, int d, int width) {
    const int r = exchange(kOpShflUp, (uint32_t)x);
    const int i = lane();
    if (width != 64) fail("shuffle width %d not emulated", width);
    return i >= d ? (int)(uint32_t)wave().slot[r][i - d] : x;
}

// ds_bpermute: every lane reads `src` of lane (addr / 4) mod 64.
inline int bpermute(int addr, int src) {
    const int r = exchange(kOpBpermute, (uint32_t)src);
    return (int)(uint32_t)wave().slot[r][((unsigned)addr >> 2) & 63];
}

inline int shfl_down(int x, int d, int width) {
    const int r = exchange(kOpShflDown, (uint32_t)x);
    const int i = lane();
    if (width != 64) fail("shuffle width %d not emulated", width);
    return i + d < kLanes ? (int)(uint32_t)wave().slot[r][i + d] : x;
}

inline uint32_t mbcnt_lo(uint32_t m, uint32_t acc) {
    const int i = lane() < 32 ? lane() : 32;
    return acc + (uint32_t)__builtin_popcountll((uint64_t)m & ((1ull << i) - 1));
}
inline uint32_t mbcnt_hi(uint32_t m, uint32_t acc) {
    const int i = lane() > 32 ? lane() - 32 : 0;
    return acc + (uint32_t)__builtin_popcountll((uint64_t)m & ((1ull << i) - 1));
}
inline uint32_t ubfe(uint32_t x, uint32_t off, uint32_t w) {
    return w >= 32 ? x >> off : (x >> off) & ((1u << w) - 1u);
}

inline Dim3 thread_idx() { return Dim3{(unsigned)lane(), 0, 0}; }

// Memory operations: lanes run one at a time, so plain accesses are atomic.
template <typename T, typename U>
inline T atomic_add(T *p, U v) { T o = *p; *p = (T)(o + (T)v); return o; }
template <typename T, typename U>
inline T atomic_sub(T *p, U v) { T o = *p; *p = (T)(o - (T)v); return o; }
template <typename T, typename U>
inline T atomic_or(T *p, U v) { T o = *p; *p = (T)(o | (T)v); return o; }
template <typename T, typename U>
inline T atomic_max(T *p, U v) { T o = *p; *p = o > (T)v ? o : (T)v; return o; }
template <typename T, typename U>
inline void atomic_store(T *p, U v) { *p = (T)v; }
template <typename T>
inline T atomic_load(const T *p) { return *p; }

}  // namespace emu

// ---- the HIP names the device code uses ------------------------------------
typedef int hipError_t;
typedef void *hipStream_t;
constexpr hipError_t hipSuccess = 0;

#define gsim_global
#define __host__
#define __device__
#define __global__
#define __shared__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define threadIdx (::emu::thread_idx())
#define __HIP_MEMORY_SCOPE_AGENT 3

#define __syncthreads() ::emu::syncthreads()
#define __ballot(p) ::emu::ballot(p)
#define __popcll(x) __builtin_popcountll((unsigned long long)(x))
#define __popc(x) __builtin_popcount((unsigned)(x))
#define __ffsll(x) __builtin_ffsll((long long)(x))
#define __clzll(x) __builtin_clzll((unsigned long long)(x))
#define __shfl_up(x, d, w) ::emu::shfl_up((x), (d), (w))
#define __shfl_down(x, d, w) ::emu::shfl_down((x), (d), (w))
#define __builtin_amdgcn_ds_bpermute(a, s) ::emu::bpermute((a), (s))
#define __builtin_nondeterministic_value(x) (x)
#define __builtin_amdgcn_readlane(x, l) ::emu::readlane((x), (l))
#define __builtin_amdgcn_readfirstlane(x) ::emu::readfirstlane((x))
#define __builtin_amdgcn_update_dpp(o, s, c, rm, bm, bc) ::emu::update_dpp((o), (s), (c), (rm), (bm), (bc))
#define __builtin_amdgcn_mov_dpp(s, c, rm, bm, bc) ::emu::mov_dpp((s), (c), (rm), (bm), (bc))
#define __builtin_amdgcn_mbcnt_lo(m, a) ::emu::mbcnt_lo((m), (a))
#define __builtin_amdgcn_mbcnt_hi(m, a) ::emu::mbcnt_hi((m), (a))
#define __builtin_amdgcn_ubfe(x, o, w) ::emu::ubfe((x), (o), (w))
#define __builtin_amdgcn_s_sleep(n) ((void)0)
#define __builtin_amdgcn_fence(...) ((void)0)
#define __hip_atomic_store(p, v, order, scope) ::emu::atomic_store((p), (v))
#define __hip_atomic_load(p, order, scope) ::emu::atomic_load((p))
#define atomicAdd(p, v) ::emu::atomic_add((p), (v))
#define atomicSub(p, v) ::emu::atomic_sub((p), (v))
#define atomicOr(p, v) ::emu::atomic_or((p), (v))
#define atomicMax(p, v) ::emu::atomic_max((p), (v))
