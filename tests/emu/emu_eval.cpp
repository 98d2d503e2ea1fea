// Runs the kernels' per-gate evaluation (eval_gate, eval_seq from
// csrc/eval_core.h, unchanged) on the CPU under the wave64 emulator, one gate
// at a time, on input waveforms given in a file (test infrastructure).
//
//   emu_eval <in.bin> <out.bin>
//
// Each input waveform and each gate's output region is a heap block of its
// own, and the wavefront's LDS is refilled with random bytes before every
// gate, so a build with AddressSanitizer reports any read outside a
// waveform, and a read of LDS the gate did not write shows up as a wrong
// result.
//
// in.bin (little endian): int64 mode, S, G, n_types, has_edge, n_eval,
// max_ops; then uint8 type[G]; int64 pin_off[G+1]; int64 pin_net[P];
// int32 rise[P]; int32 fall[P]; int32 dly[4P] if has_edge ([edge][output]
// per pin); uint8 lut[n_types*256]; int64 net_off[S+G+1]; uint64 keys[N]
// (time << 2 | value of every net's waveform); int64 gates[n_eval].
// out.bin: int64 out_off[n_eval+1]; uint64 out_keys[]; int32 err[n_eval].
// Modes: 0 level kernel's form; 1 dependency-driven kernel's form; 2 the
// dependency-driven form with the level kernel's shorter tile and
// trailing-group code; 3 the level kernel's form without that shorter code;
// 4 the segmented form (eval_gate_seg) as the level kernel runs it; 5 the
// segmented form with agent-scope stores and no prefetch.
#include <sys/mman.h>

#include <cstdarg>
#include <random>
#include <string>
#include <vector>

#include "eval_core.h"

// ---- coroutine switch (x86-64 System V: callee-saved registers + stack) ------
extern "C" void emu_ctx_switch(void **save_sp, void *load_sp);
asm(R"(
    .text
    .globl emu_ctx_switch
    .type emu_ctx_switch, @function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_ctx_switch, .-emu_ctx_switch
)");

#if EMU_ASAN
#include <sanitizer/asan_interface.h>
#endif

namespace emu {

static Wave g_wave;
static bool g_in_lane = false;
#if EMU_ASAN
static void *g_lane_fake[kLanes];
static void *g_sched_fake = nullptr;
#endif

Wave &wave() { return g_wave; }

static void to_scheduler(bool leaving) {
    Wave &w = g_wave;
    const int l = w.lane;
    g_in_lane = false;
#if EMU_ASAN
    __sanitizer_start_switch_fiber(leaving ? nullptr : &g_lane_fake[l], w.sched_bottom, w.sched_size);
#else
    (void)leaving;
#endif
    emu_ctx_switch(&w.lane_sp[l], w.sched_sp);
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(g_lane_fake[l], &w.sched_bottom, &w.sched_size);
#endif
    g_in_lane = true;
}

void yield_lane() { to_scheduler(false); }

[[noreturn]] void fail(const char *fmt, ...) {
    Wave &w = g_wave;
    if (!w.failed) {
        va_list ap;
        va_start(ap, fmt);
        int n = snprintf(w.msg, sizeof w.msg, "lane %d: ", w.lane);
        vsnprintf(w.msg + n, sizeof w.msg - n, fmt, ap);
        va_end(ap);
    }
    w.failed = true;
    if (!g_in_lane) {
        fprintf(stderr, "emulator: %s\n", w.msg);
        abort();
    }
    w.status[w.lane] = 3;
    to_scheduler(true);
    abort();  // a failed lane is never resumed
}

static void lane_main() {
    Wave &w = g_wave;
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &w.sched_bottom, &w.sched_size);
#endif
    g_in_lane = true;
    w.body(w.arg);
    w.status[w.lane] = 2;
    to_scheduler(true);
    abort();
}

static void to_lane(int l) {
    Wave &w = g_wave;
    w.lane = l;
#if EMU_ASAN
    __sanitizer_start_switch_fiber(&g_sched_fake, w.stack[l], kStackBytes);
#endif
    emu_ctx_switch(&w.sched_sp, w.lane_sp[l]);
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(g_sched_fake, nullptr, nullptr);
#endif
}

static void *fresh_stack(int l) {
    Wave &w = g_wave;
    if (!w.stack[l]) {
        const size_t page = 4096;
        char *m = (char *)mmap(nullptr, kStackBytes + page, PROT_READ | PROT_WRITE,
                               MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
        if (m == MAP_FAILED) {
            fprintf(stderr, "emulator: no memory for lane stacks\n");
            abort();
        }
        mprotect(m, page, PROT_NONE);  // overflow guard
        w.stack[l] = m + page;
    }
#if EMU_ASAN
    __asan_unpoison_memory_region(w.stack[l], kStackBytes);
#endif
    uint64_t *sp = (uint64_t *)(w.stack[l] + kStackBytes);
    *--sp = 0;                           // alignment slot: entry sees rsp = 8 mod 16
    *--sp = (uint64_t)(uintptr_t)&lane_main;
    for (int r = 0; r < 6; r++) *--sp = 0;  // rbp rbx r12-r15
    return sp;
}

void run(void (*body)(void *), void *arg) {
    Wave &w = g_wave;
    w.body = body;
    w.arg = arg;
    w.failed = false;
    w.msg[0] = 0;
    for (int l = 0; l < kLanes; l++) {
        w.status[l] = 0;
        w.ops[l] = 0;
        w.lane_sp[l] = fresh_stack(l);
    }
    for (;;) {
        for (int l = 0; l < kLanes; l++) {
            if (w.status[l] != 0) continue;
            to_lane(l);
            if (w.failed) return;
        }
        int done = 0;
        for (int l = 0; l < kLanes; l++) done += w.status[l] == 2;
        if (done == kLanes) return;
        if (done > 0) {
            snprintf(w.msg, sizeof w.msg, "%d lanes returned while the others wait at a cross-lane operation", done);
            w.failed = true;
            return;
        }
        for (int l = 1; l < kLanes; l++)
            if (w.ops[l] != w.ops[0] || w.kind[l] != w.kind[0]) {
                snprintf(w.msg, sizeof w.msg,
                         "divergent cross-lane operations: lane 0 at #%llu (kind %d), lane %d at #%llu (kind %d)",
                         (unsigned long long)w.ops[0], w.kind[0], l, (unsigned long long)w.ops[l], w.kind[l]);
                w.failed = true;
                return;
            }
        if (w.max_ops && w.ops[0] > w.max_ops) {
            snprintf(w.msg, sizeof w.msg, "more than %llu cross-lane operations: stopped",
                     (unsigned long long)w.max_ops);
            w.failed = true;
            return;
        }
        for (int l = 0; l < kLanes; l++) w.status[l] = 0;
    }
}

}  // namespace emu

// ---- one gate ------------------------------------------------------------------
namespace gsim {

struct Task {
    JobDesc *J;
    int64_t ob;
    const GateRec *R;
    int64_t gate;
    void *L;
    const uint8_t *lut;  // the gate's 256-entry table
};

template <int K, int W, bool EDGE, bool PREFETCH, bool LEAN, bool AGENT>
void gate_body(void *p) {
    Task &t = *(Task *)p;
    WaveLds<W> &L = *(WaveLds<W> *)t.L;
    reinterpret_cast<uint32_t *>(L.lut)[lane_id()] = reinterpret_cast<const uint32_t *>(t.lut)[lane_id()];
    eval_gate<K, W, EDGE, PREFETCH, LEAN, AGENT>(*t.J, t.ob, *t.R, t.gate, L);
}

template <int W, bool EDGE, bool PREFETCH, bool LEAN, bool AGENT>
void (*pick(int k))(void *) {
    switch (k) {
    case 1: return gate_body<1, W, EDGE, PREFETCH, LEAN, AGENT>;
    case 2: return gate_body<2, W, EDGE, PREFETCH, LEAN, AGENT>;
    case 3: return gate_body<3, W, EDGE, PREFETCH, LEAN, AGENT>;
    default: return gate_body<4, W, EDGE, PREFETCH, LEAN, AGENT>;
    }
}

template <int K, int W, bool EDGE, bool AGENT>
void seg_body(void *p) {
    Task &t = *(Task *)p;
    SegLds<W> &L = *(SegLds<W> *)t.L;
    reinterpret_cast<uint32_t *>(L.lut)[lane_id()] = reinterpret_cast<const uint32_t *>(t.lut)[lane_id()];
    eval_gate_seg<K, W, EDGE, !AGENT, AGENT>(*t.J, t.ob, *t.R, t.gate, L);
}

template <int W, bool EDGE, bool AGENT>
void (*pick_seg(int k))(void *) {
    switch (k) {
    case 1: return seg_body<1, W, EDGE, AGENT>;
    case 2: return seg_body<2, W, EDGE, AGENT>;
    case 3: return seg_body<3, W, EDGE, AGENT>;
    default: return seg_body<4, W, EDGE, AGENT>;
    }
}

template <bool EDGE>
void (*variant(int mode, int window, int k))(void *) {
    switch (mode) {
    case 4: return window == 64 ? pick_seg<64, EDGE, false>(k) : pick_seg<256, EDGE, false>(k);
    case 5: return pick_seg<256, EDGE, true>(k);
    case 0: return window == 64 ? pick<64, EDGE, true, true, false>(k) : pick<256, EDGE, true, true, false>(k);
    case 1: return pick<256, EDGE, !EDGE, false, true>(k);
    case 2: return pick<256, EDGE, false, true, true>(k);
    default: return window == 64 ? pick<64, EDGE, true, false, false>(k) : pick<256, EDGE, true, false, false>(k);
    }
}

}  // namespace gsim

// ---- input file ------------------------------------------------------------------
struct Reader {
    FILE *f;
    int64_t i64() {
        int64_t x;
        if (fread(&x, 8, 1, f) != 1) { fprintf(stderr, "emu_eval: short input\n"); exit(2); }
        return x;
    }
    template <typename T>
    std::vector<T> arr(int64_t n) {
        std::vector<T> v((size_t)(n > 0 ? n : 0));
        if (n > 0 && fread(v.data(), sizeof(T), (size_t)n, f) != (size_t)n) {
            fprintf(stderr, "emu_eval: short input\n");
            exit(2);
        }
        return v;
    }
};

int main(int argc, char **argv) {
    using namespace gsim;
    if (argc != 3) {
        fprintf(stderr, "usage: emu_eval in.bin out.bin\n");
        return 2;
    }
    FILE *fi = fopen(argv[1], "rb");
    if (!fi) { perror(argv[1]); return 2; }
    Reader rd{fi};
    const int64_t mode = rd.i64(), S = rd.i64(), G = rd.i64(), n_types = rd.i64(), has_edge = rd.i64(),
                  n_eval = rd.i64(), max_ops = rd.i64();
    auto type = rd.arr<uint8_t>(G);
    auto pin_off = rd.arr<int64_t>(G + 1);
    const int64_t P = pin_off[G];
    auto pin_net = rd.arr<int64_t>(P);
    auto rise = rd.arr<int32_t>(P);
    auto fall = rd.arr<int32_t>(P);
    std::vector<int32_t> dly = has_edge ? rd.arr<int32_t>(4 * P) : std::vector<int32_t>();
    auto lut = rd.arr<uint8_t>(n_types * 256);
    auto net_off = rd.arr<int64_t>(S + G + 1);
    auto keys = rd.arr<uint64_t>(net_off[S + G]);
    auto gates = rd.arr<int64_t>(n_eval);
    fclose(fi);

    emu::wave().max_ops = (uint64_t)max_ops;
    // per-gate delay table of the extended model: [pin][edge][output], inf elsewhere
    std::vector<int32_t> edly;
    if (has_edge) {
        edly.assign((size_t)G * 16, kNoRelation);
        for (int64_t g = 0; g < G; g++)
            for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
                for (int e = 0; e < 4; e++) edly[(size_t)g * 16 + (p - pin_off[g]) * 4 + e] = dly[4 * p + e];
    }
    std::vector<int64_t> off((size_t)(S + G), 0), len((size_t)(S + G), 0);
    DevState state;
    JobDesc J;
    memset(&J, 0, sizeof J);
    J.S = S;
    J.off = off.data();
    J.len = len.data();
    J.state = &state;
    J.edly = has_edge ? edly.data() : nullptr;
    alignas(16) static uint64_t anchor[2];
    uint64_t *const base = anchor;  // every block is addressed relative to this word
    J.K = base;
    auto rel = [&](const uint64_t *p) { return (int64_t)(((intptr_t)p - (intptr_t)base) / 8); };

    std::mt19937_64 rng(12345);
    size_t lds_bytes = sizeof(WaveLds<kWindowLarge>);
    lds_bytes = std::max(lds_bytes, sizeof(SegLds<kWindowLarge>));
    std::vector<uint8_t> lds(lds_bytes);
    std::vector<int64_t> out_off(1, 0);
    std::vector<uint64_t> out_keys;
    std::vector<int32_t> err((size_t)n_eval, 0);
    int64_t n_fail = 0;
    for (int64_t e = 0; e < n_eval; e++) {
        const int64_t g = gates[e];
        GateRec R;
        memset(&R, 0, sizeof R);
        R.type = type[g];
        R.k = (uint8_t)(pin_off[g + 1] - pin_off[g]);
        int32_t dmax = 0;
        for (int i = 0; i < R.k; i++) {
            const int64_t p = pin_off[g] + i;
            R.net[i] = (int32_t)pin_net[p];
            R.rise[i] = rise[p];
            R.fall[i] = fall[p];
            if (has_edge) {
                for (int x = 0; x < 4; x++)
                    if (dly[4 * p + x] != kNoRelation) dmax = std::max(dmax, dly[4 * p + x]);
            } else {
                dmax = std::max(dmax, std::max(rise[p], fall[p]));
            }
        }
        R.dmax = dmax;
        // input waveforms and the output region, each a block of its own
        std::vector<uint64_t *> blocks;
        int64_t reserved = 0;
        for (int i = 0; i < R.k; i++) {
            const int64_t n = R.net[i];
            const int64_t a = net_off[n], m = net_off[n + 1] - a;
            uint64_t *b = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
            if (m > 0) memcpy(b, keys.data() + a, sizeof(uint64_t) * (size_t)m);
            blocks.push_back(b);
            off[n] = rel(b);
            len[n] = m;
            reserved += m;
        }
        uint64_t *ob_blk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(reserved > 0 ? reserved : 1));
        const int64_t ob = rel(ob_blk);
        memset(&state, 0, sizeof state);
        off[S + g] = -1;
        len[S + g] = -1;
        for (auto &x : lds) x = (uint8_t)rng();
        Task t{&J, ob, &R, g, lds.data(), lut.data() + (size_t)R.type * 256};
        const int window = dmax <= kWindowSmall ? 64 : 256;
        const bool wave_gate = dmax <= kWindowLarge;
        const bool level_form = mode == 0 || mode == 3 || mode == 4;
        std::string msg;
        if (wave_gate) {
            void (*body)(void *) = has_edge ? variant<true>((int)mode, window, R.k)
                                            : variant<false>((int)mode, window, R.k);
            emu::run(body, &t);
            if (emu::wave().failed) msg = emu::wave().msg;
        } else {
            emu::wave().lane = 0;
            if (level_form)
                eval_seq<false>(J, R, g, ob, lut.data() + (size_t)R.type * 256);
            else
                eval_seq<true>(J, R, g, ob, lut.data() + (size_t)R.type * 256);
        }
        int64_t n_out = 0;
        if (!msg.empty()) {
            err[e] = 100;
            if (n_fail++ < 10) fprintf(stderr, "gate %lld: %s\n", (long long)g, msg.c_str());
        } else if (state.check_error) {
            err[e] = state.check_error;
            if (n_fail++ < 10) fprintf(stderr, "gate %lld: device check %d\n", (long long)g, state.check_error);
        } else if (off[S + g] != ob || len[S + g] < 0 || len[S + g] > reserved) {
            err[e] = 101;
            if (n_fail++ < 10) fprintf(stderr, "gate %lld: bad offset or length\n", (long long)g);
        } else {
            n_out = len[S + g];
            out_keys.insert(out_keys.end(), ob_blk, ob_blk + n_out);
        }
        out_off.push_back(out_off.back() + n_out);
        for (auto b : blocks) free(b);
        free(ob_blk);
    }
    FILE *fo = fopen(argv[2], "wb");
    if (!fo) { perror(argv[2]); return 2; }
    fwrite(out_off.data(), 8, out_off.size(), fo);
    fwrite(out_keys.data(), 8, out_keys.size(), fo);
    fwrite(err.data(), 4, err.size(), fo);
    fclose(fo);
    fprintf(stderr, "emu_eval: %lld gates, %lld failed\n", (long long)n_eval, (long long)n_fail);
    return 0;
}
