/*
 * oracle/o1.c -- CPU ORACLE. TEST INFRASTRUCTURE ONLY.
 *
 * This file is not part of the product. Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may build, load or call it. It shares
 * no code, header, table or constant with the HIP library: it is a plain,
 * slow, literal reading of the paper, kept deliberately simple so a reader can
 * check it against the paper by eye.
 *
 * What it computes (Section 2.1, objective statement): given a combinational
 * netlist of basic gates, per-pin delays and the 0/1/X/Z waveforms of the
 * source nets, the waveform of every gate output.
 *
 *  - 4-value logic with Z evaluated as X (Section 2.2) and the AND / OR / XOR
 *    truth tables of Table 1, typed in below. NOT, BUF, NAND, NOR, XNOR and
 *    the 3/4-input AND and OR are built from them. MUX2 is not in the paper:
 *    s=0 selects d0, s=1 selects d1, an unknown select gives the data value
 *    if both data inputs agree and X otherwise (Verilog's ?: merge rule) --
 *    parity unpinned by the paper for MUX2.
 *  - Per gate: Algorithm 2 (output waveform of an unlocked cell): a time merge
 *    of the input waveforms; at each earliest time every input that has a
 *    transition there is updated; the gate is evaluated; if the output value
 *    changed, the delay is the minimum over the inputs that changed at that
 *    time (Section 2.3 and Fig. 2; Section 3.2), and the new transition is
 *    added to the output with the "glitch eaten" rule of Eq. 1 (every earlier
 *    determined transition whose appearance time is not before the new one is
 *    denied) and the redundant-transition drop of Fig. 3 (a transition to the
 *    value the output already has is not stored).
 *  - Delay model: the paper's delay matrix is indexed by triggering pin, input
 *    edge and output value (Section 2.3). The netlists here give one rise and
 *    one fall delay per pin; the delay of a new output value 1 is the pin's
 *    rise delay, of 0 its fall delay, of X the smaller of the two (the
 *    Verilog rule for transitions to x -- parity unpinned by the paper for the
 *    X case). A pin with no transition at the merge time has no edge, which
 *    the paper's matrix expresses as an infinite delay.
 *  - Readings where the paper is silent: every input starts at X and the
 *    previous evaluated output starts at X; an empty input waveform stays X;
 *    outputs are not clipped to a window; an equal appearance time denies the
 *    older transition (Eq. 1 uses <=).
 *  - The whole circuit: gates are evaluated in a topological order that this
 *    file computes itself (Kahn's algorithm), so each gate's inputs are
 *    complete when it is evaluated (the dependency rule of Section 4.1).
 *    o1_simulate_parallel evaluates the same gates level by level on several
 *    threads (for timing the oracle on a multi-core host); its result is the
 *    same.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O1_X 2
#define O1_Z 3
#define O1_INF INT64_MAX

/* ---- Table 1: 4-value AND, OR and XOR. Row = first operand, column =
 * second operand, both in the order 0, 1, X, Z. ---------------------------- */
static const uint8_t TABLE1_AND[4][4] = {
    {0, 0, 0, 0},
    {0, 1, 2, 2},
    {0, 2, 2, 2},
    {0, 2, 2, 2},
};
static const uint8_t TABLE1_OR[4][4] = {
    {0, 1, 2, 2},
    {1, 1, 1, 1},
    {2, 1, 2, 2},
    {2, 1, 2, 2},
};
static const uint8_t TABLE1_XOR[4][4] = {
    {0, 1, 2, 2},
    {1, 0, 2, 2},
    {2, 2, 2, 2},
    {2, 2, 2, 2},
};

enum { T_BUF, T_NOT, T_AND2, T_OR2, T_NAND2, T_NOR2, T_XOR2, T_XNOR2, T_AND3, T_MUX2,
       T_AND4, T_OR4, T_COUNT };

static int arity_of(int type) {
    switch (type) {
    case T_BUF: case T_NOT: return 1;
    case T_AND3: case T_MUX2: return 3;
    case T_AND4: case T_OR4: return 4;
    default: return 2;
    }
}

/* Z is read as X (Section 2.2). */
static uint8_t z_as_x(uint8_t a) { return a == O1_Z ? O1_X : a; }

static uint8_t logic_not(uint8_t a) {
    a = z_as_x(a);
    return a == 0 ? 1 : a == 1 ? 0 : O1_X;
}

/* The module function of one basic gate over its current input values. */
uint8_t o1_calculate_signal(int type, const uint8_t *in) {
    switch (type) {
    case T_BUF: return z_as_x(in[0]);
    case T_NOT: return logic_not(in[0]);
    case T_AND2: return TABLE1_AND[in[0]][in[1]];
    case T_OR2: return TABLE1_OR[in[0]][in[1]];
    case T_NAND2: return logic_not(TABLE1_AND[in[0]][in[1]]);
    case T_NOR2: return logic_not(TABLE1_OR[in[0]][in[1]]);
    case T_XOR2: return TABLE1_XOR[in[0]][in[1]];
    case T_XNOR2: return logic_not(TABLE1_XOR[in[0]][in[1]]);
    case T_AND3: return TABLE1_AND[TABLE1_AND[in[0]][in[1]]][in[2]];
    case T_AND4: return TABLE1_AND[TABLE1_AND[TABLE1_AND[in[0]][in[1]]][in[2]]][in[3]];
    case T_OR4: return TABLE1_OR[TABLE1_OR[TABLE1_OR[in[0]][in[1]]][in[2]]][in[3]];
    case T_MUX2: {
        uint8_t d0 = z_as_x(in[0]), d1 = z_as_x(in[1]), s = z_as_x(in[2]);
        if (s == 0) return d0;
        if (s == 1) return d1;
        return d0 == d1 ? d0 : O1_X;
    }
    }
    return O1_X;
}

/* ---- A growable waveform: parallel arrays of times and values. ---------- */
typedef struct {
    int64_t *t;
    uint8_t *v;
    int64_t n, cap;
} o1_wave;

static int wave_push(o1_wave *w, uint8_t v, int64_t t) {
    if (w->n == w->cap) {
        int64_t cap = w->cap ? 2 * w->cap : 16;
        int64_t *nt = (int64_t *)realloc(w->t, (size_t)cap * sizeof(int64_t));
        if (!nt) return -1;
        w->t = nt;
        uint8_t *nv = (uint8_t *)realloc(w->v, (size_t)cap);
        if (!nv) return -1;
        w->v = nv;
        w->cap = cap;
    }
    w->t[w->n] = t;
    w->v[w->n] = v;
    w->n++;
    return 0;
}

/* Delay of one pin for a new output value (reduced delay model, see header). */
static int64_t pin_delay(int32_t rise, int32_t fall, uint8_t out_value) {
    if (out_value == 1) return rise;
    if (out_value == 0) return fall;
    return rise < fall ? rise : fall;
}

/* addSignalChange: Eq. 1 "glitch eaten", then the redundant drop of Fig. 3.
 * Every entry already in `out` was determined at an earlier merge time, and
 * the entries are in increasing appearance time, so the denied ones are the
 * tail whose appearance time is >= t_r. */
static int add_signal_change(o1_wave *out, uint8_t v, int64_t t_r) {
    while (out->n > 0 && out->t[out->n - 1] >= t_r) out->n--;
    uint8_t current = out->n > 0 ? out->v[out->n - 1] : O1_X;
    if (v == current) return 0;
    return wave_push(out, v, t_r);
}

/* Algorithm 2 for one single-output gate. `in_t[i]`, `in_v[i]`, `in_n[i]`
 * are the waveform of input pin i. */
int o1_process_cell(int type, const int64_t *const *in_t, const uint8_t *const *in_v,
                    const int64_t *in_n, const int32_t *rise, const int32_t *fall,
                    o1_wave *out) {
    int k = arity_of(type);
    uint8_t current_signals[4];
    int64_t earliest_index[4];
    int64_t earliest_timestamp[4];
    int changed[4];
    for (int i = 0; i < k; i++) {
        current_signals[i] = O1_X;
        earliest_index[i] = 0;
        earliest_timestamp[i] = in_n[i] > 0 ? in_t[i][0] : O1_INF;
    }
    uint8_t previous_output = O1_X;
    for (;;) {
        int64_t t_earliest = O1_INF;
        for (int i = 0; i < k; i++)
            if (earliest_timestamp[i] < t_earliest) t_earliest = earliest_timestamp[i];
        if (t_earliest == O1_INF) break;
        for (int i = 0; i < k; i++) {
            changed[i] = 0;
            int64_t j = earliest_index[i];
            if (earliest_timestamp[i] == t_earliest) {
                current_signals[i] = in_v[i][j];
                changed[i] = 1;
                if (j + 1 == in_n[i]) {
                    earliest_timestamp[i] = O1_INF;
                } else {
                    earliest_index[i] = j + 1;
                    earliest_timestamp[i] = in_t[i][j + 1];
                }
            }
        }
        uint8_t new_output = o1_calculate_signal(type, current_signals);
        if (new_output != previous_output) {
            int64_t del = O1_INF;
            for (int i = 0; i < k; i++) {
                if (!changed[i]) continue; /* no edge on this pin: infinite delay */
                int64_t d = pin_delay(rise[i], fall[i], new_output);
                if (d < del) del = d;
            }
            if (add_signal_change(out, new_output, t_earliest + del)) return -1;
        }
        previous_output = new_output;
    }
    return 0;
}

/* ---- Whole circuit. ------------------------------------------------------ */
typedef struct {
    int64_t S, G;
    o1_wave *gate_out; /* [G] */
} o1_result;

/* Kahn's algorithm over the gate graph; returns 0 and fills `order` with all
 * gates, or -2 if the gates do not form a DAG. */
static int topological_order(int64_t S, int64_t G, const int64_t *pin_off,
                             const int64_t *pin_net, int64_t *order) {
    int64_t *indeg = (int64_t *)calloc((size_t)(G ? G : 1), sizeof(int64_t));
    int64_t *fo_cnt = (int64_t *)calloc((size_t)(G + 1), sizeof(int64_t));
    if (!indeg || !fo_cnt) { free(indeg); free(fo_cnt); return -1; }
    int64_t P = pin_off[G];
    for (int64_t g = 0; g < G; g++)
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
            if (pin_net[p] >= S) { indeg[g]++; fo_cnt[pin_net[p] - S + 1]++; }
    for (int64_t g = 0; g < G; g++) fo_cnt[g + 1] += fo_cnt[g];
    int64_t *fo = (int64_t *)malloc((size_t)(P ? P : 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)(G ? G : 1), sizeof(int64_t));
    if (!fo || !fill) { free(indeg); free(fo_cnt); free(fo); free(fill); return -1; }
    for (int64_t g = 0; g < G; g++)
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
            if (pin_net[p] >= S) {
                int64_t d = pin_net[p] - S;
                fo[fo_cnt[d] + fill[d]++] = g;
            }
    int64_t head = 0, tail = 0;
    for (int64_t g = 0; g < G; g++)
        if (indeg[g] == 0) order[tail++] = g;
    while (head < tail) {
        int64_t d = order[head++];
        for (int64_t e = fo_cnt[d]; e < fo_cnt[d + 1]; e++)
            if (--indeg[fo[e]] == 0) order[tail++] = fo[e];
    }
    free(indeg); free(fo_cnt); free(fo); free(fill);
    return tail == G ? 0 : -2;
}

void o1_free(o1_result *r) {
    if (!r) return;
    if (r->gate_out)
        for (int64_t g = 0; g < r->G; g++) { free(r->gate_out[g].t); free(r->gate_out[g].v); }
    free(r->gate_out);
    free(r);
}

/* Simulate the whole netlist. Returns NULL on a malformed netlist (cycle,
 * bad arity, bad net id) or out of memory; *status receives the reason:
 * -1 memory, -2 cycle, -3 malformed. */
o1_result *o1_simulate(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                       const int64_t *pin_net, const int32_t *rise, const int32_t *fall,
                       const int64_t *src_off, const int64_t *src_t, const uint8_t *src_v,
                       int *status) {
    *status = 0;
    for (int64_t g = 0; g < G; g++) {
        if (type[g] >= T_COUNT || pin_off[g + 1] - pin_off[g] != arity_of(type[g])) {
            *status = -3;
            return NULL;
        }
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
            if (pin_net[p] < 0 || pin_net[p] >= S + G || pin_net[p] == S + g) {
                *status = -3;
                return NULL;
            }
    }
    o1_result *r = (o1_result *)calloc(1, sizeof(o1_result));
    int64_t *order = (int64_t *)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
    if (!r || !order) { free(r); free(order); *status = -1; return NULL; }
    r->S = S;
    r->G = G;
    r->gate_out = (o1_wave *)calloc((size_t)(G ? G : 1), sizeof(o1_wave));
    if (!r->gate_out) { free(order); free(r); *status = -1; return NULL; }
    int rc = topological_order(S, G, pin_off, pin_net, order);
    if (rc) { free(order); o1_free(r); *status = rc; return NULL; }
    for (int64_t idx = 0; idx < G; idx++) {
        int64_t g = order[idx];
        const int64_t *in_t[4];
        const uint8_t *in_v[4];
        int64_t in_n[4];
        int k = arity_of(type[g]);
        for (int i = 0; i < k; i++) {
            int64_t net = pin_net[pin_off[g] + i];
            if (net < S) {
                in_t[i] = src_t + src_off[net];
                in_v[i] = src_v + src_off[net];
                in_n[i] = src_off[net + 1] - src_off[net];
            } else {
                o1_wave *w = &r->gate_out[net - S];
                in_t[i] = w->t;
                in_v[i] = w->v;
                in_n[i] = w->n;
            }
        }
        if (o1_process_cell(type[g], in_t, in_v, in_n, rise + pin_off[g], fall + pin_off[g],
                            &r->gate_out[g])) {
            free(order); o1_free(r); *status = -1; return NULL;
        }
    }
    free(order);
    return r;
}

/* ---- Level-parallel driver (for timing the oracle on several cores). ----
 * The same per-gate procedure as o1_simulate. A gate's level is one more
 * than the highest level among the gates it reads (sources are level 0), so
 * the gates of one level read only finished waveforms of lower levels; each
 * level is split into contiguous ranges, one per thread, and the threads are
 * joined before the next level starts. The result is identical to
 * o1_simulate's: every gate sees the same complete input waveforms. */
typedef struct {
    int64_t S;
    const uint8_t *type;
    const int64_t *pin_off, *pin_net;
    const int32_t *rise, *fall;
    const int64_t *src_off, *src_t;
    const uint8_t *src_v;
    o1_result *r;
    const int64_t *gates; /* this thread's gates */
    int64_t n;
    int failed;
    /* memory-light mode (o1_simulate_fingerprints_parallel), else NULL:
     * each gate's length and fingerprint; its copy into `kept` if keep_at[g]
     * >= 0; its waveform freed at once if no gate reads it */
    int64_t *len;
    uint64_t *fp;
    const int64_t *keep_at;
    o1_result *kept;
    const int64_t *last_reader_level;
} o1_level_part;

static uint64_t fingerprint(const int64_t *t, const uint8_t *v, int64_t n);

static int eval_gate_into(const o1_level_part *a, int64_t g) {
    const int64_t *in_t[4];
    const uint8_t *in_v[4];
    int64_t in_n[4];
    int k = arity_of(a->type[g]);
    for (int i = 0; i < k; i++) {
        int64_t net = a->pin_net[a->pin_off[g] + i];
        if (net < a->S) {
            in_t[i] = a->src_t + a->src_off[net];
            in_v[i] = a->src_v + a->src_off[net];
            in_n[i] = a->src_off[net + 1] - a->src_off[net];
        } else {
            const o1_wave *w = &a->r->gate_out[net - a->S];
            in_t[i] = w->t;
            in_v[i] = w->v;
            in_n[i] = w->n;
        }
    }
    return o1_process_cell(a->type[g], in_t, in_v, in_n, a->rise + a->pin_off[g],
                           a->fall + a->pin_off[g], &a->r->gate_out[g]);
}

static int copy_wave(const o1_wave *from, o1_wave *to) {
    size_t n = (size_t)(from->n ? from->n : 1);
    to->t = (int64_t *)malloc(n * sizeof(int64_t));
    to->v = (uint8_t *)malloc(n);
    if (!to->t || !to->v) return -1;
    if (from->n) {
        memcpy(to->t, from->t, (size_t)from->n * sizeof(int64_t));
        memcpy(to->v, from->v, (size_t)from->n);
    }
    to->n = to->cap = from->n;
    return 0;
}

static void *level_part_run(void *arg) {
    o1_level_part *a = (o1_level_part *)arg;
    for (int64_t i = 0; i < a->n && !a->failed; i++) {
        const int64_t g = a->gates[i];
        if (eval_gate_into(a, g)) {
            a->failed = 1;
            break;
        }
        if (!a->len) continue;
        o1_wave *w = &a->r->gate_out[g];
        a->len[g] = w->n;
        a->fp[g] = fingerprint(w->t, w->v, w->n);
        if (a->keep_at[g] >= 0 && copy_wave(w, &a->kept->gate_out[a->keep_at[g]])) a->failed = 1;
        if (a->last_reader_level[g] == 0) { /* nothing reads it */
            free(w->t); free(w->v);
            w->t = NULL; w->v = NULL;
        }
    }
    return NULL;
}

static int check_netlist(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                         const int64_t *pin_net) {
    for (int64_t g = 0; g < G; g++) {
        if (type[g] >= T_COUNT || pin_off[g + 1] - pin_off[g] != arity_of(type[g])) return -3;
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
            if (pin_net[p] < 0 || pin_net[p] >= S + G || pin_net[p] == S + g) return -3;
    }
    return 0;
}

/* Level of every gate (1 + the highest level among the gates it reads;
 * sources are level 0) and the gates sorted by level: level l holds
 * by_level[level_start[l] .. level_start[l + 1]). level_start has n_levels + 2
 * entries and is the caller's to free. */
static int sort_by_level(int64_t S, int64_t G, const int64_t *pin_off, const int64_t *pin_net,
                         int64_t *level, int64_t *by_level, int64_t **level_start_out,
                         int64_t *n_levels_out) {
    int64_t *order = (int64_t *)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
    if (!order) return -1;
    int rc = topological_order(S, G, pin_off, pin_net, order);
    int64_t n_levels = 0, *level_start = NULL;
    if (!rc) {
        for (int64_t idx = 0; idx < G; idx++) { /* inputs precede their readers */
            int64_t g = order[idx], lv = 0;
            for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
                if (pin_net[p] >= S && level[pin_net[p] - S] > lv) lv = level[pin_net[p] - S];
            level[g] = lv + 1;
            if (lv + 1 > n_levels) n_levels = lv + 1;
        }
        level_start = (int64_t *)calloc((size_t)n_levels + 2, sizeof(int64_t));
        if (!level_start) rc = -1;
    }
    if (!rc) { /* counting sort of the gates by level */
        for (int64_t g = 0; g < G; g++) level_start[level[g] + 1]++;
        for (int64_t l = 1; l <= n_levels + 1; l++) level_start[l] += level_start[l - 1];
        for (int64_t g = 0; g < G; g++) by_level[level_start[level[g]]++] = g;
        for (int64_t l = n_levels + 1; l > 0; l--) level_start[l] = level_start[l - 1];
        level_start[0] = 0;
    }
    free(order);
    *level_start_out = level_start;
    *n_levels_out = n_levels;
    return rc;
}

/* One level's gates split into contiguous ranges, one per thread; every
 * thread is joined before this returns. `proto` holds the fields common to
 * all parts. Returns -1 if a gate failed (out of memory). */
static int run_level(const o1_level_part *proto, const int64_t *gates, int64_t n, int n_threads) {
    int nt = n < n_threads ? (int)(n ? n : 1) : n_threads;
    o1_level_part parts[256];
    pthread_t th[256];
    int started[256];
    for (int k = 0; k < nt; k++) {
        o1_level_part *pa = &parts[k];
        *pa = *proto;
        pa->failed = 0;
        const int64_t lo = n * k / nt, hi = n * (k + 1) / nt;
        pa->gates = gates + lo;
        pa->n = hi - lo;
        started[k] = k > 0 && pthread_create(&th[k], NULL, level_part_run, pa) == 0;
    }
    level_part_run(&parts[0]);
    for (int k = 1; k < nt; k++) {
        if (started[k]) pthread_join(th[k], NULL);
        else level_part_run(&parts[k]); /* no thread: run it here */
    }
    for (int k = 0; k < nt; k++)
        if (parts[k].failed) return -1;
    return 0;
}

o1_result *o1_simulate_parallel(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                                const int64_t *pin_net, const int32_t *rise, const int32_t *fall,
                                const int64_t *src_off, const int64_t *src_t, const uint8_t *src_v,
                                int n_threads, int *status) {
    *status = 0;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if ((*status = check_netlist(S, G, type, pin_off, pin_net)) != 0) return NULL;
    size_t gn = (size_t)(G ? G : 1);
    o1_result *r = (o1_result *)calloc(1, sizeof(o1_result));
    int64_t *level = (int64_t *)calloc(gn, sizeof(int64_t));
    int64_t *by_level = (int64_t *)malloc(gn * sizeof(int64_t));
    if (!r || !level || !by_level) {
        free(r); free(level); free(by_level);
        *status = -1;
        return NULL;
    }
    r->S = S;
    r->G = G;
    r->gate_out = (o1_wave *)calloc(gn, sizeof(o1_wave));
    int64_t n_levels = 0, *level_start = NULL;
    int rc = r->gate_out ? sort_by_level(S, G, pin_off, pin_net, level, by_level, &level_start, &n_levels) : -1;
    o1_level_part proto;
    memset(&proto, 0, sizeof proto);
    proto.S = S; proto.type = type; proto.pin_off = pin_off; proto.pin_net = pin_net;
    proto.rise = rise; proto.fall = fall; proto.src_off = src_off; proto.src_t = src_t;
    proto.src_v = src_v; proto.r = r;
    for (int64_t l = 1; !rc && l <= n_levels; l++)
        rc = run_level(&proto, by_level + level_start[l], level_start[l + 1] - level_start[l], n_threads);
    free(level); free(by_level); free(level_start);
    if (rc) {
        o1_free(r);
        *status = rc;
        return NULL;
    }
    return r;
}

/* Level-parallel memory-light driver for full-size parity checks: the gates
 * of o1_simulate, level by level on n_threads threads as o1_simulate_parallel,
 * each waveform reduced to len[g] and fp[g] (the fingerprint defined below
 * o1_fingerprints) and freed once the level of its last reader is done. The
 * n_keep gates listed in `keep` (distinct gate indices) are also returned
 * whole, in that order, as an o1_result of n_keep entries (free with
 * o1_free). Returns NULL with *status as o1_simulate on failure. */
o1_result *o1_simulate_fingerprints_parallel(int64_t S, int64_t G, const uint8_t *type,
                                             const int64_t *pin_off, const int64_t *pin_net,
                                             const int32_t *rise, const int32_t *fall,
                                             const int64_t *src_off, const int64_t *src_t,
                                             const uint8_t *src_v, int n_threads, int64_t *len,
                                             uint64_t *fp, int64_t n_keep, const int64_t *keep,
                                             int *status) {
    *status = 0;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if ((*status = check_netlist(S, G, type, pin_off, pin_net)) != 0) return NULL;
    for (int64_t i = 0; i < n_keep; i++)
        if (keep[i] < 0 || keep[i] >= G) {
            *status = -3;
            return NULL;
        }
    size_t gn = (size_t)(G ? G : 1);
    o1_result *work = (o1_result *)calloc(1, sizeof(o1_result));
    o1_result *kept = (o1_result *)calloc(1, sizeof(o1_result));
    int64_t *level = (int64_t *)calloc(gn, sizeof(int64_t));
    int64_t *by_level = (int64_t *)malloc(gn * sizeof(int64_t));
    int64_t *keep_at = (int64_t *)malloc(gn * sizeof(int64_t));
    int64_t *last_reader = (int64_t *)calloc(gn, sizeof(int64_t));
    int64_t *free_at = (int64_t *)malloc(gn * sizeof(int64_t));
    int rc = (work && kept && level && by_level && keep_at && last_reader && free_at) ? 0 : -1;
    if (!rc) {
        work->S = kept->S = S;
        work->G = G;
        kept->G = n_keep;
        work->gate_out = (o1_wave *)calloc(gn, sizeof(o1_wave));
        kept->gate_out = (o1_wave *)calloc((size_t)(n_keep ? n_keep : 1), sizeof(o1_wave));
        if (!work->gate_out || !kept->gate_out) rc = -1;
    }
    int64_t n_levels = 0, *level_start = NULL, *free_start = NULL;
    if (!rc) rc = sort_by_level(S, G, pin_off, pin_net, level, by_level, &level_start, &n_levels);
    if (!rc) {
        for (int64_t g = 0; g < G; g++) keep_at[g] = -1;
        for (int64_t i = 0; i < n_keep; i++) keep_at[keep[i]] = i;
        /* the level after which each gate's waveform is no longer read */
        for (int64_t g = 0; g < G; g++)
            for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
                if (pin_net[p] >= S && last_reader[pin_net[p] - S] < level[g])
                    last_reader[pin_net[p] - S] = level[g];
        free_start = (int64_t *)calloc((size_t)n_levels + 2, sizeof(int64_t));
        if (!free_start) rc = -1;
    }
    if (!rc) { /* gates grouped by the level that frees them */
        for (int64_t g = 0; g < G; g++) free_start[last_reader[g] + 1]++;
        for (int64_t l = 1; l <= n_levels + 1; l++) free_start[l] += free_start[l - 1];
        for (int64_t g = 0; g < G; g++) free_at[free_start[last_reader[g]]++] = g;
        for (int64_t l = n_levels + 1; l > 0; l--) free_start[l] = free_start[l - 1];
        free_start[0] = 0;
    }
    o1_level_part proto;
    memset(&proto, 0, sizeof proto);
    proto.S = S; proto.type = type; proto.pin_off = pin_off; proto.pin_net = pin_net;
    proto.rise = rise; proto.fall = fall; proto.src_off = src_off; proto.src_t = src_t;
    proto.src_v = src_v; proto.r = work;
    proto.len = len; proto.fp = fp; proto.keep_at = keep_at; proto.kept = kept;
    proto.last_reader_level = last_reader;
    for (int64_t l = 1; !rc && l <= n_levels; l++) {
        rc = run_level(&proto, by_level + level_start[l], level_start[l + 1] - level_start[l], n_threads);
        for (int64_t i = free_start[l]; !rc && i < free_start[l + 1]; i++) {
            o1_wave *w = &work->gate_out[free_at[i]];
            free(w->t); free(w->v);
            w->t = NULL; w->v = NULL;
        }
    }
    free(level); free(by_level); free(keep_at); free(last_reader); free(free_at);
    free(level_start); free(free_start);
    if (work) {
        if (work->gate_out)
            for (int64_t g = 0; g < G; g++) { free(work->gate_out[g].t); free(work->gate_out[g].v); }
        free(work->gate_out);
        free(work);
    }
    if (rc) {
        o1_free(kept);
        *status = rc;
        return NULL;
    }
    return kept;
}

/* Per-gate output lengths. */
void o1_lengths(const o1_result *r, int64_t *len) {
    for (int64_t g = 0; g < r->G; g++) len[g] = r->gate_out[g].n;
}

/* Copy all gate outputs into CSR arrays: off[G+1], t[off[G]], v[off[G]]. */
void o1_copy(const o1_result *r, int64_t *off, int64_t *t, uint8_t *v) {
    int64_t pos = 0;
    for (int64_t g = 0; g < r->G; g++) {
        off[g] = pos;
        memcpy(t + pos, r->gate_out[g].t, (size_t)r->gate_out[g].n * sizeof(int64_t));
        memcpy(v + pos, r->gate_out[g].v, (size_t)r->gate_out[g].n);
        pos += r->gate_out[g].n;
    }
    off[r->G] = pos;
}

/* Single-gate entry point for unit tests of Algorithm 2. Writes at most `cap`
 * entries; returns the output length, or -1 on error. */
int64_t o1_gate(int type, const int64_t *const *in_t, const uint8_t *const *in_v,
                const int64_t *in_n, const int32_t *rise, const int32_t *fall,
                int64_t *out_t, uint8_t *out_v, int64_t cap) {
    o1_wave w = {0, 0, 0, 0};
    if (o1_process_cell(type, in_t, in_v, in_n, rise, fall, &w)) { free(w.t); free(w.v); return -1; }
    int64_t n = w.n;
    if (n <= cap) {
        memcpy(out_t, w.t, (size_t)n * sizeof(int64_t));
        memcpy(out_v, w.v, (size_t)n);
    }
    free(w.t);
    free(w.v);
    return n;
}

/* ---- Memory-light mode for full-size parity checks ------------------------
 * Same procedure as o1_simulate, but each gate's waveform is reduced to its
 * length and a 64-bit fingerprint, and freed as soon as its last reader has
 * been evaluated. Fingerprint of a waveform of n transitions with
 * key_i = time_i * 4 + value_i:  fp = mix(n) + sum_i mix(key_i XOR mix(i))
 * (mod 2^64), mix being the SplitMix64 finaliser. */
static uint64_t fp_mix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static uint64_t fingerprint(const int64_t *t, const uint8_t *v, int64_t n) {
    uint64_t acc = fp_mix((uint64_t)n);
    for (int64_t i = 0; i < n; i++)
        acc += fp_mix((((uint64_t)t[i] << 2) | v[i]) ^ fp_mix((uint64_t)i));
    return acc;
}

/* Fingerprints of arbitrary CSR waveforms (for cross-checking test helpers). */
void o1_fingerprints(int64_t n_nets, const int64_t *off, const int64_t *t, const uint8_t *v,
                     uint64_t *out) {
    for (int64_t i = 0; i < n_nets; i++)
        out[i] = fingerprint(t + off[i], v + off[i], off[i + 1] - off[i]);
}

/* Returns 0, or the same codes as o1_simulate's status. Fills len[G], fp[G]. */
int o1_simulate_fingerprints(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                             const int64_t *pin_net, const int32_t *rise, const int32_t *fall,
                             const int64_t *src_off, const int64_t *src_t, const uint8_t *src_v,
                             int64_t *len, uint64_t *fp) {
    for (int64_t g = 0; g < G; g++) {
        if (type[g] >= T_COUNT || pin_off[g + 1] - pin_off[g] != arity_of(type[g])) return -3;
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
            if (pin_net[p] < 0 || pin_net[p] >= S + G || pin_net[p] == S + g) return -3;
    }
    int64_t *order = (int64_t *)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
    int64_t *readers_left = (int64_t *)calloc((size_t)(G ? G : 1), sizeof(int64_t));
    o1_wave *w = (o1_wave *)calloc((size_t)(G ? G : 1), sizeof(o1_wave));
    if (!order || !readers_left || !w) { free(order); free(readers_left); free(w); return -1; }
    int rc = topological_order(S, G, pin_off, pin_net, order);
    if (rc) { free(order); free(readers_left); free(w); return rc; }
    for (int64_t p = 0; p < (G ? pin_off[G] : 0); p++)
        if (pin_net[p] >= S) readers_left[pin_net[p] - S]++;
    for (int64_t idx = 0; idx < G; idx++) {
        int64_t g = order[idx];
        const int64_t *in_t[4];
        const uint8_t *in_v[4];
        int64_t in_n[4];
        int k = arity_of(type[g]);
        for (int i = 0; i < k; i++) {
            int64_t net = pin_net[pin_off[g] + i];
            if (net < S) {
                in_t[i] = src_t + src_off[net];
                in_v[i] = src_v + src_off[net];
                in_n[i] = src_off[net + 1] - src_off[net];
            } else {
                in_t[i] = w[net - S].t;
                in_v[i] = w[net - S].v;
                in_n[i] = w[net - S].n;
            }
        }
        if (o1_process_cell(type[g], in_t, in_v, in_n, rise + pin_off[g], fall + pin_off[g], &w[g])) {
            rc = -1;
            break;
        }
        len[g] = w[g].n;
        fp[g] = fingerprint(w[g].t, w[g].v, w[g].n);
        for (int i = 0; i < k; i++) {
            int64_t net = pin_net[pin_off[g] + i];
            if (net >= S && --readers_left[net - S] == 0) {
                free(w[net - S].t); free(w[net - S].v);
                w[net - S].t = NULL; w[net - S].v = NULL;
            }
        }
        if (readers_left[g] == 0) {
            free(w[g].t); free(w[g].v);
            w[g].t = NULL; w[g].v = NULL;
        }
    }
    for (int64_t g = 0; g < G; g++) { free(w[g].t); free(w[g].v); }
    free(order); free(readers_left); free(w);
    return rc;
}

/* ------------------------------------------------------------------------
 * Extended cell model (Section 2.3, delays of gates; Section 3.2, the delay
 * matrix; Section 3.3, module functions). Test infrastructure, like the rest
 * of this file.
 *
 *  - Module function: a built-in type (0-11) as above, or a user-defined
 *    primitive (type 12 + u) whose value is read from table u, 256 entries
 *    indexed by the packed pin values (pin i in bits 2i..2i+1); the table
 *    covers every 0/1/X/Z combination, so no Z-as-X rule applies to it.
 *  - Delay: the paper indexes the delay matrix by triggering pin, input edge
 *    and output value. Here per pin i: dly[i][edge][out] with edge 0 = rise,
 *    1 = fall and out 0 or 1; INT32_MAX means no relation (the paper's inf).
 *    Readings (the paper does not define edges of a 4-value signal): a pin
 *    change rises if its new value is 1 or it leaves 0 for X or Z, falls if
 *    its new value is 0 or it leaves 1 for X or Z, and a change between X
 *    and Z counts as both (the smaller delay). A new output value X takes the
 *    smaller of the edge's delays to 0 and to 1. The delay of a candidate is
 *    the minimum over the pins that changed at its time; when every one of
 *    them is unrelated (infinite) the candidate never appears -- appending it
 *    at infinite time and letting Eq. 1 deny it later is the same -- while
 *    the previous evaluated value still becomes the new one.
 *  - A gate is evaluated only at its input transitions, starting from an X
 *    previous value (Algorithm 2), so a table's value for all-X inputs is
 *    not output before the first input change.
 * ------------------------------------------------------------------------ */
#define O1X_NO_RELATION INT32_MAX

static int edge_of(uint8_t old_v, uint8_t new_v) {
    if (new_v == 1 || (old_v == 0 && (new_v == O1_X || new_v == O1_Z))) return 0;
    if (new_v == 0 || (old_v == 1 && (new_v == O1_X || new_v == O1_Z))) return 1;
    return 2; /* X <-> Z */
}

static int64_t edge_out_delay(const int32_t *d /* [2 edges][2 outs] */, int edge, uint8_t out) {
    int64_t best = O1_INF;
    for (int e = 0; e < 2; e++) {
        if (edge != 2 && e != edge) continue;
        for (int o = 0; o < 2; o++) {
            if (out != O1_X && o != out) continue;
            int32_t x = d[e * 2 + o];
            if (x != O1X_NO_RELATION && x < best) best = x;
        }
    }
    return best;
}

/* Algorithm 2 for one gate of the extended model. dly: [k][2][2]. */
int o1x_process_cell(int type, const uint8_t *table, const int64_t *const *in_t,
                     const uint8_t *const *in_v, const int64_t *in_n, int k,
                     const int32_t *dly, o1_wave *out) {
    uint8_t current_signals[4];
    int64_t earliest_index[4];
    int64_t earliest_timestamp[4];
    int edge[4];
    for (int i = 0; i < k; i++) {
        current_signals[i] = O1_X;
        earliest_index[i] = 0;
        earliest_timestamp[i] = in_n[i] > 0 ? in_t[i][0] : O1_INF;
    }
    uint8_t previous_output = O1_X;
    for (;;) {
        int64_t t_earliest = O1_INF;
        for (int i = 0; i < k; i++)
            if (earliest_timestamp[i] < t_earliest) t_earliest = earliest_timestamp[i];
        if (t_earliest == O1_INF) break;
        for (int i = 0; i < k; i++) {
            edge[i] = -1;
            int64_t j = earliest_index[i];
            if (earliest_timestamp[i] == t_earliest) {
                edge[i] = edge_of(current_signals[i], in_v[i][j]);
                current_signals[i] = in_v[i][j];
                if (j + 1 == in_n[i]) {
                    earliest_timestamp[i] = O1_INF;
                } else {
                    earliest_index[i] = j + 1;
                    earliest_timestamp[i] = in_t[i][j + 1];
                }
            }
        }
        uint8_t new_output;
        if (table) {
            int packed = 0;
            for (int i = 0; i < k; i++) packed |= current_signals[i] << (2 * i);
            new_output = table[packed];
        } else {
            new_output = o1_calculate_signal(type, current_signals);
        }
        if (new_output != previous_output) {
            int64_t del = O1_INF;
            for (int i = 0; i < k; i++) {
                if (edge[i] < 0) continue;
                int64_t d = edge_out_delay(dly + 4 * i, edge[i], new_output);
                if (d < del) del = d;
            }
            if (del != O1_INF && add_signal_change(out, new_output, t_earliest + del)) return -1;
        }
        previous_output = new_output;
    }
    return 0;
}

/* Whole netlist under the extended model: dly[P][2][2] per pin; udp[n_udp][256].
 * Same return convention as o1_simulate. */
o1_result *o1x_simulate(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                        const int64_t *pin_net, const int32_t *dly, int n_udp, const uint8_t *udp,
                        const int64_t *src_off, const int64_t *src_t, const uint8_t *src_v,
                        int *status) {
    *status = 0;
    for (int64_t g = 0; g < G; g++) {
        int64_t k = pin_off[g + 1] - pin_off[g];
        int ok = type[g] < T_COUNT ? k == arity_of(type[g]) : (type[g] - T_COUNT < n_udp && k >= 1 && k <= 4);
        if (!ok) { *status = -3; return NULL; }
        for (int64_t p = pin_off[g]; p < pin_off[g + 1]; p++)
            if (pin_net[p] < 0 || pin_net[p] >= S + G || pin_net[p] == S + g) { *status = -3; return NULL; }
    }
    o1_result *r = (o1_result *)calloc(1, sizeof(o1_result));
    int64_t *order = (int64_t *)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
    if (!r || !order) { free(r); free(order); *status = -1; return NULL; }
    r->S = S;
    r->G = G;
    r->gate_out = (o1_wave *)calloc((size_t)(G ? G : 1), sizeof(o1_wave));
    if (!r->gate_out) { free(order); free(r); *status = -1; return NULL; }
    int rc = topological_order(S, G, pin_off, pin_net, order);
    if (rc) { free(order); o1_free(r); *status = rc; return NULL; }
    for (int64_t idx = 0; idx < G; idx++) {
        int64_t g = order[idx];
        const int64_t *in_t[4];
        const uint8_t *in_v[4];
        int64_t in_n[4];
        int k = (int)(pin_off[g + 1] - pin_off[g]);
        for (int i = 0; i < k; i++) {
            int64_t net = pin_net[pin_off[g] + i];
            if (net < S) {
                in_t[i] = src_t + src_off[net];
                in_v[i] = src_v + src_off[net];
                in_n[i] = src_off[net + 1] - src_off[net];
            } else {
                o1_wave *w = &r->gate_out[net - S];
                in_t[i] = w->t;
                in_v[i] = w->v;
                in_n[i] = w->n;
            }
        }
        const uint8_t *table = type[g] >= T_COUNT ? udp + 256 * (size_t)(type[g] - T_COUNT) : NULL;
        if (o1x_process_cell(type[g], table, in_t, in_v, in_n, k, dly + 4 * pin_off[g], &r->gate_out[g])) {
            free(order); o1_free(r); *status = -1; return NULL;
        }
    }
    free(order);
    return r;
}
