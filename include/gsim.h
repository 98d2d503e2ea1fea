/*
 * gsim.h -- C ABI of the MI355X timing-aware 4-value gate-level re-simulator.
 *
 * The library computes, for a combinational netlist of basic gates with
 * per-pin rise/fall delays and the 0/1/X/Z waveforms of its source nets, the
 * waveform of every gate output (the re-simulation objective of Section 2.1 of
 * "Acceleration for Timing-Aware Gate-Level Logic Simulation with One-Pass GPU
 * Parallelism"). Per gate it merges the input waveforms in time, evaluates the
 * 4-value gate function (Section 2.2, Table 1; Z is read as X), takes the
 * minimum delay over the pins that changed (Section 2.3, Fig. 2; Section 3.2),
 * applies the "glitch eaten" denial of Eq. 1 and drops redundant transitions
 * (Fig. 3) -- the output-waveform procedure of Algorithm 2. All levels of a
 * job run on the GPU after one host-to-device transfer of the stimuli, and
 * results stay in device memory until fetched (Section 3, one-pass
 * parallelism).
 *
 * Conventions
 *  - Values are uint8 codes: 0, 1, X = 2, Z = 3. Gate outputs are never Z.
 *  - Times are int64 picoseconds in [0, 2^62); delays are int32 picoseconds
 *    >= 0. Times are not clipped to a window.
 *  - Nets [0, S) are sources (primary and pseudo-primary inputs); gate g
 *    (0 <= g < G, in the caller's order) drives net S + g.
 *  - A waveform is a list of (time, value) transitions with strictly
 *    increasing times, no two equal consecutive values, and a first value
 *    other than X: every net is X before its first transition.
 *  - Delay model: a transition of the output to 1 uses the triggering pin's
 *    rise delay, to 0 its fall delay, to X the smaller of the two; with
 *    several pins changing at the same time the minimum over those pins wins.
 *
 * Errors: every call returns a gsim_status and never throws. On error no
 * partial result is visible and sim_last_error() describes the failure.
 * Ownership: every caller array is read (or copied) during the call and stays
 * the caller's; device netlists belong to the context until unloaded; a job's
 * results belong to the context until sim_release_job().
 * Thread safety: one context may be used from one host thread at a time.
 */
#ifndef GSIM_H
#define GSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsim_ctx_s *gsim_ctx;
typedef int64_t gsim_netlist; /* handle, > 0 */
typedef int64_t gsim_job;     /* handle, > 0 */

typedef enum {
    GSIM_OK = 0,
    GSIM_E_ARG = -1,       /* bad argument: null pointer, bad size, bad id, bad arity */
    GSIM_E_CYCLE = -2,     /* the gates do not form a DAG */
    GSIM_E_WAVEFORM = -3,  /* a source waveform breaks the waveform conventions */
    GSIM_E_OOM = -4,       /* device memory budget exhausted (no partial result) */
    GSIM_E_DEVICE = -5,    /* HIP runtime error or no usable device */
    GSIM_E_HANDLE = -6,    /* unknown or already released handle */
    GSIM_E_OVERFLOW = -7   /* a time plus the longest path delay would leave [0, 2^62) */
} gsim_status;

/* Gate types. Pin order in brackets. Table 1 gives AND, OR and XOR; NOT, BUF,
 * NAND, NOR, XNOR and the 3/4-input AND/OR follow from it; MUX2 (not in the
 * paper) selects d0 for s=0, d1 for s=1, and for an unknown select gives the
 * data value if d0 and d1 agree, X otherwise. */
enum gsim_gate_type {
    GSIM_BUF = 0,   /* [a] */
    GSIM_NOT = 1,   /* [a] */
    GSIM_AND2 = 2,  /* [a b] */
    GSIM_OR2 = 3,
    GSIM_NAND2 = 4,
    GSIM_NOR2 = 5,
    GSIM_XOR2 = 6,
    GSIM_XNOR2 = 7,
    GSIM_AND3 = 8,  /* [a b c] */
    GSIM_MUX2 = 9,  /* [d0 d1 s] */
    GSIM_AND4 = 10, /* [a b c d] */
    GSIM_OR4 = 11,
    GSIM_NUM_TYPES = 12
};

/* Tunables, set with sim_set_option() on a context; they apply to later runs. */
enum gsim_option {
    /* Output storage per job, in transitions; 0 = automatic (see sim_run).
     * A run that needs more ends with GSIM_E_OOM from sim_wait. */
    GSIM_OPT_ARENA_TRANSITIONS = 1,
    /* Evaluate-kernel choice for netlists loaded afterwards: 0 = automatic
     * (wavefront per gate; gates whose largest pin delay exceeds the wavefront
     * kernel's window go to the lane kernel), 1 = lane-per-gate kernel for
     * every gate. */
    GSIM_OPT_KERNEL = 2,
    /* 1 = bracket every step's evaluate launches with HIP events on the
     * executor's stream; sim_job_stats then reports their summed device time
     * over the steps the job took part in. */
    GSIM_OPT_KERNEL_TIMING = 4,
    /* Dynamic binning: a gate whose inputs hold fewer than this many
     * transitions in a run is evaluated by the lane-per-gate kernel instead of
     * the wavefront-per-gate kernel (0 = never). Picked by the autotuner. */
    GSIM_OPT_LANE_THRESHOLD = 5,
    /* Schedule of later jobs: 0 = level by level (one launch chain per level,
     * shared by every admitted job); 1 = dependency-driven (Section 3.3,
     * Algorithm 1): one persistent launch per job in which a gate starts as
     * soon as its last fan-in gate has finished, with no level barrier;
     * 2 = chosen per job: dependency-driven when the netlist has fewer than
     * 800 gates per level on average (launch overhead dominates the level
     * chain) or, for stimuli given in host memory, when the per-source
     * transition counts vary with a coefficient of variation (the paper's
     * workload WCV, Eq. 5) of at least 2.5; level by level otherwise;
     * 3 = level barriers in one launch: the level order of setting 0 for one
     * job, run by persistent wavefronts (a cooperative launch, every one
     * resident) that meet at a device-wide barrier after each level, so a
     * job costs one launch instead of a chain per level; each such launch
     * waits for the context's previous one, on any stream. The barrier's
     * wait is bounded: a wait that does not end (another program holding
     * the device's wavefront slots, for instance) fails the job with
     * GSIM_E_DEVICE instead of hanging. Results are identical under every
     * setting. */
    GSIM_OPT_SCHEDULE = 6,
    /* Data-parallel form of the level schedule's wavefront-per-gate kernel
     * (Algorithm 2 per gate either way; identical results; the
     * dependency-driven kernel always uses the merged form): 1 = merged
     * positions (default),
     * the inputs merged in time across the wavefront and every step of the
     * procedure a wavefront scan; 0 = segmented, each lane runs the procedure
     * over a time segment of the gate's inputs and the lanes' candidates are
     * reconciled by Eq. 1 across lanes (measured 1.4x slower on MI355X). */
    GSIM_OPT_EVAL_FORM = 7,
    /* Dependency-driven schedule: queue slots a wavefront claims per atomic,
     * 1-16 (0 = automatic: 1 for netlists smaller than 16 gates per resident
     * wavefront, else 2). The claimed gates that are already ready run
     * between one pair of memory fences. More tickets cut the contended
     * atomics (uniform 1M-gate mid job: 2, 4, 8, 16 tickets 32.4, 25.0,
     * 46.2, 60.6 ms) but make light gates wait behind a heavy one claimed by
     * the same wavefront (sources with WCV 20: 85 ms with 2, 124 ms with 4);
     * the autotuner sets it per netlist. Passage: Algorithm 1's threads take
     * tasks from the shared queue (Section 3.3). */
    GSIM_OPT_DF_TICKETS = 8
};

/* Values of GSIM_OPT_SCHEDULE (see there). */
enum gsim_schedule {
    GSIM_SCHEDULE_LEVELS = 0,
    GSIM_SCHEDULE_DEPENDENCY = 1,
    GSIM_SCHEDULE_AUTO = 2,
    GSIM_SCHEDULE_LEVEL_BARRIERS = 3
};

/* ---- context ------------------------------------------------------------ */

/* Open a context on HIP device `device`. `hbm_budget_bytes` caps the device
 * memory the context allocates (0 = 90% of the device's free memory).
 * Passage: the device memory that holds every waveform of a job at once is
 * the premise of one-pass parallelism (Section 1, Motivation; Section 3). */
gsim_status sim_create(int device, uint64_t hbm_budget_bytes, gsim_ctx *out);
/* Release every netlist, job and buffer of the context. No passage of the
 * paper (plumbing). */
gsim_status sim_destroy(gsim_ctx ctx);
/* Message of the last failed call on `ctx` (or of the last failed
 * context-free call when ctx is NULL); owned by the library, valid until the
 * next call on the same context. Never NULL. No passage (plumbing). */
const char *sim_last_error(gsim_ctx ctx);
/* Set one of enum gsim_option on the context; each option cites its own
 * passage above. GSIM_E_ARG for an unknown option or a value out of range. */
gsim_status sim_set_option(gsim_ctx ctx, int option, int64_t value);

/* ---- netlists ------------------------------------------------------------ */

/* Validate, levelize and upload a netlist (host levelizer and CSR builder).
 * Passage: the netlist, module functions and delays given to the problem
 * (Section 2.1, Objective Statement), kept on the device for the whole run
 * with each output net stored once on its hyperedge (Section 3, the
 * figure on distributing an output waveform).
 *   S, G     number of source nets and gates (S >= 1, G >= 0)
 *   type     [G] gate types (enum gsim_gate_type)
 *   pin_off  [G+1] gate g's pins are pin_off[g] .. pin_off[g+1]-1; pin_off[0]=0,
 *            and each gate has exactly the arity of its type
 *   pin_net  [P] net read by each pin, in [0, S+G) and never the gate's own net;
 *            repeated nets on one gate are allowed
 *   rise_ps, fall_ps [P] per-pin delays, >= 0
 * Errors: GSIM_E_ARG (malformed), GSIM_E_CYCLE, GSIM_E_OOM, GSIM_E_DEVICE. */
gsim_status sim_load_netlist(gsim_ctx ctx, int64_t S, int64_t G, const uint8_t *type,
                             const int64_t *pin_off, const int64_t *pin_net,
                             const int32_t *rise_ps, const int32_t *fall_ps,
                             gsim_netlist *out);
/* A netlist under the extended cell model. The paper's delay matrix is indexed
 * by triggering pin, input edge and output value (Section 2.3; Section 3.2,
 * with inf for a pin unrelated to an output), and module functions may be
 * user-defined primitives (Section 3.3):
 *   dly[P][2][2]  per pin: [edge: 0 rise, 1 fall][output value: 0, 1], in ps,
 *                 >= 0, or GSIM_NO_RELATION for an unrelated pin. A pin change
 *                 rises if its new value is 1 or it leaves 0 for X/Z, falls if
 *                 its new value is 0 or it leaves 1 for X/Z; an X <-> Z change
 *                 takes the smaller delay of both edges; a new output value X
 *                 the smaller of the edge's delays to 0 and 1. A candidate
 *                 whose changed pins are all unrelated never appears.
 *   udp[n_udp][256] user-defined gate types 12 .. 11 + n_udp (any 1-4 pins):
 *                 the gate's value for packed pin values (pin i in bits 2i and
 *                 2i+1; entries 0, 1 or 2 = X). A gate is evaluated at its
 *                 input transitions only, from an X previous value.
 * Otherwise as sim_load_netlist (the arrays are copied; rise/fall unused). */
#define GSIM_NO_RELATION 2147483647
gsim_status sim_load_netlist_ext(gsim_ctx ctx, int64_t S, int64_t G, const uint8_t *type,
                                 const int64_t *pin_off, const int64_t *pin_net, const int32_t *dly,
                                 int32_t n_udp, const uint8_t *udp, gsim_netlist *out);

/* Free a netlist's device copy. GSIM_E_HANDLE if unknown; jobs of the
 * netlist must be released first (GSIM_E_ARG otherwise). No passage
 * (plumbing). */
gsim_status sim_unload_netlist(gsim_ctx ctx, gsim_netlist nl);

/* Per-netlist setting of GSIM_OPT_LANE_THRESHOLD, GSIM_OPT_SCHEDULE,
 * GSIM_OPT_EVAL_FORM or GSIM_OPT_DF_TICKETS (-1 = follow the context's
 * option); the other options
 * are per context. The autotuner sets them per netlist. Applies to jobs
 * submitted (schedule) or stepped (threshold, form) afterwards; a step shared
 * by jobs of several netlists takes the form of its first job's netlist.
 * Passage: a task's cost grows with its input waveforms' length (Section 5,
 * the WCV discussion), which the threshold bins on. */
gsim_status sim_set_netlist_option(gsim_ctx ctx, gsim_netlist nl, int option, int64_t value);

typedef struct {
    int64_t S, G, P;
    int32_t levels;          /* longest path length in gates (0 if G = 0) */
    int32_t max_delay_ps;    /* largest pin delay */
    int64_t max_path_delay;  /* largest sum of per-gate largest delays along a path */
    int64_t lane_gates;      /* gates routed to the lane-per-gate kernel */
} gsim_netlist_info;
/* Sizes of a loaded netlist. `levels` is the number of parallel layers a
 * level-by-level schedule needs (Section 4.1). */
gsim_status sim_netlist_info(gsim_ctx ctx, gsim_netlist nl, gsim_netlist_info *out);

/* Device memory of the context (no passage of the paper: plumbing). The
 * context carves every device buffer out of one slab of `budget_bytes`;
 * `live_bytes` is what netlists, jobs and fetch staging hold now, and
 * `largest_free_bytes` the largest buffer that can still be allocated.
 * `jobs_holding_storage` counts jobs that hold output storage (admitted and
 * not yet released). */
typedef struct {
    uint64_t budget_bytes;
    uint64_t live_bytes;
    uint64_t largest_free_bytes;
    int64_t jobs_holding_storage;
} gsim_memory_info;
gsim_status sim_memory_info(gsim_ctx ctx, gsim_memory_info *out);

/* ---- runs ----------------------------------------------------------------- */

/* Jobs run on an executor, one per HIP stream (NULL = the context's stream).
 * The executor advances its jobs one topological level per step, every
 * admitted job in the same kernel launches, with no host synchronisation
 * between levels (one host-to-device round trip per job, Section 3). A job is
 * admitted when its device storage fits the context's HBM budget; until then
 * it waits in the executor's queue. */

/* Queue one re-simulation of `nl` over host-resident source waveforms
 * (passage: the given waveforms of primary and pseudo-primary inputs,
 * Section 2.1; transferred to the device in one round, Section 1.4):
 *   src_off [S+1] source s's transitions are t/v[src_off[s] .. src_off[s+1]-1]
 *   t [N_in], v [N_in] with N_in = src_off[S]
 * The stimuli are validated and copied to the device (one transfer) before the
 * call returns; nothing runs yet. Output storage per job is
 * GSIM_OPT_ARENA_TRANSITIONS, or by default 1.5x the largest arena use per
 * input transition seen on this netlist (before any: twice the pin-read volume
 * of an input-length-preserving circuit), capped by the budget.
 * Errors: GSIM_E_ARG, GSIM_E_WAVEFORM, GSIM_E_OVERFLOW, GSIM_E_OOM, GSIM_E_HANDLE. */
gsim_status sim_submit(gsim_ctx ctx, gsim_netlist nl, const int64_t *src_off, const int64_t *t,
                       const uint8_t *v, void *hip_stream, gsim_job *out);

/* Passage as sim_submit (Section 2.1), with the given waveforms already in
 * device memory.
 * As sim_submit, but the three arrays are device pointers (e.g. owned by
 * PyTorch) holding N_in = src_off[S] transitions; the caller keeps them alive
 * and unmodified until the job completes. They are validated on the host only
 * if `validate` is non-zero (one device-to-host copy); otherwise the caller
 * guarantees the waveform conventions. Stimuli that break them give
 * unspecified waveforms, but every gate still ends: a gate whose evaluation
 * stops making progress (an input out of time order) makes sim_wait return
 * GSIM_E_DEVICE. */
gsim_status sim_submit_device(gsim_ctx ctx, gsim_netlist nl, const int64_t *d_src_off,
                              const int64_t *d_t, const uint8_t *d_v, int64_t n_in, int validate,
                              void *hip_stream, gsim_job *out);

/* sim_submit, then drive the executor until every level of the job is
 * enqueued; returns without waiting for the device. GSIM_E_OOM if the job
 * cannot be admitted because unreleased jobs hold the budget; on any error
 * the job is discarded and *out is 0. Passage: the
 * whole computation on the device with no host synchronisation in between
 * (Section 1.4, Algorithmic Flow; Section 4.1; Algorithm 2 per gate). */
gsim_status sim_run(gsim_ctx ctx, gsim_netlist nl, const int64_t *src_off, const int64_t *t,
                    const uint8_t *v, void *hip_stream, gsim_job *out);

/* sim_submit_device, then as sim_run (passage as sim_run). */
gsim_status sim_run_device(gsim_ctx ctx, gsim_netlist nl, const int64_t *d_src_off,
                           const int64_t *d_t, const uint8_t *d_v, int64_t n_in, int validate,
                           void *hip_stream, gsim_job *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the level
 * schedule of sim_run_device over buffers the caller supplies, allocating
 * nothing. Every step buffer (job state, step counters, work lists, level
 * descriptors) lives in a static device array of 32 MiB per GPU that the
 * library holds until the process ends; a netlist whose largest level needs
 * more than that (about 30 bytes per gate of its largest level, plus 96 bytes
 * per level) is refused with GSIM_E_ARG. Every call on a GPU shares that
 * array, so calls that overlap on one GPU (several streams, several host
 * threads) race and give undefined results; calls in one stream are ordered.
 * Asynchronous on `hip_stream` (NULL = the context's stream): returns after
 * enqueueing; the results are valid once the stream reaches them.
 *   d_src_off, d_t, d_v, n_in  the source waveforms in device memory, as
 *                   sim_run_device (not validated; the caller guarantees the
 *                   waveform conventions)
 *   d_off, d_len    [S+G] device int64: each net's offset into d_arena and
 *                   transition count, indexed by the library's net order
 *                   (sim_netlist_net_order gives the index of each net)
 *   d_arena         [arena_cap] device uint64: every waveform, sources first,
 *                   each transition packed as time << 2 | value
 *   d_result        [4] device int64: output transitions over all gates, 1 if
 *                   d_arena overflowed (results then incomplete: call again with
 *                   more), the device check code (0 = none), and the arena
 *                   transitions used
 * All buffers stay the caller's. Errors (nothing is enqueued): GSIM_E_ARG,
 * GSIM_E_HANDLE, GSIM_E_DEVICE. */
gsim_status sim_run_device_noalloc(gsim_ctx ctx, gsim_netlist nl, const int64_t *d_src_off,
                                   const int64_t *d_t, const uint8_t *d_v, int64_t n_in, int64_t *d_off,
                                   int64_t *d_len, uint64_t *d_arena, int64_t arena_cap, int64_t *d_result,
                                   void *hip_stream);

/* No passage (plumbing for sim_run_device_noalloc): net_index[S+G] receives,
 * for every net id of the caller (sources, then gate g's net S + g), its index
 * in the library's net order (gates are stored level by level). Host only. */
gsim_status sim_netlist_net_order(gsim_ctx ctx, gsim_netlist nl, int64_t *net_index);

/* No passage of the paper: several independent re-simulations of one
 * netlist share launches (the paper runs one task at a time).
 * Batched execution of `n_sets` stimulus sets over one resident netlist:
 * src_off[i], t[i], v[i] are set i's host arrays (as sim_submit); out[n_sets]
 * receives the job handles. All sets that fit the budget run together, level
 * by level, in shared launches; the others are admitted as released jobs free
 * memory (wait, fetch and release in submission order when the sets do not all
 * fit). Sets are admitted first fit in the order given: a caller that releases
 * jobs as they finish can pass the largest sets first, so they do not run
 * alone at the end. Every set is checked and copied before any job is made
 * (on up to 16 host threads); the caller's arrays may be freed on return.
 * Errors as sim_submit; on error no job is created. */
gsim_status sim_run_batch(gsim_ctx ctx, gsim_netlist nl, int32_t n_sets,
                          const int64_t *const *src_off, const int64_t *const *t,
                          const uint8_t *const *v, void *hip_stream, gsim_job *out);

/* No passage of the paper (serving: continuous batching across jobs).
 * One scheduling pass of the executor on `hip_stream`: admit queued jobs that
 * fit, enqueue the next level of every admitted job, then block until at most
 * `max_ahead` steps are unfinished on the device (0 = do not block; at most
 * 31). Reports the number of admitted jobs with levels left and of queued jobs.
 * Used by serving loops (continuous batching: jobs join at the next step). */
gsim_status sim_drive(gsim_ctx ctx, void *hip_stream, int32_t max_ahead, int32_t *n_active,
                      int32_t *n_queued);

/* No passage (plumbing for request loops).
 * Non-blocking: *done = 1 if the job's results are ready (or it failed). A job
 * found to have overflowed automatically sized storage is queued again with
 * twice the storage and reports 0. */
gsim_status sim_job_done(gsim_ctx ctx, gsim_job job, int32_t *done);

/* Passage: the end of the parallel computation, after which the results
 * are complete on the device (Section 1.4; Algorithm 1 ends when every
 * thread's cells are done).
 * Drive the job's executor until the job is enqueued, then block until its
 * device work is done. A job whose automatically sized output storage
 * overflowed is re-run with twice the storage (up to 6 times) before this
 * returns. GSIM_E_OOM if storage set with GSIM_OPT_ARENA_TRANSITIONS overflowed,
 * or storage could not be allocated (the job then holds no results). */
gsim_status sim_wait(gsim_ctx ctx, gsim_job job);

typedef struct {
    int64_t n_in;            /* source transitions */
    int64_t n_out;           /* output transitions over all gates */
    int64_t pin_reads;       /* sum over gates and pins of the read waveform's length */
    int64_t arena_used;      /* transitions of output storage reserved */
    int64_t arena_capacity;
    double device_ms;        /* device time of the level chain (HIP events) */
    double eval_ms;          /* with GSIM_OPT_KERNEL_TIMING: summed device time of the
                                evaluate launches, else 0 */
    int64_t eval_launches;   /* levels timed for eval_ms */
    int64_t retries;         /* automatic re-runs after an output-storage overflow */
    int64_t schedule;        /* the job's schedule: 0 level by level, 1 dependency-driven, 3 level barriers in one launch */
} gsim_job_stats;
/* Statistics of a finished job (waits for it). Passage: `pin_reads` is the
 * per-gate Eq. 2 bound summed over the job; n_out the output lengths. */
gsim_status sim_job_stats(gsim_ctx ctx, gsim_job job, gsim_job_stats *out);

/* Copy waveforms of a finished job to host memory. Passage: the results are
 * transferred back to the CPU as the output, the second and last transfer of
 * the one-pass flow (Section 1.4; Section 4.2).
 *   nets  [n] net ids to fetch (sources included); NULL = all S+G nets in id order
 *   out_off [n+1] receives offsets into out_t/out_v (out_off[0] = 0)
 *   out_t, out_v: capacity `cap` transitions; if out_t is NULL only out_off is
 *   filled (size query). GSIM_E_ARG if cap < out_off[n].
 * Buffers from hipHostMalloc (page-locked) are written by DMA directly; other
 * host memory is filled from page-locked staging by up to 16 host threads,
 * overlapped with the next batch's transfer. Returns when every byte is in
 * place; the caller keeps ownership of all arrays. */
gsim_status sim_fetch_waveforms(gsim_ctx ctx, gsim_job job, const int64_t *nets, int64_t n,
                                int64_t *out_off, int64_t *out_t, uint8_t *out_v, int64_t cap);

/* No passage of the paper (a check on results too large to copy).
 * Fingerprint of each requested net's waveform (nets as sim_fetch_waveforms;
 * NULL = all S+G nets in id order), computed on the device: with
 * mix(x) the SplitMix64 finaliser (x += 0x9E3779B97F4A7C15;
 * x = (x ^ x>>30) * 0xBF58476D1CE4E5B9; x = (x ^ x>>27) * 0x94D049BB133111EB;
 * x ^ x>>31) and key_i = time_i << 2 | value_i for the net's n transitions,
 *   out = mix(n) + sum_i mix(key_i ^ mix(i))   (mod 2^64).
 * out[n] is caller-allocated. Lets a caller compare large results without
 * copying them. */
gsim_status sim_fetch_hashes(gsim_ctx ctx, gsim_job job, const int64_t *nets, int64_t n,
                             uint64_t *out);

/* Free a job's device storage. No passage (plumbing). */
gsim_status sim_release_job(gsim_ctx ctx, gsim_job job);

/* ---- host-only helpers (no device needed) ----------------------------------- */

/* The levelizer of sim_load_netlist: level[g] = 1 + max level of its input
 * nets (sources are level 0). Passage: the parallel layers of a DAG netlist
 * (Section 4.1, the partitioning that Algorithm 1 avoids). Same validation and errors as sim_load_netlist
 * (ctx-free: read the message with sim_last_error(NULL)). */
gsim_status sim_levelize(int64_t S, int64_t G, const uint8_t *type, const int64_t *pin_off,
                         const int64_t *pin_net, const int32_t *rise_ps, const int32_t *fall_ps,
                         int32_t *level_out, int32_t *n_levels_out);

/* Check source waveforms against the conventions above and the time range
 * needed by a netlist whose longest path delay is `max_path_delay`.
 * Passage: a waveform as consecutive (value, time) transitions (Section 2.1)
 * with every signal X before its first one (Algorithm 2's initial values).
 * GSIM_E_WAVEFORM or GSIM_E_OVERFLOW with the first offending source named in
 * sim_last_error(NULL). */
gsim_status sim_validate_stimulus(int64_t S, const int64_t *src_off, const int64_t *t,
                                  const uint8_t *v, int64_t max_path_delay);

/* Library version string. No passage (plumbing). */
const char *sim_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GSIM_H */
