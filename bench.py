#!/usr/bin/env python3
"""Throughput of the re-simulation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--seed S] [--headline-only]
                    [--no-cpu-baseline] [--served-full] ...

A step is one whole job of the industrial-shaped workload: every level of a
10M-gate netlist (8,192 PIs + 50,000 pseudo-PIs, 150 levels, fan-in 1-4,
power-law fanout up to 5,000, 1-200 ps rise/fall delays, 200 transitions per
source) simulated from stimuli already resident in HBM, through the C ABI
(sim_run_device), on one stream, with jobs enqueued two deep so host enqueue
overlaps device work. The evaluate launches are bracketed with HIP events on
that stream. The same measurement on the 1M-gate mid-size workload, the
dependency-driven schedule, latency of the 1,000-gate job, batching, serving,
time windows and the end-to-end rate follow as nested sections. Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0
CU_COUNT, CLOCK_HZ = 256, 2.4e9   # MI355X: 256 CUs at 2.4 GHz; one wave64 VALU instruction per CU per cycle
ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(ROOT, "profiles")
# device code: the kernels and the per-gate evaluation they share
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2304_13398_amd", "csrc", f)
                  for f in ("kernels.hip", "eval_core.h", "gsim_internal.h")]

# Committed counter profiles of each workload's dominant evaluate kernel; a
# figure is used only while the kernel source hash recorded there matches.
PROFILE_FILES = {
    "industrial": ("eval_wave256_industrial_hbm_traffic.txt", "eval_wave256_industrial_sq_counters.txt"),
    "mid": ("eval_wave64_mid_hbm_traffic.txt", "eval_wave64_mid_sq_counters.txt"),
}


def kernel_source_hash():
    try:
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(f, "rb").read())
        return h.hexdigest()[:16]
    except OSError:
        return None


def profile_value(fname, key):
    """A figure from a committed profile summary ("key: value" or "key value"
    line), or None if the file is missing or was taken on other kernel source."""
    try:
        text = open(os.path.join(PROFILES, fname)).read()
    except OSError:
        return None
    h = kernel_source_hash()
    if not h or f"sha256 prefix: {h}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(key):
            rest = line[len(key):].lstrip(": \t").split()
            if rest:
                return float(rest[0])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed industrial steps (for profiler runs)")
    ap.add_argument("--served-only", action="store_true", help="only the served section")
    ap.add_argument("--batched-only", action="store_true", help="only the batched section")
    ap.add_argument("--skewed-only", action="store_true", help="only the skewed-activity section")
    ap.add_argument("--mid-only", action="store_true",
                    help="only the timed mid-size steps (for profiler runs)")
    ap.add_argument("--eval-form", choices=("segmented", "merged"), default="merged",
                    help="data-parallel form of the wavefront-per-gate kernel (same results)")
    ap.add_argument("--schedule", choices=("levels", "dataflow", "levelsync"), default="levels",
                    help="schedule of the --mid-only job")
    ap.add_argument("--df-tickets", type=int, default=0,
                    help="dependency-driven schedule: queue slots claimed per atomic (0 = automatic)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mid", action="store_true", help="skip the 1M-gate mid-size sections")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny-configuration latency")
    ap.add_argument("--no-e2e", action="store_true",
                    help="skip the host-to-host run of the mid job (all waveforms fetched)")
    ap.add_argument("--no-windows", action="store_true",
                    help="skip the exact time-window chunking measurement")
    ap.add_argument("--no-skewed", action="store_true",
                    help="skip the uneven-source-activity (WCV) runs")
    ap.add_argument("--no-dataflow", action="store_true",
                    help="skip the one-launch schedules (dependency-driven, level barriers)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched section (64 stimulus sets over the 1M-gate netlist)")
    ap.add_argument("--batched-sets", type=int, default=64)
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served section (Poisson requests over 8 resident netlists)")
    ap.add_argument("--served-rates", default="10,25,50,100,250,500",
                    help="request rates (jobs/s), comma separated")
    ap.add_argument("--served-seconds", type=float, default=8.0,
                    help="arrival span per rate (jobs = rate x span, at least 100 and at most 1,000)")
    ap.add_argument("--served-full", action="store_true",
                    help="1,000 requests at every rate (about six minutes of arrivals)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="instead of the workload, time a plain device-to-device copy of BYTES "
                         "(the practical HBM ceiling, and the reference for the profiler's "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---- bytes the method must move ---------------------------------------------

def b_min_bytes(nl, lengths):
    """Bytes a job must move at least: every waveform that some gate reads is
    read once and every output written once, at 9 bytes a transition (int64
    time + int8 value, the paper's element), plus each gate's output offset
    (8 B) and the netlist (type and pin offset, 1 + 8 B per gate; pin net and
    rise/fall, 4 + 8 B per pin)."""
    read = np.zeros(nl.S + nl.G, dtype=bool)
    read[nl.pin_net] = True
    consumed = int(lengths[read].sum())
    n_out = int(lengths[nl.S:].sum())
    return 9 * consumed + 9 * n_out + 8 * nl.G + 9 * nl.G + 12 * nl.P


def b_pin_bytes(nl, lengths):
    """As b_min_bytes, but every pin reads its waveform itself (no reuse
    across a net's readers)."""
    pin_reads = int(lengths[nl.pin_net].sum())
    n_out = int(lengths[nl.S:].sum())
    return 9 * pin_reads + 9 * n_out + 8 * nl.G + 9 * nl.G + 12 * nl.P


def per_level_bytes(nl, lengths):
    """Bytes the level-by-level evaluate launches touch: per level, every net
    the level reads once (8 B a packed transition), every output written once,
    the 64-byte gate record and 16 B of offset and length per pin read and per
    output."""
    S = nl.S
    total = 0
    pin_gate = np.repeat(np.arange(nl.G), np.diff(nl.pin_off))
    order = np.argsort(nl.level[pin_gate], kind="stable")
    lv_pin = nl.level[pin_gate][order]
    nets_sorted = nl.pin_net[order]
    bounds = np.searchsorted(lv_pin, np.arange(1, int(nl.level.max()) + 2))
    gates_per_level = np.bincount(nl.level, minlength=int(nl.level.max()) + 1)
    out_len = np.bincount(nl.level, weights=lengths[S:S + nl.G].astype(np.float64),
                          minlength=int(nl.level.max()) + 1)
    for lv in range(1, int(nl.level.max()) + 1):
        nets = np.unique(nets_sorted[bounds[lv - 1]:bounds[lv]])
        pins = bounds[lv] - bounds[lv - 1]
        total += 8 * int(lengths[nets].sum()) + 8 * int(out_len[lv]) + 64 * int(gates_per_level[lv])
        total += 16 * int(pins) + 16 * int(gates_per_level[lv])
    return total


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ---- one workload, timed -------------------------------------------------------

def timed_job(G, sim, nl, st, steps, warmup, name, profile_key):
    """Jobs of one workload from stimuli resident in HBM, two deep on torch's
    current stream: wall time per job over `steps` after `warmup`, the device
    time of the evaluate launches (HIP events on that stream), and the
    roofline of the evaluate kernel against HBM bandwidth."""
    import torch
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
    stream = torch.cuda.current_stream()
    sim.set_option(G.OPT_KERNEL_TIMING, 1)
    h = sim.load_netlist(nl)
    info = sim.netlist_info(h)

    def launch(validate=False):
        return sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                              stream=stream.cuda_stream, validate=validate)

    stats = []

    def finish(j, keep):
        sim.wait(j)
        if keep:
            stats.append(sim.stats(j))
        sim.release(j)

    finish(launch(validate=True), False)  # also validates the stimuli once on the device copy
    for _ in range(max(0, warmup - 1)):
        finish(launch(), False)
    # two jobs in flight when two fit the HBM budget, else one at a time
    depth = 2
    a = launch()
    try:
        finish(launch(), False)
    except G.GsimError as e:
        if e.status != G.E_OOM:
            raise
        depth = 1
    finish(a, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prev = None
    for _ in range(steps):
        if depth == 1 and prev is not None:
            finish(prev, True)
            prev = None
        try:
            j = launch()
        except G.GsimError as e:
            # the pool could not place a second arena next to the first
            # (fragmentation): one at a time from here on
            if e.status != G.E_OOM or prev is None:
                raise
            depth = 1
            finish(prev, True)
            prev = None
            j = launch()
        if prev is not None:
            finish(prev, True)
        prev = j
    if prev is not None:
        finish(prev, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_out = stats[-1].n_out
    assert all(s.n_out == n_out for s in stats), "steps disagree on the output size"
    ms = wall / steps * 1000.0
    eval_ms = statistics.median(s.eval_ms for s in stats)
    launches = stats[-1].eval_launches
    say(f"{name}: {steps} steps in {wall:.3f}s, {ms:.2f} ms per job ({depth} in flight), evaluate "
        f"{eval_ms:.2f} ms over {launches} launches")

    # every net's length from one more run: the bytes the method must move
    j = launch()
    sim.wait(j)
    lengths = sim.lengths(j)
    pin_reads = sim.stats(j).pin_reads
    sim.release(j)
    sim.set_option(G.OPT_KERNEL_TIMING, 0)
    b_min = b_min_bytes(nl, lengths)
    avg_launch_s = eval_ms / launches / 1000.0
    achieved = b_min / launches / avg_launch_s / 1e9
    traffic_file, sq_file = PROFILE_FILES[profile_key]
    # per level: both delay windows' evaluate kernels, as the live timing brackets them
    traffic_per_launch = profile_value(traffic_file, "level_traffic_bytes")
    valu = profile_value(sq_file, "level_valu")
    roof = {
        "kernel": "eval_wave_kernel (one wavefront per gate; per level, the 64 ps and 256 ps window launches "
                  "bracketed together by HIP events on the job's stream)",
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBPS,
        "traffic": (traffic_per_launch / avg_launch_s / 1e9) if traffic_per_launch else None,
        "traffic_bytes_per_launch": traffic_per_launch,
        "algorithmic_bytes_per_launch": b_min / launches,
        "algorithmic_bytes_per_output_transition": b_min / n_out,
        "output_transitions_per_launch": n_out / launches,
        "avg_launch_ms": eval_ms / launches,
        "launches_per_step": launches,
        "b_min_bytes_per_job": b_min,
        "b_pin_gbps": b_pin_bytes(nl, lengths) / launches / avg_launch_s / 1e9,
        "per_level_reads_gbps": per_level_bytes(nl, lengths) / launches / avg_launch_s / 1e9,
        "profiles": {"traffic": f"profiles/{traffic_file}", "sq": f"profiles/{sq_file}"},
    }
    if valu:
        # issue bound: the VALU stream's time at one wave64 instruction per CU per cycle
        busy = valu / (CU_COUNT * CLOCK_HZ) / avg_launch_s
        roof["alu"] = {"valu_instr_per_launch": valu, "issue_busy_frac": busy,
                       "lane_ops_per_s": valu * 64 / avg_launch_s,
                       "peak_lane_ops_per_s": CU_COUNT * 64 * CLOCK_HZ}
        roof["binds"] = "alu (VALU issue)" if busy > 0.8 else "neither fully (latency)"
    res = {"ms_per_step": ms, "value": n_out / (ms / 1000.0), "n_out": int(n_out), "jobs_in_flight": depth,
           "device_ms_per_step": statistics.median(s.device_ms for s in stats),
           "eval_ms_per_step": eval_ms, "pin_reads": int(pin_reads), "roofline": roof,
           "levels": info.levels}
    return h, d, res, lengths


def oracle_whole_job(O, nl, st, n_threads, single=True):
    """The oracle (plain C; each waveform freed after its last reader) on the
    whole job: output transitions and seconds level-parallel on n_threads, and
    on one thread. Both runs must give the same lengths and fingerprints."""
    t = time.perf_counter()
    ln_p, fp_p, _ = O.o1_simulate_fingerprints_parallel(nl, st, n_threads)
    par_s = time.perf_counter() - t
    n_o = int(ln_p.sum())
    single_s = None
    if single:
        t = time.perf_counter()
        ln_s, fp_s = O.o1_simulate_fingerprints(nl, st)
        single_s = time.perf_counter() - t
        assert np.array_equal(ln_s, ln_p) and np.array_equal(fp_s, fp_p), \
            "level-parallel oracle disagrees with the sequential one"
    return n_o, par_s, single_s


def copy_rate(nbytes, reps=5):
    """Read-plus-write GB/s of a plain device copy of nbytes (the practical
    HBM ceiling; both events on torch's current stream, where the copy runs)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    a.fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    return ms, 2 * nbytes / (ms / 1000.0) / 1e9


def copy_probe(nbytes, reps=5):
    ms, gbps = copy_rate(nbytes, reps)
    print(json.dumps({"copy_probe_bytes": nbytes, "ms_per_copy": ms,
                      "read_plus_write_gbps": gbps}), flush=True)
    return 0


def _gen_stimulus(args):
    from paper_2304_13398_amd import workloads as W
    S, n, window, seed = args
    return W.make_stimulus(S=S, n_per_src=n, window=window, seed=seed)


def pool_map(fn, items):
    """Map over CPU worker processes started fresh (spawn): this process holds
    the GPU, and forked children would inherit its runtime state."""
    import concurrent.futures
    import multiprocessing
    workers = max(1, min(16, len(os.sched_getaffinity(0)), len(items)))
    if workers == 1:
        return [fn(x) for x in items]
    with concurrent.futures.ProcessPoolExecutor(
            max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        return list(ex.map(fn, items))


# Unfinished steps the request loop lets the executor enqueue ahead of it (a
# request that arrives waits at most this many steps, well under a
# millisecond here, to join). Measured with 300 requests: at 100 jobs/s p50/p99
# 18/120 ms with two, 16/98 ms with eight; at 500 jobs/s 538/1626 and 338/1520.
SERVE_LOOKAHEAD = 8

# Unfinished steps the batched loop lets the executor enqueue ahead of it: with
# two, the host loop could not keep the device busy (1.01 s for the 64 sets);
# from eight on the device never waits (0.75 s).
BATCH_LOOKAHEAD = 8


def oracle_threads():
    """Host threads for the level-parallel oracle: the cores this process may
    use, at most 16 (the CPU share of one GPU)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def bench_end_to_end(G, sim, nl, h, st, reps=3):
    """The headline job from host stimuli to every net's waveform in host
    memory: stimulus upload, validation and the run (sim_run + sim_wait), then
    sim_fetch_waveforms of all S+G nets into host buffers allocated and
    touched beforehand. Best of ``reps``."""
    n = nl.S + nl.G
    off = np.zeros(n + 1, dtype=np.int64)
    best = None
    t_buf = v_buf = None
    for _ in range(reps):
        t0 = time.perf_counter()
        j = sim.run(h, st)
        sim.wait(j)
        t1 = time.perf_counter()
        sim._ck(sim.lib.sim_fetch_waveforms(sim.ctx, j, None, n, off.ctypes.data_as(G.ctypes.c_void_p),
                                            None, None, 0))
        total = int(off[-1])
        if t_buf is None or len(t_buf) < total:
            t_buf = np.zeros(max(total, 1), dtype=np.int64)
            v_buf = np.zeros(max(total, 1), dtype=np.uint8)
        t2 = time.perf_counter()
        sim._ck(sim.lib.sim_fetch_waveforms(sim.ctx, j, None, n, off.ctypes.data_as(G.ctypes.c_void_p),
                                            t_buf.ctypes.data_as(G.ctypes.c_void_p),
                                            v_buf.ctypes.data_as(G.ctypes.c_void_p), total))
        t3 = time.perf_counter()
        sim.release(j)
        r = (t1 - t0, t3 - t2, total)
        if best is None or r[0] + r[1] < best[0] + best[1]:
            best = r
    run_s, fetch_s, total = best
    n_out = total - st.n
    return {
        "workload": "the headline job, host stimuli to host waveforms of all nets",
        "upload_and_run_ms": run_s * 1e3,
        "fetch_all_ms": fetch_s * 1e3,
        "fetch_gbps": 9.0 * total / fetch_s / 1e9,
        "total_ms": (run_s + fetch_s) * 1e3,
        "transitions_per_s": n_out / (run_s + fetch_s),
        "runs": reps,
    }


def bench_tiny_latency(G, sim, seed, reps=200):
    """Latency of the tiny configuration (1,000 gates, 32 PIs, 20 levels, 100
    transitions per PI): one job at a time, stimuli resident in HBM (submit to
    completion), and from host stimuli to every gate output in host memory."""
    import torch
    from paper_2304_13398_amd import workloads as W
    nl, st = W.config1(seed=seed)
    h = sim.load_netlist(nl)
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
    stream = torch.cuda.current_stream()
    gates = np.arange(nl.S, nl.S + nl.G)
    resident, host = [], []
    for i in range(reps + 5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        j = sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                           stream=stream.cuda_stream)
        sim.wait(j)
        t1 = time.perf_counter()
        sim.release(j)
        t2 = time.perf_counter()
        j = sim.run(h, st)
        sim.wait(j)
        off, t, v = sim.fetch(j, gates)
        t3 = time.perf_counter()
        sim.release(j)
        if i >= 5:
            resident.append((t1 - t0) * 1e6)
            host.append((t3 - t2) * 1e6)
    n_out = int(off[-1])
    sim.unload_netlist(h)
    return {
        "workload": "tiny: 1,000 gates, 32 PIs, 20 levels, 10 gate types, 100 transitions per PI",
        "n_out": n_out,
        "resident_p50_us": float(np.percentile(resident, 50)),
        "resident_p99_us": float(np.percentile(resident, 99)),
        "host_to_host_p50_us": float(np.percentile(host, 50)),
        "host_to_host_p99_us": float(np.percentile(host, 99)),
        "runs": reps,
    }


def bench_skewed(G, sim, nl, h, seed, wcvs=(5.0, 20.0), steps=3):
    """Uneven source activity on the resident 1M-gate netlist: the same
    2,048,000 given transitions with per-source counts of coefficient of
    variation WCV (the paper's Eq. 5), under each schedule."""
    import torch
    from paper_2304_13398_amd import autotune
    from paper_2304_13398_amd import workloads as W
    out = {"workload": "1M-gate mid netlist, 2,048,000 given transitions, per-source counts "
                       "log-normal with the stated WCV", "runs": {}}
    tuner = autotune.Autotuner(sim, reps=1)
    for wcv in wcvs:
        st = W.make_stimulus_skewed(S=nl.S, mean_per_src=1000, wcv=wcv, window=1_000_000, seed=seed)
        dev = torch.device("cuda:0")
        d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
        stream = torch.cuda.current_stream()
        row = {}
        for name, sched in (("levels", 0), ("dataflow", 1), ("levelsync", 3)):
            sim.set_option(G.OPT_SCHEDULE, sched)
            times, n_out = [], 0
            for i in range(steps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                j = sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                                   stream=stream.cuda_stream)
                sim.wait(j)
                if i > 0:
                    times.append(time.perf_counter() - t0)
                n_out = sim.stats(j).n_out
                sim.release(j)
            ms = statistics.median(times) * 1000.0
            row[name] = {"ms_per_job": ms, "transitions_per_s": n_out / (ms / 1000.0), "n_out": int(n_out)}
        sim.set_option(G.OPT_SCHEDULE, 0)
        # the tuner's choice for this stimulus (its key includes the skew)
        c, tms = tuner.tune(nl, h, st)
        row["tuned_setting"], row["tuning_device_ms"] = autotune.setting_name(c), tms
        tuner.clear(h)
        n = np.diff(st.off)
        row["wcv_given"] = float(n.std() / n.mean())
        out["runs"][str(wcv)] = row
        print(f"[bench] skewed wcv {wcv}: levels {row['levels']['ms_per_job']:.1f} ms, "
              f"dataflow {row['dataflow']['ms_per_job']:.1f} ms, tuner chose {row['tuned_setting']}",
              file=sys.stderr, flush=True)
    return out


def bench_windows(G, sim, nl, h, st, n_out_whole, ms_whole, n_windows=4):
    """Exact time-window chunking of the mid job: device time and output
    volume of the windows (each with its halo) against the whole job; the
    windows' outputs inside their own ranges add up to the whole job's. Also
    wall time from host stimuli to finished jobs: the whole job, the windows
    one after another, and the windows submitted together (shared launches)."""
    from paper_2304_13398_amd import windows as WN
    H = WN.window_halo(nl)
    wins = WN.window_stimuli(nl, st, n_windows, halo=H)
    dev_ms, n_out = 0.0, 0
    for _, _, sub in wins:
        j = sim.run(h, sub)
        sim.wait(j)
        s = sim.stats(j)
        dev_ms += s.device_ms
        n_out += s.n_out
        sim.release(j)

    def whole():
        t0 = time.perf_counter()
        j = sim.run(h, st)
        sim.wait(j)
        sim.release(j)
        return time.perf_counter() - t0

    def one_by_one():
        t0 = time.perf_counter()
        for _, _, sub in wins:
            j = sim.run(h, sub)
            sim.wait(j)
            sim.release(j)
        return time.perf_counter() - t0

    def together():
        t0 = time.perf_counter()
        pending = [sim.submit(h, sub) for _, _, sub in wins]
        while pending:
            sim.drive(max_ahead=BATCH_LOOKAHEAD)
            for j in [j for j in pending if sim.done(j)]:
                sim.release(j)
                pending.remove(j)
        return time.perf_counter() - t0

    for f in (whole, one_by_one, together):  # untimed pass: staging allocation
        f()
    w_s, seq_s, tog_s = (min(f() for _ in range(2)) for f in (whole, one_by_one, together))
    return {"windows": len(wins), "halo_ps": H, "device_ms_sum": dev_ms,
            "device_ms_whole": ms_whole, "n_out_sum": int(n_out), "n_out_whole": int(n_out_whole),
            "overhead": dev_ms / ms_whole - 1.0,
            "wall_ms": {"whole_job": w_s * 1e3, "windows_one_by_one": seq_s * 1e3,
                        "windows_together": tog_s * 1e3},
            "wall_includes": "stimulus copy and upload from host memory, all levels, completion"}


def workload_stats(nl, lengths):
    """The paper's workload statistics (Table 2 columns and Eq. 5): coefficient
    of variation of the given (source) waveform lengths and of the generated
    ones, and the mean generated length per level."""
    src = lengths[:nl.S].astype(np.float64)
    gen = lengths[nl.S:nl.S + nl.G].astype(np.float64)
    cv = lambda a: float(a.std() / a.mean()) if len(a) and a.mean() > 0 else None
    per_level = [float(gen[nl.level == lv].mean()) for lv in range(1, int(nl.level.max()) + 1)]
    return {"wcv_given": cv(src), "wcv_generated": cv(gen),
            "given_transitions": int(src.sum()), "generated_transitions": int(gen.sum()),
            "mean_generated_length_per_level": [round(x, 1) for x in per_level]}


def W_loguniform(rng, lo, hi, n):
    from paper_2304_13398_amd import workloads as W
    return W.loguniform_int(rng, lo, hi, size=n)


# Unfinished steps the request loop lets the executor enqueue ahead of it (a
# request that arrives waits at most this many steps, well under a
# millisecond here, to join). Measured with 300 requests: at 100 jobs/s p50/p99
# 18/120 ms with two, 16/98 ms with eight; at 500 jobs/s 538/1626 and 338/1520.
SERVE_LOOKAHEAD = 8

# Unfinished steps the batched loop lets the executor enqueue ahead of it: with
# two, the host loop could not keep the device busy (1.01 s for the 64 sets);
# from eight on the device never waits (0.75 s).
BATCH_LOOKAHEAD = 8


def bench_batched(G, sim, nl, h, n_sets, seed):
    """Batched: n_sets stimulus sets over the resident netlist, per-set
    transitions per PI log-uniform in [50, 5000] (the sets the full-size
    parity test checks); all sets through the executor (shared launches,
    admitted as HBM allows, largest sets first) vs one set per launch chain.
    The schedule, evaluation form and lane threshold are autotuned on a
    sample set first."""
    from paper_2304_13398_amd import autotune
    from paper_2304_13398_amd import workloads as W
    t = time.perf_counter()
    set_args = W.config4_set_args(S=nl.S, n_sets=n_sets, seed=seed)
    sets = pool_map(_gen_stimulus, set_args)
    ns = np.array([a[1] for a in set_args])
    say(f"batched: {n_sets} sets generated in {time.perf_counter() - t:.1f}s "
        f"({sum(x.n for x in sets)} transitions)")
    tuner = autotune.Autotuner(sim, reps=1)
    median = sets[int(np.argsort(ns)[len(ns) // 2])]
    setting, tms = tuner.tune(nl, h, median)

    def one_per_launch():
        t0 = time.perf_counter()
        n_out = 0
        for st in sets:
            j = sim.run(h, st)
            sim.wait(j)
            n_out += sim.stats(j).n_out
            sim.release(j)
        return n_out, time.perf_counter() - t0

    diag = {}

    def batched():
        t0 = time.perf_counter()
        # largest first (first-fit decreasing): jobs are released as they finish
        pending = sim.run_batch(h, sorted(sets, key=lambda x: -x.n))
        diag["run_batch_return_s"] = time.perf_counter() - t0
        n_out, retries, drives = 0, 0, 0
        while pending:
            sim.drive(max_ahead=BATCH_LOOKAHEAD)  # admit sets as memory frees, advance all
            drives += 1
            for j in [j for j in pending if sim.done(j)]:
                st = sim.stats(j)
                n_out += st.n_out
                retries += st.retries
                sim.release(j)
                pending.remove(j)
        diag["retries"], diag["drive_calls"] = retries, drives
        return n_out, time.perf_counter() - t0

    # one untimed pass of each first: the first batch allocates page-locked
    # staging for all its sets at once (the one-per-launch loop reuses one set)
    one_per_launch()
    batched()
    n1, t1 = one_per_launch()
    n2, t2 = batched()
    assert n1 == n2, "batched and one-per-launch runs disagree on the output size"
    say(f"batched: one-per-launch {t1:.2f}s, batched {t2:.2f}s")
    return {
        "workload": f"{n_sets} stimulus sets over the 1M-gate netlist, transitions per PI "
                    f"log-uniform 50-5,000 (mean {float(ns.mean()):.0f})",
        "sets": n_sets, "n_in": int(sum(x.n for x in sets)), "n_out": int(n2),
        "batched_transitions_per_s": n2 / t2, "batched_s": t2,
        "one_per_launch_transitions_per_s": n1 / t1, "one_per_launch_s": t1,
        "speedup": t1 / t2,
        "tuned_setting": autotune.setting_name(setting), "tuning_device_ms": tms, "batched_diagnostics": diag,
        "lookahead_steps": BATCH_LOOKAHEAD,
        "includes": "stimulus upload (pageable H2D), all levels, per-set completion wait",
    }


def bench_served(G, sim, rates, seed, seconds, full):
    """Served: Poisson requests over 8 resident netlists (10k-2M gates), each
    request log-uniform 20-2,000 transitions per PI and asking for the
    waveforms of its netlist's deepest level plus every net's fingerprint;
    continuous batching vs one job at a time, on the same arrivals."""
    from paper_2304_13398_amd import autotune, serve
    t = time.perf_counter()
    nls = serve.served_netlists(seed=seed)
    rng = np.random.default_rng(seed + 5_000_011)
    items = []
    per = 6
    for k, nl in enumerate(nls):
        for i, n in enumerate(W_loguniform(rng, 20, 2000, per)):
            items.append((nl.S, int(n), 1_000_000, seed * 100_000 + k * 1000 + i))
    stims = pool_map(_gen_stimulus, items)
    pool = [stims[per * k:per * k + per] for k in range(len(nls))]
    hs = [sim.load_netlist(nl) for nl in nls]
    say(f"served: netlists and stimuli ready in {time.perf_counter() - t:.1f}s")
    # the request loop shares level steps across requests: the tuner chooses
    # among level-schedule settings only
    tuner = autotune.Autotuner(sim, reps=1, candidates=[c for c in autotune.CANDIDATES
                                                        if c[0] == G.SCHEDULE_LEVELS])
    tuned = []
    for nl, h, p in zip(nls, hs, pool):
        c, _ = tuner.tune(nl, h, sorted(p, key=lambda x: x.n)[len(p) // 2])
        tuned.append(autotune.setting_name(c))
        big = max(p, key=lambda x: x.n)
        j = sim.run(h, big)          # learn the arena use of the largest request
        sim.wait(j)
        sim.release(j)
    out = {"workload": "8 resident netlists of 10k-2M gates (mid-size generator, 60 levels); "
                       "requests uniform over netlists, 20-2,000 transitions per PI (log-uniform), "
                       "Poisson arrivals; each request fetches its deepest level's waveforms and "
                       "every net's fingerprint",
           "tuned_settings": tuned, "rates": {}}
    for rate in rates:
        n_jobs = 1000 if full else int(min(1000, max(100, rate * seconds)))
        reqs = serve.served_workload(n_jobs, rate, nls, pool, seed=seed + int(rate))
        rc, mc = serve.serve_continuous(sim, hs, reqs, max_ahead=SERVE_LOOKAHEAD,
                                        progress=lambda m: say(f"served rate {rate} continuous: {m}"))
        rs, ms = serve.serve_sequential(sim, hs, reqs,
                                        progress=lambda m: say(f"served rate {rate} sequential: {m}"))
        c, s = serve.summarize(rc, mc), serve.summarize(rs, ms)
        out["rates"][str(rate)] = {"jobs": n_jobs, "continuous": c, "sequential": s}
        say(f"served rate {rate} ({n_jobs} jobs): continuous p50/p99 {c['p50_ms']:.1f}/{c['p99_ms']:.1f} ms, "
            f"sequential {s['p50_ms']:.1f}/{s['p99_ms']:.1f} ms")
    for h in hs:
        sim.unload_netlist(h)
    return out


def eq6_speedups(per):
    """GPU over oracle per configuration (the paper's Eq. 6 speedup, here as a
    ratio of output-transition rates on the same work) and their geometric
    mean, against the level-parallel and the single-thread oracle."""
    for v in per.values():
        v["speedup"] = v["gpu_transitions_per_s"] / v["oracle_parallel_per_s"]
        if v.get("oracle_single_per_s"):
            v["speedup_single_thread"] = v["gpu_transitions_per_s"] / v["oracle_single_per_s"]
            # the faster CPU form (threads cost more than they give on a tiny job)
            v["speedup_best_cpu"] = min(v["speedup"], v["speedup_single_thread"])
        else:
            v["speedup_best_cpu"] = v["speedup"]
    g = lambda key: float(np.exp(np.mean([np.log(v[key]) for v in per.values() if key in v])))
    return {"per_config": per, "geomean_speedup_best_cpu": g("speedup_best_cpu"),
            "geomean_speedup": g("speedup")}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path (one job splits across GPUs by time windows, each window a "
              "single-GPU job).", file=sys.stderr, flush=True)
        return 2
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    import torch
    from paper_2304_13398_amd import gsim as G
    from paper_2304_13398_amd import workloads as W
    sim = G.Sim(0)
    sim.set_option(G.OPT_EVAL_FORM, G.FORM_SEGMENTED if args.eval_form == "segmented" else G.FORM_MERGED)
    n_threads = oracle_threads()
    eq6 = {}

    if args.served_only:
        rates = [float(x) for x in args.served_rates.split(",") if x]
        print(json.dumps({"served": bench_served(G, sim, rates, args.seed, args.served_seconds,
                                                 args.served_full)}), flush=True)
        sim.close()
        return 0
    if args.skewed_only:
        sim.set_option(G.OPT_DF_TICKETS, args.df_tickets)
        nl = W.config2_netlist(seed=args.seed)
        h = sim.load_netlist(nl)
        print(json.dumps({"skewed": bench_skewed(G, sim, nl, h, args.seed)}), flush=True)
        sim.close()
        return 0
    if args.batched_only:
        nl = W.config2_netlist(seed=args.seed)
        h = sim.load_netlist(nl)
        print(json.dumps({"batched": bench_batched(G, sim, nl, h, args.batched_sets, args.seed)}), flush=True)
        sim.close()
        return 0
    if args.mid_only:
        if args.schedule == "dataflow":
            sim.set_option(G.OPT_SCHEDULE, 1)
            sim.set_option(G.OPT_DF_TICKETS, args.df_tickets)
        elif args.schedule == "levelsync":
            sim.set_option(G.OPT_SCHEDULE, 3)
        nl, st = W.config2(seed=args.seed)
        h, d, res, _ = timed_job(G, sim, nl, st, args.steps, args.warmup, "mid", "mid")
        print(json.dumps({"mid": res}), flush=True)
        sim.close()
        return 0

    # ---- headline: the industrial-shaped job --------------------------------
    t = time.perf_counter()
    nl, st = W.config3(seed=args.seed)
    say(f"industrial workload generated in {time.perf_counter() - t:.1f}s: G={nl.G} S={nl.S} "
        f"P={nl.P} N_in={st.n}")
    h, d, res, lengths = timed_job(G, sim, nl, st, args.steps, args.warmup, "industrial", "industrial")
    out = {
        "metric": "output transitions/sec",
        "value": res["value"],
        "unit": "transitions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "industrial-shaped re-simulation: 10M-gate levelled random DAG, 8,192 PIs + "
                        "50,000 pseudo-PIs, 150 levels, fan-in 1-4, power-law fanout (alpha 2.2, "
                        "cap 5,000), rise/fall 1-200 ps, 200 transitions per source over [0, 1e6] ps, "
                        "values 0/1/X/Z p=.49/.49/.01/.01",
            "seed": args.seed, "gates": nl.G, "sources": nl.S, "pins": nl.P,
            "levels": res["levels"], "n_in": st.n, "n_out": res["n_out"],
            "parallelism": "single GPU",
        },
        "device_ms_per_step": res["device_ms_per_step"],
        "eval_ms_per_step": res["eval_ms_per_step"],
        "roofline": res["roofline"],
    }
    if args.headline_only:
        print(json.dumps(out), flush=True)
        sim.close()
        return 0
    _, copy_gbps = copy_rate(1 << 30)
    out["roofline"]["copy_ceiling_gbps"] = copy_gbps
    out["roofline"]["frac_of_copy_ceiling"] = out["roofline"]["achieved"] / copy_gbps
    out["workload_stats"] = workload_stats(nl, lengths)
    sim.unload_netlist(h)
    del d
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        n_o, par_s, _ = oracle_whole_job(O, nl, st, n_threads, single=False)
        assert n_o == res["n_out"], "the oracle's output size differs from the GPU's"
        # one thread on a closed prefix of the netlist (levels 1-15, about 20 s)
        n_gates = int(np.searchsorted(nl.level, 15, side="right"))
        t1 = time.perf_counter()
        ln_s, _ = O.o1_simulate_fingerprints(nl.prefix(n_gates), st)
        single_s = time.perf_counter() - t1
        single_rate = int(ln_s.sum()) / single_s
        out["cpu_baseline"] = {
            "value": n_o / par_s,
            "unit": "transitions/s",
            "cores": n_threads,
            "kind": "oracle",
            "sample": f"the whole job (oracle O1 in plain C, each level's gates split over {n_threads} "
                      f"threads; {n_o} output transitions in {par_s:.1f}s); one thread on levels 1-15 "
                      f"({n_gates} gates, {int(ln_s.sum())} output transitions in {single_s:.1f}s)",
            "single_thread_value": single_rate,
            "cpu_model": cpu_model(),
            "gpu_speedup": res["value"] / (n_o / par_s),
            "gpu_speedup_single_thread": res["value"] / single_rate,
        }
        eq6["industrial"] = {"gpu_transitions_per_s": res["value"], "oracle_parallel_per_s": n_o / par_s,
                             "oracle_single_per_s": single_rate, "oracle_single_sample": "levels 1-15"}
        say(f"oracle on the whole industrial job: {par_s:.1f}s on {n_threads} threads; one thread "
            f"{single_rate:.3g} transitions/s on levels 1-15")
    del nl, st, lengths

    # ---- the 1M-gate mid-size job and the sections built on it -----------------
    if not args.no_mid:
        nl, st = W.config2(seed=args.seed)
        h, d, mid, m_lengths = timed_job(G, sim, nl, st, min(args.steps, 10), args.warmup, "mid", "mid")
        mid["workload"] = ("mid-size re-simulation: 1M-gate levelled random DAG, 2,048 PIs, 60 levels, "
                           "fan-in 1-4, power-law fanout (alpha 2.2, cap 1,000), rise/fall 1-50 ps, "
                           "1,000 transitions per PI over [0, 1e6] ps, values 0/1/X/Z p=.45/.45/.05/.05")
        mid["workload_stats"] = workload_stats(nl, m_lengths)
        out["mid"] = mid
        stream = torch.cuda.current_stream()

        def launch():
            return sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                                  stream=stream.cuda_stream)

        # the same jobs under the one-launch schedules
        for key, sched, desc in (
                ("dataflow", 1, "dependency-driven: one persistent launch per job, no level barrier"),
                ("levelsync", 3, "level barriers: one persistent launch per job, a device-wide "
                                 "barrier after each level")):
            if args.no_dataflow:
                break
            sim.set_option(G.OPT_SCHEDULE, sched)
            sim.set_option(G.OPT_KERNEL_TIMING, 1)
            j = launch()
            sim.wait(j)
            sim.release(j)
            torch.cuda.synchronize()
            steps = min(args.steps, 10)
            t0 = time.perf_counter()
            dstats = []
            for _ in range(steps):
                j = launch()
                sim.wait(j)
                dstats.append(sim.stats(j))
                sim.release(j)
            dwall = time.perf_counter() - t0
            sim.set_option(G.OPT_SCHEDULE, 0)
            sim.set_option(G.OPT_KERNEL_TIMING, 0)
            assert all(x.n_out == mid["n_out"] for x in dstats), f"{key} runs disagree"
            d_ms = dwall / steps * 1000.0
            d_eval = statistics.median(x.eval_ms for x in dstats)
            out[key] = {
                "workload": "the mid-size job", "schedule": desc,
                "ms_per_step": d_ms, "value": mid["n_out"] / (d_ms / 1000.0), "kernel_ms": d_eval,
                "b_min_gbps": mid["roofline"]["b_min_bytes_per_job"] / (d_eval / 1000.0) / 1e9,
                "vs_levels": mid["ms_per_step"] / d_ms,
            }
            say(f"{key}: {d_ms:.2f} ms per mid job (levels {mid['ms_per_step']:.2f})")
        if not args.no_cpu_baseline:
            from oracle import oracle as O
            n_o, par_s, _ = oracle_whole_job(O, nl, st, n_threads, single=False)
            assert n_o == mid["n_out"], "the oracle's output size differs from the GPU's"
            # one thread on a closed prefix of the netlist (levels 1-15)
            n_gates = int(np.searchsorted(nl.level, 15, side="right"))
            t1 = time.perf_counter()
            ln_s, _ = O.o1_simulate_fingerprints(nl.prefix(n_gates), st)
            single_s = time.perf_counter() - t1
            eq6["mid"] = {"gpu_transitions_per_s": mid["value"], "oracle_parallel_per_s": n_o / par_s,
                          "oracle_single_per_s": int(ln_s.sum()) / single_s,
                          "oracle_single_sample": "levels 1-15"}
            mid["cpu_oracle"] = {"whole_job_parallel_s": par_s, "threads": n_threads,
                                 "single_thread_levels_1_15_s": single_s}
        if not args.no_e2e:
            out["end_to_end"] = bench_end_to_end(G, sim, nl, h, st)
            say(f"end to end: {out['end_to_end']}")
        if not args.no_windows:
            out["time_windows"] = bench_windows(G, sim, nl, h, st, mid["n_out"], mid["device_ms_per_step"])
            say(f"time windows: {out['time_windows']}")
        if not args.no_skewed:
            out["skewed"] = bench_skewed(G, sim, nl, h, args.seed)
        if not args.no_batched:
            out["batched"] = bench_batched(G, sim, nl, h, args.batched_sets, args.seed)
        sim.unload_netlist(h)
        del d
    if not args.no_tiny:
        out["tiny_latency"] = bench_tiny_latency(G, sim, args.seed)
        if not args.no_dataflow:
            for key, sched in (("tiny_latency_dataflow", 1), ("tiny_latency_levelsync", 3)):
                sim.set_option(G.OPT_SCHEDULE, sched)
                out[key] = bench_tiny_latency(G, sim, args.seed)
            sim.set_option(G.OPT_SCHEDULE, 0)
        if not args.no_cpu_baseline:
            from oracle import oracle as O
            nl1, st1 = W.config1(seed=args.seed)
            n_o, par_s, single_s = oracle_whole_job(O, nl1, st1, n_threads)
            key = min((k for k in ("tiny_latency", "tiny_latency_dataflow", "tiny_latency_levelsync") if k in out),
                      key=lambda k: out[k]["resident_p50_us"])
            gpu_s = out[key]["resident_p50_us"] / 1e6
            eq6["tiny"] = {"gpu_transitions_per_s": n_o / gpu_s, "oracle_parallel_per_s": n_o / par_s,
                           "oracle_single_per_s": n_o / single_s, "gpu_schedule": key}
    if not args.no_served:
        rates = [float(x) for x in args.served_rates.split(",") if x]
        out["served"] = bench_served(G, sim, rates, args.seed, args.served_seconds, args.served_full)
    if eq6 and "cpu_baseline" in out:
        out["cpu_baseline"].update(eq6_speedups(eq6))
    print(json.dumps(out), flush=True)
    sim.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
