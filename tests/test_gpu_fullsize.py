"""Full-size configurations on the GPU, compared with the oracle gate by gate.

Every workload runs in the launch configuration bench.py times (stimuli
resident in HBM for single jobs; the batch and request loops as the bench
drives them). For every gate of every job the waveform's length and 64-bit
fingerprint (sim_fetch_hashes; the definition is in include/gsim.h) must
equal the oracle's, and for a 1% sample of gates the waveforms are compared
transition for transition. The oracle is O1 (Algorithm 2 per gate, Eq. 1,
Fig. 3 drop), run level by level on the host's cores in its memory-light mode
(each waveform freed after the level of its last reader), which CPU tests pin
byte for byte to the sequential oracle.

Besides the oracle, two properties that hold at any size are checked on a
sample of gates: the steady state (a waveform's last value is the
combinational value of the sources' last values) and the structural
invariants of a waveform against its inputs.
"""
import os
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import gsim as G
from paper_2304_13398_amd import workloads as W

pytestmark = pytest.mark.gpu

# host threads for the oracle (16: the host cores a GPU job is given)
THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
SAMPLE_FRACTION = 0.01


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = G.Sim(0)
    yield s
    s.close()


def run_resident(sim, nl, st):
    import torch
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
    stream = torch.cuda.current_stream()
    h = sim.load_netlist(nl)
    j = sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                       stream=stream.cuda_stream)
    sim.wait(j)
    torch.cuda.synchronize()
    return h, j, d


def sample_gates(G_, seed=7, fraction=SAMPLE_FRACTION):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(G_, size=max(1, int(G_ * fraction)), replace=False))


class OracleRun:
    """The oracle's lengths and fingerprints of every gate, and the whole
    waveforms of a sample of gates."""

    def __init__(self, nl, st, sample):
        t0 = time.perf_counter()
        self.len, self.fp, self.kept = O.o1_simulate_fingerprints_parallel(nl, st, THREADS, keep=sample)
        self.sample = sample
        self.seconds = time.perf_counter() - t0
        say(f"  oracle: {int(self.len.sum())} output transitions, {self.seconds:.1f} s on {THREADS} threads")


def first_difference(a, b):
    bad = np.nonzero(a != b)[0]
    return f"{len(bad)} gates differ, first gate {int(bad[0])}" if len(bad) else ""


def compare_job(sim, j, nl, want: OracleRun):
    """Every gate's length and fingerprint, and the sample element by element."""
    gates = np.arange(nl.S, nl.S + nl.G)
    got_len = sim.lengths(j, gates)
    assert np.array_equal(got_len, want.len), "lengths: " + first_difference(got_len, want.len)
    got_fp = sim.hashes(j, gates)
    assert np.array_equal(got_fp, want.fp), "fingerprints: " + first_difference(got_fp, want.fp)
    off, t, v = sim.fetch(j, nl.S + want.sample)
    k_off, k_t, k_v = want.kept
    assert np.array_equal(off, k_off), "sample offsets differ"
    assert np.array_equal(t, k_t) and np.array_equal(v, k_v), "sampled waveforms differ"
    say(f"  all {nl.G} gates equal (length + fingerprint); {len(want.sample)} gates "
        f"({int(off[-1])} transitions) equal element by element")


def gate_lut():
    lut = np.zeros((12, 256), dtype=np.uint8)
    for t in range(12):
        k = O.ARITY[t]
        for packed in range(256):
            lut[t, packed] = O.gate_eval(t, [(packed >> (2 * i)) & 3 for i in range(k)])
    return lut


def combinational_final(nl, st):
    """Combinational value of every gate for the sources' last values,
    evaluated level by level (the generator's levels)."""
    lut = gate_lut()
    n_src = np.diff(st.off)
    last = np.where(n_src > 0, st.v[np.maximum(st.off[1:] - 1, 0)], 2).astype(np.uint8)
    val = np.concatenate([last, np.full(nl.G + 1, 2, dtype=np.uint8)])
    zero_net = nl.S + nl.G  # reads as 0 in the padding of absent pins
    val[zero_net] = 0
    ar = np.diff(nl.pin_off)
    pins = np.full((nl.G, 4), zero_net, dtype=np.int64)
    for p in range(4):
        has = ar > p
        pins[has, p] = nl.pin_net[nl.pin_off[:-1][has] + p]
    for lv in range(1, int(nl.level.max()) + 1):
        g = np.nonzero(nl.level == lv)[0]
        packed = np.zeros(len(g), dtype=np.int64)
        for p in range(4):
            packed |= val[pins[g, p]].astype(np.int64) << (2 * p)
        val[nl.S + g] = lut[nl.type[g], packed]
    return val[nl.S:nl.S + nl.G]


def check_properties(sim, j, nl, st, n_sample=2000):
    """Steady state and structural invariants on sampled gates (no oracle)."""
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(nl.G, size=min(n_sample, nl.G), replace=False))
    want_final = combinational_final(nl, st)[sample]
    off, t, v = sim.fetch(j, nl.S + sample)
    sub_nets = np.unique(nl.pin_net[np.concatenate([np.arange(nl.pin_off[g], nl.pin_off[g + 1])
                                                    for g in sample.tolist()])])
    in_off, in_t, _ = sim.fetch(j, sub_nets)
    pos = {int(n): k for k, n in enumerate(sub_nets.tolist())}
    for i, g in enumerate(sample.tolist()):
        tt, vv = t[off[i]:off[i + 1]], v[off[i]:off[i + 1]]
        last = int(vv[-1]) if len(vv) else 2
        assert last == want_final[i], f"gate {g}: steady state {last} != {want_final[i]}"
        if len(tt) == 0:
            continue
        assert np.all(np.diff(tt) > 0) and vv[0] != 2 and np.all(vv[1:] != vv[:-1]) and np.all(vv < 3)
        ins = [in_t[in_off[pos[int(n)]]:in_off[pos[int(n)] + 1]]
               for n in nl.pin_net[nl.pin_off[g]:nl.pin_off[g + 1]]]
        distinct = np.unique(np.concatenate(ins))
        assert len(tt) <= len(distinct)
        ds = np.unique(np.concatenate([nl.rise[nl.pin_off[g]:nl.pin_off[g + 1]],
                                       nl.fall[nl.pin_off[g]:nl.pin_off[g + 1]]]))
        assert np.isin(tt[:, None] - ds[None, :], distinct).any(axis=1).all()
    say(f"  {len(sample)} sampled gates: steady state and invariants hold")


# ---- mid: 1M gates, 2,048 PIs, 60 levels, 1,000 transitions per PI ------------

@pytest.fixture(scope="module")
def mid():
    nl, st = W.config2()
    say(f"mid: G={nl.G} S={nl.S} N_in={st.n}")
    return nl, st, OracleRun(nl, st, sample_gates(nl.G))


@pytest.mark.parametrize("schedule", [0, 1, 3], ids=["levels", "dataflow", "levelsync"])
def test_mid_full_size(sim, mid, schedule):
    nl, st, want = mid
    sim.set_option(G.OPT_SCHEDULE, schedule)
    try:
        h, j, keep = run_resident(sim, nl, st)
        s = sim.stats(j)
        assert s.schedule == schedule
        say(f"  gpu ({['levels', 'dependency-driven', '', 'level barriers'][schedule]}): {s.n_out} output "
            f"transitions, {s.device_ms:.1f} ms device")
        compare_job(sim, j, nl, want)
        if schedule == 0:
            check_properties(sim, j, nl, st)
        sim.release(j)
        sim.unload_netlist(h)
    finally:
        sim.set_option(G.OPT_SCHEDULE, 0)


# ---- industrial-shaped: 10M gates, 58,192 sources, 150 levels, 1-200 ps -------

def test_industrial_full_size(sim):
    nl, st = W.config3()
    say(f"industrial: G={nl.G} S={nl.S} N_in={st.n}")
    h, j, keep = run_resident(sim, nl, st)
    s = sim.stats(j)
    say(f"  gpu: {s.n_out} output transitions, {s.device_ms:.1f} ms device")
    want = OracleRun(nl, st, sample_gates(nl.G))
    compare_job(sim, j, nl, want)
    check_properties(sim, j, nl, st)
    sim.release(j)
    sim.unload_netlist(h)


# ---- batched: 64 stimulus sets over the resident 1M-gate netlist ---------------

BATCH_GROUPS = 4


@pytest.fixture(scope="module")
def batched(sim):
    """All 64 sets through the batch path as the bench drives it (largest set
    first, eight steps ahead, each set released as it finishes); the GPU's
    lengths and fingerprints of every gate of every set."""
    nl = W.config2_netlist()
    sets = W.config4_sets(S=nl.S)
    h = sim.load_netlist(nl)
    order = sorted(range(len(sets)), key=lambda i: -sets[i].n)
    jobs = sim.run_batch(h, [sets[i] for i in order])
    set_of = dict(zip(jobs, order))
    gates = np.arange(nl.S, nl.S + nl.G)
    got = {}
    pending = list(jobs)
    t0 = time.perf_counter()
    while pending:
        sim.drive(max_ahead=8)
        for j in [j for j in pending if sim.done(j)]:
            sim.wait(j)
            got[set_of[j]] = (sim.lengths(j, gates), sim.hashes(j, gates), sim.stats(j).n_out)
            sim.release(j)
            pending.remove(j)
    say(f"batched: {len(sets)} sets over G={nl.G}, {sum(x.n for x in sets)} given transitions, "
        f"{sum(g[2] for g in got.values())} output transitions, {time.perf_counter() - t0:.1f} s")
    sim.unload_netlist(h)
    return nl, sets, got


@pytest.mark.parametrize("group", range(BATCH_GROUPS))
def test_batched_sets_full_size(batched, group):
    nl, sets, got = batched
    ids = list(range(group, len(sets), BATCH_GROUPS))
    t0 = time.perf_counter()
    for i in ids:
        ln, fp = O.o1_simulate_fingerprints_parallel(nl, sets[i], THREADS)[:2]
        g_len, g_fp, _ = got[i]
        assert np.array_equal(g_len, ln), f"set {i} lengths: " + first_difference(g_len, ln)
        assert np.array_equal(g_fp, fp), f"set {i} fingerprints: " + first_difference(g_fp, fp)
        say(f"  set {i}: {sets[i].n} given, {int(ln.sum())} output transitions, every gate equal")
    say(f"  sets {ids}: every gate equal ({time.perf_counter() - t0:.1f} s of oracle)")


# ---- served: requests over the 8 resident netlists of 10k-2M gates ------------

def test_served_full_size_netlists(sim):
    """Requests over the full-size served netlists (10k to 2M gates), several
    on the 2M-gate one, arriving together so that they share steps
    (continuous batching); then the same requests one at a time. Every
    request's fingerprints of all nets equal the oracle's for that request
    alone."""
    from paper_2304_13398_amd import serve
    from tests import net_hash
    nls = serve.served_netlists(scale=1.0, seed=1)
    pool = serve.make_stim_pool(nls, per_netlist=2, seed=3)
    hs = [sim.load_netlist(nl) for nl in nls]
    reqs = serve.served_workload(12, 500.0, nls, pool, seed=5)
    big = len(nls) - 1
    reqs += [serve.Request(reqs[-1].arrival + 0.001 * (k + 1), big, pool[big][k], serve.observed_outputs(nls[big]))
             for k in range(2)]
    say(f"served: {len(reqs)} requests, netlists {sorted(set(r.netlist for r in reqs))} "
        f"(sizes {[nl.G for nl in nls]})")
    want = {}
    t0 = time.perf_counter()
    for r in reqs:
        key = id(r.stim)
        if key not in want:
            nl = nls[r.netlist]
            ln, fp = O.o1_simulate_fingerprints_parallel(nl, r.stim, THREADS)[:2]
            want[key] = (np.concatenate([net_hash.fingerprints(r.stim.off, r.stim.t, r.stim.v), fp]),
                         int(ln.sum()))
    say(f"  oracle: {len(want)} distinct requests, {time.perf_counter() - t0:.1f} s")
    for loop in (serve.serve_continuous, serve.serve_sequential):
        res, span = loop(sim, hs, reqs)
        assert len(res) == len(reqs)
        for x in res:
            fp, n_out = want[id(x.request.stim)]
            assert x.n_out == n_out, loop.__name__
            assert np.array_equal(x.fingerprints, fp), f"{loop.__name__}: netlist {x.request.netlist}"
        say(f"  {loop.__name__}: {len(res)} requests equal the oracle ({span:.2f} s)")
    for h in hs:
        sim.unload_netlist(h)
