"""Executor paths on the GPU: batched stimulus sets, jobs of different netlists
sharing launches (continuous batching), dynamic binning by input volume, and
admission limited by the HBM budget. Every result is compared exactly with
the oracle run on the same job alone."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import gsim as G
from paper_2304_13398_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = G.Sim(0)
    yield s
    s.close()


def fetch_gates(sim, j, nl):
    return sim.fetch(j, np.arange(nl.S, nl.S + nl.G))


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_batch_of_uneven_sets(sim):
    nl = W.config2_netlist(G=6000, S=48, L=30, seed=3)
    rng = np.random.default_rng(3)
    sets = [W.make_stimulus(S=nl.S, n_per_src=int(n), window=1_000_000, seed=100 + i)
            for i, n in enumerate(W.loguniform_int(rng, 50, 1500, size=7))]
    say(f"batch: G={nl.G} sets={len(sets)} lengths={[s.n for s in sets]}")
    h = sim.load_netlist(nl)
    jobs = sim.run_batch(h, sets)
    for j, st in zip(jobs, sets):
        sim.wait(j)
        assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, st))
        sim.release(j)
    sim.unload_netlist(h)


def test_batch_with_a_bad_set_leaves_nothing(sim):
    """Sets are checked (on host threads) before any job is made: a batch
    with one unordered set fails as a whole, and the netlist can be unloaded
    at once (no job of it is left); the same batch without that set runs
    exactly."""
    nl = W.config2_netlist(G=3000, S=40, L=20, seed=8)
    sets = [W.make_stimulus(S=nl.S, n_per_src=200 + 50 * i, window=1_000_000, seed=200 + i) for i in range(12)]
    bad = W.Stimulus(off=sets[5].off.copy(), t=sets[5].t.copy(), v=sets[5].v.copy())
    a = int(bad.off[3])
    bad.t[a], bad.t[a + 1] = bad.t[a + 1], bad.t[a]  # times out of order in source 3
    say(f"bad batch: G={nl.G} sets={len(sets)}")
    h = sim.load_netlist(nl)
    with pytest.raises(G.GsimError) as e:
        sim.run_batch(h, sets[:5] + [bad] + sets[6:])
    assert e.value.status == G.E_WAVEFORM
    sim.unload_netlist(h)
    h = sim.load_netlist(nl)
    good = sets[:5] + sets[6:]
    for j, st in zip(sim.run_batch(h, good), good):
        sim.wait(j)
        assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, st))
        sim.release(j)
    sim.unload_netlist(h)


def test_continuous_batching_mixed_netlists(sim):
    """Jobs of three netlists (different sizes and depths) join a running
    executor at different steps; each result equals the job run alone."""
    nls = [W.config1(seed=4)[0], W.config2_netlist(G=4000, S=40, L=25, seed=5),
           W.config3(G=5000, S=120, L=40, seed=6)[0]]
    hs = [sim.load_netlist(nl) for nl in nls]
    rng = np.random.default_rng(7)
    pending = []
    for k in range(9):
        which = k % 3
        nl = nls[which]
        n = int(rng.integers(20, 400))
        st = W.make_stimulus(S=nl.S, n_per_src=n, window=100_000, seed=200 + k)
        j = sim.submit(hs[which], st)
        pending.append((j, nl, st))
        for _ in range(int(rng.integers(1, 6))):   # a few steps before the next arrival
            sim.drive()
    say(f"mixed: {len(pending)} jobs submitted")
    while any(not sim.done(j) for j, _, _ in pending):
        sim.drive(max_ahead=2)
    for j, nl, st in pending:
        sim.wait(j)
        assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, st)), f"job {j}"
        sim.release(j)
    for h in hs:
        sim.unload_netlist(h)


@pytest.mark.parametrize("threshold", [0, 200, 1 << 30])
def test_dynamic_binning_thresholds(sim, threshold):
    """Gates reading fewer than `threshold` input transitions go to the lane
    kernel: none, some, all."""
    nl, st = W.config2(G=8000, S=40, L=30, n_per_src=150)
    sim.set_option(G.OPT_LANE_THRESHOLD, threshold)
    try:
        got = sim.simulate(nl, st)
    finally:
        sim.set_option(G.OPT_LANE_THRESHOLD, 0)
    assert same(got, O.o1_simulate(nl, st))


def test_autotuner_settings_are_exact(sim):
    """Every setting the autotuner may choose (schedule, evaluation form, lane
    threshold) gives the oracle's waveforms when set on the netlist, also for
    a batch of sets that share steps; the tuner applies the fastest one."""
    from paper_2304_13398_amd import autotune
    nl, st = W.config2(G=6000, S=40, L=30, n_per_src=200, seed=12)
    want = O.o1_simulate(nl, st)
    h = sim.load_netlist(nl)
    try:
        tuner = autotune.Autotuner(sim, reps=1)
        for c in tuner.candidates:
            tuner.apply(h, c)
            j = sim.run(h, st)
            sim.wait(j)
            assert same(fetch_gates(sim, j, nl), want), autotune.setting_name(c)
            assert sim.stats(j).schedule == c[0]
            sim.release(j)
        c, ms = tuner.tune(nl, h, st)
        assert c in tuner.candidates and len(ms) == len(tuner.candidates)
        sets = [W.make_stimulus(S=nl.S, n_per_src=n, window=1_000_000, seed=40 + n) for n in (30, 120, 400)]
        for j, x in zip(sim.run_batch(h, sets), sets):
            sim.wait(j)
            assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, x)), autotune.setting_name(c)
            sim.release(j)
    finally:
        for opt in (G.OPT_SCHEDULE, G.OPT_EVAL_FORM, G.OPT_LANE_THRESHOLD, G.OPT_DF_TICKETS):
            sim.set_netlist_option(h, opt, -1)
        sim.unload_netlist(h)


def test_admission_waves_under_a_small_budget():
    """A context whose HBM budget holds about two jobs: five sets are admitted
    as earlier ones are released, and every result is still exact."""
    nl = W.config2_netlist(G=3000, S=32, L=20, seed=8)
    sets = [W.make_stimulus(S=nl.S, n_per_src=300, window=1_000_000, seed=300 + i) for i in range(5)]
    with G.Sim(0) as probe:
        h = probe.load_netlist(nl)
        j = probe.run(h, sets[0])
        probe.wait(j)
        need = probe.stats(j).arena_used
        probe.release(j)
        probe.unload_netlist(h)
    arena = int(need * 1.5)
    per_job = arena * 8 + 64 << 20     # arena + per-net tables and pool rounding
    with G.Sim(0, hbm_budget_bytes=2 * per_job + (96 << 20)) as s:
        s.set_option(G.OPT_ARENA_TRANSITIONS, arena)
        h = s.load_netlist(nl)
        jobs = s.run_batch(h, sets)
        for j, st in zip(jobs, sets):
            s.wait(j)
            assert same(fetch_gates(s, j, nl), O.o1_simulate(nl, st))
            s.release(j)
        s.unload_netlist(h)


def test_learned_arena_size_and_automatic_retry(sim):
    """A dense stimulus teaches the netlist's arena use per input transition:
    3,000 transitions per source packed into 6 ns, so that most of them are
    eaten as glitches at the first gates and deeper levels reserve little
    (about 46 slots per input transition, from the oracle's lengths). Sparse
    stimuli spread over 1 us need about 500 per input transition, far more
    than 1.5x that, so the first of them overflows and is re-run with twice
    the storage until it fits. Results stay exact, and the overflowed runs
    leave nothing allocated."""
    nl = W.config2_netlist(G=6000, S=32, L=40, seed=9)
    h = sim.load_netlist(nl)
    dense = W.make_stimulus(S=nl.S, n_per_src=3000, window=6_000, seed=31)
    j = sim.run(h, dense)
    sim.wait(j)
    sim.release(j)
    held = sim.memory_info()
    retries = []
    for n in (40, 15, 5):
        st = W.make_stimulus(S=nl.S, n_per_src=n, window=1_000_000, seed=32 + n)
        j = sim.run(h, st)
        sim.wait(j)
        retries.append(sim.stats(j).retries)
        assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, st))
        sim.release(j)
    say(f"retries per sparse job: {retries}")
    assert sum(retries) > 0, "the sparse jobs were meant to overflow their first arena"
    # every buffer of an overflowed run went back to the pool: after the
    # retried jobs are released the context holds what it held before them
    after = sim.memory_info()
    assert after.jobs_holding_storage == held.jobs_holding_storage == 0
    assert after.live_bytes == held.live_bytes, (held.live_bytes, after.live_bytes)
    sim.unload_netlist(h)


def test_request_loop_results_equal_alone(sim):
    """The served request loop on small resident netlists: every request's
    fingerprints (all nets) equal those of the oracle run on that request
    alone, under continuous batching and one-at-a-time service."""
    from paper_2304_13398_amd import serve
    from tests import net_hash
    nls = serve.served_netlists(scale=0.01, seed=9)[:4]
    pool = serve.make_stim_pool(nls, per_netlist=3, seed=9, lo=5, hi=60)
    hs = [sim.load_netlist(nl) for nl in nls]
    reqs = serve.served_workload(24, 2000.0, nls, pool, seed=9)
    say(f"served: {len(reqs)} requests over netlists {[nl.G for nl in nls]}")
    want = {}
    for r in reqs:
        key = id(r.stim)
        if key not in want:
            nl = nls[r.netlist]
            off, t, v = O.o1_simulate(nl, r.stim)
            want[key] = np.concatenate([net_hash.fingerprints(r.stim.off, r.stim.t, r.stim.v),
                                        net_hash.fingerprints(off, t, v)])
    for loop in (serve.serve_continuous, serve.serve_sequential):
        res, _ = loop(sim, hs, reqs)
        assert len(res) == len(reqs)
        for x in res:
            assert np.array_equal(x.fingerprints, want[id(x.request.stim)]), loop.__name__
    for h in hs:
        sim.unload_netlist(h)


def test_dependency_driven_batch_and_mix(sim):
    """Jobs under the dependency-driven schedule: a batch of uneven sets and
    jobs of two netlists submitted while others run; each equals the oracle."""
    sim.set_option(G.OPT_SCHEDULE, 1)
    try:
        nl = W.config2_netlist(G=5000, S=40, L=25, seed=11)
        nl2 = W.config3(G=4000, S=100, L=30, seed=12)[0]
        h, h2 = sim.load_netlist(nl), sim.load_netlist(nl2)
        rng = np.random.default_rng(11)
        sets = [W.make_stimulus(S=nl.S, n_per_src=int(n), window=1_000_000, seed=300 + i)
                for i, n in enumerate(W.loguniform_int(rng, 20, 800, size=5))]
        jobs = sim.run_batch(h, sets)
        st2 = W.make_stimulus(S=nl2.S, n_per_src=150, window=500_000, seed=399)
        j2 = sim.submit(h2, st2)
        sim.drive()
        for j, st in zip(jobs, sets):
            sim.wait(j)
            assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, st))
            sim.release(j)
        sim.wait(j2)
        assert same(fetch_gates(sim, j2, nl2), O.o1_simulate(nl2, st2))
        sim.release(j2)
        sim.unload_netlist(h)
        sim.unload_netlist(h2)
    finally:
        sim.set_option(G.OPT_SCHEDULE, 0)


def test_level_barrier_batch_and_two_streams(sim):
    """Jobs under the level-barrier schedule: a batch of uneven sets, then two
    jobs started on two streams before either is waited for (each launch
    waits for the context's previous one, so two grids never share the
    device); each equals the oracle."""
    import torch
    sim.set_option(G.OPT_SCHEDULE, 3)
    try:
        nl = W.config2_netlist(G=30000, S=64, L=30, seed=13)
        h = sim.load_netlist(nl)
        rng = np.random.default_rng(13)
        sets = [W.make_stimulus(S=nl.S, n_per_src=int(n), window=1_000_000, seed=500 + i)
                for i, n in enumerate(W.loguniform_int(rng, 20, 800, size=4))]
        for j, st in zip(sim.run_batch(h, sets), sets):
            sim.wait(j)
            assert sim.stats(j).schedule == 3
            assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, st))
            sim.release(j)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        jobs = [sim.run(h, st, stream=s.cuda_stream) for s, st in zip(streams, sets[:2])]
        for j, st in zip(jobs, sets[:2]):
            sim.wait(j)
            assert same(fetch_gates(sim, j, nl), O.o1_simulate(nl, st))
            sim.release(j)
        sim.unload_netlist(h)
    finally:
        sim.set_option(G.OPT_SCHEDULE, 0)


@pytest.mark.parametrize("n_windows", [3, 8])
def test_time_windows_on_the_gpu_equal_the_oracle(sim, n_windows):
    """A job cut into exact time windows (halo from the netlist's delays), each
    window run on the GPU, the pieces concatenated: equal to the oracle's run
    of the whole job."""
    from paper_2304_13398_amd import windows as WN
    nl, st = W.config3(G=6000, S=150, L=30, n_per_src=120, seed=13)
    run, run_many, close = WN.gpu_engine(sim, nl)
    try:
        got = WN.simulate_windowed(nl, st, run, n_windows)
        together = WN.simulate_windowed(nl, st, None, n_windows, run_many=run_many)
    finally:
        close()
    say(f"windows: {n_windows}, halo {WN.window_halo(nl)} ps")
    want = O.o1_simulate(nl, st)
    assert same(got, want)
    assert same(together, want)


def test_mixed_delay_models_share_steps(sim):
    """Jobs of a basic netlist, an extended one (edge delays, user tables) and
    a cell netlist advance in the same steps: every evaluate variant and each
    job's own gate tables in shared launches; each equals its oracle."""
    from paper_2304_13398_amd import cells as CL
    nl_a = W.config2_netlist(G=4000, S=40, L=25, seed=21)
    nl_b = W.config2_netlist(G=3000, S=32, L=20, seed=22)
    type_b, dly_b, udp_b = W.make_cell_model(nl_b, seed=22, edge_spread=0.7, inf_prob=0.1, n_udp=6, udp_frac=0.3)
    ext_b = W.with_types(nl_b, type_b)
    nl_c, dly_c, udp_c = CL.random_cell_netlist(1500, S=24, seed=23, dmax=120)
    h_a, h_b = sim.load_netlist(nl_a), sim.load_netlist_ext(ext_b, dly_b, udp_b)
    h_c = sim.load_netlist_ext(nl_c, dly_c, udp_c)
    jobs = []
    for k in range(6):
        which = k % 3
        nl, h = ((nl_a, h_a), (ext_b, h_b), (nl_c, h_c))[which]
        st = W.make_stimulus(S=nl.S, n_per_src=60 + 40 * k, window=200_000, seed=400 + k)
        jobs.append((sim.submit(h, st), which, nl, st))
        sim.drive()
    while any(not sim.done(j) for j, _, _, _ in jobs):
        sim.drive(max_ahead=2)
    for j, which, nl, st in jobs:
        sim.wait(j)
        if which == 0:
            want = O.o1_simulate(nl, st)
        elif which == 1:
            want = O.o1x_simulate(nl, st, dly_b, udp_b)
        else:
            want = O.o1x_simulate(nl, st, dly_c, udp_c)
        assert same(fetch_gates(sim, j, nl), want), f"job {j} (netlist {which})"
        sim.release(j)
    for h in (h_a, h_b, h_c):
        sim.unload_netlist(h)


def test_automatic_schedule_choice():
    """GSIM_OPT_SCHEDULE = 2 picks the dependency-driven launch for a small
    netlist and for uneven source activity, level by level for a large
    netlist with even activity; results equal the explicit schedules'."""
    sim = G.Sim(0)
    try:
        cases = []
        nl_t, st_t = W.config1(seed=1)
        cases.append(("tiny", nl_t, st_t, 1))
        nl_u, st_u = W.config2(seed=3, G=100_000, S=205)
        cases.append(("uniform 100k", nl_u, st_u, 0))
        st_s = W.make_stimulus_skewed(S=nl_u.S, mean_per_src=1000, wcv=5.0, window=1_000_000, seed=3)
        cases.append(("skewed 100k", nl_u, st_s, 1))
        for name, nl, st, want_sched in cases:
            h = sim.load_netlist(nl)
            hashes = {}
            for sched in (2, 0, 1):
                sim.set_option(G.OPT_SCHEDULE, sched)
                j = sim.run(h, st)
                sim.wait(j)
                if sched == 2:
                    got = sim.stats(j).schedule
                    say(f"auto schedule on {name}: {got}")
                    assert got == want_sched, name
                hashes[sched] = sim.hashes(j)
                sim.release(j)
            sim.set_option(G.OPT_SCHEDULE, 0)
            assert np.array_equal(hashes[2], hashes[0]) and np.array_equal(hashes[2], hashes[1]), name
            sim.unload_netlist(h)
    finally:
        sim.close()
