"""HIP path vs the CPU oracle O1, element by element, through the C ABI,
under every schedule (level by level; dependency-driven; level barriers in
one launch).

Every comparison is exact (integer times and 2-bit values: tolerance 0).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import gsim as G
from paper_2304_13398_amd import workloads as W
from tests import oracle_pins as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=[0, 1, 3], ids=["levels", "dataflow", "levelsync"])
def sim(request):
    """Every case runs under every schedule: level by level, dependency-driven
    (one persistent launch per job), and level barriers in one launch."""
    s = G.Sim(0)
    s.set_option(G.OPT_SCHEDULE, request.param)
    say(f"schedule {request.param}")
    yield s
    s.close()


def gpu(sim, nl, st, kernel=0):
    sim.set_option(G.OPT_KERNEL, kernel)
    try:
        return sim.simulate(nl, st)
    finally:
        sim.set_option(G.OPT_KERNEL, 0)


def assert_same(got, want, nl=None):
    goff, gt, gv = got
    woff, wt, wv = want
    if np.array_equal(goff, woff) and np.array_equal(gt, wt) and np.array_equal(gv, wv):
        return
    glen, wlen = np.diff(goff), np.diff(woff)
    for g in range(len(wlen)):
        a = list(zip(gt[goff[g]:goff[g + 1]].tolist(), gv[goff[g]:goff[g + 1]].tolist()))
        b = list(zip(wt[woff[g]:woff[g + 1]].tolist(), wv[woff[g]:woff[g + 1]].tolist()))
        if a != b:
            info = ""
            if nl is not None:
                info = (f" type={int(nl.type[g])} pins={nl.pin_net[nl.pin_off[g]:nl.pin_off[g + 1]].tolist()}"
                        f" rise={nl.rise[nl.pin_off[g]:nl.pin_off[g + 1]].tolist()}"
                        f" fall={nl.fall[nl.pin_off[g]:nl.pin_off[g + 1]].tolist()}")
            n_bad = int(np.sum(glen != wlen))
            pytest.fail(f"gate {g} differs ({n_bad} gates with other lengths){info}\n"
                        f" gpu   ({len(a)}): {a[:12]}\n oracle({len(b)}): {b[:12]}")
    pytest.fail("arrays differ")


def check(sim, nl, st, kernel=0):
    say(f"case {nl.name or 'netlist'} G={nl.G} S={nl.S} N_in={st.n} kernel={kernel}")
    want = O.o1_simulate(nl, st)
    got = gpu(sim, nl, st, kernel)
    assert_same(got, want, nl)
    return got


def test_config1_tiny(sim):
    check(sim, *W.config1(seed=1))


@pytest.mark.parametrize("seed", [2, 3])
def test_config1_other_seeds(sim, seed):
    check(sim, *W.config1(seed=seed))


def test_config1_lane_kernel(sim):
    check(sim, *W.config1(seed=1), kernel=1)


def test_config2_generator_20k(sim):
    """The mid-size generator (power-law fanout, fan-in 1-4) at 20k gates and
    full depth, 1,000 transitions per PI: many 64-transition tiles per pin and
    ragged tails."""
    check(sim, *W.config2(G=20_000, S=64))


def test_config3_generator_30k(sim):
    """Industrial-shaped generator (delays up to 200 ps, 150 levels) at 30k gates."""
    check(sim, *W.config3(G=30_000, S=300))


def test_worked_examples_on_gpu(sim):
    # Fig. 2: simultaneous falls, minimum delay
    nl = P.netlist_of(2, [(W.AND2, [0, 1])], [3, 7], [5, 10])
    st = P.stimulus_of([[(0, 1), (100, 0)], [(0, 1), (100, 0)]])
    off, t, v = gpu(sim, nl, st)
    assert list(zip(t.tolist(), v.tolist())) == [(3, 1), (105, 0)]
    # Fig. 3: glitch eaten, redundant fall dropped
    nl = P.netlist_of(2, [(W.AND2, [0, 1])], [15, 1], [4, 5])
    st = P.stimulus_of([[(0, 0), (5, 1)], [(0, 1), (10, 0)]])
    off, t, v = gpu(sim, nl, st)
    assert list(zip(t.tolist(), v.tolist())) == [(4, 0)]
    # several denials by one candidate (4-value logic)
    nl = P.netlist_of(2, [(W.XOR2, [0, 1])], [100, 1], [100, 1])
    st = P.stimulus_of([[(10, 1), (11, 2), (12, 0)], [(0, 0), (13, 1)]])
    off, t, v = gpu(sim, nl, st)
    assert list(zip(t.tolist(), v.tolist())) == [(14, 1)]


@pytest.mark.parametrize("kernel", [0, 1])
def test_zero_delays(sim, kernel):
    nl = W.make_netlist(G=3000, S=24, L=12, types=W.TYPES_ALL, dmin=0, dmax=0, seed=7,
                        name="zero-delay")
    st = W.make_stimulus(S=24, n_per_src=150, window=2000, seed=7)
    check(sim, nl, st, kernel)


def test_delays_at_tentative_window_edge(sim):
    """Largest pin delay = 256 = the wavefront kernel's tentative window."""
    nl = W.make_netlist(G=2000, S=16, L=10, types=W.TYPES_ALL, dmin=200, dmax=256, seed=8,
                        name="dmax256")
    st = W.make_stimulus(S=16, n_per_src=300, window=3000, seed=8)
    h = sim.load_netlist(nl)
    assert sim.netlist_info(h).lane_gates == 0
    sim.unload_netlist(h)
    check(sim, nl, st)


def test_large_delays_use_lane_kernel(sim):
    nl = W.make_netlist(G=2000, S=16, L=10, types=W.TYPES_ALL, dmin=0, dmax=900, seed=9,
                        name="dmax900")
    st = W.make_stimulus(S=16, n_per_src=300, window=3000, seed=9)
    h = sim.load_netlist(nl)
    info = sim.netlist_info(h)
    assert 0 < info.lane_gates < nl.G
    sim.unload_netlist(h)
    check(sim, nl, st)


def test_dense_short_pulses(sim):
    """Transitions 1 ps apart against delays up to 40 ps: long chains of
    tentative transitions and denials across tile boundaries."""
    nl = W.make_netlist(G=1500, S=8, L=15, types=W.TYPES_ALL, dmin=0, dmax=40, seed=10,
                        name="dense")
    st = W.make_stimulus(S=8, n_per_src=700, window=800, seed=10)
    check(sim, nl, st)


def test_empty_and_single_transition_sources(sim):
    nl = W.make_netlist(G=800, S=10, L=8, types=W.TYPES_ALL, dmin=1, dmax=30, seed=11,
                        name="ragged-sources")
    waves = []
    rng = np.random.default_rng(11)
    for s in range(10):
        n = [0, 1, 0, 2, 63, 64, 65, 127, 128, 129][s]
        waves.append(P._random_wave(rng, n, 400))
    check(sim, nl, P.stimulus_of(waves))


def test_duplicate_pins_and_z_sources(sim):
    gates = [(W.XOR2, [0, 0]), (W.AND2, [1, 1]), (W.MUX2, [0, 1, 1]), (W.OR4, [2, 2, 3, 3]),
             (W.AND4, [4, 5, 4, 6]), (W.NOT, [7]), (W.BUF, [2])]
    k = sum(len(g[1]) for g in gates)
    rng = np.random.default_rng(12)
    nl = P.netlist_of(3, gates, rng.integers(0, 9, k).tolist(), rng.integers(0, 9, k).tolist())
    waves = [[(0, 3), (5, 1), (9, 3), (12, 2), (20, 0)], [(1, 1), (2, 3), (3, 0)], [(4, 3)]]
    check(sim, nl, P.stimulus_of(waves))


def test_no_gates(sim):
    nl = P.netlist_of(2, [], [], [])
    st = P.stimulus_of([[(0, 1)], []])
    h = sim.load_netlist(nl)
    j = sim.run(h, st)
    sim.wait(j)
    off, t, v = sim.fetch(j)
    assert off.tolist() == [0, 1, 1] and t.tolist() == [0] and v.tolist() == [1]
    sim.release(j)
    sim.unload_netlist(h)


def layered(widths, S, seed):
    """Gates in strict levels of the given widths; each gate reads 1-4 nets of
    the previous level (sources for the first), delays 1-60 ps."""
    rng = np.random.default_rng(seed)
    arity = {O.BUF: 1, O.NOT: 1, O.AND2: 2, O.XOR2: 2, O.NOR2: 2, O.AND3: 3, O.MUX2: 3, O.OR4: 4}
    types = list(arity)
    gates, prev, first = [], np.arange(S), S
    for w in widths:
        for _ in range(w):
            ty = types[rng.integers(len(types))]
            gates.append((ty, [int(x) for x in rng.choice(prev, size=arity[ty])]))
        prev = np.arange(first, first + w)
        first += w
    P_ = sum(len(g[1]) for g in gates)
    return P.netlist_of(S, gates, rng.integers(1, 61, P_), rng.integers(1, 61, P_))


def test_level_shapes(sim):
    """Shapes that set the level-barrier grid: a 300-level chain (one
    wavefront, 299 barriers), one level of 9,000 gates (the full grid, no
    barrier), and 1,000-gate levels (a grid of 1,000: a partial last group of
    40 wavefronts)."""
    for name, widths, S in (("chain", [1] * 300, 3), ("one wide level", [9000], 64),
                            ("1,000 per level", [1000] * 4, 64)):
        nl = layered(widths, S, seed=len(widths))
        nl.name = name
        st = W.make_stimulus(S=S, n_per_src=60, window=50_000, seed=3)
        check(sim, nl, st)


def test_shuffled_gate_order(sim):
    nl, st = W.config1(seed=5)
    rng = np.random.default_rng(1)
    perm = rng.permutation(nl.G)
    inv = np.argsort(perm)
    remap = np.concatenate([np.arange(nl.S), nl.S + inv])
    gates = [(int(nl.type[g]), [int(remap[x]) for x in nl.pin_net[nl.pin_off[g]:nl.pin_off[g + 1]]])
             for g in perm]
    rise = np.concatenate([nl.rise[nl.pin_off[g]:nl.pin_off[g + 1]] for g in perm])
    fall = np.concatenate([nl.fall[nl.pin_off[g]:nl.pin_off[g + 1]] for g in perm])
    check(sim, P.netlist_of(nl.S, gates, rise, fall), st)


def test_fetch_subset_sources_and_stats(sim):
    nl, st = W.config1(seed=6)
    want = O.o1_simulate(nl, st)
    h = sim.load_netlist(nl)
    j = sim.run(h, st)
    sim.wait(j)
    nets = np.array([nl.S + 5, 3, nl.S + nl.G - 1, 0, nl.S + 5])
    off, t, v = sim.fetch(j, nets)
    for i, n in enumerate(nets.tolist()):
        a, b = off[i], off[i + 1]
        if n < nl.S:
            wt, wv = st.t[st.off[n]:st.off[n + 1]], st.v[st.off[n]:st.off[n + 1]]
        else:
            g = n - nl.S
            wt, wv = want[1][want[0][g]:want[0][g + 1]], want[2][want[0][g]:want[0][g + 1]]
        assert np.array_equal(t[a:b], wt) and np.array_equal(v[a:b], wv)
    s = sim.stats(j)
    assert s.n_in == st.n and s.n_out == int(want[0][-1])
    assert s.pin_reads >= s.n_out and s.device_ms > 0
    with pytest.raises(G.GsimError) as e:
        sim.fetch(j, np.array([nl.S + nl.G]))
    assert e.value.status == G.E_ARG
    sim.release(j)
    with pytest.raises(G.GsimError) as e:
        sim.wait(j)
    assert e.value.status == G.E_HANDLE
    sim.unload_netlist(h)


def test_two_runs_identical(sim):
    nl, st = W.config2(G=5000, S=32, L=30, n_per_src=400)
    a = gpu(sim, nl, st)
    b = gpu(sim, nl, st)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_arena_overflow_reports_oom(sim):
    nl, st = W.config1(seed=1)
    h = sim.load_netlist(nl)
    sim.set_option(G.OPT_ARENA_TRANSITIONS, st.n + 1000)
    try:
        j = sim.run(h, st)
        with pytest.raises(G.GsimError) as e:
            sim.wait(j)
        assert e.value.status == G.E_OOM
        sim.release(j)
    finally:
        sim.set_option(G.OPT_ARENA_TRANSITIONS, 0)
    j = sim.run(h, st)          # the context still works afterwards
    sim.wait(j)
    off, t, v = sim.fetch(j, np.arange(nl.S, nl.S + nl.G))
    assert_same((off, t, v), O.o1_simulate(nl, st), nl)
    sim.release(j)
    sim.unload_netlist(h)


def test_invalid_stimulus_rejected(sim):
    nl, st = W.config1(seed=1)
    h = sim.load_netlist(nl)
    bad_v = st.v.copy()
    bad_v[5] = bad_v[4]
    with pytest.raises(G.GsimError) as e:
        sim.run(h, W.Stimulus(st.off, st.t, bad_v))
    assert e.value.status == G.E_WAVEFORM
    sim.unload_netlist(h)


def test_invalid_large_stimulus_names_the_first_bad_source(sim):
    """A stimulus above a million transitions is checked over ranges of
    sources on host threads; the error names the first bad source, as the
    serial check does, and a good copy of it runs exactly."""
    nl = W.config2_netlist(G=2000, S=512, L=10, seed=9)
    st = W.make_stimulus(S=nl.S, n_per_src=2500, window=1_000_000, seed=9)
    assert st.n > (1 << 20)
    h = sim.load_netlist(nl)
    for bad_sources in ((400,), (77, 400), (3, 77, 400)):
        t = st.t.copy()
        for s in bad_sources:
            a = int(st.off[s]) + 10
            t[a], t[a + 1] = t[a + 1], t[a]
        with pytest.raises(G.GsimError) as e:
            sim.run(h, W.Stimulus(st.off, t, st.v))
        assert e.value.status == G.E_WAVEFORM
        assert f"source {bad_sources[0]}:" in str(e.value)
    j = sim.run(h, st)
    sim.wait(j)
    assert_same(sim.fetch(j, np.arange(nl.S, nl.S + nl.G)), O.o1_simulate(nl, st), nl)
    sim.release(j)
    sim.unload_netlist(h)


def test_run_device_from_torch(sim):
    import torch
    nl, st = W.config1(seed=2)
    want = O.o1_simulate(nl, st)
    dev = torch.device("cuda:0")
    d_off = torch.from_numpy(st.off).to(dev)
    d_t = torch.from_numpy(st.t).to(dev)
    d_v = torch.from_numpy(st.v).to(dev)
    stream = torch.cuda.current_stream()
    h = sim.load_netlist(nl)
    j = sim.run_device(h, d_off.data_ptr(), d_t.data_ptr(), d_v.data_ptr(), st.n,
                       stream=stream.cuda_stream, validate=True)
    sim.wait(j)
    got = sim.fetch(j, np.arange(nl.S, nl.S + nl.G))
    assert_same(got, want, nl)
    sim.release(j)
    sim.unload_netlist(h)


@pytest.mark.parametrize("kernel", [0, 1])
def test_time_gaps_beyond_32_bits(sim, kernel):
    """Source times spread over ~2^40 ps with dense bursts: rounds whose span
    would exceed the 32-bit in-round offsets, and tentative transitions left
    when a round's horizon is capped."""
    rng = np.random.default_rng(21)
    S = 6
    waves = []
    for s in range(S):
        bursts = np.sort(rng.choice(2 ** 40, size=5, replace=False))
        ts = np.unique(np.concatenate([b + np.sort(rng.choice(200, size=40, replace=False))
                                       for b in bursts]))
        vals, prev = [], 2
        for _ in ts:
            v = int(rng.choice([c for c in range(4) if c != prev]))
            vals.append(v)
            prev = v
        waves.append(list(zip(ts.tolist(), vals)))
    nl = W.make_netlist(G=400, S=S, L=8, types=W.TYPES_ALL, dmin=0, dmax=60, seed=21,
                        name="time-gaps")
    check(sim, nl, P.stimulus_of(waves), kernel)


@pytest.mark.parametrize("kernel", [0, 1])
def test_times_near_the_limit(sim, kernel):
    """Source times just below 2^61 and just below 2^62 minus the longest path
    delay (the largest the library accepts): tiles whose keys' high words sit
    at the top of their range and change inside a tile, dense bursts across
    several 2^30 ps boundaries, through 12 levels of gates."""
    rng = np.random.default_rng(31)
    S = 8
    nl = W.make_netlist(G=600, S=S, L=12, types=W.TYPES_ALL, dmin=0, dmax=60, seed=31, name="near-limit")
    top = (1 << 62) - 1 - 12 * 61 - 1_000  # every output stays below 2^62
    waves = []
    for s in range(S):
        starts = [(1 << 61) - 5_000, (1 << 61) + (1 << 30) - 700, top - 600_000, top - 3_000]
        ts = np.unique(np.concatenate([b + np.sort(rng.choice(2_500, size=90, replace=False)) for b in starts]))
        vals, prev = [], 2
        for _ in ts:
            v = int(rng.choice([c for c in range(4) if c != prev]))
            vals.append(v)
            prev = v
        waves.append(list(zip(ts.tolist(), vals)))
    check(sim, nl, P.stimulus_of(waves), kernel)


def test_one_huge_gap_at_round_edge(sim):
    """A burst, a gap of 2^31 ps, then a second burst, through a chain of gates."""
    a = [(t, 1 if i % 2 == 0 else 0) for i, t in enumerate(range(0, 300, 3))]
    b = [(t, 0 if i % 2 == 0 else 1) for i, t in enumerate(range(1, 301, 3))]
    a += [(2 ** 31 + t, 0 if i % 2 else 1) for i, t in enumerate(range(0, 30, 2))]
    b += [(2 ** 31 + 7 + t, 1 if i % 2 else 0) for i, t in enumerate(range(0, 30, 2))]
    gates = [(W.XOR2, [0, 1]), (W.AND2, [0, 2]), (W.OR2, [3, 1]), (W.NOT, [4]), (W.XNOR2, [5, 2])]
    k = sum(len(g[1]) for g in gates)
    nl = P.netlist_of(2, gates, [40] * k, [7] * k)
    check(sim, nl, P.stimulus_of([a, b]))


def test_fingerprints_match_oracle(sim):
    from tests import net_hash
    nl, st = W.config2(G=20_000, S=64)
    off, t, v = O.o1_simulate(nl, st)
    h = sim.load_netlist(nl)
    j = sim.run(h, st)
    got = sim.hashes(j)                      # all nets, sources first
    src = net_hash.fingerprints(st.off, st.t, st.v)
    assert np.array_equal(got[:nl.S], src)
    assert np.array_equal(got[nl.S:], net_hash.fingerprints(off, t, v))
    sub = np.array([nl.S + 3, 1, nl.S + nl.G - 1])
    assert np.array_equal(sim.hashes(j, sub), got[sub])
    sim.release(j)
    sim.unload_netlist(h)


@pytest.mark.parametrize("wcv", [4.0, 12.0])
def test_skewed_source_activity(sim, wcv):
    """Uneven source activity (coefficient of variation of the given lengths
    as in the paper's WCV): heavy-tailed gate sizes, some silent sources."""
    nl, st = W.config2_skewed(wcv, G=20_000, S=256, L=30, seed=5)
    check(sim, nl, st)


def ext_check(sim, nl, st, dly, udp, kernel=0):
    say(f"extended model {nl.name} G={nl.G} N_in={st.n} udp={len(udp)} kernel={kernel}")
    want = O.o1x_simulate(nl, st, dly, udp)
    sim.set_option(G.OPT_KERNEL, kernel)
    try:
        h = sim.load_netlist_ext(nl, dly, udp)
        try:
            j = sim.run(h, st)
            got = sim.fetch(j, np.arange(nl.S, nl.S + nl.G))
            sim.release(j)
        finally:
            sim.unload_netlist(h)
    finally:
        sim.set_option(G.OPT_KERNEL, 0)
    assert_same(got, want, nl)


@pytest.mark.parametrize("kernel", [0, 1])
def test_edge_delays_and_user_tables_tiny(sim, kernel):
    """Delays by pin, input edge and output value, with unrelated (inf)
    entries; user-defined gate tables (including ones that map all-X inputs
    to 0 or 1); wavefront and lane kernels."""
    nl, st = W.config1(seed=6)
    type_, dly, udp = W.make_cell_model(nl, seed=6, edge_spread=0.8, inf_prob=0.2, n_udp=8, udp_frac=0.4)
    ext_check(sim, W.with_types(nl, type_), st, dly, udp, kernel)


def test_edge_delays_mid_generator(sim):
    """20k gates under the extended model. Under the dependency-driven
    schedule one run of an earlier kernel version never finished; the per-gate
    procedure of that version is exact on every gate of this case under the
    CPU wave emulator (tests/test_emu_eval.py), and the publication of a
    gate's outputs to its consumers now has a formal happens-before edge."""
    nl, st = W.config2(G=20_000, S=64, L=30, n_per_src=400, seed=7)
    type_, dly, udp = W.make_cell_model(nl, seed=7, edge_spread=0.5, inf_prob=0.05, n_udp=6, udp_frac=0.2)
    ext_check(sim, W.with_types(nl, type_), st, dly, udp)


def test_edge_delays_across_windows_and_xz_sources(sim):
    """Delays from 0 to 400 ps (small and large windows and the lane kernel),
    X and Z as likely as 0 and 1 at the sources."""
    nl = W.make_netlist(G=3000, S=40, L=20, types=W.TYPES_ALL, dmin=0, dmax=400, seed=8, name="wide")
    st = W.make_stimulus(S=40, n_per_src=300, window=50_000, probs=(0.25, 0.25, 0.25, 0.25), seed=8)
    type_, dly, udp = W.make_cell_model(nl, seed=8, edge_spread=0.9, inf_prob=0.15, n_udp=8, udp_frac=0.5)
    ext_check(sim, W.with_types(nl, type_), st, dly, udp)


def test_edge_free_extended_load_equals_basic(sim):
    """The extended loader with delays that do not depend on the edge gives
    the basic model's result (different kernel variant, same definition)."""
    nl, st = W.config2(G=8000, S=48, L=25, n_per_src=300, seed=9)
    d = np.zeros((nl.P, 2, 2), dtype=np.int32)
    d[:, :, 0] = nl.fall[:, None]
    d[:, :, 1] = nl.rise[:, None]
    ext_check(sim, nl, st, d, np.zeros((0, 256), np.uint8))


def test_standard_cell_netlist(sim):
    """Multi-output library cells (adders, AOI, decoder, gated mux) expanded
    into table gates with per-output delay matrices."""
    from paper_2304_13398_amd import cells as CL
    nl, dly, udp = CL.random_cell_netlist(3000, S=48, seed=10)
    st = W.make_stimulus(S=48, n_per_src=200, window=100_000, seed=10)
    ext_check(sim, nl, st, dly, udp)
