"""Exact time-window chunking: windows run independently (with the halo)
and concatenated equal one run of the whole job. The windowing is checked
here with the oracle as the engine; the GPU test runs it on the library."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import windows as WN
from paper_2304_13398_amd import workloads as W


def oracle_engine(nl):
    return lambda sub: O.o1_simulate(nl, sub)


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("n_windows", [2, 3, 7])
def test_windows_equal_whole_run_tiny(n_windows):
    nl, st = W.config1(seed=2)
    assert same(WN.simulate_windowed(nl, st, oracle_engine(nl), n_windows), O.o1_simulate(nl, st))


def test_windows_equal_whole_run_mid_generator():
    nl, st = W.config2(G=3000, S=48, L=25, n_per_src=300, seed=4)
    assert same(WN.simulate_windowed(nl, st, oracle_engine(nl), 5), O.o1_simulate(nl, st))


def test_windows_with_large_delays_and_dense_glitches():
    nl = W.make_netlist(G=400, S=12, L=12, types=W.TYPES_ALL, dmin=0, dmax=400, seed=9, name="wide")
    st = W.make_stimulus(S=12, n_per_src=400, window=3000, seed=9)
    assert same(WN.simulate_windowed(nl, st, oracle_engine(nl), 6), O.o1_simulate(nl, st))


def test_a_halo_too_short_is_detected():
    """Mutant of the halo: one level's worth too short must break exactness
    somewhere (so the test above is not vacuous)."""
    nl = W.make_netlist(G=400, S=12, L=12, types=W.TYPES_ALL, dmin=0, dmax=400, seed=9, name="wide")
    st = W.make_stimulus(S=12, n_per_src=400, window=3000, seed=9)
    H = WN.window_halo(nl)
    short = WN.simulate_windowed(nl, st, oracle_engine(nl), 6, halo=H // 4)
    assert not same(short, O.o1_simulate(nl, st))


def test_window_stimulus_holds_the_value_at_the_cut():
    st = W.Stimulus(np.array([0, 3, 3, 5]), np.array([10, 20, 30, 5, 40]),
                    np.array([1, 0, 2, 3, 1], dtype=np.uint8))
    sub = WN.window_stimulus(st, 3, 25, 41)
    # source 0: holds 0 at 25, then X at 30; source 1: empty; source 2: Z from 5, then 1 at 40
    assert sub.off.tolist() == [0, 2, 2, 4]
    assert sub.t.tolist() == [25, 30, 25, 40]
    assert sub.v.tolist() == [0, 2, 3, 1]
    # a source holding X at the cut gets no transition there
    sub2 = WN.window_stimulus(st, 3, 35, 41)
    assert sub2.t.tolist() == [35, 40] and sub2.v.tolist() == [3, 1]


def test_window_starting_on_a_change_to_x():
    st = W.Stimulus(np.array([0, 3]), np.array([10, 20, 30]), np.array([1, 2, 0], dtype=np.uint8))
    sub = WN.window_stimulus(st, 1, 20, 100)
    assert sub.t.tolist() == [30] and sub.v.tolist() == [0]
    nl = W.make_netlist(G=30, S=1, L=3, types=W.TYPES_ALL, seed=1, name="x-at-cut")
    full = O.o1_simulate(nl, st)
    assert same(WN.simulate_windowed(nl, st, oracle_engine(nl), 3, halo=WN.window_halo(nl)), full)


def test_mid_generator_windows_are_valid_stimuli():
    from paper_2304_13398_amd import gsim as G
    nl, st = W.config2(G=2000, S=256, L=20, n_per_src=2000, seed=1)
    H = WN.window_halo(nl)
    edges = [None] + WN.window_bounds(st, 6) + [None]
    for lo, hi in zip(edges[:-1], edges[1:]):
        sub = WN.window_stimulus(st, nl.S, 0 if lo is None else max(0, lo - H),
                                 np.iinfo(np.int64).max if hi is None else hi)
        G.validate_stimulus(nl.S, sub.off, sub.t, sub.v)
    assert same(WN.simulate_windowed(nl, st, oracle_engine(nl), 6), O.o1_simulate(nl, st))


def _window_stimulus_by_source(st, S, t_lo, t_hi):
    """The window's stimulus source by source, as its definition reads."""
    offs, ts, vs = [0], [], []
    for s in range(S):
        t, v = st.t[st.off[s]:st.off[s + 1]], st.v[st.off[s]:st.off[s + 1]]
        inside = (t >= t_lo) & (t < t_hi)
        tt, vv = list(t[inside]), list(v[inside])
        before = v[t < t_lo]
        held = int(before[-1]) if len(before) else 2
        if held != 2 and not (tt and tt[0] == t_lo):
            tt, vv = [t_lo] + tt, [held] + vv
        elif tt and vv[0] == 2:
            tt, vv = tt[1:], vv[1:]
        ts += tt
        vs += vv
        offs.append(len(ts))
    return np.array(offs, np.int64), np.array(ts, np.int64), np.array(vs, np.uint8)


def test_window_stimulus_equals_its_definition():
    """Random cuts, cuts on transition times, X/Z values and empty sources."""
    rng = np.random.default_rng(11)
    st = W.make_stimulus(S=60, n_per_src=40, window=10_000, probs=(0.3, 0.3, 0.2, 0.2), seed=11)
    # a few empty sources
    keep = np.ones(st.n, dtype=bool)
    for s in (0, 17, 59):
        keep[st.off[s]:st.off[s + 1]] = False
    lens = np.diff(st.off) * np.isin(np.arange(60), (0, 17, 59), invert=True)
    st = W.Stimulus(np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), st.t[keep], st.v[keep])
    cuts = list(rng.integers(0, 12_000, size=40)) + list(st.t[rng.integers(0, st.n, size=40)])
    for lo in cuts:
        for hi in (lo + 1, lo + int(rng.integers(1, 5000)), np.iinfo(np.int64).max):
            got = WN.window_stimulus(st, 60, int(lo), int(hi))
            want = _window_stimulus_by_source(st, 60, int(lo), int(hi))
            assert np.array_equal(got.off, want[0]) and np.array_equal(got.t, want[1]) \
                and np.array_equal(got.v, want[2]), (lo, hi)
