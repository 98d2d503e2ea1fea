"""Checks that pin the CPU oracle to facts outside itself.

Each ``check_*`` takes the path of an O1 shared library (the real one, or a
copy with a planted mistake) and returns a list of failure strings, empty when
the check holds. The facts come from the paper (Table 1; the Fig. 2 and Fig. 3
worked examples; Eq. 1), from closed forms (zero-delay simulation is
combinational evaluation at every source change; a strictly levelled circuit
with one uniform delay d shifts that by level*d; the final value of every net
is the combinational value of the final source values) and from brute force
(the dense-time definition O3 on tiny inputs).
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

from oracle import oracle as O
from paper_2304_13398_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
VAL = {"0": 0, "1": 1, "X": 2, "Z": 3}


def table1():
    tabs, cur = {}, None
    with open(os.path.join(GOLDEN, "table1_truth_tables.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line in ("AND", "OR", "XOR"):
                cur = tabs.setdefault(line, [])
            else:
                cur.append([VAL[c] for c in line.split()])
    return tabs


def netlist_of(S, gates, rise, fall):
    """gates: list of (type, [nets]); rise/fall: flat per-pin lists."""
    types = np.array([g[0] for g in gates], dtype=np.uint8)
    pin_off = np.zeros(len(gates) + 1, dtype=np.int64)
    pin_off[1:] = np.cumsum([len(g[1]) for g in gates])
    pin_net = np.array([n for g in gates for n in g[1]], dtype=np.int64)
    return W.Netlist(S, len(gates), types, pin_off, pin_net, np.array(rise, dtype=np.int32),
                     np.array(fall, dtype=np.int32), np.zeros(len(gates), dtype=np.int32))


def stimulus_of(waves):
    off = np.zeros(len(waves) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(w) for w in waves])
    t = np.array([x[0] for w in waves for x in w], dtype=np.int64)
    v = np.array([x[1] for w in waves for x in w], dtype=np.uint8)
    return W.Stimulus(off, t, v)


def o1_lists(nl, st, lib):
    return O.csr_to_lists(*O.o1_simulate(nl, st, lib))


# ---------------------------------------------------------------------------

def check_table1(lib):
    bad = []
    tabs = table1()
    for name, gt in (("AND", O.AND2), ("OR", O.OR2), ("XOR", O.XOR2)):
        for a in range(4):
            for b in range(4):
                want = tabs[name][a][b]
                got = O.o1_eval(gt, [a, b], lib)
                if got != want:
                    bad.append(f"Table 1 {name}({a},{b}) = {got}, want {want}")
    return bad


def check_derived_gates(lib):
    """NOT/BUF by the Z-as-X rule of Section 2.2; NAND/NOR/XNOR as the negation
    of Table 1; 3/4-input AND/OR as folds of Table 1 (both tables are
    associative); MUX2 by its stated definition."""
    bad = []
    t = table1()
    neg = [1, 0, 2, 2]
    zx = [0, 1, 2, 2]
    for a in range(4):
        if O.o1_eval(O.NOT, [a], lib) != neg[a]:
            bad.append(f"NOT({a})")
        if O.o1_eval(O.BUF, [a], lib) != zx[a]:
            bad.append(f"BUF({a})")
    for a, b in itertools.product(range(4), repeat=2):
        for gt, want in ((O.NAND2, neg[t["AND"][a][b]]), (O.NOR2, neg[t["OR"][a][b]]),
                         (O.XNOR2, neg[t["XOR"][a][b]])):
            if O.o1_eval(gt, [a, b], lib) != want:
                bad.append(f"type {gt}({a},{b})")
    for v in itertools.product(range(4), repeat=3):
        want = t["AND"][t["AND"][v[0]][v[1]]][v[2]]
        if O.o1_eval(O.AND3, list(v), lib) != want:
            bad.append(f"AND3{v}")
        d0, d1, s = zx[v[0]], zx[v[1]], zx[v[2]]
        want = d0 if s == 0 else d1 if s == 1 else (d0 if d0 == d1 else 2)
        if O.o1_eval(O.MUX2, list(v), lib) != want:
            bad.append(f"MUX2{v}")
    for v in itertools.product(range(4), repeat=4):
        wa = t["AND"][t["AND"][t["AND"][v[0]][v[1]]][v[2]]][v[3]]
        wo = t["OR"][t["OR"][t["OR"][v[0]][v[1]]][v[2]]][v[3]]
        if O.o1_eval(O.AND4, list(v), lib) != wa:
            bad.append(f"AND4{v}")
        if O.o1_eval(O.OR4, list(v), lib) != wo:
            bad.append(f"OR4{v}")
    return bad


def check_fig2(lib):
    fx = json.load(open(os.path.join(GOLDEN, "fig2_min_delay.json")))
    a, b = fx["pins"]["a"], fx["pins"]["b"]
    bad = []
    for ra, rb in fx["rise_choices"]:
        got = O.o1_gate(O.AND2, [(a["t"], a["v"]), (b["t"], b["v"])], [ra, rb],
                        [a["fall"], b["fall"]], lib)
        want = [(min(ra, rb), 1), (fx["expected_fall_time"], 0)]
        if got != want:
            bad.append(f"Fig. 2 rise=({ra},{rb}): {got} != {want}")
    return bad


def check_fig3(lib):
    fx = json.load(open(os.path.join(GOLDEN, "fig3_glitch_eaten.json")))
    a, b = fx["pins"]["a"], fx["pins"]["b"]
    bad = []
    for fa in fx["a_fall_choices"]:
        for rb in fx["b_rise_choices"]:
            got = O.o1_gate(O.AND2, [(a["t"], a["v"]), (b["t"], b["v"])], [a["rise"], rb],
                            [fa, b["fall"]], lib)
            want = [(min(fa, b["fall"]), 0)]
            if got != want:
                bad.append(f"Fig. 3 fall_a={fa} rise_b={rb}: {got} != {want}")
    return bad


def check_multipop(lib):
    """Recursive denial in 4-value logic (Section 4.2): XOR with b low; a goes
    1, X, 0 at 10, 11, 12 through a 100 ps pin, giving three scheduled
    transitions at 110, 111, 112; b rises at 13 through a 1 ps pin, so the
    output 1 at 14 denies all three (Eq. 1), and nothing is dropped because the
    output is still X."""
    got = O.o1_gate(O.XOR2, [([10, 11, 12], [1, 2, 0]), ([0, 13], [0, 1])], [100, 1],
                    [100, 1], lib)
    want = [(14, 1)]
    return [] if got == want else [f"multi-pop: {got} != {want}"]


def _random_wave(rng, n, tmax):
    times = sorted(rng.choice(tmax + 1, size=n, replace=False).tolist())
    vals, prev = [], 2
    for _ in times:
        v = int(rng.choice([c for c in range(4) if c != prev]))
        vals.append(v)
        prev = v
    return list(zip(times, vals))


def check_bruteforce_o3(lib, cases_per_type=150, seed=0, exhaustive2=False):
    """O1 equals the dense-time definition O3 on single gates with short
    waveforms, small times and small delays (including zero)."""
    rng = np.random.default_rng(seed)
    bad = []
    for gt in range(12):
        k = O.ARITY[gt]
        for _ in range(cases_per_type):
            waves = [_random_wave(rng, int(rng.integers(0, 4)), 6) for _ in range(k)]
            rise = rng.integers(0, 4, size=k).tolist()
            fall = rng.integers(0, 4, size=k).tolist()
            nl = netlist_of(k, [(gt, list(range(k)))], rise, fall)
            st = stimulus_of(waves)
            a = o1_lists(nl, st, lib)[0]
            b = O.o3_simulate(nl, st)[0]
            if a != b:
                bad.append(f"type {gt} waves={waves} rise={rise} fall={fall}: O1 {a} O3 {b}")
                if len(bad) > 5:
                    return bad
    if exhaustive2:
        bad += check_exhaustive_pairs(lib)
    return bad


def _all_short_waves(times=(0, 1, 2, 3), maxlen=2):
    out = [[]]
    for n in range(1, maxlen + 1):
        for ts in itertools.combinations(times, n):
            for vs in itertools.product(range(4), repeat=n):
                if vs[0] == 2 or any(vs[i] == vs[i - 1] for i in range(1, n)):
                    continue
                out.append(list(zip(ts, vs)))
    return out


def check_exhaustive_pairs(lib, gtypes=(O.AND2, O.XOR2, O.OR2), delays=((0, 2), (2, 1), (3, 3))):
    """Every pair of waveforms of length <= 2 over times {0..3} on the
    2-input Table 1 gates, for a few delay pairs per pin: O1 == O3."""
    bad = []
    waves = _all_short_waves()
    for gt in gtypes:
        for wa, wb in itertools.product(waves, repeat=2):
            for (ra, fa), (rb, fb) in itertools.product(delays, repeat=2):
                nl = netlist_of(2, [(gt, [0, 1])], [ra, rb], [fa, fb])
                st = stimulus_of([wa, wb])
                a = o1_lists(nl, st, lib)[0]
                b = O.o3_simulate(nl, st, t_max=12)[0]
                if a != b:
                    bad.append(f"type {gt} {wa} {wb} d={ra, fa, rb, fb}: O1 {a} O3 {b}")
                    if len(bad) > 5:
                        return bad
    return bad


def _small_circuit(seed, G=24, S=5, L=4, dmin=0, dmax=4, strict=False, n=6, window=40):
    nl = W.make_netlist(G=G, S=S, L=L, types=W.TYPES_ALL, dmin=dmin, dmax=dmax,
                        strict=strict, seed=seed)
    st = W.make_stimulus(S=S, n_per_src=n, window=window, seed=seed)
    return nl, st


def _src_value_at(st, s, T):
    t = st.t[st.off[s]:st.off[s + 1]]
    i = int(np.searchsorted(t, T, side="right"))
    return 2 if i == 0 else int(st.v[st.off[s] + i - 1])


def _zero_delay_waves(nl, st):
    """Combinational evaluation at every source-change time; the waveform of
    each gate is the list of points where that value sequence changes."""
    times = sorted(set(st.t.tolist()))
    waves = [[] for _ in range(nl.G)]
    prev = [2] * nl.G
    for T in times:
        vals = O.combinational(nl, [_src_value_at(st, s, T) for s in range(nl.S)])
        for g in range(nl.G):
            if vals[g] != prev[g]:
                waves[g].append((T, vals[g]))
                prev[g] = vals[g]
    return waves


def check_zero_delay(lib, seeds=range(8)):
    bad = []
    for seed in seeds:
        nl, st = _small_circuit(seed, dmin=0, dmax=0)
        want = _zero_delay_waves(nl, st)
        got = o1_lists(nl, st, lib)
        if got != want:
            g = next(i for i in range(nl.G) if got[i] != want[i])
            bad.append(f"zero delay seed {seed} gate {g}: {got[g]} != {want[g]}")
    return bad


def check_uniform_shift(lib, seeds=range(8), d=3):
    """Strictly levelled circuit, rise = fall = d on every pin: no transition
    is ever denied, and every level-l net is its zero-delay waveform shifted
    by l*d."""
    bad = []
    for seed in seeds:
        nl, st = _small_circuit(seed + 100, strict=True)
        nl.rise[:] = d
        nl.fall[:] = d
        zero = _zero_delay_waves(nl, st)
        got = o1_lists(nl, st, lib)
        for g in range(nl.G):
            want = [(t + int(nl.level[g]) * d, v) for t, v in zero[g]]
            if got[g] != want:
                bad.append(f"uniform shift seed {seed} gate {g}: {got[g]} != {want}")
                break
    return bad


def check_steady_state(lib, seeds=range(8)):
    """Whatever the delays, the last value of every gate equals the
    combinational value of the sources' last values (X for an empty output)."""
    bad = []
    for seed in seeds:
        nl, st = _small_circuit(seed + 200, G=60, S=6, L=6, dmin=0, dmax=9, n=10, window=60)
        final_src = [int(st.v[st.off[s + 1] - 1]) if st.off[s + 1] > st.off[s] else 2
                     for s in range(nl.S)]
        want = O.combinational(nl, final_src)
        got = o1_lists(nl, st, lib)
        for g in range(nl.G):
            last = got[g][-1][1] if got[g] else 2
            if last != want[g]:
                bad.append(f"steady state seed {seed} gate {g}: {last} != {want[g]}")
                break
    return bad


def check_invariants_on(nl, st, off, t, v):
    """Structural invariants of every output waveform (Section 2.1 waveform
    definition; Eq. 2 applied to one gate)."""
    bad = []
    S = nl.S
    for g in range(nl.G):
        tt = t[off[g]:off[g + 1]]
        vv = v[off[g]:off[g + 1]]
        if len(tt) == 0:
            continue
        if np.any(np.diff(tt) <= 0):
            bad.append(f"gate {g}: times not strictly increasing")
        if vv[0] == 2 or np.any(vv[1:] == vv[:-1]):
            bad.append(f"gate {g}: repeated value or leading X")
        if np.any(vv > 2):
            bad.append(f"gate {g}: Z on a gate output")
        ins_t = []
        for p in range(nl.pin_off[g], nl.pin_off[g + 1]):
            n = int(nl.pin_net[p])
            if n < S:
                ins_t.append(st.t[st.off[n]:st.off[n + 1]])
            else:
                ins_t.append(t[off[n - S]:off[n - S + 1]])
        distinct = np.unique(np.concatenate(ins_t)) if ins_t else np.empty(0, np.int64)
        if len(tt) > len(distinct) or len(distinct) > sum(len(x) for x in ins_t):
            bad.append(f"gate {g}: length bound (Eq. 2) violated")
        ds = np.unique(np.concatenate([nl.rise[nl.pin_off[g]:nl.pin_off[g + 1]],
                                       nl.fall[nl.pin_off[g]:nl.pin_off[g + 1]]]))
        ok = np.isin(tt[:, None] - ds[None, :], distinct).any(axis=1)
        if not ok.all():
            bad.append(f"gate {g}: output time not an input time plus a pin delay")
        if len(bad) > 5:
            break
    return bad


def check_invariants(lib):
    nl, st = W.config1(seed=3)
    return check_invariants_on(nl, st, *O.o1_simulate(nl, st, lib))


def check_o2_agrees(lib, seeds=range(10)):
    bad = []
    for seed in seeds:
        nl, st = _small_circuit(seed + 300, G=40, S=6, L=5, dmin=0, dmax=6, n=8, window=50)
        a = o1_lists(nl, st, lib)
        b = O.o2_simulate(nl, st)
        if a != b:
            g = next(i for i in range(nl.G) if a[i] != b[i])
            bad.append(f"O1 vs O2 seed {seed} gate {g}: {a[g]} != {b[g]}")
    return bad


FAST_CHECKS = (check_table1, check_derived_gates, check_fig2, check_fig3, check_multipop,
               check_zero_delay, check_uniform_shift, check_steady_state, check_invariants,
               check_o2_agrees)
