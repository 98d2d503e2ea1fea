"""The extended cell model of the oracle (delays by pin, input edge and output
value, with the paper's inf for unrelated pins; user-defined gate tables),
pinned by: reduction to the pinned oracle in the special cases the extended
model contains, the independent dense-time definition on tiny circuits, and
a worked example written out by hand."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INF = W.NO_RELATION


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def collapsed_delays(nl):
    """dly with no edge dependence: rise for output 1, fall for output 0."""
    d = np.zeros((nl.P, 2, 2), dtype=np.int32)
    d[:, :, 0] = nl.fall[:, None]
    d[:, :, 1] = nl.rise[:, None]
    return d


@pytest.mark.parametrize("cfg", ["tiny", "mid"])
def test_edge_free_delays_reduce_to_the_pinned_oracle(cfg):
    nl, st = W.config1(seed=3) if cfg == "tiny" else W.config2(G=2000, S=40, L=20, n_per_src=200, seed=3)
    assert same(O.o1x_simulate(nl, st, collapsed_delays(nl)), O.o1_simulate(nl, st))


def test_tables_equal_to_builtin_types_reduce_to_the_pinned_oracle():
    nl, st = W.config2(G=1500, S=32, L=15, n_per_src=150, seed=4)
    udp = np.zeros((12, 256), dtype=np.uint8)
    for t in range(12):
        k = O.ARITY[t]
        for packed in range(4 ** k):
            udp[t, packed] = O.gate_eval(t, [(packed >> (2 * i)) & 3 for i in range(k)])
    ext = W.with_types(nl, nl.type.astype(np.int64) + 12)
    assert same(O.o1x_simulate(ext, st, collapsed_delays(nl), udp), O.o1_simulate(nl, st))


@pytest.mark.parametrize("seed", range(6))
def test_matches_the_dense_time_definition(seed):
    nl = W.make_netlist(G=14, S=4, L=5, types=W.TYPES_ALL, dmin=0, dmax=6, seed=seed, name="ext")
    st = W.make_stimulus(S=4, n_per_src=6, window=30, seed=seed)
    type_, dly, udp = W.make_cell_model(nl, seed=seed, edge_spread=0.9, inf_prob=0.25,
                                        n_udp=4, udp_frac=0.4)
    ext = W.with_types(nl, type_)
    got = O.csr_to_lists(*O.o1x_simulate(ext, st, dly, udp))
    assert got == O.o3x_simulate(ext, st, dly, udp)


def test_edge_worked_example():
    case = json.load(open(os.path.join(GOLDEN, "edge_delays.json")))
    for c in case["cases"]:
        nl = W.Netlist(2, 1, np.array([O.AND2], np.uint8), np.array([0, 2]), np.array([0, 1]),
                       np.zeros(2, np.int32), np.zeros(2, np.int32), np.array([1], np.int32), "and")
        st = W.Stimulus(np.array([0, len(c["a"]), len(c["a"]) + len(c["b"])]),
                        np.array([t for t, _ in c["a"]] + [t for t, _ in c["b"]]),
                        np.array([v for _, v in c["a"]] + [v for _, v in c["b"]], dtype=np.uint8))
        dly = np.array([c["dly_a"], c["dly_b"]], dtype=np.int64)
        dly[dly < 0] = INF
        got = O.csr_to_lists(*O.o1x_simulate(nl, st, dly.astype(np.int32)))
        assert got == [[tuple(x) for x in c["expected"]]], c["name"]
        assert O.o3x_simulate(nl, st, dly.astype(np.int32)) == got


def test_unrelated_pins_never_cause_an_output():
    """A pin whose every entry is inf can change the gate's value, but that
    candidate never appears; the output still follows the related pin."""
    nl, st = W.config1(seed=5)
    d = collapsed_delays(nl)
    # every gate's last pin unrelated
    last = nl.pin_off[1:] - 1
    d[last] = INF
    off, t, v = O.o1x_simulate(nl, st, d)
    assert same(O.o1x_simulate(nl, st, d), (off, t, v))
    assert off[-1] < O.o1_simulate(nl, st)[0][-1]


def check_ext(lib=None, seeds=range(12)):
    """Every extended-model pin against the oracle library at ``lib``; returns
    the failures (used by the mutant tests with planted mistakes)."""
    fails = []
    for seed in seeds:
        nl = W.make_netlist(G=14, S=4, L=5, types=W.TYPES_ALL, dmin=0, dmax=6, seed=seed, name="ext")
        # odd seeds: X and Z as likely as 0 and 1 (X <-> Z changes reach table gates)
        probs = (0.25, 0.25, 0.25, 0.25) if seed % 2 else (0.45, 0.45, 0.05, 0.05)
        st = W.make_stimulus(S=4, n_per_src=6, window=30, probs=probs, seed=seed)
        type_, dly, udp = W.make_cell_model(nl, seed=seed, edge_spread=0.9, inf_prob=0.25,
                                            n_udp=4, udp_frac=0.7 if seed % 2 else 0.4)
        ext = W.with_types(nl, type_)
        if O.csr_to_lists(*O.o1x_simulate(ext, st, dly, udp, lib=lib)) != O.o3x_simulate(ext, st, dly, udp):
            fails.append(f"dense-time seed {seed}")
    case = json.load(open(os.path.join(GOLDEN, "edge_delays.json")))
    for c in case["cases"]:
        nl = W.Netlist(2, 1, np.array([O.AND2], np.uint8), np.array([0, 2]), np.array([0, 1]),
                       np.zeros(2, np.int32), np.zeros(2, np.int32), np.array([1], np.int32), "and")
        st = W.Stimulus(np.array([0, len(c["a"]), len(c["a"]) + len(c["b"])]),
                        np.array([t for t, _ in c["a"]] + [t for t, _ in c["b"]]),
                        np.array([v for _, v in c["a"]] + [v for _, v in c["b"]], dtype=np.uint8))
        dly = np.array([c["dly_a"], c["dly_b"]], dtype=np.int64)
        dly[dly < 0] = INF
        if O.csr_to_lists(*O.o1x_simulate(nl, st, dly.astype(np.int32), lib=lib)) != \
                [[tuple(x) for x in c["expected"]]]:
            fails.append(f"golden {c['name']}")
    return fails


def test_all_extended_pins_hold():
    assert check_ext() == []
