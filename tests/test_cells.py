"""Standard-cell templates compiled into user-defined gate tables (one gate
per cell output with that output's slice of the delay matrix). The compiled
tables are checked against compositions of the oracle's gate function; the
expansion against the same circuit written with built-in gates."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import cells as C
from paper_2304_13398_amd import workloads as W


@pytest.mark.parametrize("gtype", range(12))
def test_single_gate_template_is_the_gate(gtype):
    k = O.ARITY[gtype]
    pins = [f"i{n}" for n in range(k)]
    tab = C.compile_template(C.CellTemplate("g", pins, ["y"], [(gtype, pins, "y")]))[0]
    for combo in itertools.product(range(4), repeat=k):
        packed = sum(v << (2 * i) for i, v in enumerate(combo))
        assert tab[packed] == O.gate_eval(gtype, list(combo))


def test_full_adder_tables_are_the_composition():
    s_tab, co_tab = C.compile_template(C.FULL_ADDER)
    for a, b, ci in itertools.product(range(4), repeat=3):
        x = O.gate_eval(O.XOR2, [a, b])
        s = O.gate_eval(O.XOR2, [x, ci])
        co = O.gate_eval(O.OR2, [O.gate_eval(O.AND2, [a, b]), O.gate_eval(O.AND2, [x, ci])])
        packed = a | b << 2 | ci << 4
        assert (s_tab[packed], co_tab[packed]) == (s, co)


def test_half_adder_cells_equal_the_gate_circuit():
    """A chain of half adders expanded into table gates, with delays that do
    not depend on the edge, equals the same circuit of XOR2/AND2 gates."""
    rng = np.random.default_rng(2)
    S, n = 6, 40
    insts, nl_type, nl_pins, rise, fall = [], [], [], [], []
    n_nets = S
    for c in range(n):
        a, b = (int(x) for x in rng.integers(n_nets, size=2))
        r = rng.integers(1, 40, size=(2, 2))  # [input][output]
        f = rng.integers(1, 40, size=(2, 2))
        d = np.zeros((2, 2, 2, 2), dtype=np.int64)
        for i in range(2):
            for o in range(2):
                d[i, o, :, 0] = f[i, o]
                d[i, o, :, 1] = r[i, o]
        insts.append(C.CellInstance(0, [a, b], d))
        for o, gt in enumerate((O.XOR2, O.AND2)):
            nl_type.append(gt)
            nl_pins += [a, b]
            rise += [int(r[0, o]), int(r[1, o])]
            fall += [int(f[0, o]), int(f[1, o])]
        n_nets += 2
    ext, dly, udp = C.expand(S, [C.HALF_ADDER], insts)
    G = len(nl_type)
    basic = W.Netlist(S, G, np.array(nl_type, np.uint8), np.arange(0, 2 * G + 1, 2), np.array(nl_pins),
                      np.array(rise, np.int32), np.array(fall, np.int32), np.zeros(G, np.int32), "ha")
    st = W.make_stimulus(S=S, n_per_src=50, window=3000, seed=2)
    got = O.o1x_simulate(ext, st, dly, udp)
    want = O.o1_simulate(basic, st)
    assert all(np.array_equal(x, y) for x, y in zip(got, want))


def test_random_cell_netlist_is_well_formed():
    nl, dly, udp = C.random_cell_netlist(200, S=10, seed=3)
    assert nl.P == dly.shape[0] and udp.shape[1] == 256 and (udp <= 2).all()
    assert (nl.type >= 12).all() and (nl.type < 12 + len(udp)).all()
    st = W.make_stimulus(S=10, n_per_src=40, window=5000, seed=3)
    off, t, v = O.o1x_simulate(nl, st, dly, udp)
    assert off[-1] > 0
