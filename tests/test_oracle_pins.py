"""The CPU oracle against facts outside itself (paper tables and worked
examples, closed forms, brute force, invariants, cross-formulation)."""
import pytest

from oracle import oracle as O
from tests import oracle_pins as P


@pytest.fixture(scope="module")
def lib():
    return O.build(force=False)


@pytest.mark.parametrize("check", P.FAST_CHECKS, ids=lambda c: c.__name__)
def test_pin(lib, check):
    assert check(lib) == []


def test_bruteforce_dense_time_definition(lib):
    assert P.check_bruteforce_o3(lib, cases_per_type=250, seed=11) == []


def test_exhaustive_short_waveform_pairs(lib):
    assert P.check_exhaustive_pairs(lib) == []


def test_python_gate_functions_match_table1():
    """The possibility-reading gate functions used by O2/O3 against Table 1."""
    t = P.table1()
    for name, gt in (("AND", O.AND2), ("OR", O.OR2), ("XOR", O.XOR2)):
        for a in range(4):
            for b in range(4):
                assert O.gate_eval(gt, [a, b]) == t[name][a][b]


def test_o2_o3_agree_on_small_circuits():
    for seed in range(6):
        nl, st = P._small_circuit(seed + 500, G=16, S=4, L=4, dmin=0, dmax=3, n=5, window=20)
        assert O.o2_simulate(nl, st) == O.o3_simulate(nl, st)


def test_o1_o2_on_tiny_config_prefix(lib):
    from paper_2304_13398_amd import workloads as W
    nl, st = W.config1(seed=2)
    sub = nl.prefix(150)
    assert P.o1_lists(sub, st, lib) == O.o2_simulate(sub, st)


def test_cycle_is_rejected(lib):
    nl = P.netlist_of(1, [(O.AND2, [0, 2]), (O.BUF, [1])], [1, 1, 1], [1, 1, 1])
    st = P.stimulus_of([[(0, 1)]])
    with pytest.raises(O.OracleError):
        O.o1_simulate(nl, st, lib)
