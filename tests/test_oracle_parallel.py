"""The level-parallel O1 driver (used to time the oracle on several cores)
gives exactly the result of the sequential O1, whatever the thread count."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import workloads as W

from tests import oracle_pins as P


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_equals_sequential_tiny(threads):
    nl, st = W.config1(seed=4)
    ref = O.o1_simulate(nl, st)
    got = O.o1_simulate(nl, st, threads=threads)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_parallel_equals_sequential_mid_shaped():
    nl, st = W.config2(seed=6, G=20_000, S=64, L=12, n_per_src=300)
    ref = O.o1_simulate(nl, st)
    got = O.o1_simulate(nl, st, threads=7)
    assert int(ref[0][-1]) > 100_000
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_parallel_rejects_a_cycle():
    nl = P.netlist_of(1, [(O.AND2, [0, 2]), (O.BUF, [1])], [1, 1, 1], [1, 1, 1])
    st = P.stimulus_of([[(0, 1)]])
    with pytest.raises(O.OracleError):
        O.o1_simulate(nl, st, threads=4)
