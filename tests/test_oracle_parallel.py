"""The level-parallel O1 driver (used to time the oracle on several cores)
gives exactly the result of the sequential O1, whatever the thread count."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import workloads as W

from tests import net_hash
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


@pytest.mark.parametrize("threads", [1, 5, 16])
def test_parallel_fingerprints_equal_the_sequential_oracle(threads):
    """The level-parallel memory-light driver used by the full-size parity
    tests: lengths and fingerprints equal those of the sequential O1's full
    waveforms (and of the sequential memory-light driver), and the kept gates
    come back transition for transition, in the order asked."""
    nl, st = W.config2(seed=6, G=20_000, S=64, L=12, n_per_src=300)
    off, t, v = O.o1_simulate(nl, st)
    keep = np.random.default_rng(threads).choice(nl.G, size=200, replace=False)
    ln, fp, (k_off, k_t, k_v) = O.o1_simulate_fingerprints_parallel(nl, st, threads, keep=keep)
    assert np.array_equal(ln, np.diff(off))
    assert np.array_equal(fp, net_hash.fingerprints(off, t, v))
    s_ln, s_fp = O.o1_simulate_fingerprints(nl, st)
    assert np.array_equal(ln, s_ln) and np.array_equal(fp, s_fp)
    for i, g in enumerate(keep.tolist()):
        assert np.array_equal(k_t[k_off[i]:k_off[i + 1]], t[off[g]:off[g + 1]])
        assert np.array_equal(k_v[k_off[i]:k_off[i + 1]], v[off[g]:off[g + 1]])


def test_parallel_fingerprints_without_a_sample_and_on_a_cycle():
    nl, st = W.config1(seed=3)
    off, t, v = O.o1_simulate(nl, st)
    ln, fp, (k_off, _, _) = O.o1_simulate_fingerprints_parallel(nl, st, 4)
    assert np.array_equal(ln, np.diff(off)) and len(k_off) == 1
    assert np.array_equal(fp, net_hash.fingerprints(off, t, v))
    cyc = P.netlist_of(1, [(O.AND2, [0, 2]), (O.BUF, [1])], [1, 1, 1], [1, 1, 1])
    with pytest.raises(O.OracleError):
        O.o1_simulate_fingerprints_parallel(cyc, P.stimulus_of([[(0, 1)]]), 2)
