"""The waveform fingerprint used for large parity checks: the C oracle's
implementation, the test helper's, and the whole-netlist memory-light oracle
mode agree; permuting or changing a transition changes it."""
import numpy as np

from oracle import oracle as O
from paper_2304_13398_amd import workloads as W
from tests import net_hash


def test_c_and_numpy_fingerprints_agree():
    nl, st = W.config1(seed=2)
    off, t, v = O.o1_simulate(nl, st)
    assert np.array_equal(O.o1_fingerprints_of(off, t, v), net_hash.fingerprints(off, t, v))


def test_memory_light_oracle_matches_full_oracle():
    nl, st = W.config2(G=4000, S=32, L=30, n_per_src=300)
    off, t, v = O.o1_simulate(nl, st)
    ln, fp = O.o1_simulate_fingerprints(nl, st)
    assert np.array_equal(ln, np.diff(off))
    assert np.array_equal(fp, net_hash.fingerprints(off, t, v))


def test_fingerprint_sees_order_and_values():
    off = np.array([0, 3, 3])
    t = np.array([1, 5, 9])
    v = np.array([1, 0, 2], dtype=np.uint8)
    base = net_hash.fingerprints(off, t, v)
    assert base[1] == net_hash.mix(np.uint64(0))  # empty waveform
    assert net_hash.fingerprints(off, t, np.array([1, 2, 0], dtype=np.uint8))[0] != base[0]
    assert net_hash.fingerprints(off, np.array([1, 6, 9]), v)[0] != base[0]


def test_skewed_lengths_hit_the_target_cv():
    import numpy as np
    from paper_2304_13398_amd import workloads as W
    for wcv in (2.0, 5.0, 20.0):
        st = W.make_stimulus_skewed(S=2048, mean_per_src=300, wcv=wcv, window=1_000_000, seed=3)
        n = np.diff(st.off)
        assert abs(n.std() / n.mean() - wcv) < 0.02 * wcv
        assert abs(int(n.sum()) - 2048 * 300) < 2048
        assert n.max() <= 1_000_001
        again = W.make_stimulus_skewed(S=2048, mean_per_src=300, wcv=wcv, window=1_000_000, seed=3)
        assert np.array_equal(st.t, again.t) and np.array_equal(st.v, again.v)
