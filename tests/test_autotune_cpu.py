"""The autotuner's table key on the CPU: stimuli of one netlist differ in
their key by mean source waveform length and by the unevenness of source
activity (WCV), the two stimulus properties on which the best setting was
measured to change."""
import numpy as np

from paper_2304_13398_amd import autotune
from paper_2304_13398_amd import workloads as W


def test_skew_bucket_by_wcv():
    S = 512
    uniform = W.make_stimulus(S=S, n_per_src=200, window=1_000_000, seed=1)
    assert autotune.skew_bucket(uniform, S) == 0
    seen = []
    for wcv in (1.5, 3.0, 5.0, 20.0):
        st = W.make_stimulus_skewed(S=S, mean_per_src=200, wcv=wcv, window=1_000_000, seed=2)
        n = np.diff(st.off)
        measured = n.std() / n.mean()
        assert autotune.skew_bucket(st, S) == 1 + int(np.floor(np.log2(measured))), (wcv, measured)
        seen.append(autotune.skew_bucket(st, S))
    assert seen == sorted(seen) and len(set(seen)) == 4  # one bucket per doubling


def test_length_bucket_is_log2_of_mean_length():
    S = 256
    for n_per_src, bucket in ((16, 4), (1000, 10), (3000, 12)):
        st = W.make_stimulus(S=S, n_per_src=n_per_src, window=10_000_000, seed=3)
        assert autotune.length_bucket(st, S) == bucket
