"""Waveform fingerprints in NumPy (test helper): fp = mix(n) + sum_i
mix(key_i ^ mix(i)) mod 2^64, key_i = time_i << 2 | value_i, mix = the
SplitMix64 finaliser -- the definition the library's sim_fetch_hashes states."""
import numpy as np

_U = np.uint64


def mix(x):
    with np.errstate(over="ignore"):  # arithmetic mod 2^64 by definition
        x = np.asarray(x, dtype=np.uint64) + _U(0x9E3779B97F4A7C15)
        x = (x ^ (x >> _U(30))) * _U(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> _U(27))) * _U(0x94D049BB133111EB)
        return x ^ (x >> _U(31))


def fingerprints(off, t, v):
    off = np.asarray(off, dtype=np.int64)
    n = np.diff(off)
    key = (np.asarray(t, dtype=np.int64).astype(np.uint64) << _U(2)) | np.asarray(v, dtype=np.uint64)
    idx = (np.arange(len(key), dtype=np.int64) - np.repeat(off[:-1], n)).astype(np.uint64)
    with np.errstate(over="ignore"):
        terms = mix(key ^ mix(idx))
        cs = np.concatenate([np.zeros(1, dtype=np.uint64), np.cumsum(terms, dtype=np.uint64)])
        return (cs[off[1:]] - cs[off[:-1]]) + mix(n.astype(np.uint64))
