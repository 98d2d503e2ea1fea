"""Autotuner for the evaluate path.

The tunable is the dynamic-binning threshold (GSIM_OPT_LANE_THRESHOLD): gates
whose inputs hold fewer transitions than the threshold run one per lane
instead of one per wavefront. Which is faster depends on the netlist (fan-in
mix, delays) and on how long the waveforms are, so the tuner times candidate
thresholds on a sample job and keeps the fastest, per (netlist, stimulus
length bucket). Results are cached in memory and, if a path is given, in a
JSON file.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

import numpy as np

from . import gsim as G

CANDIDATES = (0, 64, 192, 512, 2048)


def netlist_key(nl) -> str:
    h = hashlib.sha1()
    for a in (nl.type, nl.pin_off, nl.pin_net, nl.rise, nl.fall):
        h.update(np.ascontiguousarray(a).tobytes())
    return f"G{nl.G}-S{nl.S}-{h.hexdigest()[:12]}"


def length_bucket(st, S: int) -> int:
    """log2 of the mean source waveform length, rounded."""
    mean = st.n / max(S, 1)
    return int(round(math.log2(max(mean, 1.0))))


class Autotuner:
    def __init__(self, sim: G.Sim, path: str | None = None, candidates=CANDIDATES, reps: int = 2):
        self.sim = sim
        self.path = path
        self.candidates = tuple(candidates)
        self.reps = reps
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def _time(self, h, st, threshold):
        self.sim.set_netlist_option(h, G.OPT_LANE_THRESHOLD, threshold)
        best = float("inf")
        for _ in range(self.reps):
            j = self.sim.run(h, st)
            self.sim.wait(j)
            best = min(best, self.sim.stats(j).device_ms)
            self.sim.release(j)
        return best

    def tune(self, nl, h, st):
        """Pick the lane threshold for netlist ``nl`` (loaded as ``h``) on
        stimuli like ``st``; applies it to ``h`` and returns (threshold, ms by
        candidate)."""
        key = f"{netlist_key(nl)}/b{length_bucket(st, nl.S)}"
        if key in self.table:
            thr = int(self.table[key]["threshold"])
            self.sim.set_netlist_option(h, G.OPT_LANE_THRESHOLD, thr)
            return thr, self.table[key]["ms"]
        ms = {str(c): self._time(h, st, c) for c in self.candidates}
        thr = int(min(ms, key=ms.get))
        self.sim.set_netlist_option(h, G.OPT_LANE_THRESHOLD, thr)
        self.table[key] = {"threshold": thr, "ms": ms}
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.table, f, indent=1)
        return thr, ms
