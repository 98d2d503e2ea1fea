"""Autotuner for the evaluate path.

Knobs, each with a measurable effect that depends on the netlist and on how
long its waveforms are:

* schedule (GSIM_OPT_SCHEDULE): level by level, with every admitted job's
  level in shared launches, or dependency-driven, one persistent launch per
  job with no level barrier (wins on small or unevenly active netlists), or
  the level order in one persistent launch with a device-wide barrier per
  level (no launch chain);
* evaluation form of the level schedule (GSIM_OPT_EVAL_FORM): merged
  positions or time segments per lane;
* dynamic-binning threshold (GSIM_OPT_LANE_THRESHOLD): gates whose inputs hold
  fewer transitions than it run one per lane instead of one per wavefront;
* tickets per claim of the dependency-driven schedule (GSIM_OPT_DF_TICKETS):
  more cut the contended atomics, fewer keep light gates from waiting behind
  heavy ones.

The tuner times each candidate setting on a sample job and keeps the
fastest, per (netlist, stimulus length bucket, source skew bucket), applying it to the netlist
with sim_set_netlist_option. Results are cached in memory and, if a path is
given, in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

import numpy as np

from . import gsim as G

# (schedule, evaluation form, lane threshold, dependency-driven tickets per claim; 0 = automatic)
CANDIDATES = (
    (G.SCHEDULE_LEVELS, G.FORM_MERGED, 0, 0),
    (G.SCHEDULE_LEVELS, G.FORM_MERGED, 64, 0),
    (G.SCHEDULE_LEVELS, G.FORM_MERGED, 512, 0),
    (G.SCHEDULE_LEVELS, G.FORM_SEGMENTED, 0, 0),
    (G.SCHEDULE_DEPENDENCY, G.FORM_MERGED, 0, 0),
    (G.SCHEDULE_DEPENDENCY, G.FORM_MERGED, 0, 4),
    (G.SCHEDULE_LEVEL_BARRIERS, G.FORM_MERGED, 0, 0),
)
SCHEDULE_NAMES = {G.SCHEDULE_LEVELS: "levels", G.SCHEDULE_DEPENDENCY: "dataflow",
                  G.SCHEDULE_LEVEL_BARRIERS: "levelsync"}
FORM_NAMES = {G.FORM_MERGED: "merged", G.FORM_SEGMENTED: "segmented"}


def setting_name(c) -> str:
    if c[0] == G.SCHEDULE_DEPENDENCY:
        return f"dataflow/tickets{c[3] if c[3] else 'auto'}"
    if c[0] == G.SCHEDULE_LEVEL_BARRIERS:
        return "levelsync"
    return f"levels/{FORM_NAMES[c[1]]}/lane{c[2]}"


def netlist_key(nl) -> str:
    h = hashlib.sha1()
    for a in (nl.type, nl.pin_off, nl.pin_net, nl.rise, nl.fall):
        h.update(np.ascontiguousarray(a).tobytes())
    return f"G{nl.G}-S{nl.S}-{h.hexdigest()[:12]}"


def length_bucket(st, S: int) -> int:
    """log2 of the mean source waveform length, rounded."""
    mean = st.n / max(S, 1)
    return int(round(math.log2(max(mean, 1.0))))


def skew_bucket(st, S: int) -> int:
    """Unevenness of the sources' activity (the coefficient of variation of
    their transition counts, the paper's WCV): 0 below 1, then one bucket per
    doubling (1 + floor(log2 WCV)). The two schedules cross near WCV 2.4 on
    the mid-size netlist, and the level schedule's loss grows with WCV."""
    n = np.diff(np.asarray(st.off[:S + 1], dtype=np.int64))
    m = n.mean() if len(n) else 0.0
    wcv = float(n.std() / m) if m > 0 else 0.0
    return 0 if wcv < 1.0 else 1 + int(math.floor(math.log2(wcv)))


class Autotuner:
    def __init__(self, sim: G.Sim, path: str | None = None, candidates=CANDIDATES, reps: int = 2):
        self.sim = sim
        self.path = path
        self.candidates = tuple(tuple(c) for c in candidates)
        self.reps = reps
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def apply(self, h, c):
        self.sim.set_netlist_option(h, G.OPT_SCHEDULE, c[0])
        self.sim.set_netlist_option(h, G.OPT_EVAL_FORM, c[1])
        self.sim.set_netlist_option(h, G.OPT_LANE_THRESHOLD, c[2])
        self.sim.set_netlist_option(h, G.OPT_DF_TICKETS, c[3] if c[3] else -1)

    def clear(self, h):
        """Back to the context's settings on ``h``."""
        for opt in (G.OPT_SCHEDULE, G.OPT_EVAL_FORM, G.OPT_LANE_THRESHOLD, G.OPT_DF_TICKETS):
            self.sim.set_netlist_option(h, opt, -1)

    def _time(self, h, st, c):
        self.apply(h, c)
        best = float("inf")
        for _ in range(self.reps):
            j = self.sim.run(h, st)
            self.sim.wait(j)
            best = min(best, self.sim.stats(j).device_ms)
            self.sim.release(j)
        return best

    def tune(self, nl, h, st):
        """Pick the setting for netlist ``nl`` (loaded as ``h``) on stimuli like
        ``st``; applies it to ``h`` and returns (setting, device ms by
        candidate name)."""
        key = f"{netlist_key(nl)}/b{length_bucket(st, nl.S)}/s{skew_bucket(st, nl.S)}"
        if key in self.table:
            c = tuple(self.table[key]["setting"])
            self.apply(h, c)
            return c, self.table[key]["ms"]
        ms = {setting_name(c): self._time(h, st, c) for c in self.candidates}
        c = min(self.candidates, key=lambda x: ms[setting_name(x)])
        self.apply(h, c)
        self.table[key] = {"setting": list(c), "name": setting_name(c), "ms": ms}
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.table, f, indent=1)
        return c, ms
