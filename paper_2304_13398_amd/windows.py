"""Exact time-window chunking of one re-simulation job.

A gate's output at time T depends on its inputs only through the gate value
just before some earlier time A and the input transitions after A, as soon as
T >= A + D_max + 1 (D_max: the gate's largest pin delay). Every candidate
decided before A appears by A + D_max, and the last one's value is the gate
value at A; Eq. 1 only lets later candidates deny earlier ones. Applied level
by level, every net is exact from T_k on when its window's sources are
exact from T_k - H, with

    H = max over source-to-gate paths of the sum of (D_max(g) + 1) + 1.

So the stimulus can be cut into windows [T_k, T_(k+1)): window k runs the
whole netlist on the source transitions in [T_k - H, T_(k+1)), each source
starting with the value it holds at T_k - H, and keeps the transitions of
every gate that fall in [T_k, T_(k+1)). Outputs before T_(k+1) depend only on
inputs before it (an output appears no earlier than its cause, and a later
candidate can only deny outputs that appear at or after it), and each
window's list is already free of repeats at T_k (the value just before T_k is
exact within the window), so the windows' pieces concatenate into the full
result with no seam repair.

Uses: jobs whose output does not fit the HBM budget at once (windows run one
after another, each fetched before the next), and the multi-GPU split of one
job (one window per GPU, no exchange between them).

``run`` is any engine mapping a stimulus to the gate waveforms (off[G+1], t,
v) of the netlist: the GPU library in the product path.
"""
from __future__ import annotations

import numpy as np

from . import workloads as W


def window_halo(nl) -> int:
    """H for the netlist: longest source-to-gate path in sum of (D_max + 1),
    plus one. Gates are visited in level order (levels from the library's own
    levelizer, so any valid netlist works)."""
    from . import gsim as G
    level, n_levels = G.levelize(nl.S, nl.G, nl.type, nl.pin_off, nl.pin_net, nl.rise, nl.fall)
    dmax = np.zeros(nl.G, dtype=np.int64)
    arity = np.diff(nl.pin_off)
    pin_gate = np.repeat(np.arange(nl.G), arity)
    np.maximum.at(dmax, pin_gate, np.maximum(nl.rise, nl.fall).astype(np.int64))
    dist = np.zeros(nl.S + nl.G, dtype=np.int64)
    order = np.argsort(level, kind="stable")
    bounds = np.searchsorted(level[order], np.arange(1, n_levels + 2))
    for lv in range(n_levels):
        gates = order[bounds[lv]:bounds[lv + 1]]
        if len(gates) == 0:
            continue
        pins = np.concatenate([np.arange(nl.pin_off[g], nl.pin_off[g + 1]) for g in gates])
        owner = pin_gate[pins]
        best = np.zeros(nl.G, dtype=np.int64)
        np.maximum.at(best, owner, dist[nl.pin_net[pins]])
        dist[nl.S + gates] = best[gates] + dmax[gates] + 1
    return int(dist.max()) + 1 if nl.G else 1


def window_stimulus(st, S, t_lo, t_hi) -> W.Stimulus:
    """Source transitions in [t_lo, t_hi), each source first set to the value
    it holds at t_lo (a transition at t_lo, unless that value is X or the
    source already changes at t_lo; a change to X exactly at t_lo is dropped,
    since every window starts at X)."""
    offs, ts, vs = [0], [], []
    for s in range(S):
        a, b = int(st.off[s]), int(st.off[s + 1])
        t, v = st.t[a:b], st.v[a:b]
        i0 = int(np.searchsorted(t, t_lo, side="left"))
        i1 = int(np.searchsorted(t, t_hi, side="left"))
        tt, vv = t[i0:i1], v[i0:i1]
        if i0 > 0 and v[i0 - 1] != 2 and (len(tt) == 0 or tt[0] != t_lo):
            tt = np.concatenate([[t_lo], tt])
            vv = np.concatenate([[v[i0 - 1]], vv])
        elif len(tt) and vv[0] == 2:  # a change to X exactly at t_lo: the window starts at X
            tt, vv = tt[1:], vv[1:]
        ts.append(tt)
        vs.append(vv)
        offs.append(offs[-1] + len(tt))
    t = np.concatenate(ts).astype(np.int64) if ts else np.zeros(0, np.int64)
    v = np.concatenate(vs).astype(np.uint8) if vs else np.zeros(0, np.uint8)
    return W.Stimulus(np.asarray(offs, dtype=np.int64), t, v)


def window_bounds(st, n_windows: int) -> list[int]:
    """Inner boundaries T_1 < ... < T_(n-1) at quantiles of the source
    transition times (equal input volume per window)."""
    if n_windows <= 1 or st.n == 0:
        return []
    ts = np.sort(st.t)
    qs = [int(ts[min(len(ts) - 1, (k * len(ts)) // n_windows)]) for k in range(1, n_windows)]
    return sorted(set(q for q in qs if q > 0))


def window_stimuli(nl, st, n_windows: int, halo: int | None = None):
    """The windows' ranges [lo, hi) (None: open) and their stimuli."""
    H = window_halo(nl) if halo is None else halo
    inner = window_bounds(st, n_windows)
    edges = [None] + inner + [None]
    out = []
    for k in range(len(edges) - 1):
        lo, hi = edges[k], edges[k + 1]
        if lo is None and hi is None:
            sub = st
        else:
            t_lo = 0 if lo is None else max(0, lo - H)
            t_hi = np.iinfo(np.int64).max if hi is None else hi
            sub = window_stimulus(st, nl.S, t_lo, t_hi)
        out.append((lo, hi, sub))
    return out


def simulate_windowed(nl, st, run, n_windows: int, halo: int | None = None, run_many=None):
    """The job's gate waveforms assembled from ``n_windows`` independent runs.
    Returns (off[G+1], t, v) in gate order, like one run of the whole job.
    ``run`` maps one window's stimulus to its gate waveforms; ``run_many``,
    if given, maps the list of all windows' stimuli to the list of results
    (so the windows can run together)."""
    wins = window_stimuli(nl, st, n_windows, halo)
    results = run_many([w[2] for w in wins]) if run_many is not None else [run(w[2]) for w in wins]
    gid_parts, t_parts, v_parts = [], [], []
    for (lo, hi, _), (off, t, v) in zip(wins, results):
        gid = np.repeat(np.arange(nl.G, dtype=np.int64), np.diff(off))
        keep = np.ones(len(t), dtype=bool)
        if lo is not None:
            keep &= t >= lo
        if hi is not None:
            keep &= t < hi
        gid_parts.append(gid[keep])
        t_parts.append(t[keep])
        v_parts.append(v[keep])
    gid = np.concatenate(gid_parts) if gid_parts else np.zeros(0, np.int64)
    order = np.argsort(gid, kind="stable")  # windows are in time order: stable keeps it
    out_off = np.zeros(nl.G + 1, dtype=np.int64)
    np.cumsum(np.bincount(gid, minlength=nl.G)[:nl.G], out=out_off[1:])
    out_t = np.concatenate(t_parts)[order].astype(np.int64)
    out_v = np.concatenate(v_parts)[order].astype(np.uint8)
    return out_off, out_t, out_v


def gpu_engine(sim, nl):
    """Engine for ``simulate_windowed``: the library on one resident netlist.
    Returns (run, run_many, close): run_many submits every window at once and
    lets the executor advance them in shared launches."""
    h = sim.load_netlist(nl)
    gates = np.arange(nl.S, nl.S + nl.G)

    def run(sub):
        j = sim.run(h, sub)
        try:
            sim.wait(j)
            return sim.fetch(j, gates)
        finally:
            sim.release(j)

    def run_many(subs):
        jobs = [sim.submit(h, sub) for sub in subs]
        try:
            for j in jobs:
                sim.wait(j)
            return [sim.fetch(j, gates) for j in jobs]
        finally:
            for j in jobs:
                sim.release(j)

    def close():
        sim.unload_netlist(h)

    return run, run_many, close
