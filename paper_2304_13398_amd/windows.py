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
    since every window starts at X). Vectorised over all sources."""
    off = np.asarray(st.off, dtype=np.int64)
    t = np.asarray(st.t, dtype=np.int64)
    v = np.asarray(st.v, dtype=np.uint8)
    a, b = off[:S], off[1:S + 1]
    before = np.concatenate([[0], np.cumsum(t < t_lo)])     # per source: transitions before t_lo
    below = np.concatenate([[0], np.cumsum(t < t_hi)])      # ... and before t_hi
    i0 = a + (before[b] - before[a])
    i1 = a + (below[b] - below[a])
    has = i1 > i0
    first_t = np.where(has, t[np.minimum(i0, max(len(t) - 1, 0))] if len(t) else 0, -1)
    first_v = np.where(has, v[np.minimum(i0, max(len(v) - 1, 0))] if len(v) else 0, 0)
    prev_v = np.where(i0 > a, v[np.maximum(i0 - 1, 0)] if len(v) else 2, 2)
    add = (i0 > a) & (prev_v != 2) & ~(has & (first_t == t_lo))   # the held value, at t_lo
    drop = ~add & has & (first_v == 2)                             # a change to X at t_lo
    start = i0 + drop                                              # first kept transition
    n_keep = i1 - start
    counts = n_keep + add
    out_off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(counts, out=out_off[1:])
    out_t = np.empty(int(out_off[-1]), dtype=np.int64)
    out_v = np.empty(int(out_off[-1]), dtype=np.uint8)
    ia = np.nonzero(add)[0]
    out_t[out_off[ia]] = t_lo
    out_v[out_off[ia]] = prev_v[ia]
    # kept transitions: source s's [start_s, i1_s) to [out_off_s + add_s, ...)
    src = np.repeat(np.arange(S, dtype=np.int64), n_keep)
    k = np.arange(int(n_keep.sum()), dtype=np.int64) - np.repeat(np.cumsum(n_keep) - n_keep, n_keep)
    out_t[out_off[src] + add[src] + k] = t[start[src] + k]
    out_v[out_off[src] + add[src] + k] = v[start[src] + k]
    return W.Stimulus(out_off, out_t, out_v)


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
    # each window keeps its gates' transitions in [lo, hi); gate g's pieces
    # follow each other in window (time) order: a scatter, no sort
    G = nl.G
    kept = []
    counts = np.zeros((len(wins), G), dtype=np.int64)
    for k, ((lo, hi, _), (off, t, v)) in enumerate(zip(wins, results)):
        off = np.asarray(off, dtype=np.int64)
        t = np.asarray(t, dtype=np.int64)
        # the kept part of each gate's sorted list is [off_g + below(lo), off_g + below(hi))
        def below(x):
            if x is None:
                return None
            c = np.concatenate([[0], np.cumsum(t < x)])
            return c[off[1:]] - c[off[:-1]]
        n = np.diff(off)
        lo_n = np.zeros(G, dtype=np.int64) if lo is None else below(lo)
        hi_n = n if hi is None else below(hi)
        counts[k] = hi_n - lo_n
        kept.append((off[:-1] + lo_n, t, np.asarray(v, dtype=np.uint8)))
    out_off = np.zeros(G + 1, dtype=np.int64)
    np.cumsum(counts.sum(axis=0), out=out_off[1:])
    out_t = np.empty(int(out_off[-1]), dtype=np.int64)
    out_v = np.empty(int(out_off[-1]), dtype=np.uint8)
    dest0 = out_off[:-1].copy()
    for k, (src0, t, v) in enumerate(kept):
        c = counts[k]
        gid = np.repeat(np.arange(G, dtype=np.int64), c)
        r = np.arange(int(c.sum()), dtype=np.int64) - np.repeat(np.cumsum(c) - c, c)
        out_t[dest0[gid] + r] = t[src0[gid] + r]
        out_v[dest0[gid] + r] = v[src0[gid] + r]
        dest0 += c
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
