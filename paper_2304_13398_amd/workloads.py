"""Seeded synthetic workloads: combinational netlists and source waveforms.

This module only draws inputs. It holds none of the simulation's arithmetic
(no gate function, no delay rule, no merge): the same arrays are handed to the
HIP library and to the CPU oracle, and each computes on them independently.

The paper measures on re-simulation designs that are not available here
(Section 5, Table 2); the workloads below stand in for them with the shapes
the benchmark configurations name: a levelled random DAG of basic gates with
per-pin rise/fall delays, power-law fanout, and 0/1/X/Z source waveforms with
strictly increasing times and no repeated consecutive values.

Conventions shared by every consumer of these arrays:
  * nets ``[0, S)`` are sources (primary and pseudo-primary inputs), gate ``g``
    drives net ``S + g``;
  * values are ``uint8`` codes 0, 1, X=2, Z=3; times are ``int64`` ps;
    delays are ``int32`` ps;
  * a gate's pins are ``pin_net[pin_off[g]:pin_off[g+1]]`` in the pin order of
    its type (MUX2: d0, d1, s).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Gate type codes of the C ABI (include/gsim.h).
BUF, NOT, AND2, OR2, NAND2, NOR2, XOR2, XNOR2, AND3, MUX2, AND4, OR4 = range(12)
TYPE_NAMES = ("BUF", "NOT", "AND2", "OR2", "NAND2", "NOR2", "XOR2", "XNOR2",
              "AND3", "MUX2", "AND4", "OR4")
# Pin count of each type: a property of the netlist format, needed to draw pins.
ARITY = np.array([1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 4, 4], dtype=np.int64)

TYPES_TINY = np.array([BUF, NOT, AND2, OR2, NAND2, NOR2, XOR2, XNOR2, AND3, MUX2])
TYPES_ALL = np.arange(12)

V0, V1, VX, VZ = 0, 1, 2, 3


@dataclasses.dataclass
class Netlist:
    S: int
    G: int
    type: np.ndarray      # uint8 [G]
    pin_off: np.ndarray   # int64 [G+1]
    pin_net: np.ndarray   # int64 [P]
    rise: np.ndarray      # int32 [P]
    fall: np.ndarray      # int32 [P]
    level: np.ndarray     # int32 [G], the level the generator built the gate at
    name: str = ""

    @property
    def P(self) -> int:
        return int(self.pin_off[-1])

    def prefix(self, n_gates: int) -> "Netlist":
        """The sub-netlist of the first ``n_gates`` gates.

        Gates are generated level by level and only read nets of lower levels,
        so any prefix is a closed netlist over the same sources.
        """
        p = int(self.pin_off[n_gates])
        return Netlist(self.S, n_gates, self.type[:n_gates], self.pin_off[:n_gates + 1],
                       self.pin_net[:p], self.rise[:p], self.fall[:p],
                       self.level[:n_gates], self.name + f"[:{n_gates}]")


@dataclasses.dataclass
class Stimulus:
    off: np.ndarray   # int64 [S+1]
    t: np.ndarray     # int64 [N_in]
    v: np.ndarray     # uint8 [N_in]

    @property
    def n(self) -> int:
        return int(self.off[-1])


def _child_rngs(seed: int, n: int):
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(n)]


def _powerlaw_weights(rng, n, alpha=2.2, wmax=1000):
    w = np.arange(1, wmax + 1, dtype=np.float64)
    p = w ** (-alpha)
    p /= p.sum()
    return rng.choice(np.arange(1, wmax + 1), size=n, p=p).astype(np.float64)


def _level_sizes(G, L):
    base, rem = divmod(G, L)
    return np.array([base + (1 if i < rem else 0) for i in range(L)], dtype=np.int64)


def _draw_weighted(rng, lo, hi, weight, count):
    """``count`` net ids from [lo, hi), each with probability proportional to weight."""
    if count == 0:
        return np.empty(0, dtype=np.int64)
    c = np.cumsum(weight[lo:hi])
    total = c[-1]
    if total <= 0:
        raise RuntimeError("no eligible net left for a pin")
    u = rng.random(count) * total
    return lo + np.searchsorted(c, u, side="right").astype(np.int64)


def _assign_pins(rng, lo, hi, weight, fanout, cap, count):
    """Weighted draw with a fanout cap: a net whose fanout reaches ``cap`` stops
    being eligible, and the draws beyond the cap are drawn again."""
    out = _draw_weighted(rng, lo, hi, weight, count)
    if cap is None:
        np.add.at(fanout, out, 1)
        return out
    todo = np.arange(count)
    while True:
        nets = out[todo]
        room = cap - fanout[lo:hi]
        cnt = np.bincount(nets - lo, minlength=hi - lo)
        if not (cnt > room).any():
            fanout[lo:hi] += cnt
            return out
        # keep a uniformly chosen `room` of the draws of each over-full net
        perm = rng.permutation(len(todo))
        nets_p = nets[perm]
        order = np.argsort(nets_p, kind="stable")
        srt = nets_p[order]
        rank_p = np.empty(len(todo), dtype=np.int64)
        rank_p[order] = np.arange(len(todo)) - np.searchsorted(srt, srt, side="left")
        keep = np.empty(len(todo), dtype=bool)
        keep[perm] = rank_p < room[nets_p - lo]
        fanout[lo:hi] += np.bincount(nets[keep] - lo, minlength=hi - lo)
        weight[lo:hi][fanout[lo:hi] >= cap] = 0.0
        todo = todo[~keep]
        out[todo] = _draw_weighted(rng, lo, hi, weight, len(todo))


def make_netlist(*, G, S, L, types, dmin=1, dmax=50, powerlaw=False, fanout_cap=None,
                 strict=False, seed=1, name="") -> Netlist:
    """Levelled random DAG.

    Gate types are uniform over ``types``. One randomly chosen pin of a level-l
    gate reads a net of level l-1 (sources are level 0), the other pins read
    nets of any level below l. With ``powerlaw`` every net draws a weight
    w ~ P(w) proportional to w^-2.2 on [1, 1000] and pins pick nets with
    probability proportional to w; ``fanout_cap`` bounds each net's fanout.
    Per-pin rise and fall delays are uniform integers in [dmin, dmax].
    With ``strict`` every pin of a level-l gate reads a net of level l-1.
    """
    r_type, r_pin, r_delay, r_weight = _child_rngs(seed, 4)
    sizes = _level_sizes(G, L)
    gtype = r_type.choice(np.asarray(types), size=G).astype(np.uint8)
    arity = ARITY[gtype]
    pin_off = np.zeros(G + 1, dtype=np.int64)
    np.cumsum(arity, out=pin_off[1:])
    P = int(pin_off[-1])
    N = S + G
    weight = _powerlaw_weights(r_weight, N) if powerlaw else np.ones(N)
    fanout = np.zeros(N, dtype=np.int64)
    pin_net = np.empty(P, dtype=np.int64)
    level = np.repeat(np.arange(1, L + 1, dtype=np.int32), sizes)
    lvl_start = np.concatenate([[0, S], S + np.cumsum(sizes)])  # first net id of each level
    g0 = 0
    for lv in range(1, L + 1):
        g1 = g0 + int(sizes[lv - 1])
        a = arity[g0:g1]
        first = pin_off[g0:g1]
        prim = first + (r_pin.random(g1 - g0) * a).astype(np.int64)
        allp = np.arange(pin_off[g0], pin_off[g1])
        is_prim = np.zeros(len(allp), dtype=bool)
        is_prim[prim - pin_off[g0]] = True
        others = allp[~is_prim]
        pin_net[prim] = _assign_pins(r_pin, lvl_start[lv - 1], lvl_start[lv], weight, fanout,
                                     fanout_cap, len(prim))
        pin_net[others] = _assign_pins(r_pin, lvl_start[lv - 1] if strict else 0,
                                       lvl_start[lv], weight, fanout, fanout_cap, len(others))
        g0 = g1
    rise = r_delay.integers(dmin, dmax + 1, size=P).astype(np.int32)
    fall = r_delay.integers(dmin, dmax + 1, size=P).astype(np.int32)
    return Netlist(S, G, gtype, pin_off, pin_net, rise, fall, level, name)


def _distinct_sorted_times(rng, rows, n, window):
    """``rows`` independent uniform n-subsets of the integers [0, window], sorted."""
    if n > window + 1:
        raise ValueError("more transitions than distinct times in the window")
    t = rng.integers(0, window + 1, size=(rows, n))
    t.sort(axis=1)
    while True:
        dup = np.zeros_like(t, dtype=bool)
        dup[:, 1:] = t[:, 1:] == t[:, :-1]
        k = int(dup.sum())
        if k == 0:
            return t
        t[dup] = rng.integers(0, window + 1, size=k)
        t.sort(axis=1)


def _values_no_repeat(rng, lengths, probs):
    """Values drawn from ``probs`` over {0,1,X,Z}; a value equal to the previous
    one of the same source (X before the first) is drawn again, all such
    positions at once, until none is left. Only redrawn positions and their
    successors can change status, so later passes look at those alone."""
    n = int(lengths.sum())
    v = rng.choice(4, size=n, p=probs).astype(np.uint8)
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    is_start = np.zeros(n + 1, dtype=bool)
    is_start[starts[lengths > 0]] = True

    def bad_among(idx):
        prev = np.where(is_start[idx], VX, v[np.maximum(idx - 1, 0)])
        return idx[v[idx] == prev]

    bad = bad_among(np.arange(n, dtype=np.int64))
    while len(bad):
        v[bad] = rng.choice(4, size=len(bad), p=probs).astype(np.uint8)
        cand = np.union1d(bad, bad + 1)
        cand = cand[cand < n]
        bad = bad_among(cand)
    return v


def make_stimulus(*, S, n_per_src, window, probs=(0.45, 0.45, 0.05, 0.05), seed=1) -> Stimulus:
    """Every source gets ``n_per_src`` transitions at distinct times in [0, window]."""
    r_t, r_v = _child_rngs(seed + 1_000_003, 2)
    t = _distinct_sorted_times(r_t, S, n_per_src, window).reshape(-1).astype(np.int64)
    lengths = np.full(S, n_per_src, dtype=np.int64)
    v = _values_no_repeat(r_v, lengths, np.asarray(probs))
    off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return Stimulus(off, t, v)


def skewed_lengths(rng, S, mean, wcv, cap):
    """Per-source transition counts with mean ``mean`` (so the total is
    S * mean up to rounding) and a coefficient of variation near ``wcv``:
    log-normal shape, its sigma found by bisection on the sample's own CV.
    Counts are capped at ``cap`` (the distinct times of the window)."""
    z = rng.standard_normal(S)

    def lengths(sigma):
        x = np.exp(sigma * (z - z.max()))  # scaled so the largest is 1: no overflow
        n = np.minimum(np.rint(mean * S * x / x.sum()), cap).astype(np.int64)
        return n

    def cv(n):
        return float(n.std() / n.mean()) if n.mean() > 0 else 0.0

    lo, hi = 0.0, 8.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if cv(lengths(mid)) < wcv:
            lo = mid
        else:
            hi = mid
    return lengths(0.5 * (lo + hi))


def make_stimulus_skewed(*, S, mean_per_src, wcv, window, probs=(0.45, 0.45, 0.05, 0.05),
                         seed=1) -> Stimulus:
    """Sources with uneven waveform lengths (the paper's WCV, Eq. 5: the
    coefficient of variation of the given waveforms' lengths): counts from
    ``skewed_lengths``, each source's times a uniform subset of [0, window]."""
    r_n, r_t, r_v = _child_rngs(seed + 2_000_029, 3)
    lengths = skewed_lengths(r_n, S, mean_per_src, wcv, window + 1)
    t = np.concatenate([np.sort(r_t.choice(window + 1, size=int(n), replace=False))
                        for n in lengths] + [np.zeros(0, dtype=np.int64)]).astype(np.int64)
    v = _values_no_repeat(r_v, lengths, np.asarray(probs))
    off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return Stimulus(off, t, v)


NO_RELATION = 2**31 - 1  # a delay entry of a pin unrelated to the output (the paper's inf)


def make_cell_model(nl, *, seed, edge_spread=0.5, inf_prob=0.0, n_udp=0, udp_frac=0.0):
    """The extended cell model over an existing netlist (delays by pin, input
    edge and output value; user-defined gate tables):

    * dly[p][edge][out], edge 0 = rise / 1 = fall, out 0 / 1: the pin's fall
      (out 0) or rise (out 1) delay times a factor drawn per entry from
      [1 - edge_spread, 1 + edge_spread]; each entry is NO_RELATION with
      probability inf_prob;
    * n_udp tables of 256 output values in {0, 1, X}, for arities 1-4 in
      turn; a fraction udp_frac of the gates whose pin count matches a table's
      arity switch to type 12 + that table.
    Returns (type[G] uint8, dly[P, 2, 2] int32, udp[n_udp, 256] uint8)."""
    r_d, r_i, r_u, r_g = _child_rngs(seed + 3_000_017, 4)
    P = nl.P
    base = np.stack([nl.fall, nl.rise], axis=1).astype(np.float64)        # [P, out]
    fac = r_d.uniform(1 - edge_spread, 1 + edge_spread, size=(P, 2, 2))
    dly = np.rint(base[:, None, :] * fac).astype(np.int64)
    dly = np.clip(dly, 0, NO_RELATION - 1).astype(np.int32)
    if inf_prob > 0:
        dly[r_i.random(size=(P, 2, 2)) < inf_prob] = NO_RELATION
    udp = r_u.choice(3, size=(n_udp, 256)).astype(np.uint8)
    arity = np.array([1 + u % 4 for u in range(n_udp)], dtype=np.int64)
    type_ = nl.type.copy()
    if n_udp and udp_frac > 0:
        k = np.diff(nl.pin_off)
        pick = r_g.random(nl.G) < udp_frac
        for g in np.nonzero(pick)[0]:
            cands = np.nonzero(arity == k[g])[0]
            if len(cands):
                type_[g] = 12 + int(cands[int(r_g.integers(len(cands)))])
    return type_, dly, udp


def with_types(nl, type_) -> "Netlist":
    return Netlist(nl.S, nl.G, np.asarray(type_, dtype=np.uint8), nl.pin_off, nl.pin_net,
                   nl.rise, nl.fall, nl.level, nl.name + "+cells")


# --------------------------------------------------------------------------
# The benchmark configurations.

def config1(seed=1):
    """Tiny: 1,000 gates, 32 PIs, 20 levels, 10 gate types, delays 1-50 ps,
    100 transitions per PI over [0, 10,000] ps."""
    nl = make_netlist(G=1000, S=32, L=20, types=TYPES_TINY, dmax=50, seed=seed,
                      name=f"cfg1-tiny-s{seed}")
    st = make_stimulus(S=32, n_per_src=100, window=10_000, seed=seed)
    return nl, st


def config2_netlist(G=1_000_000, S=2048, L=60, seed=1):
    """Mid: the generator at 1M gates, 2,048 PIs, 60 levels, fan-in 1-4,
    power-law fanout (alpha 2.2, cap 1,000), delays 1-50 ps."""
    return make_netlist(G=G, S=S, L=L, types=TYPES_ALL, dmax=50, powerlaw=True,
                        fanout_cap=1000, seed=seed, name=f"cfg2-mid-G{G}-s{seed}")


def config2(seed=1, G=1_000_000, S=2048, L=60, n_per_src=1000):
    nl = config2_netlist(G=G, S=S, L=L, seed=seed)
    st = make_stimulus(S=S, n_per_src=n_per_src, window=1_000_000, seed=seed)
    return nl, st


def config2_skewed(wcv, seed=1, G=1_000_000, S=2048, L=60, mean_per_src=1000):
    """The mid netlist with uneven source activity: the same 2,048,000 given
    transitions, per-source counts with coefficient of variation ``wcv``."""
    nl = config2_netlist(G=G, S=S, L=L, seed=seed)
    st = make_stimulus_skewed(S=S, mean_per_src=mean_per_src, wcv=wcv, window=1_000_000, seed=seed)
    return nl, st


def config3(seed=1, G=10_000_000, S=8192 + 50_000, L=150, n_per_src=200):
    """Industrial-shaped: 10M gates, 8,192 PIs + 50,000 pseudo-PIs, 150 levels,
    fanout cap 5,000, delays 1-200 ps, 200 transitions per source with 2% X/Z."""
    nl = make_netlist(G=G, S=S, L=L, types=TYPES_ALL, dmax=200, powerlaw=True,
                      fanout_cap=5000, seed=seed, name=f"cfg3-ind-G{G}-s{seed}")
    st = make_stimulus(S=S, n_per_src=n_per_src, window=1_000_000,
                       probs=(0.49, 0.49, 0.01, 0.01), seed=seed)
    return nl, st


def loguniform_int(rng, lo, hi, size=None):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


def config4_set_args(S=2048, n_sets=64, seed=1, lo=50, hi=5000, window=1_000_000):
    """Arguments of make_stimulus for each batched set: (S, n_s, window, seed_s)
    with n_s ~ round(exp U(ln lo, ln hi)) transitions on every PI."""
    rng = _child_rngs(seed + 7_000_001, 1)[0]
    ns = loguniform_int(rng, lo, hi, size=n_sets)
    return [(S, int(n), window, seed * 1000 + s) for s, n in enumerate(ns)]


def config4_sets(S=2048, n_sets=64, seed=1, lo=50, hi=5000, window=1_000_000):
    """Batched: ``n_sets`` stimulus sets, set s has n_s ~ round(exp U(ln lo, ln hi))
    transitions on every PI."""
    return [make_stimulus(S=a, n_per_src=n, window=w, seed=sd)
            for a, n, w, sd in config4_set_args(S, n_sets, seed, lo, hi, window)]


def config5_netlist_sizes():
    """Served: 8 resident netlists, G_i = round(1e4 * 200^(i/7)), S_i = max(32, round(2048 G_i / 1e6))."""
    G = [int(round(1e4 * 200 ** (i / 7))) for i in range(8)]
    S = [max(32, int(round(2048 * g / 1e6))) for g in G]
    return list(zip(G, S))
