"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module. It shares no code with the HIP library
(``paper_2304_13398_amd``) and never imports it; the only thing both sides see
is the arrays drawn by ``paper_2304_13398_amd.workloads``.

Three independent formulations of the same result (all in plain code):

* **O1** (``o1.c``, called through ctypes): Algorithm 2 per gate with the
  Eq. 1 "glitch eaten" rule and the redundant-transition drop of Fig. 3, gates
  in a topological order. This is the parity authority for the GPU.
* **O2** (``o2_simulate``, pure Python): a global discrete-event simulator. A
  time-ordered agenda; at each time the gates are visited in level order, each
  gate is evaluated if one of its inputs changed at that time (scheduling its
  new transition with the Eq. 1 denial and the Fig. 3 drop against its pending
  list), then its pending transition due at that time, if any, is applied to
  its output net.
* **O3** (``o3_simulate``, pure Python, tiny inputs only): the dense-time
  definition. Every net has a value y(T) at every integer T (X before its first
  transition). A gate's candidate transitions are the times where its
  evaluated value changes, each with appearance time T + the minimum delay
  over the pins whose value changed at T; the output at T is the value of the
  last-determined candidate whose appearance time is <= T. (Eq. 1 denies
  exactly the candidates that a later-determined one overtakes, and the Fig. 3
  drop does not change the value function, so this is the same waveform.)

The gate functions in this file use the possibility reading of Section 2.2
(X may be 0 or 1, Z is read as X): a gate's result is 0 or 1 when every
combination of possible input values gives that result, X otherwise. It is a
different formulation from the table look-ups of ``o1.c``; both are pinned to
Table 1 by the tests.

Parity unpinned by the paper: MUX2 (not in the paper), the delay of a
transition to X (min of rise and fall), and 3/4-input types beyond what
associativity of Table 1 fixes. See the module docstring of ``o1.c``.
"""
from __future__ import annotations

import ctypes
import heapq
import itertools
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libo1.so")
SRC = os.path.join(HERE, "o1.c")

X, Z = 2, 3
BUF, NOT, AND2, OR2, NAND2, NOR2, XOR2, XNOR2, AND3, MUX2, AND4, OR4 = range(12)
ARITY = (1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 4, 4)


# ---------------------------------------------------------------------------
# Build and load O1.

def build(force: bool = True, src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile ``o1.c`` with gcc into a shared library (plain -O2)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread", *extra, "-o", tmp, src])
        os.replace(tmp, out)
    return out


class _O1:
    def __init__(self, path):
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.o1_simulate.restype = P
        lib.o1_simulate.argtypes = [i64, i64, P, P, P, P, P, P, P, P, ctypes.POINTER(ctypes.c_int)]
        lib.o1_simulate_parallel.restype = P
        lib.o1_simulate_parallel.argtypes = [i64, i64, P, P, P, P, P, P, P, P, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int)]
        lib.o1_lengths.argtypes = [P, P]
        lib.o1_copy.argtypes = [P, P, P, P]
        lib.o1_free.argtypes = [P]
        lib.o1_gate.restype = i64
        lib.o1_gate.argtypes = [ctypes.c_int, P, P, P, P, P, P, P, i64]
        lib.o1_calculate_signal.restype = ctypes.c_uint8
        lib.o1_calculate_signal.argtypes = [ctypes.c_int, P]
        lib.o1_simulate_fingerprints.restype = ctypes.c_int
        lib.o1_simulate_fingerprints.argtypes = [i64, i64, P, P, P, P, P, P, P, P, P, P]
        lib.o1_fingerprints.argtypes = [i64, P, P, P, P]
        lib.o1_simulate_fingerprints_parallel.restype = P
        lib.o1_simulate_fingerprints_parallel.argtypes = [i64, i64, P, P, P, P, P, P, P, P,
                                                          ctypes.c_int, P, P, i64, P,
                                                          ctypes.POINTER(ctypes.c_int)]
        lib.o1x_simulate.restype = P
        lib.o1x_simulate.argtypes = [i64, i64, P, P, P, P, ctypes.c_int, P, P, P, P,
                                     ctypes.POINTER(ctypes.c_int)]
        self.lib = lib


_o1_cache = {}


def o1_lib(path: str | None = None) -> _O1:
    path = path or LIB
    if path not in _o1_cache:
        if path == LIB and not os.path.exists(LIB):
            build(force=False)
        _o1_cache[path] = _O1(path)
    return _o1_cache[path]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def o1_simulate(nl, st, lib: str | None = None, threads: int = 0):
    """O1 on a whole netlist. Returns (off[G+1], t, v): gate g's waveform is
    t[off[g]:off[g+1]], v[off[g]:off[g+1]]. With ``threads`` > 0 the gates of
    each level are split over that many threads (same result)."""
    L = o1_lib(lib).lib
    type_ = np.ascontiguousarray(nl.type, dtype=np.uint8)
    pin_off = np.ascontiguousarray(nl.pin_off, dtype=np.int64)
    pin_net = np.ascontiguousarray(nl.pin_net, dtype=np.int64)
    rise = np.ascontiguousarray(nl.rise, dtype=np.int32)
    fall = np.ascontiguousarray(nl.fall, dtype=np.int32)
    soff = np.ascontiguousarray(st.off, dtype=np.int64)
    st_t = np.ascontiguousarray(st.t, dtype=np.int64)
    st_v = np.ascontiguousarray(st.v, dtype=np.uint8)
    status = ctypes.c_int(0)
    if threads > 0:
        h = L.o1_simulate_parallel(nl.S, nl.G, _ptr(type_), _ptr(pin_off), _ptr(pin_net), _ptr(rise),
                                   _ptr(fall), _ptr(soff), _ptr(st_t), _ptr(st_v), threads,
                                   ctypes.byref(status))
    else:
        h = L.o1_simulate(nl.S, nl.G, _ptr(type_), _ptr(pin_off), _ptr(pin_net), _ptr(rise),
                          _ptr(fall), _ptr(soff), _ptr(st_t), _ptr(st_v), ctypes.byref(status))
    if not h:
        raise OracleError({-1: "out of memory", -2: "cycle", -3: "malformed netlist"}
                          .get(status.value, str(status.value)))
    try:
        ln = np.empty(nl.G, dtype=np.int64)
        L.o1_lengths(h, _ptr(ln))
        n = int(ln.sum())
        off = np.empty(nl.G + 1, dtype=np.int64)
        t = np.empty(n, dtype=np.int64)
        v = np.empty(n, dtype=np.uint8)
        L.o1_copy(h, _ptr(off), _ptr(t), _ptr(v))
    finally:
        L.o1_free(h)
    return off, t, v


def o1x_simulate(nl, st, dly, udp=None, lib: str | None = None):
    """O1 under the extended cell model (delays by pin, input edge and output
    value; user-defined gate tables for types 12 and up). ``dly`` is int32
    [P, 2, 2] (edge rise/fall, output 0/1; INT32_MAX = no relation), ``udp``
    uint8 [n, 256]. Returns (off[G+1], t, v) like o1_simulate."""
    L = o1_lib(lib).lib
    type_ = np.ascontiguousarray(nl.type, dtype=np.uint8)
    pin_off = np.ascontiguousarray(nl.pin_off, dtype=np.int64)
    pin_net = np.ascontiguousarray(nl.pin_net, dtype=np.int64)
    d = np.ascontiguousarray(dly, dtype=np.int32).reshape(-1)
    assert d.size == 4 * nl.P
    u = np.ascontiguousarray(udp if udp is not None else np.zeros((0, 256)), dtype=np.uint8)
    soff = np.ascontiguousarray(st.off, dtype=np.int64)
    st_t = np.ascontiguousarray(st.t, dtype=np.int64)
    st_v = np.ascontiguousarray(st.v, dtype=np.uint8)
    status = ctypes.c_int(0)
    h = L.o1x_simulate(nl.S, nl.G, _ptr(type_), _ptr(pin_off), _ptr(pin_net), _ptr(d), len(u),
                       _ptr(u) if len(u) else None, _ptr(soff), _ptr(st_t), _ptr(st_v),
                       ctypes.byref(status))
    if not h:
        raise OracleError({-1: "out of memory", -2: "cycle", -3: "malformed netlist"}
                          .get(status.value, str(status.value)))
    try:
        ln = np.empty(nl.G, dtype=np.int64)
        L.o1_lengths(h, _ptr(ln))
        off = np.empty(nl.G + 1, dtype=np.int64)
        t = np.empty(int(ln.sum()), dtype=np.int64)
        v = np.empty(int(ln.sum()), dtype=np.uint8)
        L.o1_copy(h, _ptr(off), _ptr(t), _ptr(v))
    finally:
        L.o1_free(h)
    return off, t, v


def o1_fingerprints_of(off, t, v, lib: str | None = None):
    """Fingerprint (see o1.c) of each waveform of CSR arrays."""
    L = o1_lib(lib).lib
    off = np.ascontiguousarray(off, dtype=np.int64)
    t = np.ascontiguousarray(t, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.uint8)
    out = np.zeros(max(len(off) - 1, 1), dtype=np.uint64)
    L.o1_fingerprints(len(off) - 1, _ptr(off), _ptr(t), _ptr(v), _ptr(out))
    return out[:len(off) - 1]


def o1_simulate_fingerprints(nl, st, lib: str | None = None):
    """O1 on a whole netlist, keeping only each gate's output length and
    fingerprint (waveforms are freed after their last reader): (len[G], fp[G])."""
    L = o1_lib(lib).lib
    arrs = [np.ascontiguousarray(a, dtype=d) for a, d in (
        (nl.type, np.uint8), (nl.pin_off, np.int64), (nl.pin_net, np.int64), (nl.rise, np.int32),
        (nl.fall, np.int32), (st.off, np.int64), (st.t, np.int64), (st.v, np.uint8))]
    ln = np.zeros(max(nl.G, 1), dtype=np.int64)
    fp = np.zeros(max(nl.G, 1), dtype=np.uint64)
    rc = L.o1_simulate_fingerprints(nl.S, nl.G, *[_ptr(a) for a in arrs], _ptr(ln), _ptr(fp))
    if rc:
        raise OracleError({-1: "out of memory", -2: "cycle", -3: "malformed netlist"}.get(rc, str(rc)))
    return ln[:nl.G], fp[:nl.G]


def o1_simulate_fingerprints_parallel(nl, st, threads: int, keep=None, lib: str | None = None):
    """O1 on a whole netlist, level by level on ``threads`` threads, keeping
    each gate's output length and fingerprint (waveforms freed after the level
    of their last reader) and the whole waveforms of the gates in ``keep``:
    (len[G], fp[G], (off, t, v) of the kept gates in the order given)."""
    L = o1_lib(lib).lib
    arrs = [np.ascontiguousarray(a, dtype=d) for a, d in (
        (nl.type, np.uint8), (nl.pin_off, np.int64), (nl.pin_net, np.int64), (nl.rise, np.int32),
        (nl.fall, np.int32), (st.off, np.int64), (st.t, np.int64), (st.v, np.uint8))]
    keep = np.ascontiguousarray(np.zeros(0) if keep is None else keep, dtype=np.int64)
    ln = np.zeros(max(nl.G, 1), dtype=np.int64)
    fp = np.zeros(max(nl.G, 1), dtype=np.uint64)
    status = ctypes.c_int(0)
    h = L.o1_simulate_fingerprints_parallel(nl.S, nl.G, *[_ptr(a) for a in arrs], int(threads),
                                            _ptr(ln), _ptr(fp), len(keep),
                                            _ptr(keep) if len(keep) else None, ctypes.byref(status))
    if not h:
        raise OracleError({-1: "out of memory", -2: "cycle", -3: "malformed netlist"}.get(
            status.value, str(status.value)))
    try:
        n = np.zeros(max(len(keep), 1), dtype=np.int64)
        L.o1_lengths(h, _ptr(n))
        off = np.zeros(len(keep) + 1, dtype=np.int64)
        off[1:] = np.cumsum(n[:len(keep)])
        t = np.zeros(max(int(off[-1]), 1), dtype=np.int64)
        v = np.zeros(max(int(off[-1]), 1), dtype=np.uint8)
        L.o1_copy(h, _ptr(off), _ptr(t), _ptr(v))
    finally:
        L.o1_free(h)
    return ln[:nl.G], fp[:nl.G], (off, t[:off[-1]], v[:off[-1]])


def o1_gate(gtype, waves, rise, fall, lib: str | None = None):
    """O1 on one gate. ``waves`` = list of (times, values) per pin."""
    L = o1_lib(lib).lib
    k = ARITY[gtype]
    assert len(waves) == k
    ts = [np.ascontiguousarray(w[0], dtype=np.int64) for w in waves]
    vs = [np.ascontiguousarray(w[1], dtype=np.uint8) for w in waves]
    pt = (ctypes.c_void_p * 4)(*[t.ctypes.data for t in ts], *([0] * (4 - k)))
    pv = (ctypes.c_void_p * 4)(*[v.ctypes.data for v in vs], *([0] * (4 - k)))
    n = np.array([len(t) for t in ts] + [0] * (4 - k), dtype=np.int64)
    r = np.ascontiguousarray(rise, dtype=np.int32)
    f = np.ascontiguousarray(fall, dtype=np.int32)
    cap = int(n.sum()) + 1
    ot = np.empty(cap, dtype=np.int64)
    ov = np.empty(cap, dtype=np.uint8)
    m = L.o1_gate(gtype, ctypes.cast(pt, ctypes.c_void_p), ctypes.cast(pv, ctypes.c_void_p),
                  _ptr(n), _ptr(r), _ptr(f), _ptr(ot), _ptr(ov), cap)
    if m < 0:
        raise OracleError("o1_gate failed")
    return list(zip(ot[:m].tolist(), ov[:m].tolist()))


def o1_eval(gtype, vals, lib: str | None = None) -> int:
    """O1's gate function on one input combination."""
    a = np.zeros(4, dtype=np.uint8)
    a[:len(vals)] = vals
    return int(o1_lib(lib).lib.o1_calculate_signal(gtype, _ptr(a)))


# ---------------------------------------------------------------------------
# Gate functions, possibility reading (Section 2.2).

def _possible(v):
    return (0,) if v == 0 else (1,) if v == 1 else (0, 1)   # X and Z: either level


def _collapse(results):
    s = set(results)
    return s.pop() if len(s) == 1 else X


_BOOL = {
    BUF: lambda a: a[0],
    NOT: lambda a: 1 - a[0],
    AND2: lambda a: a[0] & a[1],
    OR2: lambda a: a[0] | a[1],
    NAND2: lambda a: 1 - (a[0] & a[1]),
    NOR2: lambda a: 1 - (a[0] | a[1]),
    XOR2: lambda a: a[0] ^ a[1],
    XNOR2: lambda a: 1 - (a[0] ^ a[1]),
    AND3: lambda a: a[0] & a[1] & a[2],
    MUX2: lambda a: a[1] if a[2] else a[0],
    AND4: lambda a: a[0] & a[1] & a[2] & a[3],
    OR4: lambda a: a[0] | a[1] | a[2] | a[3],
}


def gate_eval(gtype, vals) -> int:
    """Value of a gate: 0 or 1 if every combination of possible input levels
    agrees, else X."""
    f = _BOOL[gtype]
    return _collapse(f(c) for c in itertools.product(*(_possible(v) for v in vals)))


def pin_delay(rise, fall, value):
    return rise if value == 1 else fall if value == 0 else min(rise, fall)


# ---------------------------------------------------------------------------
# Shared helpers of O2/O3 (structure only).

def _levels(nl):
    """Longest-path level of every gate (sources are level 0), by repeated
    relaxation over the pins; raises on a cycle."""
    S, G = nl.S, nl.G
    lvl = np.zeros(S + G, dtype=np.int64)
    for _ in range(G + 1):
        changed = False
        for g in range(G):
            pins = nl.pin_net[nl.pin_off[g]:nl.pin_off[g + 1]]
            want = 1 + max(int(lvl[p]) for p in pins)
            if lvl[S + g] != want:
                lvl[S + g] = want
                changed = True
        if not changed:
            return lvl
    raise OracleError("cycle")


def _pins(nl, g):
    a, b = int(nl.pin_off[g]), int(nl.pin_off[g + 1])
    return ([int(x) for x in nl.pin_net[a:b]], [int(x) for x in nl.rise[a:b]],
            [int(x) for x in nl.fall[a:b]])


def _source_waves(st, S):
    return [list(zip(st.t[st.off[s]:st.off[s + 1]].tolist(),
                     st.v[st.off[s]:st.off[s + 1]].tolist())) for s in range(S)]


# ---------------------------------------------------------------------------
# O2: global discrete-event simulation.

def o2_simulate(nl, st):
    """Returns a list of G waveforms, each a list of (time, value)."""
    S, G = nl.S, nl.G
    lvl = _levels(nl)
    order = sorted(range(G), key=lambda g: (lvl[S + g], g))
    fanout = [[] for _ in range(S + G)]
    pins = [_pins(nl, g) for g in range(G)]
    for g in range(G):
        for p in pins[g][0]:
            fanout[p].append(g)
    value = [X] * (S + G)           # committed value of every net
    last_eval = [X] * G             # previous evaluated output of every gate
    pending = [[] for _ in range(G)]  # scheduled (time, value), increasing time
    out = [[] for _ in range(G)]
    agenda = []                     # heap of times at which something may happen
    src_events = {}
    for s, w in enumerate(_source_waves(st, S)):
        for t, v in w:
            src_events.setdefault(t, []).append((s, v))
            heapq.heappush(agenda, t)
    seen = set()
    while agenda:
        T = heapq.heappop(agenda)
        if T in seen:
            continue
        seen.add(T)
        changed_nets = set()
        for s, v in src_events.get(T, ()):
            value[s] = v
            changed_nets.add(s)
        for g in order:
            nets, rise, fall = pins[g]
            hit = [i for i, n in enumerate(nets) if n in changed_nets]
            if hit:
                e = gate_eval(nl.type[g], [value[n] for n in nets])
                if e != last_eval[g]:
                    d = min(pin_delay(rise[i], fall[i], e) for i in hit)
                    tr = T + d
                    pend = pending[g]
                    while pend and pend[-1][0] >= tr:      # Eq. 1
                        pend.pop()
                    proj = pend[-1][1] if pend else value[S + g]
                    if e != proj:                           # Fig. 3 drop
                        pend.append((tr, e))
                        heapq.heappush(agenda, tr)
                last_eval[g] = e
            pend = pending[g]
            if pend and pend[0][0] == T:
                _, v = pend.pop(0)
                value[S + g] = v
                out[g].append((T, v))
                changed_nets.add(S + g)
    return out


# ---------------------------------------------------------------------------
# O3: dense-time definition (tiny inputs only).

def o3_simulate(nl, st, t_max=None):
    S, G = nl.S, nl.G
    lvl = _levels(nl)
    srcw = _source_waves(st, S)
    if t_max is None:
        last = max([w[-1][0] for w in srcw if w] + [0])
        dm = int(max(nl.rise.max(initial=0), nl.fall.max(initial=0)))
        t_max = last + (int(lvl.max(initial=0)) + 1) * (dm + 1) + 1
    n_t = t_max + 2                       # index 0 is time -1, index i is time i-1
    y = np.full((S + G, n_t), X, dtype=np.int64)
    for s, w in enumerate(srcw):
        for t, v in w:
            y[s, t + 1:] = v
    order = sorted(range(G), key=lambda g: (lvl[S + g], g))
    for g in order:
        nets, rise, fall = _pins(nl, g)
        gt = int(nl.type[g])
        e = [X] + [gate_eval(gt, [int(y[n, i]) for n in nets]) for i in range(1, n_t)]
        cands = []                         # (appearance time, value), in determination order
        for i in range(1, n_t):
            if e[i] != e[i - 1]:
                ch = [k for k, n in enumerate(nets) if y[n, i] != y[n, i - 1]]
                d = min(pin_delay(rise[k], fall[k], e[i]) for k in ch)
                cands.append((i - 1 + d, e[i]))
        for i in range(1, n_t):
            T = i - 1
            j = [c for c in cands if c[0] <= T]
            y[S + g, i] = j[-1][1] if j else X
    out = []
    for g in range(G):
        row = y[S + g]
        out.append([(i - 1, int(row[i])) for i in range(1, n_t) if row[i] != row[i - 1]])
    return out


# ---------------------------------------------------------------------------
# O3 under the extended cell model (tiny inputs only): the same dense-time
# definition, with the gate value from a table for types 12 and up and the
# delay of a candidate = min over the changed pins of their delay for their
# edge and the new value; a candidate with no related changed pin never
# appears; the gate's value is X until its first input change. Edge readings
# as in the C oracle's extended model.

NO_RELATION = 2**31 - 1


def edge_class(old, new):
    if new == 1 or (old == 0 and new in (X, Z)):
        return 0
    if new == 0 or (old == 1 and new in (X, Z)):
        return 1
    return 2


def edge_delay(d22, edge, out):
    """d22[edge][out]; edge 2 = both edges; out X = both outputs."""
    vals = [d22[e][o] for e in (0, 1) if edge in (e, 2) for o in (0, 1) if out in (o, X)]
    vals = [x for x in vals if x != NO_RELATION]
    return min(vals) if vals else None


def o3x_simulate(nl, st, dly, udp=None, t_max=None):
    S, G = nl.S, nl.G
    lvl = _levels(nl)
    srcw = _source_waves(st, S)
    if t_max is None:
        last = max([w[-1][0] for w in srcw if w] + [0])
        finite = [int(x) for x in np.asarray(dly).reshape(-1) if x != NO_RELATION]
        dm = max(finite + [0])
        t_max = last + (int(lvl.max(initial=0)) + 1) * (dm + 1) + 1
    n_t = t_max + 2
    y = np.full((S + G, n_t), X, dtype=np.int64)
    for s, w in enumerate(srcw):
        for t, v in w:
            y[s, t + 1:] = v
    for g in sorted(range(G), key=lambda g: (lvl[S + g], g)):
        a, b = int(nl.pin_off[g]), int(nl.pin_off[g + 1])
        nets = [int(x) for x in nl.pin_net[a:b]]
        gt = int(nl.type[g])

        def f(vals):
            if gt >= 12:
                return int(udp[gt - 12][sum(v << (2 * i) for i, v in enumerate(vals))])
            return gate_eval(gt, vals)

        # the gate is evaluated from its first input change on; before that its
        # value is X (Algorithm 2 starts from an X previous value), which only
        # matters for tables that map all-X inputs to 0 or 1
        started = np.cumsum(np.any(y[nets, 1:] != y[nets, :-1], axis=0)) > 0
        e = [X] + [f([int(y[n, i]) for n in nets]) if started[i - 1] else X for i in range(1, n_t)]
        cands = []
        for i in range(1, n_t):
            if e[i] != e[i - 1]:
                ds = [edge_delay(dly[a + k], edge_class(int(y[n, i - 1]), int(y[n, i])), e[i])
                      for k, n in enumerate(nets) if y[n, i] != y[n, i - 1]]
                ds = [x for x in ds if x is not None]
                if ds:
                    cands.append((i - 1 + min(ds), e[i]))
        for i in range(1, n_t):
            j = [c for c in cands if c[0] <= i - 1]
            y[S + g, i] = j[-1][1] if j else X
    out = []
    for g in range(G):
        row = y[S + g]
        out.append([(i - 1, int(row[i])) for i in range(1, n_t) if row[i] != row[i - 1]])
    return out


def combinational(nl, src_values):
    """Textbook zero-delay evaluation: the value of every gate for one vector of
    source values, gates in level order."""
    S, G = nl.S, nl.G
    lvl = _levels(nl)
    val = list(src_values) + [X] * G
    for g in sorted(range(G), key=lambda g: (lvl[S + g], g)):
        nets, _, _ = _pins(nl, g)
        val[S + g] = gate_eval(int(nl.type[g]), [val[n] for n in nets])
    return val[S:]


def csr_to_lists(off, t, v):
    return [list(zip(t[off[g]:off[g + 1]].tolist(), v[off[g]:off[g + 1]].tolist()))
            for g in range(len(off) - 1)]
