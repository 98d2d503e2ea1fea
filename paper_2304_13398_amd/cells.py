"""Standard-cell templates compiled into the library's gate model.

A cell template (Section 3.3: a module function is a combination of basic
gates, shared by every cell made from the same template) names its input and
output pins and lists its internal basic gates over pins and internal nets.
Delays are given per cell instance by input pin, output pin, input edge and
output value (the delay matrix of Section 3.2); inside a cell the basic
gates act without delay. So each output pin of an instance becomes one gate
of the expanded netlist:

* its function is a user-defined table (sim_load_netlist_ext): the
  composition of the internal gates, evaluated once per 0/1/X/Z combination
  of the cell's inputs (at most four);
* its pin delays are that output's slice of the instance's delay matrix.

Nets of a cell-level netlist: sources are 0 .. S-1; output o of instance c is
net S + (outputs of instances before c) + o, which is also its gate index in
the expanded netlist.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np

from . import workloads as W

X, Z = 2, 3
BUF, NOT, AND2, OR2, NAND2, NOR2, XOR2, XNOR2, AND3, MUX2, AND4, OR4 = range(12)


def _x(v):
    return X if v == Z else v


def _and(vals):
    vals = [_x(v) for v in vals]
    if 0 in vals:
        return 0
    return 1 if all(v == 1 for v in vals) else X


def _or(vals):
    vals = [_x(v) for v in vals]
    if 1 in vals:
        return 1
    return 0 if all(v == 0 for v in vals) else X


def _xor(vals):
    vals = [_x(v) for v in vals]
    return X if X in vals else sum(vals) & 1


def _not(v):
    v = _x(v)
    return X if v == X else 1 - v


def basic_value(gtype: int, vals) -> int:
    """4-value value of a built-in gate (Z read as X; AND, OR, XOR as in
    Table 1 and their n-input extensions; MUX2 (d0, d1, s): an unknown select
    gives the data value if both agree, else X)."""
    if gtype == BUF:
        return _x(vals[0])
    if gtype == NOT:
        return _not(vals[0])
    if gtype in (AND2, AND3, AND4):
        return _and(vals)
    if gtype in (OR2, OR4):
        return _or(vals)
    if gtype == NAND2:
        return _not(_and(vals))
    if gtype == NOR2:
        return _not(_or(vals))
    if gtype == XOR2:
        return _xor(vals)
    if gtype == XNOR2:
        return _not(_xor(vals))
    if gtype == MUX2:
        d0, d1, s = (_x(v) for v in vals)
        if s == 0:
            return d0
        if s == 1:
            return d1
        return d0 if d0 == d1 else X
    raise ValueError(f"unknown gate type {gtype}")


@dataclasses.dataclass
class CellTemplate:
    name: str
    inputs: list            # pin names (1-4)
    outputs: list           # pin names
    gates: list             # (type, [net names], output net name), in dependency order


def compile_template(tpl: CellTemplate) -> list:
    """One 256-entry table per output pin: the value for every packed 0/1/X/Z
    combination of the inputs (pin i in bits 2i and 2i+1)."""
    k = len(tpl.inputs)
    if not 1 <= k <= 4:
        raise ValueError("a cell has 1-4 inputs")
    tables = [np.zeros(256, dtype=np.uint8) for _ in tpl.outputs]
    for combo in itertools.product(range(4), repeat=k):
        val = dict(zip(tpl.inputs, combo))
        for gtype, ins, out in tpl.gates:
            val[out] = basic_value(gtype, [val[n] for n in ins])
        packed = sum(v << (2 * i) for i, v in enumerate(combo))
        for o, name in enumerate(tpl.outputs):
            tables[o][packed] = val[name]
    for tab in tables:   # unused pin bits read as 0 for arities below 4
        for packed in range(4 ** k, 256):
            tab[packed] = tab[packed & (4 ** k - 1)]
    return tables


@dataclasses.dataclass
class CellInstance:
    template: int           # index into the template list
    inputs: list            # net ids read by the cell's input pins
    dly: np.ndarray         # int32 [n_inputs, n_outputs, 2 edges, 2 output values]


def expand(S: int, templates: list, instances: list):
    """Expanded netlist: one gate per (instance, output pin), each a
    user-defined type. Returns (Netlist, dly[P, 2, 2], udp[n, 256])."""
    tables, udp_of = [], []
    for tpl in templates:
        first = len(tables)
        tables += compile_template(tpl)
        udp_of.append(first)
    types, pin_off, pin_net, dly = [], [0], [], []
    for inst in instances:
        tpl = templates[inst.template]
        d = np.asarray(inst.dly, dtype=np.int64)
        if d.shape != (len(tpl.inputs), len(tpl.outputs), 2, 2):
            raise ValueError(f"instance of {tpl.name}: delay matrix shape {d.shape}")
        for o in range(len(tpl.outputs)):
            types.append(12 + udp_of[inst.template] + o)
            pin_net += list(inst.inputs)
            pin_off.append(len(pin_net))
            dly += [d[i, o] for i in range(len(tpl.inputs))]
    G = len(types)
    nl = W.Netlist(S, G, np.array(types, dtype=np.uint8), np.array(pin_off, dtype=np.int64),
                   np.array(pin_net, dtype=np.int64), np.zeros(len(pin_net), np.int32),
                   np.zeros(len(pin_net), np.int32), np.zeros(G, np.int32), "cells")
    return nl, np.array(dly, dtype=np.int32).reshape(-1, 2, 2), np.array(tables, dtype=np.uint8)


# A few standard-cell templates (the usual library cells; internal basic gates).
HALF_ADDER = CellTemplate("HA", ["a", "b"], ["s", "co"],
                          [(XOR2, ["a", "b"], "s"), (AND2, ["a", "b"], "co")])
FULL_ADDER = CellTemplate("FA", ["a", "b", "ci"], ["s", "co"],
                          [(XOR2, ["a", "b"], "x"), (XOR2, ["x", "ci"], "s"),
                           (AND2, ["a", "b"], "g"), (AND2, ["x", "ci"], "p"), (OR2, ["g", "p"], "co")])
AOI21 = CellTemplate("AOI21", ["a", "b", "c"], ["y"],
                     [(AND2, ["a", "b"], "ab"), (OR2, ["ab", "c"], "o"), (NOT, ["o"], "y")])
DECODER2 = CellTemplate("DEC2", ["a", "b"], ["y0", "y1", "y2", "y3"],
                        [(NOT, ["a"], "na"), (NOT, ["b"], "nb"),
                         (AND2, ["na", "nb"], "y0"), (AND2, ["a", "nb"], "y1"),
                         (AND2, ["na", "b"], "y2"), (AND2, ["a", "b"], "y3")])
MUX4_ENABLE = CellTemplate("MUX2EN", ["d0", "d1", "s", "en"], ["y", "yn"],
                           [(MUX2, ["d0", "d1", "s"], "m"), (AND2, ["m", "en"], "y"), (NOT, ["y"], "yn")])
LIBRARY = [HALF_ADDER, FULL_ADDER, AOI21, DECODER2, MUX4_ENABLE]


def random_cell_netlist(n_cells: int, S: int, seed: int, dmax: int = 60, inf_prob: float = 0.05,
                        edge_spread: float = 0.5, templates=LIBRARY):
    """A levelled random netlist of library cells: each instance reads sources
    or outputs of earlier instances; delays per (input, output, edge, value)
    drawn around a per-pin base, some unrelated (inf)."""
    rng = np.random.default_rng(seed)
    instances, n_nets = [], S
    for _ in range(n_cells):
        ti = int(rng.integers(len(templates)))
        tpl = templates[ti]
        ins = [int(rng.integers(n_nets)) for _ in tpl.inputs]
        base = rng.integers(1, dmax + 1, size=(len(tpl.inputs), len(tpl.outputs), 1, 2))
        fac = rng.uniform(1 - edge_spread, 1 + edge_spread, size=(len(tpl.inputs), len(tpl.outputs), 2, 2))
        d = np.rint(base * fac).astype(np.int64)
        d[rng.random(d.shape) < inf_prob] = W.NO_RELATION
        instances.append(CellInstance(ti, ins, d))
        n_nets += len(tpl.outputs)
    return expand(S, templates, instances)
