"""C-ABI library on the CPU: it loads, exports every declared symbol, and its
host logic (levelizer, validation) behaves; no device calls."""
import os
import re

import numpy as np
import pytest

from paper_2304_13398_amd import gsim as G
from paper_2304_13398_amd import workloads as W
from tests import oracle_pins as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gsim.h")).read()
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = G.load_library()
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(G.EXPORTED)


def test_version():
    assert "gfx950" in G.version()


def test_levelizer_matches_generator_levels():
    nl = W.config2_netlist(G=20000, S=64, L=60)
    level, n = G.levelize(nl.S, nl.G, nl.type, nl.pin_off, nl.pin_net, nl.rise, nl.fall)
    assert n == 60
    # one pin of every generated gate reads the level below, so the longest-path
    # level equals the level it was built at
    assert np.array_equal(level, nl.level)


def test_levelizer_on_shuffled_gate_order():
    nl, _ = W.config1(seed=4)
    rng = np.random.default_rng(0)
    perm = rng.permutation(nl.G)          # new gate i = old gate perm[i]
    inv = np.argsort(perm)
    remap = np.concatenate([np.arange(nl.S), nl.S + inv])
    gates = [(int(nl.type[g]), [int(remap[x]) for x in nl.pin_net[nl.pin_off[g]:nl.pin_off[g + 1]]])
             for g in perm]
    rise = np.concatenate([nl.rise[nl.pin_off[g]:nl.pin_off[g + 1]] for g in perm])
    fall = np.concatenate([nl.fall[nl.pin_off[g]:nl.pin_off[g + 1]] for g in perm])
    sh = P.netlist_of(nl.S, gates, rise, fall)
    level, n = G.levelize(sh.S, sh.G, sh.type, sh.pin_off, sh.pin_net, sh.rise, sh.fall)
    assert n == 20 and np.array_equal(level, nl.level[perm])


def _expect(status, fn, *args):
    with pytest.raises(G.GsimError) as e:
        fn(*args)
    assert e.value.status == status, str(e.value)
    return str(e.value)


def test_netlist_validation_errors():
    ok = P.netlist_of(2, [(W.AND2, [0, 1]), (W.NOT, [2])], [1, 1, 1], [1, 1, 1])
    G.levelize(ok.S, ok.G, ok.type, ok.pin_off, ok.pin_net, ok.rise, ok.fall)
    cyc = P.netlist_of(2, [(W.AND2, [0, 3]), (W.NOT, [2])], [1, 1, 1], [1, 1, 1])
    _expect(G.E_CYCLE, G.levelize, cyc.S, cyc.G, cyc.type, cyc.pin_off, cyc.pin_net, cyc.rise, cyc.fall)
    selfloop = P.netlist_of(2, [(W.AND2, [0, 2])], [1, 1], [1, 1])
    _expect(G.E_CYCLE, G.levelize, 2, 1, selfloop.type, selfloop.pin_off, selfloop.pin_net,
            selfloop.rise, selfloop.fall)
    bad_arity = P.netlist_of(2, [(W.AND2, [0])], [1], [1])
    _expect(G.E_ARG, G.levelize, 2, 1, bad_arity.type, bad_arity.pin_off, bad_arity.pin_net,
            bad_arity.rise, bad_arity.fall)
    bad_net = P.netlist_of(2, [(W.AND2, [0, 7])], [1, 1], [1, 1])
    _expect(G.E_ARG, G.levelize, 2, 1, bad_net.type, bad_net.pin_off, bad_net.pin_net,
            bad_net.rise, bad_net.fall)
    neg = P.netlist_of(2, [(W.AND2, [0, 1])], [1, -1], [1, 1])
    _expect(G.E_ARG, G.levelize, 2, 1, neg.type, neg.pin_off, neg.pin_net, neg.rise, neg.fall)
    bad_type = P.netlist_of(2, [(W.AND2, [0, 1])], [1, 1], [1, 1])
    bad_type.type[0] = 12
    _expect(G.E_ARG, G.levelize, 2, 1, bad_type.type, bad_type.pin_off, bad_type.pin_net,
            bad_type.rise, bad_type.fall)


def test_stimulus_validation_errors():
    def st(waves):
        s = P.stimulus_of(waves)
        return s.off, s.t, s.v
    G.validate_stimulus(2, *st([[(0, 1), (5, 3)], []]))
    _expect(G.E_WAVEFORM, G.validate_stimulus, 1, *st([[(0, 2)]]))            # leading X
    _expect(G.E_WAVEFORM, G.validate_stimulus, 1, *st([[(0, 1), (3, 1)]]))    # repeat
    _expect(G.E_WAVEFORM, G.validate_stimulus, 1, *st([[(4, 1), (4, 0)]]))    # equal times
    _expect(G.E_WAVEFORM, G.validate_stimulus, 1, *st([[(4, 1), (2, 0)]]))    # decreasing
    _expect(G.E_WAVEFORM, G.validate_stimulus, 1, *st([[(-1, 1)]]))           # negative
    _expect(G.E_WAVEFORM, G.validate_stimulus, 1, *st([[(0, 4)]]))            # bad value
    _expect(G.E_OVERFLOW, G.validate_stimulus, 1, *st([[(2 ** 62 - 10, 1)]]), 10)
    G.validate_stimulus(1, *st([[(2 ** 62 - 11, 1)]]), 10)


def test_context_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    _expect(G.E_DEVICE, G.Sim)


def header_struct(name):
    """(field, C type) pairs of `typedef struct { ... } name;` in gsim.h."""
    src = open(os.path.join(ROOT, "include", "gsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        fields += [(n.strip(), ctype) for n in names.split(",")]
    return fields


@pytest.mark.parametrize("c_name,py_cls", [("gsim_job_stats", "JobStats"),
                                           ("gsim_netlist_info", "NetlistInfo"),
                                           ("gsim_memory_info", "MemoryInfo")])
def test_binding_structs_match_the_header(c_name, py_cls):
    import ctypes
    ctype_of = {"int64_t": ctypes.c_int64, "int32_t": ctypes.c_int32, "double": ctypes.c_double,
                "uint64_t": ctypes.c_uint64}
    want = [(n, ctype_of[t]) for n, t in header_struct(c_name)]
    got = list(getattr(G, py_cls)._fields_)
    assert got == want


def header_enum(name):
    """{member: value} of `enum name { ... };` in gsim.h (comments removed)."""
    src = open(os.path.join(ROOT, "include", "gsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"enum " + name + r"\s*\{([^}]*)\}", src).group(1)
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"(\w+)\s*=\s*(-?\d+)", body)}


def test_binding_constants_match_the_header():
    """The binding's option, schedule and gate-type numbers are the header's."""
    opts = header_enum("gsim_option")
    for name, value in opts.items():
        assert getattr(G, name[len("GSIM_"):]) == value, name
    for name, value in header_enum("gsim_schedule").items():
        assert getattr(G, name[len("GSIM_"):]) == value, name
    gates = header_enum("gsim_gate_type")
    n = gates.pop("GSIM_NUM_TYPES")
    assert sorted(gates.values()) == list(range(n))
    from oracle import oracle as O
    for name, value in gates.items():
        assert getattr(O, name[len("GSIM_"):]) == value, name
