"""The kernels' per-gate evaluation code, run on the CPU under a wave64
emulator (tests/emu), compared with the oracle gate by gate.

The emulator runs csrc/eval_core.h unchanged: every lane is a coroutine, and
every cross-lane operation (ballot, readlane, DPP, barrier) is a rendezvous
of all 64 lanes. It fails a gate if lanes reach cross-lane operations
divergently, if a value passed to readfirstlane differs across lanes, or if a
gate runs more cross-lane operations than a limit (a round that never ends).
Each gate gets the oracle's waveforms of its input nets, so the comparison is
of the per-gate procedure alone (Algorithm 2 with Eq. 1 and the Fig. 3 drop),
independent of the schedule that feeds it.

Forms: "seg" (the segmented form, eval_gate_seg, as the level kernel runs
it), "seg_dataflow" (the same with agent-scope stores and no prefetch),
"levels" (the merged form
of the level kernel: tiles prefetched, shorter tile and trailing-group code),
"levels_long" (that form without the shorter code), "dataflow" (the merged
form of the dependency-driven kernel), and
"dataflow_lean" (the dependency-driven kernel with the level kernel's shorter
code, a form withdrawn after one GPU run of the 20k-gate extended-model case
did not finish). No GPU is used.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import workloads as W
from tests.emu import run_emu as E

MAX_OPS = 20_000_000


def compare(got, err, want, gates):
    off, t, v = got
    assert not np.any(err), f"{int(np.count_nonzero(err))} gates failed, codes {sorted(set(err[err != 0].tolist()))}"
    bad = []
    for i, g in enumerate(gates.tolist()):
        a, b = want[0][g], want[0][g + 1]
        if not (np.array_equal(t[off[i]:off[i + 1]], want[1][a:b]) and
                np.array_equal(v[off[i]:off[i + 1]], want[2][a:b])):
            bad.append(g)
    assert not bad, f"{len(bad)} gates differ from the oracle, first {bad[:5]}"


@pytest.fixture(scope="module")
def tiny():
    nl, st = W.config1(seed=1)
    return nl, st, O.o1_simulate(nl, st), E.builtin_lut(O.gate_eval)


@pytest.mark.parametrize("mode", ["seg", "seg_dataflow", "levels", "dataflow", "dataflow_lean", "levels_long"])
def test_tiny_every_gate(tiny, mode):
    nl, st, want, lut = tiny
    gates = np.arange(nl.G)
    got, err, _ = E.run(mode, nl, st, want, lut, gates=gates, max_ops=MAX_OPS)
    compare(got, err, want, gates)


def test_tiny_under_address_sanitizer(tiny):
    """Every input waveform and output region is its own heap block: any
    read or write outside them is reported."""
    nl, st, want, lut = tiny
    gates = np.arange(0, nl.G, 3)
    for mode in ("seg", "levels"):
        got, err, log = E.run(mode, nl, st, want, lut, gates=gates, max_ops=MAX_OPS, asan=True)
        assert "AddressSanitizer" not in log
        compare(got, err, want, gates)


def test_a_wrong_table_entry_is_seen(tiny):
    """The comparison is not vacuous: one flipped truth-table entry of AND2
    changes some gate's output."""
    nl, st, want, lut = tiny
    lut = lut.copy()
    lut[W.AND2, 1 | (1 << 2)] = 0  # AND2(1, 1) -> 0
    gates = np.nonzero(nl.type == W.AND2)[0]
    got, err, _ = E.run("levels", nl, st, want, lut, gates=gates, max_ops=MAX_OPS)
    with pytest.raises(AssertionError):
        compare(got, err, want, gates)


@pytest.fixture(scope="module")
def edge_mid():
    """The 20k-gate extended-model workload (delays by pin, input edge and
    output value with unrelated entries; user-defined tables), seed 7."""
    nl, st = W.config2(G=20_000, S=64, L=30, n_per_src=400, seed=7)
    type_, dly, udp = W.make_cell_model(nl, seed=7, edge_spread=0.5, inf_prob=0.05, n_udp=6, udp_frac=0.2)
    nl = W.with_types(nl, type_)
    want = O.o1x_simulate(nl, st, dly, udp)
    lut = np.concatenate([E.builtin_lut(O.gate_eval), udp])
    return nl, st, dly, want, lut


@pytest.mark.parametrize("mode", ["dataflow_lean", "seg", "dataflow", "levels"])
def test_edge_model_mid_generator(edge_mid, mode):
    """Every gate in the withdrawn form; a third of them in the forms in use."""
    nl, st, dly, want, lut = edge_mid
    gates = np.arange(nl.G) if mode == "dataflow_lean" else np.arange(0, nl.G, 3)
    got, err, _ = E.run(mode, nl, st, want, lut, gates=gates, dly=dly, max_ops=MAX_OPS)
    compare(got, err, want, gates)


def test_wide_delays_xz_sources():
    """Delays 0-400 ps (both windows and the lane procedure), X and Z as
    likely as 0 and 1 at the sources, extended model."""
    nl = W.make_netlist(G=1500, S=40, L=15, types=W.TYPES_ALL, dmin=0, dmax=400, seed=8, name="wide")
    st = W.make_stimulus(S=40, n_per_src=300, window=50_000, probs=(0.25, 0.25, 0.25, 0.25), seed=8)
    type_, dly, udp = W.make_cell_model(nl, seed=8, edge_spread=0.9, inf_prob=0.15, n_udp=8, udp_frac=0.5)
    nl = W.with_types(nl, type_)
    want = O.o1x_simulate(nl, st, dly, udp)
    lut = np.concatenate([E.builtin_lut(O.gate_eval), udp])
    for mode in ("seg", "seg_dataflow", "levels", "dataflow"):
        got, err, _ = E.run(mode, nl, st, want, lut, dly=dly, max_ops=MAX_OPS)
        compare(got, err, want, np.arange(nl.G))


def test_long_waveforms_every_pin_count():
    """Industrial-shaped netlist (all cell types, power-law fanout, 1-200 ps
    delays) with 600 transitions per source: gates of every pin count whose
    inputs span several rounds, so that rounds end at the 512-slot cut, the
    four-pin merge pairs its pins both ways, and time groups straddle two
    lanes of a round."""
    nl = W.make_netlist(G=20_000, S=200, L=40, types=W.TYPES_ALL, dmax=200, powerlaw=True,
                        fanout_cap=5000, seed=3, name="long")
    st = W.make_stimulus(S=200, n_per_src=600, window=1_000_000, probs=(0.49, 0.49, 0.01, 0.01), seed=3)
    want = O.o1_simulate(nl, st, threads=4)
    lut = E.builtin_lut(O.gate_eval)
    k = np.diff(nl.pin_off)
    n_in = np.concatenate([np.diff(st.off), np.diff(want[0])])[nl.pin_net]
    wg = np.add.reduceat(n_in, nl.pin_off[:-1])
    gates = np.unique(np.concatenate([np.nonzero((k == kk) & (wg > 1500))[0][:80] for kk in (1, 2, 3, 4)] +
                                     [np.arange(0, nl.G, 211)]))
    assert all(np.count_nonzero(k[gates] == kk) >= 40 for kk in (1, 2, 3, 4))
    for mode in ("levels", "dataflow"):
        got, err, _ = E.run(mode, nl, st, want, lut, gates=gates, max_ops=MAX_OPS)
        compare(got, err, want, gates)
