"""Full-size configurations on the GPU, in the launch configuration bench.py
times (stimuli resident in HBM, sim_run_device):

* every gate of the first levels is compared exactly with the oracle (length
  and fingerprint of its waveform) -- those levels form a closed netlist the
  oracle finishes in seconds;
* for a random sample of gates across all levels: structural invariants of
  the waveform and of how it relates to its input waveforms, and the steady
  state (last value = combinational value of the sources' last values);
* with GSIM_FULLSIZE_ORACLE=1, every gate is compared with the oracle
  (memory-light mode; minutes of CPU).
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import gsim as G
from paper_2304_13398_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim():
    s = G.Sim(0)
    yield s
    s.close()


def run_resident(sim, nl, st):
    import torch
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
    stream = torch.cuda.current_stream()
    h = sim.load_netlist(nl)
    j = sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                       stream=stream.cuda_stream)
    sim.wait(j)
    torch.cuda.synchronize()
    return h, j, d


def gate_lut():
    lut = np.zeros((12, 256), dtype=np.uint8)
    for t in range(12):
        k = O.ARITY[t]
        for packed in range(256):
            lut[t, packed] = O.gate_eval(t, [(packed >> (2 * i)) & 3 for i in range(k)])
    return lut


def combinational_final(nl, st):
    """Combinational value of every gate for the sources' last values,
    evaluated level by level (the generator's levels)."""
    lut = gate_lut()
    n_src = np.diff(st.off)
    last = np.where(n_src > 0, st.v[np.maximum(st.off[1:] - 1, 0)], 2).astype(np.uint8)
    val = np.concatenate([last, np.full(nl.G + 1, 2, dtype=np.uint8)])
    zero_net = nl.S + nl.G  # reads as 0 in the padding of absent pins
    val[zero_net] = 0
    ar = np.diff(nl.pin_off)
    pins = np.full((nl.G, 4), zero_net, dtype=np.int64)
    for p in range(4):
        has = ar > p
        pins[has, p] = nl.pin_net[nl.pin_off[:-1][has] + p]
    for lv in range(1, int(nl.level.max()) + 1):
        g = np.nonzero(nl.level == lv)[0]
        packed = np.zeros(len(g), dtype=np.int64)
        for p in range(4):
            packed |= val[pins[g, p]].astype(np.int64) << (2 * p)
        val[nl.S + g] = lut[nl.type[g], packed]
    return val[nl.S:nl.S + nl.G]


def check_full_size(sim, nl, st, prefix_levels, n_sample=3000):
    say(f"full size {nl.name}: G={nl.G} S={nl.S} N_in={st.n}")
    h, j, keep = run_resident(sim, nl, st)
    s = sim.stats(j)
    say(f"  gpu: {s.n_out} output transitions, {s.device_ms:.1f} ms device")

    # 1) exact on the closed prefix of the first levels
    n_pre = int(np.searchsorted(nl.level, prefix_levels, side="right"))
    o_len, o_fp = O.o1_simulate_fingerprints(nl.prefix(n_pre), st)
    gates = np.arange(nl.S, nl.S + n_pre)
    assert np.array_equal(sim.lengths(j, gates), o_len), "lengths differ on the first levels"
    assert np.array_equal(sim.hashes(j, gates), o_fp), "waveforms differ on the first levels"
    say(f"  levels 1-{prefix_levels}: {n_pre} gates exact")

    # 2) sampled gates over all levels: invariants and steady state
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(nl.G, size=min(n_sample, nl.G), replace=False))
    want_final = combinational_final(nl, st)[sample]
    off, t, v = sim.fetch(j, nl.S + sample)
    for i, g in enumerate(sample.tolist()):
        tt, vv = t[off[i]:off[i + 1]], v[off[i]:off[i + 1]]
        last = int(vv[-1]) if len(vv) else 2
        assert last == want_final[i], f"gate {g}: steady state {last} != {want_final[i]}"
    sub_nets = np.unique(nl.pin_net[np.concatenate([np.arange(nl.pin_off[g], nl.pin_off[g + 1])
                                                    for g in sample.tolist()])])
    in_off, in_t, in_v = sim.fetch(j, sub_nets)
    pos = {int(n): k for k, n in enumerate(sub_nets.tolist())}
    for i, g in enumerate(sample.tolist()):
        tt, vv = t[off[i]:off[i + 1]], v[off[i]:off[i + 1]]
        if len(tt) == 0:
            continue
        assert np.all(np.diff(tt) > 0) and vv[0] != 2 and np.all(vv[1:] != vv[:-1]) and np.all(vv < 3)
        ins = [in_t[in_off[pos[int(n)]]:in_off[pos[int(n)] + 1]]
               for n in nl.pin_net[nl.pin_off[g]:nl.pin_off[g + 1]]]
        distinct = np.unique(np.concatenate(ins))
        assert len(tt) <= len(distinct)
        ds = np.unique(np.concatenate([nl.rise[nl.pin_off[g]:nl.pin_off[g + 1]],
                                       nl.fall[nl.pin_off[g]:nl.pin_off[g + 1]]]))
        assert np.isin(tt[:, None] - ds[None, :], distinct).any(axis=1).all()
    say(f"  {len(sample)} sampled gates: invariants and steady state hold")

    # 3) opt-in: every gate against the oracle
    if os.environ.get("GSIM_FULLSIZE_ORACLE") == "1":
        o_len, o_fp = O.o1_simulate_fingerprints(nl, st)
        all_gates = np.arange(nl.S, nl.S + nl.G)
        assert np.array_equal(sim.lengths(j, all_gates), o_len)
        assert np.array_equal(sim.hashes(j, all_gates), o_fp)
        say(f"  all {nl.G} gates exact against the oracle")
    sim.release(j)
    sim.unload_netlist(h)


@pytest.mark.parametrize("schedule", [0, 1], ids=["levels", "dataflow"])
def test_mid_full_size(sim, schedule):
    """1M gates, 2,048 PIs, 60 levels, 1,000 transitions per PI."""
    nl, st = W.config2()
    sim.set_option(G.OPT_SCHEDULE, schedule)
    try:
        check_full_size(sim, nl, st, prefix_levels=10)
    finally:
        sim.set_option(G.OPT_SCHEDULE, 0)


@pytest.mark.timeout(300)
def test_industrial_full_size(sim):
    """10M gates, 58,192 sources, 150 levels, delays up to 200 ps."""
    nl, st = W.config3()
    check_full_size(sim, nl, st, prefix_levels=6)
