"""Fetching waveforms of a job larger than the fetch staging buffers (8M
transitions per batch, two batches in flight): into pageable and into pinned
host memory, all nets and a reordered subset, split nets across batches, and
the first levels compared exactly with the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2304_13398_amd import gsim as G
from paper_2304_13398_amd import workloads as W

pytestmark = pytest.mark.gpu

STAGE = 8 << 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def job():
    sim = G.Sim(0)
    nl, st = W.config2(seed=5, G=100_000, S=205)
    h = sim.load_netlist(nl)
    say(f"fetch job: G={nl.G} S={nl.S} N_in={st.n}")
    j = sim.run(h, st)
    sim.wait(j)
    yield sim, nl, st, j
    sim.release(j)
    sim.unload_netlist(h)
    sim.close()


def fetch_into(sim, j, nets, n, t_buf, v_buf):
    off = np.zeros(n + 1, dtype=np.int64)
    p_nets = None if nets is None else nets.ctypes.data_as(G.ctypes.c_void_p)
    sim._ck(sim.lib.sim_fetch_waveforms(sim.ctx, j, p_nets, n, off.ctypes.data_as(G.ctypes.c_void_p),
                                        None, None, 0))
    total = int(off[-1])
    assert len(t_buf) >= total and len(v_buf) >= total
    sim._ck(sim.lib.sim_fetch_waveforms(sim.ctx, j, p_nets, n, off.ctypes.data_as(G.ctypes.c_void_p),
                                        G.ctypes.c_void_p(t_buf.ctypes.data), G.ctypes.c_void_p(v_buf.ctypes.data),
                                        total))
    return off, t_buf[:total], v_buf[:total]


def pinned(n, dtype):
    import torch
    return torch.empty(max(n, 1), dtype=dtype, pin_memory=True).numpy()


def test_fetch_all_pageable_and_pinned_agree(job):
    import torch
    sim, nl, st, j = job
    off, t, v = sim.fetch(j)
    total = int(off[-1])
    say(f"fetch all: {total} transitions, {total / STAGE:.1f} staging batches")
    assert total > 3 * STAGE, "the job must span several staging batches"
    assert np.array_equal(off[1:nl.S + 1], st.off[1:])
    assert np.array_equal(t[:st.n], st.t) and np.array_equal(v[:st.n], st.v)
    pt, pv = pinned(total, torch.int64), pinned(total, torch.uint8)
    off2, t2, v2 = fetch_into(sim, j, None, nl.S + nl.G, pt, pv)
    assert np.array_equal(off, off2)
    assert np.array_equal(t, t2) and np.array_equal(v, v2)


def test_fetch_subset_reversed(job):
    import torch
    sim, nl, st, j = job
    off, t, v = sim.fetch(j)
    rng = np.random.default_rng(3)
    nets = np.sort(rng.choice(nl.S + nl.G, size=(nl.S + nl.G) // 2, replace=False))[::-1].copy()
    lens = np.diff(off)[nets]
    want_off = np.concatenate([[0], np.cumsum(lens)])
    for mode in ("pageable", "pinned"):
        n_tot = int(want_off[-1])
        if mode == "pinned":
            bt, bv = pinned(n_tot, torch.int64), pinned(n_tot, torch.uint8)
        else:
            bt, bv = np.zeros(max(n_tot, 1), np.int64), np.zeros(max(n_tot, 1), np.uint8)
        o2, t2, v2 = fetch_into(sim, j, nets, len(nets), bt, bv)
        say(f"fetch subset ({mode}): {len(nets)} nets, {n_tot} transitions")
        assert np.array_equal(o2, want_off)
        for k in rng.choice(len(nets), size=2000, replace=False):
            a, b = off[nets[k]], off[nets[k] + 1]
            assert np.array_equal(t2[o2[k]:o2[k + 1]], t[a:b])
            assert np.array_equal(v2[o2[k]:o2[k + 1]], v[a:b])


def test_fetch_first_levels_match_oracle(job):
    sim, nl, st, j = job
    n_gates = int(np.searchsorted(nl.level, 2, side="right"))
    o_off, o_t, o_v = O.o1_simulate(nl.prefix(n_gates), st)
    off, t, v = sim.fetch(j, np.arange(nl.S, nl.S + n_gates))
    say(f"oracle levels 1-2: {n_gates} gates, {int(o_off[-1])} transitions")
    assert np.array_equal(off, o_off)
    assert np.array_equal(t, o_t) and np.array_equal(v, o_v)
