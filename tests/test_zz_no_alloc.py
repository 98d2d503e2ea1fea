"""The allocation-free entry point (sim_run_device_noalloc) against the
regular one (sim_run_device): every net's waveform equal, on two calls in a
row over the same output buffers (filled with garbage first), the second with
a smaller input; an arena overflow is reported; a netlist too large for the
static scratch is refused."""
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


def regular(sim, h, nl, st):
    """sim_run_device on the same device-resident stimuli; all nets fetched."""
    import torch
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
    stream = torch.cuda.current_stream()
    j = sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n, stream=stream.cuda_stream)
    sim.wait(j)
    got = sim.fetch(j)
    stats = sim.stats(j)
    sim.release(j)
    return got, stats.n_out, stats.arena_used


def no_alloc(sim, h, nl, st, bufs):
    """The allocation-free run into the caller's buffers `bufs`; decoded per
    net in the caller's net order."""
    import torch
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
    d_off, d_len, d_arena, d_res = bufs
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    sim.run_device_noalloc(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n, d_off.data_ptr(),
                           d_len.data_ptr(), d_arena.data_ptr(), d_arena.numel(), d_res.data_ptr(),
                           stream=stream.cuda_stream)
    torch.cuda.synchronize()
    res = d_res.cpu().numpy()
    order = sim.net_order(h)
    off = d_off.cpu().numpy()[order]
    ln = d_len.cpu().numpy()[order]
    arena = d_arena.cpu().numpy().view(np.uint64)
    out_off = np.concatenate([[0], np.cumsum(ln)])
    idx = np.concatenate([np.arange(o, o + n) for o, n in zip(off.tolist(), ln.tolist())]) if ln.sum() else \
        np.zeros(0, np.int64)
    keys = arena[idx]
    return res, (out_off, (keys >> np.uint64(2)).astype(np.int64), (keys & np.uint64(3)).astype(np.uint8))


def buffers(N, cap):
    import torch
    dev = torch.device("cuda:0")
    # filled with garbage so that nothing depends on zeroed outputs
    return (torch.full((N,), -7, dtype=torch.int64, device=dev), torch.full((N,), -7, dtype=torch.int64, device=dev),
            torch.full((cap,), -1, dtype=torch.int64, device=dev), torch.full((4,), -7, dtype=torch.int64, device=dev))


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("case", ["tiny", "mid20k"])
def test_two_calls_second_smaller(sim, case):
    if case == "tiny":
        nl, st = W.config1(seed=2)
        st_small = W.make_stimulus(S=nl.S, n_per_src=40, window=10_000, seed=9)
    else:
        nl, st = W.config2(G=20_000, S=64, L=30, n_per_src=400, seed=4)
        st_small = W.make_stimulus(S=nl.S, n_per_src=150, window=1_000_000, seed=9)
    h = sim.load_netlist(nl)
    try:
        N = nl.S + nl.G
        want1, n1, used1 = regular(sim, h, nl, st)
        want2, n2, _ = regular(sim, h, nl, st_small)
        cap = used1 + 1024  # what the regular run reserved (every gate's bound), and some
        bufs = buffers(N, cap)
        say(f"{case}: G={nl.G} N_in={st.n} then {st_small.n}; outputs {n1}, {n2}; arena {cap}")
        res1, got1 = no_alloc(sim, h, nl, st, bufs)
        assert res1[1] == 0 and res1[2] == 0, res1
        assert res1[0] == n1
        assert same(got1, want1)
        res2, got2 = no_alloc(sim, h, nl, st_small, bufs)
        assert res2[1] == 0 and res2[2] == 0, res2
        assert res2[0] == n2
        assert same(got2, want2)
        if case == "tiny":
            # and both equal the oracle
            o_off, o_t, o_v = O.o1_simulate(nl, st_small)
            g_off, g_t, g_v = got2
            base = int(g_off[nl.S])
            assert np.array_equal(g_off[nl.S:] - base, o_off)
            assert np.array_equal(g_t[base:], o_t) and np.array_equal(g_v[base:], o_v)
    finally:
        sim.unload_netlist(h)


def test_overflow_is_reported(sim):
    nl, st = W.config1(seed=3)
    h = sim.load_netlist(nl)
    try:
        bufs = buffers(nl.S + nl.G, st.n + 10)
        res, _ = no_alloc(sim, h, nl, st, bufs)
        assert res[1] == 1
    finally:
        sim.unload_netlist(h)


def test_too_large_for_the_scratch_is_refused(sim):
    """1.5M one-pin gates in one level need more step scratch than the
    static array holds: GSIM_E_ARG, nothing enqueued."""
    import torch
    G_ = 1_500_000
    S = 4
    nl = W.Netlist(S=S, G=G_, type=np.zeros(G_, np.uint8), pin_off=np.arange(G_ + 1, dtype=np.int64),
                   pin_net=(np.arange(G_) % S).astype(np.int64), rise=np.full(G_, 3, np.int32),
                   fall=np.full(G_, 4, np.int32), level=np.ones(G_, np.int32), name="wide-level")
    st = W.make_stimulus(S=S, n_per_src=10, window=1000, seed=1)
    h = sim.load_netlist(nl)
    try:
        dev = torch.device("cuda:0")
        d = [torch.from_numpy(a).to(dev) for a in (st.off, st.t, st.v)]
        bufs = buffers(S + G_, st.n + 4 * G_)
        with pytest.raises(G.GsimError) as e:
            sim.run_device_noalloc(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                                   bufs[0].data_ptr(), bufs[1].data_ptr(), bufs[2].data_ptr(), bufs[2].numel(),
                                   bufs[3].data_ptr())
        assert e.value.status == G.E_ARG
        assert "scratch" in str(e.value)
    finally:
        sim.unload_netlist(h)
