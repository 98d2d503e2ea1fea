"""Device stimuli passed without validation that break the waveform
conventions (times out of order): every gate still ends, and the job reports
an error or returns waveforms -- it never loops. Each round of a gate either
takes an input transition or makes a tentative survivor final; a round that
does neither stops the gate with a device error."""
import sys

import numpy as np
import pytest

from paper_2304_13398_amd import gsim as G
from paper_2304_13398_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_out_of_order_device_stimulus_ends():
    import torch
    nl, st = W.config1(seed=3)
    t = st.t.copy()
    for s in range(0, nl.S, 3):  # every third source's times reversed
        a, b = int(st.off[s]), int(st.off[s + 1])
        t[a:b] = t[a:b][::-1]
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(x).to(dev) for x in (st.off, t, st.v)]
    sim = G.Sim(0)
    try:
        h = sim.load_netlist(nl)
        say("out-of-order device stimulus, level schedule, tiny netlist")
        j = sim.run_device(h, d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), st.n,
                           stream=torch.cuda.current_stream().cuda_stream)
        try:
            sim.wait(j)
            outcome = "finished"
        except G.GsimError as e:
            outcome = f"error: {e}"
        say(f"outcome: {outcome}")
        sim.release(j)
        # the context stays usable: a valid job afterwards matches a fresh run
        j = sim.run(h, st)
        sim.wait(j)
        got = sim.fetch(j, np.arange(nl.S, nl.S + nl.G))
        sim.release(j)
        ref = G.Sim(0)
        try:
            want = ref.simulate(nl, st)
        finally:
            ref.close()
        for a, b in zip(got, want):
            assert np.array_equal(a, b)
        sim.unload_netlist(h)
    finally:
        sim.close()
