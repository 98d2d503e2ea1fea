"""Request loop over resident netlists: continuous batching vs one job at a time.

A request names a resident netlist, carries its source waveforms, and asks for
the waveforms of the netlist's observed outputs (the gates of its deepest
level) plus an 8-byte fingerprint of every net's waveform (sim_fetch_hashes),
which lets a client compare whole results without copying them. Latency is
measured from the request's arrival to the moment both are in host memory.

* ``serve_continuous``: requests are submitted to the library's executor when
  they arrive; every scheduling pass (``sim_drive``) admits what fits the HBM
  budget and advances every admitted job by one level in shared launches, so
  requests that arrive while others run join at the next level.
* ``serve_sequential``: the plain form -- one ``sim_run`` at a time, in arrival
  order, on the same GPU and stream.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import gsim as G
from . import workloads as W


@dataclasses.dataclass
class Request:
    arrival: float          # seconds after the start of the run
    netlist: int            # index into the resident netlists
    stim: W.Stimulus
    outputs: np.ndarray     # net ids whose waveforms are fetched
    digest: bool = True     # also fetch the fingerprints of all nets


@dataclasses.dataclass
class Result:
    latency: float
    n_out: int              # output transitions the job computed (all gates)
    fetched: int            # transitions returned to the caller
    fingerprints: np.ndarray | None = None
    request: Request | None = None


def primary_outputs(nl) -> np.ndarray:
    """Gate outputs that no pin reads."""
    read = np.zeros(nl.S + nl.G, dtype=bool)
    read[nl.pin_net] = True
    return np.nonzero(~read[nl.S:])[0] + nl.S


def observed_outputs(nl) -> np.ndarray:
    """Net ids of the gates of the deepest level."""
    return np.nonzero(nl.level == nl.level.max())[0] + nl.S


def poisson_arrivals(rng, rate: float, n: int) -> np.ndarray:
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def _finish(sim, j, req, t0):
    off, t, v = sim.fetch(j, req.outputs)
    fp = sim.hashes(j) if req.digest else None
    lat = time.perf_counter() - t0 - req.arrival
    n_out = sim.stats(j).n_out
    sim.release(j)
    return Result(lat, int(n_out), int(off[-1]), fp, req)


def _progress(progress, results, total):
    if progress and len(results) % 100 == 0:
        progress(f"{len(results)}/{total} requests done")


def serve_continuous(sim: G.Sim, handles, requests, max_ahead: int = 8, progress=None):
    reqs = sorted(requests, key=lambda r: r.arrival)
    results = []
    running = {}
    i = 0
    t0 = time.perf_counter()
    while i < len(reqs) or running:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i].arrival <= now:
            r = reqs[i]
            running[sim.submit(handles[r.netlist], r.stim)] = r
            i += 1
        if running:
            sim.drive(max_ahead=max_ahead)
            for j in [j for j in running if sim.done(j)]:
                results.append(_finish(sim, j, running.pop(j), t0))
                _progress(progress, results, len(reqs))
        elif i < len(reqs):
            time.sleep(max(0.0, min(0.001, reqs[i].arrival - now)))
    return results, time.perf_counter() - t0


def serve_sequential(sim: G.Sim, handles, requests, progress=None):
    reqs = sorted(requests, key=lambda r: r.arrival)
    results = []
    t0 = time.perf_counter()
    for r in reqs:
        wait = r.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        j = sim.run(handles[r.netlist], r.stim)
        sim.wait(j)
        results.append(_finish(sim, j, r, t0))
        _progress(progress, results, len(reqs))
    return results, time.perf_counter() - t0


def summarize(results, makespan):
    lat = np.array([r.latency for r in results]) * 1000.0
    n_out = sum(r.n_out for r in results)
    return {
        "jobs": len(results),
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_ms": float(lat.mean()) if len(lat) else None,
        "transitions_per_s": n_out / makespan if makespan > 0 else None,
        "makespan_s": makespan,
    }


def served_workload(n_jobs: int, rate: float, netlists, stim_pool, seed: int = 1):
    """Requests over the resident netlists: netlist uniform, stimulus drawn from
    that netlist's pre-generated pool, Poisson arrivals at ``rate`` per second."""
    rng = np.random.default_rng(seed)
    arrivals = poisson_arrivals(rng, rate, n_jobs)
    outs = [observed_outputs(nl) for nl in netlists]
    reqs = []
    for a in arrivals:
        k = int(rng.integers(len(netlists)))
        pool = stim_pool[k]
        reqs.append(Request(float(a), k, pool[int(rng.integers(len(pool)))], outs[k]))
    return reqs


def make_stim_pool(netlists, per_netlist: int, seed: int = 1, lo: int = 20, hi: int = 2000,
                   window: int = 1_000_000):
    """Per netlist, stimuli with n ~ round(exp U(ln lo, ln hi)) transitions per source."""
    rng = np.random.default_rng(seed + 5_000_011)
    pool = []
    for k, nl in enumerate(netlists):
        ns = W.loguniform_int(rng, lo, hi, size=per_netlist)
        pool.append([W.make_stimulus(S=nl.S, n_per_src=int(n), window=window,
                                     seed=seed * 100_000 + k * 1000 + i)
                     for i, n in enumerate(ns)])
    return pool


def served_netlists(scale: float = 1.0, seed: int = 1):
    """The 8 resident netlists of the served configuration (mid-size generator),
    G_i = round(1e4 * 200^(i/7)) gates (times ``scale``), 60 levels."""
    out = []
    for i, (g, s) in enumerate(W.config5_netlist_sizes()):
        g = max(600, int(round(g * scale)))
        s = max(32, int(round(2048 * g / 1e6)))
        out.append(W.config2_netlist(G=g, S=s, L=60, seed=seed * 10 + i))
    return out

