"""ctypes binding of libgsim (include/gsim.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; this module
converts NumPy arrays (or device pointers, e.g. from PyTorch tensors) to the
C ABI and raises :class:`GsimError` on a non-zero status. There is no
fallback: if ``libgsim.so`` is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgsim.so")

OK, E_ARG, E_CYCLE, E_WAVEFORM, E_OOM, E_DEVICE, E_HANDLE, E_OVERFLOW = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "GSIM_E_ARG", -2: "GSIM_E_CYCLE", -3: "GSIM_E_WAVEFORM",
                -4: "GSIM_E_OOM", -5: "GSIM_E_DEVICE", -6: "GSIM_E_HANDLE", -7: "GSIM_E_OVERFLOW"}
OPT_ARENA_TRANSITIONS, OPT_KERNEL, OPT_KERNEL_TIMING, OPT_LANE_THRESHOLD, OPT_SCHEDULE = 1, 2, 4, 5, 6
OPT_EVAL_FORM = 7
OPT_DF_TICKETS = 8
# values of OPT_EVAL_FORM
FORM_SEGMENTED, FORM_MERGED = 0, 1  # the library default is FORM_MERGED
# values of OPT_SCHEDULE
SCHEDULE_LEVELS, SCHEDULE_DEPENDENCY, SCHEDULE_AUTO, SCHEDULE_LEVEL_BARRIERS = 0, 1, 2, 3
NO_RELATION = 2**31 - 1

EXPORTED = ("sim_create", "sim_destroy", "sim_last_error", "sim_set_option", "sim_load_netlist",
            "sim_load_netlist_ext",
            "sim_unload_netlist", "sim_set_netlist_option", "sim_netlist_info", "sim_memory_info", "sim_submit", "sim_submit_device", "sim_run",
            "sim_run_device", "sim_run_batch", "sim_drive", "sim_job_done", "sim_wait",
            "sim_job_stats", "sim_fetch_waveforms", "sim_fetch_hashes", "sim_release_job", "sim_levelize",
            "sim_validate_stimulus", "sim_version", "sim_run_device_noalloc", "sim_netlist_net_order")


class GsimError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class NetlistInfo(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int64), ("G", ctypes.c_int64), ("P", ctypes.c_int64),
                ("levels", ctypes.c_int32), ("max_delay_ps", ctypes.c_int32),
                ("max_path_delay", ctypes.c_int64), ("lane_gates", ctypes.c_int64)]


class MemoryInfo(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("live_bytes", ctypes.c_uint64),
                ("largest_free_bytes", ctypes.c_uint64), ("jobs_holding_storage", ctypes.c_int64)]


class JobStats(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int64), ("n_out", ctypes.c_int64),
                ("pin_reads", ctypes.c_int64), ("arena_used", ctypes.c_int64),
                ("arena_capacity", ctypes.c_int64), ("device_ms", ctypes.c_double),
                ("eval_ms", ctypes.c_double), ("eval_launches", ctypes.c_int64),
                ("retries", ctypes.c_int64), ("schedule", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgsim.so (built by ``paper_2304_13398_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2304_13398_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname. Loading it first
    # makes libgsim bind to that copy, so a process that uses both has exactly
    # one HIP runtime (two would each try to own the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, i64, i32, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    sig = {
        "sim_create": ([ctypes.c_int, ctypes.c_uint64, P], st),
        "sim_destroy": ([P], st),
        "sim_last_error": ([P], ctypes.c_char_p),
        "sim_set_option": ([P, ctypes.c_int, i64], st),
        "sim_load_netlist": ([P, i64, i64, P, P, P, P, P, P], st),
        "sim_load_netlist_ext": ([P, i64, i64, P, P, P, P, ctypes.c_int32, P, P], st),
        "sim_unload_netlist": ([P, i64], st),
        "sim_netlist_info": ([P, i64, P], st),
        "sim_memory_info": ([P, P], st),
        "sim_set_netlist_option": ([P, i64, ctypes.c_int, i64], st),
        "sim_submit": ([P, i64, P, P, P, P, P], st),
        "sim_submit_device": ([P, i64, P, P, P, i64, ctypes.c_int, P, P], st),
        "sim_run": ([P, i64, P, P, P, P, P], st),
        "sim_run_device": ([P, i64, P, P, P, i64, ctypes.c_int, P, P], st),
        "sim_run_batch": ([P, i64, i32, P, P, P, P, P], st),
        "sim_drive": ([P, P, i32, P, P], st),
        "sim_job_done": ([P, i64, P], st),
        "sim_wait": ([P, i64], st),
        "sim_job_stats": ([P, i64, P], st),
        "sim_fetch_waveforms": ([P, i64, P, i64, P, P, P, i64], st),
        "sim_fetch_hashes": ([P, i64, P, i64, P], st),
        "sim_release_job": ([P, i64], st),
        "sim_levelize": ([i64, i64, P, P, P, P, P, P, P], st),
        "sim_validate_stimulus": ([i64, P, P, P, i64], st),
        "sim_version": ([], ctypes.c_char_p),
        "sim_run_device_noalloc": ([P, i64, P, P, P, i64, P, P, P, i64, P, P], st),
        "sim_netlist_net_order": ([P, i64, P], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(status, ctx=None):
    if status != OK:
        msg = load_library().sim_last_error(ctx)
        raise GsimError(status, msg.decode() if msg else "")


def version() -> str:
    return load_library().sim_version().decode()


def levelize(S, G, type_, pin_off, pin_net, rise, fall):
    """Host levelizer (no device needed): (level[G], n_levels)."""
    lib = load_library()
    type_, pin_off, pin_net = _c(type_, np.uint8), _c(pin_off, np.int64), _c(pin_net, np.int64)
    rise, fall = _c(rise, np.int32), _c(fall, np.int32)
    level = np.zeros(max(G, 1), dtype=np.int32)
    nl = ctypes.c_int32(0)
    _check(lib.sim_levelize(S, G, _p(type_), _p(pin_off), _p(pin_net), _p(rise), _p(fall),
                            _p(level), ctypes.byref(nl)))
    return level[:G], nl.value


def validate_stimulus(S, off, t, v, max_path_delay=0):
    lib = load_library()
    off, t, v = _c(off, np.int64), _c(t, np.int64), _c(v, np.uint8)
    _check(lib.sim_validate_stimulus(S, _p(off), _p(t), _p(v), max_path_delay))


class Sim:
    """A library context on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.lib = load_library()
        h = ctypes.c_void_p()
        _check(self.lib.sim_create(device, hbm_budget_bytes, ctypes.byref(h)))
        self.ctx = h
        self._nl_nets = {}    # netlist handle -> S + G
        self._job_nets = {}   # job handle -> S + G of its netlist

    def close(self):
        if self.ctx:
            _check(self.lib.sim_destroy(self.ctx))
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _ck(self, status):
        _check(status, self.ctx)

    def set_option(self, option: int, value: int):
        self._ck(self.lib.sim_set_option(self.ctx, option, int(value)))

    def load_netlist_ext(self, nl, dly, udp=None) -> int:
        """Extended cell model: ``dly`` int32 [P, 2, 2] (input edge rise/fall,
        output 0/1; NO_RELATION = unrelated pin); ``udp`` uint8 [n, 256] tables
        of user-defined types 12 + i. nl.type may use those types."""
        d = _c(dly, np.int32).reshape(-1)
        if d.size != 4 * int(nl.pin_off[-1] if len(nl.pin_off) else 0):
            raise ValueError("dly must have shape [P, 2, 2]")
        u = _c(udp if udp is not None else np.zeros((0, 256)), np.uint8)
        arrs = (_c(nl.type, np.uint8), _c(nl.pin_off, np.int64), _c(nl.pin_net, np.int64))
        h = ctypes.c_int64()
        self._ck(self.lib.sim_load_netlist_ext(self.ctx, nl.S, nl.G, *[_p(a) for a in arrs], _p(d),
                                               len(u), _p(u) if len(u) else None, ctypes.byref(h)))
        self._nl_nets[h.value] = nl.S + nl.G
        return h.value

    def load_netlist(self, nl) -> int:
        """``nl`` has S, G, type, pin_off, pin_net, rise, fall (workloads.Netlist)."""
        arrs = (_c(nl.type, np.uint8), _c(nl.pin_off, np.int64), _c(nl.pin_net, np.int64),
                _c(nl.rise, np.int32), _c(nl.fall, np.int32))
        h = ctypes.c_int64()
        self._ck(self.lib.sim_load_netlist(self.ctx, nl.S, nl.G, *[_p(a) for a in arrs],
                                           ctypes.byref(h)))
        self._nl_nets[h.value] = nl.S + nl.G
        return h.value

    def unload_netlist(self, h: int):
        self._ck(self.lib.sim_unload_netlist(self.ctx, h))
        self._nl_nets.pop(h, None)

    def set_netlist_option(self, h: int, option: int, value: int):
        self._ck(self.lib.sim_set_netlist_option(self.ctx, h, option, int(value)))

    def netlist_info(self, h: int) -> NetlistInfo:
        info = NetlistInfo()
        self._ck(self.lib.sim_netlist_info(self.ctx, h, ctypes.byref(info)))
        return info

    def memory_info(self) -> MemoryInfo:
        """Device memory of the context (budget, held, largest free)."""
        m = MemoryInfo()
        self._ck(self.lib.sim_memory_info(self.ctx, ctypes.byref(m)))
        return m

    def run(self, h: int, st, stream: int | None = None) -> int:
        """Start a job over host-resident stimuli (st: off, t, v)."""
        off, t, v = _c(st.off, np.int64), _c(st.t, np.int64), _c(st.v, np.uint8)
        j = ctypes.c_int64()
        self._ck(self.lib.sim_run(self.ctx, h, _p(off), _p(t), _p(v),
                                  ctypes.c_void_p(stream) if stream else None, ctypes.byref(j)))
        self._job_nets[j.value] = self._nl_nets.get(h, 0)
        return j.value

    def run_device(self, h: int, d_off: int, d_t: int, d_v: int, n_in: int,
                   stream: int | None = None, validate: bool = False) -> int:
        """Start a job over device-resident stimuli given as raw device pointers."""
        j = ctypes.c_int64()
        self._ck(self.lib.sim_run_device(self.ctx, h, ctypes.c_void_p(d_off), ctypes.c_void_p(d_t),
                                         ctypes.c_void_p(d_v), n_in, 1 if validate else 0,
                                         ctypes.c_void_p(stream) if stream else None,
                                         ctypes.byref(j)))
        self._job_nets[j.value] = self._nl_nets.get(h, 0)
        return j.value

    def run_device_noalloc(self, h: int, d_src_off: int, d_t: int, d_v: int, n_in: int, d_off: int,
                           d_len: int, d_arena: int, arena_cap: int, d_result: int,
                           stream: int | None = None):
        """The allocation-free run over caller-owned device buffers (raw device
        pointers); asynchronous on `stream`."""
        self._ck(self.lib.sim_run_device_noalloc(
            self.ctx, h, ctypes.c_void_p(d_src_off), ctypes.c_void_p(d_t), ctypes.c_void_p(d_v), n_in,
            ctypes.c_void_p(d_off), ctypes.c_void_p(d_len), ctypes.c_void_p(d_arena), arena_cap,
            ctypes.c_void_p(d_result), ctypes.c_void_p(stream) if stream else None))

    def net_order(self, h: int) -> np.ndarray:
        """Index of every net (caller's ids) in the library's net order."""
        n = self.netlist_info(h)
        out = np.empty(n.S + n.G, dtype=np.int64)
        self._ck(self.lib.sim_netlist_net_order(self.ctx, h, _p(out)))
        return out

    def submit(self, h: int, st, stream: int | None = None) -> int:
        """Queue a job over host-resident stimuli (nothing runs until driven)."""
        off, t, v = _c(st.off, np.int64), _c(st.t, np.int64), _c(st.v, np.uint8)
        j = ctypes.c_int64()
        self._ck(self.lib.sim_submit(self.ctx, h, _p(off), _p(t), _p(v),
                                     ctypes.c_void_p(stream) if stream else None, ctypes.byref(j)))
        self._job_nets[j.value] = self._nl_nets.get(h, 0)
        return j.value

    def submit_device(self, h: int, d_off: int, d_t: int, d_v: int, n_in: int,
                      stream: int | None = None, validate: bool = False) -> int:
        j = ctypes.c_int64()
        self._ck(self.lib.sim_submit_device(self.ctx, h, ctypes.c_void_p(d_off),
                                            ctypes.c_void_p(d_t), ctypes.c_void_p(d_v), n_in,
                                            1 if validate else 0,
                                            ctypes.c_void_p(stream) if stream else None,
                                            ctypes.byref(j)))
        self._job_nets[j.value] = self._nl_nets.get(h, 0)
        return j.value

    def run_batch(self, h: int, stims, stream: int | None = None):
        """Batched execution of several stimulus sets over one netlist: job handles."""
        n = len(stims)
        arrs = [(_c(s.off, np.int64), _c(s.t, np.int64), _c(s.v, np.uint8)) for s in stims]
        P = ctypes.c_void_p
        offs = (P * n)(*[a[0].ctypes.data for a in arrs])
        ts = (P * n)(*[a[1].ctypes.data for a in arrs])
        vs = (P * n)(*[a[2].ctypes.data for a in arrs])
        out = np.zeros(n, dtype=np.int64)
        self._ck(self.lib.sim_run_batch(self.ctx, h, n, ctypes.cast(offs, P), ctypes.cast(ts, P),
                                        ctypes.cast(vs, P), ctypes.c_void_p(stream) if stream else None,
                                        _p(out)))
        for j in out.tolist():
            self._job_nets[j] = self._nl_nets.get(h, 0)
        return out.tolist()

    def drive(self, max_ahead: int = 0, stream: int | None = None):
        """One scheduling pass: (active jobs, queued jobs)."""
        a, q = ctypes.c_int32(), ctypes.c_int32()
        self._ck(self.lib.sim_drive(self.ctx, ctypes.c_void_p(stream) if stream else None,
                                    max_ahead, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def done(self, job: int) -> bool:
        d = ctypes.c_int32()
        self._ck(self.lib.sim_job_done(self.ctx, job, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, job: int):
        self._ck(self.lib.sim_wait(self.ctx, job))

    def stats(self, job: int) -> JobStats:
        s = JobStats()
        self._ck(self.lib.sim_job_stats(self.ctx, job, ctypes.byref(s)))
        return s

    def fetch(self, job: int, nets=None):
        """Waveforms of ``nets`` (all S+G nets in id order if None): (off[n+1], t, v)."""
        if nets is None:
            n = self._job_nets[job]
        else:
            nets = _c(nets, np.int64)
            n = len(nets)
        off = np.zeros(n + 1, dtype=np.int64)
        self._ck(self.lib.sim_fetch_waveforms(self.ctx, job, _p(nets), n, _p(off), None, None, 0))
        total = int(off[-1])
        t = np.empty(max(total, 1), dtype=np.int64)
        v = np.empty(max(total, 1), dtype=np.uint8)
        self._ck(self.lib.sim_fetch_waveforms(self.ctx, job, _p(nets), n, _p(off), _p(t), _p(v),
                                              total))
        return off, t[:total], v[:total]

    def lengths(self, job: int, nets=None) -> np.ndarray:
        """Transition counts of ``nets`` (all if None), without copying waveforms."""
        if nets is None:
            n = self._job_nets[job]
        else:
            nets = _c(nets, np.int64)
            n = len(nets)
        off = np.zeros(n + 1, dtype=np.int64)
        self._ck(self.lib.sim_fetch_waveforms(self.ctx, job, _p(nets), n, _p(off), None, None, 0))
        return np.diff(off)

    def hashes(self, job: int, nets=None) -> np.ndarray:
        """Per-net fingerprints (see sim_fetch_hashes) of ``nets`` (all if None)."""
        if nets is None:
            n = self._job_nets[job]
        else:
            nets = _c(nets, np.int64)
            n = len(nets)
        out = np.zeros(max(n, 1), dtype=np.uint64)
        self._ck(self.lib.sim_fetch_hashes(self.ctx, job, _p(nets), n, _p(out)))
        return out[:n]

    def release(self, job: int):
        self._ck(self.lib.sim_release_job(self.ctx, job))
        self._job_nets.pop(job, None)

    def simulate(self, nl, st):
        """Load, run, fetch every gate output, release: (off[G+1], t, v) in gate order."""
        h = self.load_netlist(nl)
        try:
            j = self.run(h, st)
            try:
                self.wait(j)
                return self.fetch(j, np.arange(nl.S, nl.S + nl.G))
            finally:
                self.release(j)
        finally:
            self.unload_netlist(h)
