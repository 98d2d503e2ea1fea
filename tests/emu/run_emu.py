"""Build and drive the wave64 emulator of the kernels' per-gate evaluation
(test infrastructure; see emu_eval.cpp).

The emulator runs the device code of csrc/eval_core.h unchanged on the CPU,
one gate at a time, on input waveforms the caller supplies (in the tests: the
oracle's waveforms of the gate's input nets), so that the kernels' per-gate
procedure can be compared with the oracle gate by gate without a GPU.
"""
from __future__ import annotations

import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2304_13398_amd", "csrc")
BUILD = os.path.join(HERE, "_build")

MODES = {"levels": 0, "dataflow": 1, "dataflow_lean": 2, "levels_long": 3, "seg": 4, "seg_dataflow": 5}


def build(asan: bool = False) -> str:
    """Compile the emulator (g++; with AddressSanitizer on the host code if
    asan). Rebuilt when a source is newer than the binary."""
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "emu_eval_asan" if asan else "emu_eval")
    srcs = [os.path.join(HERE, "emu_eval.cpp"), os.path.join(HERE, "wave_emu.h"),
            os.path.join(CSRC, "eval_core.h"), os.path.join(CSRC, "gsim_internal.h")]
    if os.path.exists(exe) and os.path.getmtime(exe) >= max(os.path.getmtime(s) for s in srcs):
        return exe
    cmd = ["g++", "-O2", "-g", "-std=c++17", "-I", os.path.join(HERE, "shim"), "-I", CSRC,
           os.path.join(HERE, "emu_eval.cpp"), "-o", f"{exe}.{os.getpid()}.tmp"]
    if asan:
        cmd[1:1] = ["-fsanitize=address", "-fno-omit-frame-pointer"]
    subprocess.check_call(cmd)
    # a name of its own per process: parallel test workers may build at once
    os.replace(f"{exe}.{os.getpid()}.tmp", exe)
    return exe


def builtin_lut(gate_eval, n_builtin=12, arity=(1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 4, 4)):
    """[type][packed pin values] of the built-in gates from a gate function."""
    lut = np.zeros((n_builtin, 256), dtype=np.uint8)
    for t in range(n_builtin):
        for packed in range(256):
            lut[t, packed] = gate_eval(t, [(packed >> (2 * i)) & 3 for i in range(arity[t])])
    return lut


def run(mode, nl, st, gate_waves, lut, gates=None, dly=None, max_ops=0, asan=False, timeout=1800):
    """Evaluate `gates` (default: all) of netlist `nl` under the emulator,
    with the sources' waveforms `st` and the gates' input waveforms taken from
    `gate_waves` = (off[G+1], t, v). Returns (off, t, v) of the evaluated
    gates' outputs, the per-gate error codes, and the emulator's log."""
    exe = build(asan)
    g_off, g_t, g_v = gate_waves
    net_off = np.concatenate([np.asarray(st.off, np.int64), int(st.off[-1]) + np.asarray(g_off[1:], np.int64)])
    t = np.concatenate([np.asarray(st.t, np.int64), np.asarray(g_t, np.int64)])
    v = np.concatenate([np.asarray(st.v, np.uint8), np.asarray(g_v, np.uint8)])
    keys = (t.astype(np.uint64) << np.uint64(2)) | v.astype(np.uint64)
    gates = np.arange(nl.G, dtype=np.int64) if gates is None else np.asarray(gates, np.int64)
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fin, "wb") as f:
            np.array([MODES[mode] if isinstance(mode, str) else mode, nl.S, nl.G, len(lut),
                      0 if dly is None else 1, len(gates), max_ops], np.int64).tofile(f)
            np.asarray(nl.type, np.uint8).tofile(f)
            np.asarray(nl.pin_off, np.int64).tofile(f)
            np.asarray(nl.pin_net, np.int64).tofile(f)
            np.asarray(nl.rise, np.int32).tofile(f)
            np.asarray(nl.fall, np.int32).tofile(f)
            if dly is not None:
                np.asarray(dly, np.int32).reshape(-1).tofile(f)
            np.asarray(lut, np.uint8).reshape(-1).tofile(f)
            net_off.tofile(f)
            keys.tofile(f)
            gates.tofile(f)
        p = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=timeout)
        if p.returncode != 0:
            raise RuntimeError(f"emulator exited with {p.returncode}:\n{p.stderr[-4000:]}")
        raw = np.fromfile(fout, dtype=np.uint8)
    n = len(gates)
    off = raw[:8 * (n + 1)].view(np.int64)
    m = int(off[-1])
    k = raw[8 * (n + 1):8 * (n + 1 + m)].view(np.uint64)
    err = raw[8 * (n + 1 + m):].view(np.int32)
    return (off.copy(), (k >> np.uint64(2)).astype(np.int64), (k & np.uint64(3)).astype(np.uint8)), err.copy(), p.stderr
