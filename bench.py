#!/usr/bin/env python3
"""Benchmark of the fused Lax-Wendroff Teukolsky step on one MI355X.

A bench "step" is one time step of the whole hot path over the full grid:
predictor and corrector (paper Eqs. 13-14) with the coefficients of
Eqs. (5)-(12), the particle source, the boundary conditions and the
waveform recorder, all in the library's fused kernel (by default two steps
per launch, bitwise identical to single steps).  The workload is the
largest single-mode grid: a = 0.99, m = 2, s = -2, source at r0 = 8,
32768 x 1024 (r*, theta) points, zero initial data.  Prints one JSON line.

Roofline: the algorithmic traffic of one launch is one read of u^n and one
write of u^{n+k} (64 B per grid point in FP64, 32 B in FP32) whatever the
number k of fused steps; it is divided by the launch's average duration.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
TARGET_FRAC = 0.70         # per-launch fraction of HBM_PEAK the step kernel is built towards
BYTES_PER_UPDATE = {64: 64, 32: 32}   # read (Phi, Pi) + write (Phi', Pi'), complex
KERNEL_SRCS = [os.path.join(ROOT, "paper_0909_4039_amd", "csrc", f) for f in ("teuk_kernels.hip", "teuk_device.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lw_step_traffic.json")


def kernel_code_hash():
    """sha256 of the kernel sources with comments removed and whitespace
    collapsed, so that a comment edit does not void measured counters."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        src = open(f).read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def measured_traffic(prec, rows, order):
    """HBM bytes per launch of the two-step launch at this tiling (theta rows
    per wave, launch form) from rocprofv3 FETCH_SIZE/WRITE_SIZE runs, if they
    were taken on the current kernel code (else None)."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_code_sha256") != kernel_code_hash():
            return None
        e = rec["fp%d" % prec]["%d:%d" % (rows, order)]
        return {"bytes_per_launch": e["fetch_bytes"] + e["write_bytes"], "fetch_bytes": e["fetch_bytes"],
                "write_bytes": e["write_bytes"],
                "source": (f"{os.path.relpath(TRAFFIC_FILE, ROOT)}: rocprofv3 counters taken on the kernel code of "
                           f"commit {rec.get('kernel_commit', '?')} (the same kernel code as the library measured here) at {rows} rows "
                           f"per wave, launch form {order}; not this run's")}
    except (OSError, KeyError, ValueError):
        return None


# Two-step tilings (theta rows per wave, launch form: 0 one wavefront per
# tile in chunk-major block order, 1 the same in group-major order, 2 a
# pair) that --tiling-sweep times, and whose HBM counters the traffic record
# holds: the autotuner's usual choices on 32768 x 1024 and their neighbours.
SWEEP_TILINGS = {64: [(64, 0), (80, 0), (96, 0), (112, 0), (128, 0), (192, 0), (256, 0), (64, 1), (80, 1), (96, 1),
                      (112, 1), (128, 1), (192, 1), (64, 2), (96, 2)],
                 32: [(48, 0), (64, 0), (80, 0), (96, 0), (112, 0), (128, 0), (192, 0), (48, 1), (64, 1), (80, 1),
                      (96, 1), (112, 1), (128, 1), (48, 2), (64, 2), (80, 2), (96, 2)]}


def tiling_sweep(W, steps, warmup):
    """Milliseconds per two-step launch of the largest workload at each of
    SWEEP_TILINGS (no autotuning), FP64 and FP32."""
    import torch
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
    out = {}
    for prec, tilings in SWEEP_TILINGS.items():
        s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, prec=prec)
        s.set_source(W.r0, W.amp)
        s.set_blocking(2)
        res = {}
        for rows, order in tilings:
            s.set_tiling(rows, order)
            s.step(warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.step(steps)
            e1.record(s.stream)
            torch.cuda.synchronize()
            res["%d:%d" % (rows, order)] = e0.elapsed_time(e1) / steps * 2
        s.check_finite()
        s.close()
        out["fp%d" % prec] = {"ms_per_launch": res}
    return out


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2000)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp32", action="store_true")
    p.add_argument("--no-adjoint", action="store_true")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-others", action="store_true")
    p.add_argument("--no-copy", action="store_true")
    p.add_argument("--no-fp32-long", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--tiling-sweep", action="store_true",
                   help="time the largest workload at fixed two-step tilings instead of the benchmark (profiling aid)")
    return p.parse_args()


def time_solver(W, prec, steps, warmup):
    import torch
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
    s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, prec=prec)
    s.set_source(W.r0, W.amp)
    # 40 launches per trial: the best few tilings differ by 1-2 %, about the
    # spread of a 10-launch trial (setup, outside the timed region)
    s.autotune(40)
    kb = s.get_blocking()
    tiling = s.get_tiling()
    s.set_observer(W.rstar_obs, warmup + steps + 1)
    s.step(warmup)
    torch.cuda.synchronize()
    stream = s.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    s.check_finite()
    ms = e0.elapsed_time(e1)
    s.close()
    return ms, dt, kb, tiling


def time_single_step(W, prec, steps=200, warmup=20):
    """The same workload with one step per launch (the unblocked kernel at its
    default tiling): milliseconds per launch, for the per-launch roofline of
    the kernel without temporal blocking."""
    import torch
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
    s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, prec=prec)
    s.set_source(W.r0, W.amp)
    s.set_blocking(1)
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    rows = s.get_tiling()[0]
    s.close()
    return ms, rows


def time_adjoint(steps=None):
    """Adjoint workload (a = 0.6, m = 2, 4096 x 256, 20000 steps, source r0 = 10,
    observer r* = 300): wall time of the forward run with the waveform
    recorded, and of the reverse sweep that returns dL/dPhi0, dL/dPi0,
    dL/dr0 and dL/damp for L = sum |w|^2 (no forward state kept); then the
    same for an inspiralling source, whose sweep returns the gradient of
    every orbit-table entry."""
    import torch
    from paper_0909_4039_amd import inputs, workloads
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    import numpy as np
    W = workloads.ADJOINT
    n = steps or W.steps
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
    s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt)
    s.set_source(W.r0, W.amp)
    phi, pi = inputs.pulse(W.nr, W.nth, W.rstar_min, W.rstar_max, W.m, W.pulse["center"], W.pulse["width"],
                           inputs.seeded_amplitude(W.pulse["seed"]))

    s.set_state(phi, pi)
    tuned = s.autotune(10)
    adj_tuned = s.adjoint_autotune(10)

    table = None

    def forward():
        s.set_state(phi, pi)
        s.set_time(0.0, 0)
        if table is not None:
            s.set_trajectory(table)   # the run starts at the table's first entry
        s.set_observer(W.rstar_obs, n + 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.step(n)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    forward()                       # warm-up
    fwd = min(forward() for _ in range(3))
    g = (2.0 * s.wave).contiguous()
    s.adjoint(g, n, W.rstar_obs)    # warm-up
    adj = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.adjoint(g, n, W.rstar_obs)
        adj.append(time.perf_counter() - t)
    # dL/da (the Kerr spin) by the checkpointed sweep: the forward states
    # are needed, sqrt(N) of them are kept and each segment is recomputed
    s.set_state(phi, pi)
    torch.cuda.synchronize()
    p0, q0 = s.phi.clone(), s.pi.clone()
    t = time.perf_counter()
    dLda = s.param_gradient("a", g, n, W.rstar_obs, p0, q0, h=1e-5)
    torch.cuda.synchronize()
    spin_s = time.perf_counter() - t
    ck = int(np.ceil(np.sqrt(n)))
    # (the cost does not depend on g; at r* = 300 the waveform of this run,
    # hence g and dL/da, is zero: see the adjoint FD test for values)
    del dLda
    spin = {"ms": spin_s * 1e3, "over_forward": spin_s / fwd, "checkpoint_interval": ck,
            "stored_states": int(np.ceil(n / ck)) + ck + 1}
    del p0, q0
    # the same grid and run with an inspiralling source (mass ratio 1e-4):
    # forward with the orbit table, and the reverse sweep that also returns
    # dL/dr0 and dL/dphi of every table entry
    table = inputs.inspiral_trajectory(W.r0, W.a, W.M, 1e-4, dt, n)
    forward()
    fwd_m = min(forward() for _ in range(3))
    g = (2.0 * s.wave).contiguous()
    s.adjoint_moving(g, n, W.rstar_obs)
    adj_m = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.adjoint_moving(g, n, W.rstar_obs)
        adj_m.append(time.perf_counter() - t)
    s.close()
    return {"workload": W.name, "steps": n, "forward_ms": fwd * 1e3, "adjoint_ms": min(adj) * 1e3,
            "adjoint_over_forward": min(adj) / fwd, "stored_forward_states": 0,
            "rows_per_wave": tuned[0], "steps_per_launch": tuned[1],
            "adjoint_rows_per_wave": adj_tuned[0], "adjoint_steps_per_launch": adj_tuned[1],
            "spin_gradient": spin,
            "inspiral": {"forward_ms": fwd_m * 1e3, "adjoint_ms": min(adj_m) * 1e3,
                         "adjoint_over_forward": min(adj_m) / fwd_m, "gradient_entries": 2 * n}}


def _pulse(w):
    from paper_0909_4039_amd import inputs
    p = w.pulse
    return inputs.pulse(w.nr, w.nth, w.rstar_min, w.rstar_max, w.m, p["center"], p["width"], p["amplitude"])


def time_batched(steps=200, graph_steps=20):
    """The 32-instance batch (m = 1..8 x a in {0, 0.3, 0.6, 0.9}, uneven grids
    from seed 3, pulses and sources, FP64, waveforms recorded): updates/s of
    32 single-mode solvers stepped one after another (each autotuned) against
    one batch (autotuned, one persistent launch per two steps, replayed from
    a captured graph).  Results are bitwise identical between the two."""
    import torch
    from paper_0909_4039_amd import workloads
    from paper_0909_4039_amd.batch import Batch, make_desc
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    ws = workloads.batched_instances()
    pts = sum(w.nr * w.nth for w in ws)
    dts = [suggest_dt(w.nr, w.nth, w.rstar_min, w.rstar_max, w.a, w.M, w.m, w.s, w.steps) for w in ws]
    # per mode
    solvers = []
    for w, dt in zip(ws, dts):
        s = Solver(w.nr, w.nth, w.rstar_min, w.rstar_max, w.a, w.M, w.m, w.s, dt)
        s.set_source(w.r0, w.amp)
        s.set_state(*_pulse(w))
        s.set_observer(w.rstar_obs, 2 * steps + 1)
        s.autotune(5)
        solvers.append(s)
    for s in solvers:
        s.step(steps // 10)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s in solvers:
        s.step(steps)
    torch.cuda.synchronize()
    per_mode = time.perf_counter() - t
    for s in solvers:
        s.close()
    del solvers
    torch.cuda.empty_cache()
    # batched
    descs = [make_desc(w.nr, w.nth, w.rstar_min, w.rstar_max, w.a, w.m, dt, s=w.s, r0=w.r0, amp=w.amp,
                       rstar_obs=w.rstar_obs) for w, dt in zip(ws, dts)]
    b = Batch(descs, 2 * steps + 2 * graph_steps)
    for i, w in enumerate(ws):
        b.set_state(i, *_pulse(w))
    rows, kb, persistent = b.autotune(5)
    b.capture_graph(graph_steps)
    b.step(graph_steps)
    b.synchronize()
    t = time.perf_counter()
    b.step(steps)
    b.synchronize()
    batched = time.perf_counter() - t
    b.close()
    del b
    torch.cuda.empty_cache()
    return {"workload": "batch_32_modes_seed3", "instances": len(ws), "points": pts, "steps": steps,
            "per_mode_updates_per_s": pts * steps / per_mode, "batched_updates_per_s": pts * steps / batched,
            "batched_over_per_mode": per_mode / batched, "batch_rows_per_wave": rows, "batch_steps_per_launch": kb,
            "batch_persistent": persistent,
            "graph_steps": graph_steps}


def time_inspiral_modes(steps=1000, graph_steps=20):
    """The m = 1..8 modes of one inspiral (a = 0.9, s = -2, 8192 x 256 each,
    source from r0 = 10 decaying with mass ratio 1e-4, zero initial data,
    waveforms recorded): updates/s of 8 single-mode solvers stepped one
    after another (each autotuned) against one batch of the 8 modes (moving
    build, autotuned, replayed from a captured graph).  Results are bitwise
    identical between the two."""
    import torch
    from paper_0909_4039_amd import inputs, workloads
    from paper_0909_4039_amd.batch import Batch, make_desc
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    W = workloads.KERR_SOURCE   # the 8192 x 256 single-mode workload's grid and orbit
    modes = list(range(1, 9))
    total = steps + 2 * graph_steps
    dts = [suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, m, W.s, W.steps) for m in modes]
    dt = min(dts)   # one time step for all modes, so they share the orbit table
    table = inputs.inspiral_trajectory(W.r0, W.a, W.M, 1e-4, dt, total)
    pts = W.nr * W.nth * len(modes)
    solvers = []
    for m in modes:
        s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, m, W.s, dt)
        s.set_source(W.r0, W.amp)
        s.set_trajectory(table)
        s.set_observer(W.rstar_obs, total + 1)
        s.autotune(5)
        solvers.append(s)
    for s in solvers:
        s.step(graph_steps)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for s in solvers:
        s.step(steps)
    torch.cuda.synchronize()
    per_mode = time.perf_counter() - t
    for s in solvers:
        s.close()
    del solvers
    torch.cuda.empty_cache()
    descs = [make_desc(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, m, dt, s=W.s, r0=W.r0, amp=W.amp,
                       rstar_obs=W.rstar_obs) for m in modes]
    b = Batch(descs, total)
    for i in range(len(modes)):
        b.set_trajectory(i, table)
    rows, kb, persistent = b.autotune(5)
    b.capture_graph(graph_steps)
    b.step(graph_steps)
    b.synchronize()
    t = time.perf_counter()
    b.step(steps)
    b.synchronize()
    batched = time.perf_counter() - t
    b.close()
    del b
    torch.cuda.empty_cache()
    return {"workload": "inspiral_modes_m1-8_a0.9_8192x256", "instances": len(modes), "points": pts,
            "steps": steps, "mass_ratio": 1e-4, "per_mode_updates_per_s": pts * steps / per_mode,
            "batched_updates_per_s": pts * steps / batched, "batched_over_per_mode": per_mode / batched,
            "batch_rows_per_wave": rows, "batch_steps_per_launch": kb, "batch_persistent": persistent}


def time_small_and_mid():
    """Two more single-mode workloads, each autotuned.

    - Schwarzschild pulse, 256 x 64, 2000 steps: a launch-bound grid (16k
      points), stepped by direct launches and as a batch of one replayed from
      a captured HIP graph (bitwise identical results).
    - Kerr a = 0.9 with source, 8192 x 256, 50000 steps, FP64 and FP32.
    """
    import torch
    from paper_0909_4039_amd import inputs, workloads
    from paper_0909_4039_amd.batch import Batch, make_desc
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    out = {}
    W = workloads.SCHWARZSCHILD_PULSE
    n = W.steps
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, n)
    phi, pi = inputs.pulse(W.nr, W.nth, W.rstar_min, W.rstar_max, W.m, W.pulse["center"], W.pulse["width"],
                           inputs.seeded_amplitude(W.pulse["seed"]))
    s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt)
    s.set_state(phi, pi)
    rows, kb = s.autotune(20)
    s.set_observer(W.rstar_obs, 2 * n + 1)
    s.step(n // 10)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.step(n)
    torch.cuda.synchronize()
    direct = time.perf_counter() - t
    s.close()
    b = Batch([make_desc(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.m, dt, s=W.s, rstar_obs=W.rstar_obs)],
              2 * n)
    b.set_state(0, phi, pi)
    brows, bkb, bpers = b.autotune(20)
    g = 200
    b.capture_graph(g)
    b.step(g)
    b.synchronize()
    t = time.perf_counter()
    b.step(n)
    b.synchronize()
    graph = time.perf_counter() - t
    b.close()
    pts = W.nr * W.nth
    out[W.name] = {"steps": n, "direct_us_per_step": direct / n * 1e6, "graph_us_per_step": graph / n * 1e6,
                   "direct_updates_per_s": pts * n / direct, "graph_updates_per_s": pts * n / graph,
                   "rows_per_wave": rows, "steps_per_launch": kb, "graph_steps": g}
    W = workloads.KERR_SOURCE
    n = W.steps
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, n)
    res = {"steps": n}
    for prec in (64, 32):
        s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, prec=prec)
        s.set_source(W.r0, W.amp)
        rows, kb = s.autotune(20)
        s.set_observer(W.rstar_obs, n + 1)
        s.step(100)
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.step(n - 100)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        s.check_finite()
        s.close()
        res[f"fp{prec}"] = {"updates_per_s": W.nr * W.nth * (n - 100) / el, "rows_per_wave": rows,
                            "steps_per_launch": kb}
    out[W.name] = res
    # the same grid with the particle inspiralling (mass ratio 1e-4) from r0 = 10
    from paper_0909_4039_amd import inputs as _inputs
    s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt)
    s.set_source(W.r0, W.amp)
    s.set_trajectory(_inputs.inspiral_trajectory(W.r0, W.a, W.M, 1e-4, dt, n))
    rows, kb = s.autotune(20)
    s.set_observer(W.rstar_obs, n + 1)
    s.step(100)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.step(n - 100)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    s.check_finite()
    s.close()
    out[W.name + "_inspiral"] = {"steps": n, "mass_ratio": 1e-4, "fp64_updates_per_s": W.nr * W.nth * (n - 100) / el,
                                 "rows_per_wave": rows, "steps_per_launch": kb}
    return out


def copy_bandwidth(gib=2.0, reps=20):
    """HBM bandwidth of a plain streaming copy (the library's teuk_stream_copy
    kernel: 16-byte loads and stores, nothing else), read + write bytes over
    time: the practical ceiling beside the 8 TB/s published peak."""
    import ctypes
    import torch
    from paper_0909_4039_amd import _lib
    n = int(gib * 2 ** 30 / 16)
    a = torch.zeros(n, dtype=torch.complex128, device="cuda:0")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    h = ctypes.c_void_p(st.cuda_stream)
    nbytes = n * 16
    _lib.check(_lib.lib().teuk_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, h))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        _lib.check(_lib.lib().teuk_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, h))
    e1.record(st)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    return {"kernel": "stream_copy_kernel (teuk_stream_copy)", "bytes_per_copy": 2 * nbytes,
            "GBs": 2 * nbytes / sec / 1e9, "copy_checked": ok}


def fp32_error_full_length():
    """FP32 waveform error at the workloads' own run lengths.

    - Kerr a = 0.9 with the source, 8192 x 256, zero data, the full 50,000
      steps, read at r* = 20: against the FP64 oracle's waveform of the same
      run (tests/golden/long_kerr_a0.9_source_8192x256_full.npz, written by
      tests/golden/make_long_runs.py from the oracle alone) on its sampled
      steps and rows, and against the GPU's FP64 run on every row.
    - a = 0.99 with the source at r0 = 8, 32768 x 1024, zero data, the full
      100,000 steps, read at r* = 20: against the GPU's FP64 run (the FP64
      path matches the oracle over 2000 steps of this grid in
      tests/test_gpu_long_parity.py).
    Errors are relative L2 over the waveform and max |w32 - w64| / max |w64|."""
    import json as _json
    import numpy as np
    import torch
    from paper_0909_4039_amd import workloads
    from paper_0909_4039_amd.solver import Solver, suggest_dt

    def run(W, n, robs, prec, dt):
        s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, prec=prec)
        s.set_source(W.r0, W.amp)
        s.set_observer(robs, n + 1)
        s.step(n)
        torch.cuda.synchronize()
        s.check_finite()
        w = s.wave.cpu().numpy().astype(np.complex128)
        s.close()
        return w

    def errs(a, b):
        return {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                "max_elem": float(np.max(np.abs(a - b)) / np.max(np.abs(b)))}

    out = {}
    gpath = os.path.join(ROOT, "tests", "golden", "long_kerr_a0.9_source_8192x256_full.npz")
    W = workloads.KERR_SOURCE
    n, robs = W.steps, 20.0
    golden = None
    if os.path.exists(gpath):
        z = np.load(gpath, allow_pickle=False)
        golden = (_json.loads(str(z["meta"])), z["wave"], z["wave_steps"], z["wave_rows"])
    dt = golden[0]["dt"] if golden else suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, n)
    w32 = run(W, n, robs, 32, dt)
    w64 = run(W, n, robs, 64, dt)
    w32s = run(W, n, robs, 48, dt)
    rec = {"steps": n, "rstar_obs": robs, "dt": dt, "vs_gpu_fp64": errs(w32, w64), "bound": 1e-5,
           "fp32_storage_fp64_math": {"vs_gpu_fp64": errs(w32s, w64)}}
    if golden:
        sl = np.ix_(golden[2], golden[3])
        rec["vs_oracle_fp64"] = errs(w32[sl], golden[1])
        rec["fp32_storage_fp64_math"]["vs_oracle_fp64"] = errs(w32s[sl], golden[1])
        rec["gpu_fp64_vs_oracle"] = errs(w64[sl], golden[1])
        rec["oracle_sample"] = f"{len(golden[2])} steps x {len(golden[3])} theta rows"
    out[W.name] = rec
    W = workloads.LARGE
    n, robs = W.steps, 20.0
    dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, n)
    w32 = run(W, n, robs, 32, dt)
    w64 = run(W, n, robs, 64, dt)
    w32s = run(W, n, robs, 48, dt)
    out[W.name] = {"steps": n, "rstar_obs": robs, "dt": dt, "vs_gpu_fp64": errs(w32, w64), "bound": 1e-5,
                   "fp32_storage_fp64_math": {"vs_gpu_fp64": errs(w32s, w64)}}
    return out


_CPU_SAMPLE = """
import json, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import oracle
from paper_0909_4039_amd import workloads
W = workloads.LARGE
oracle.build()
j0, nj = W.nth // 2 - 32, 64
dt = oracle.stable_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
o = oracle.Oracle(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, r0=W.r0, amp=W.amp,
                  rstar_obs=W.rstar_obs, window=(0, W.nr, j0, nj))
phi = np.zeros((nj, W.nr), complex)
pi = np.zeros((nj, W.nr), complex)
t = time.perf_counter()
phi, pi = o.step(phi, pi, 0.0)
one = time.perf_counter() - t
n = max(1, int({seconds} / max(one, 1e-6)) - 1)
t = time.perf_counter()
for k in range(n):
    phi, pi = o.step(phi, pi, (k + 1) * dt)
el = time.perf_counter() - t
print(json.dumps({{"updates_per_s": W.nr * nj * n / el, "steps": n, "seconds": el, "threads": oracle.threads()}}))
"""


def cpu_baseline_single_thread(seconds):
    """The same oracle sample on one thread, in a child process (OMP_NUM_THREADS=1)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _CPU_SAMPLE.format(root=ROOT, seconds=seconds)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def fp32_error():
    """FP32 against FP64 on the GPU path (FP64 matches the oracle to 1e-12):
    relative L2 error of the extracted waveform for the Schwarzschild pulse
    (256 x 64, 2000 steps, read at r* = 30 where the pulse arrives) and for
    the Kerr a = 0.9 source grid (8192 x 256, smooth seeded data, 2000
    steps, read at r* = 20)."""
    import numpy as np
    import torch
    from paper_0909_4039_amd import inputs, workloads
    from paper_0909_4039_amd.solver import Solver, suggest_dt
    out = {}
    for W, n, robs in ((workloads.SCHWARZSCHILD_PULSE, 2000, 30.0), (workloads.KERR_SOURCE, 2000, 20.0)):
        dt = suggest_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
        if W.pulse:
            phi, pi = inputs.pulse(W.nr, W.nth, W.rstar_min, W.rstar_max, W.m, W.pulse["center"], W.pulse["width"],
                                   inputs.seeded_amplitude(W.pulse["seed"]))
        else:
            phi, pi = inputs.smooth_random_state(W.nr, W.nth, W.rstar_min, W.rstar_max, seed=5)
        waves = {}
        for prec in (64, 32):
            s = Solver(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, prec=prec)
            if W.amp:
                s.set_source(W.r0, W.amp)
            s.set_state(phi, pi)
            s.set_observer(robs, n + 1)
            s.step(n)
            torch.cuda.synchronize()
            waves[prec] = s.wave.cpu().numpy().astype(np.complex128)
            s.close()
        err = float(np.linalg.norm(waves[32] - waves[64]) / np.linalg.norm(waves[64]))
        out[W.name] = {"steps": n, "rstar_obs": robs, "waveform_rel_err": err, "bound": 1e-5}
    return out


def cpu_model():
    """The host CPU's model name, its family / model / stepping numbers and
    clock (which name the core generation where a virtual machine shortens
    the name), and the logical core count, as the kernel reports them."""
    fields = {"model name": "model", "cpu family": "family", "model": "model_number", "stepping": "stepping",
              "cpu MHz": "mhz"}
    out = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break          # the first processor's block only
                key, _, val = line.partition(":")
                key = key.strip()
                if key in fields:
                    out[fields[key]] = val.strip()
    except OSError:
        pass
    return {"model": out.get("model"), "family": out.get("family"), "model_number": out.get("model_number"),
            "stepping": out.get("stepping"), "mhz": out.get("mhz"), "logical_cpus": os.cpu_count()}


_CPU_FULL_RUN = """
import json, sys, time
sys.path.insert(0, {root!r})
import oracle
from paper_0909_4039_amd import inputs, workloads
W = workloads.SCHWARZSCHILD_PULSE
oracle.build()
dt = oracle.stable_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
phi, pi = inputs.pulse(W.nr, W.nth, W.rstar_min, W.rstar_max, W.m, W.pulse["center"], W.pulse["width"],
                       inputs.seeded_amplitude(W.pulse["seed"]))
o = oracle.Oracle(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, rstar_obs=W.rstar_obs)
o.run(phi, pi, 10)
t = time.perf_counter()
o.run(phi, pi, W.steps)
el = time.perf_counter() - t
print(json.dumps({{"workload": W.name, "steps": W.steps, "seconds": el,
                  "updates_per_s": W.nr * W.nth * W.steps / el, "threads": oracle.threads()}}))
"""


def cpu_full_run_small():
    """The oracle over the whole Schwarzschild pulse workload (256 x 64, its
    2000 steps, waveform recorded), on one thread in a child process (a grid
    this small gains nothing from more): a full run beside the sampled one."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _CPU_FULL_RUN.format(root=ROOT)], env=env, capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_windows(steps=200):
    """The oracle (all host cores) on 200-step windows of the other workloads'
    full grids: the 8192 x 256 source grid (zero data), the adjoint
    workload's 4096 x 256 grid (pulse and source), and the smallest and the
    largest instance of the 32-mode batch."""
    import time
    import numpy as np
    import oracle
    from paper_0909_4039_amd import inputs, workloads
    oracle.build()
    batch = workloads.batched_instances(3)
    by_size = sorted(batch, key=lambda w: w.nr * w.nth)
    out = {}
    for W in (workloads.KERR_SOURCE, workloads.ADJOINT, by_size[0], by_size[-1]):
        dt = oracle.stable_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
        o = oracle.Oracle(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, r0=W.r0, amp=W.amp,
                          rstar_obs=W.rstar_obs)
        if W.pulse:
            amp = W.pulse.get("amplitude") or inputs.seeded_amplitude(W.pulse["seed"])
            phi, pi = inputs.pulse(W.nr, W.nth, W.rstar_min, W.rstar_max, W.m, W.pulse["center"], W.pulse["width"],
                                   amp)
        else:
            phi = np.zeros((W.nth, W.nr), complex)
            pi = np.zeros((W.nth, W.nr), complex)
        phi, pi, _ = o.run(phi, pi, 2, record=False)   # thread start-up and page faults
        t = time.perf_counter()
        o.run(phi, pi, steps, 2 * dt, record=False)
        el = time.perf_counter() - t
        out[W.name] = {"grid": [W.nr, W.nth], "steps": steps, "seconds": el,
                       "updates_per_s": W.nr * W.nth * steps / el}
    out["threads"] = oracle.threads()
    return out


def cpu_baseline(W, seconds):
    import numpy as np
    import oracle
    from paper_0909_4039_amd import inputs
    oracle.build()
    j0, nj = W.nth // 2 - 32, 64
    dt = oracle.stable_dt(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, W.steps)
    o = oracle.Oracle(W.nr, W.nth, W.rstar_min, W.rstar_max, W.a, W.M, W.m, W.s, dt, r0=W.r0, amp=W.amp,
                      rstar_obs=W.rstar_obs, window=(0, W.nr, j0, nj))
    phi = np.zeros((nj, W.nr), complex)
    pi = np.zeros((nj, W.nr), complex)
    # the first steps pay for thread start-up and page faults: size the
    # timed run from warm steps
    for k in range(3):
        phi, pi = o.step(phi, pi, k * dt)
    t = time.perf_counter()
    for k in range(3, 8):
        phi, pi = o.step(phi, pi, k * dt)
    one = (time.perf_counter() - t) / 5
    n = max(1, int(seconds / max(one, 1e-6)))
    t = time.perf_counter()
    for k in range(n):
        phi, pi = o.step(phi, pi, (k + 8) * dt)
    el = time.perf_counter() - t
    pts = W.nr * nj
    return {"value": pts * n / el, "unit": "grid-point updates/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"theta rows {j0}-{j0 + nj - 1} of the {W.nr}x{W.nth} grid ({pts} points), all r* "
                      f"columns, {n} FP64 steps ({el:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); libteuk has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)
    from paper_0909_4039_amd import workloads
    W = workloads.LARGE
    pts = W.nr * W.nth
    if args.tiling_sweep:
        # the copy kernel runs too: it calibrates the HBM counters of a profiled sweep
        print(json.dumps({"tiling_sweep": tiling_sweep(W, args.steps, args.warmup), "workload": W.name,
                          "hbm_copy": copy_bandwidth()}), flush=True)
        return
    # the oracle's CPU baselines run first, before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, args.cpu_seconds)
        cpu["host"] = cpu_model()
        cpu["single_thread"] = cpu_baseline_single_thread(args.cpu_seconds / 2)
        cpu["full_run"] = cpu_full_run_small()
        cpu["windows"] = cpu_windows()
    import torch
    ms, dt, kb, tiling = time_solver(W, 64, args.steps, args.warmup)
    ms_step = ms / args.steps
    ups = pts * args.steps / (ms * 1e-3)
    launch_s = ms_step * kb * 1e-3               # average duration of one launch (kb steps)
    traffic64 = measured_traffic(64, tiling[0], tiling[1]) if kb == 2 else None
    achieved = BYTES_PER_UPDATE[64] * pts / launch_s
    out = {
        "metric": "grid-point updates/s FP64/FP32 + % HBM roofline; batched vs per-mode; adjoint/fwd",
        "value": ups,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": W.name, "n_rstar": W.nr, "n_theta": W.nth, "rstar": [W.rstar_min, W.rstar_max],
                   "a": W.a, "m": W.m, "s": W.s, "r0": W.r0, "rstar_obs": W.rstar_obs, "dt": dt,
                   "initial_data": "zero, source on", "steps_per_launch": kb,
                   "rows_per_wave": tiling[0],
                   "launch_form": {0: "one wavefront per tile, chunk-major blocks",
                                   1: "one wavefront per tile, group-major blocks"}.get(tiling[1],
                                                                                       "pair of wavefronts per tile")},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK,
                     # measured HBM bytes per launch (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE), or None
                     "traffic": (lambda t: t["bytes_per_launch"] if t else None)(traffic64),
                     "traffic_detail": traffic64,
                     "kernel": ("lw_step_split_kernel<double, double>" if (kb == 2 and tiling[1] == 2)
                                else f"lw_step_kernel<double, double, {kb}, "
                                     f"{'true' if (kb == 2 and 64 * pts > 256 * 2 ** 20) else 'false'}>"),
                     "bytes_per_launch": BYTES_PER_UPDATE[64] * pts, "launch_ms": launch_s * 1e3,
                     "target_frac": TARGET_FRAC, "gap_to_target": TARGET_FRAC - achieved / HBM_PEAK},
        # update rate expressed as the bandwidth an unblocked step would need
        "effective": {"update_bandwidth_GBs": BYTES_PER_UPDATE[64] * ups / 1e9,
                      "frac_of_hbm_peak": BYTES_PER_UPDATE[64] * ups / HBM_PEAK,
                      "note": "not a roofline figure: two fused steps move the bytes of one, and this counts "
                              "64 B per update; roofline.frac is the per-launch fraction"},
    }
    # the kernel without temporal blocking, for comparison: one step per launch
    ms1, rows1 = time_single_step(W, 64)
    out["roofline"]["single_step_kernel"] = {
        "kernel": "lw_step_kernel<double, double, 1, false>", "rows_per_wave": rows1, "launch_ms": ms1,
        "achieved": BYTES_PER_UPDATE[64] * pts / (ms1 * 1e-3) / 1e9,
        "frac": BYTES_PER_UPDATE[64] * pts / (ms1 * 1e-3) / HBM_PEAK,
        "note": "one step per launch: slower per step than the two-step launch above, which is what runs"}
    if not args.no_fp32:
        ms32, _, kb32, tiling32 = time_solver(W, 32, args.steps, args.warmup)
        ups32 = pts * args.steps / (ms32 * 1e-3)
        l32 = ms32 / args.steps * kb32 * 1e-3
        out["fp32"] = {"value": ups32, "unit": "grid-point updates/s", "ms_per_step": ms32 / args.steps,
                       "steps_per_launch": kb32,
                       "hbm_frac_per_launch": BYTES_PER_UPDATE[32] * pts / l32 / HBM_PEAK,
                       "effective_frac": BYTES_PER_UPDATE[32] * ups32 / HBM_PEAK,
                       "rows_per_wave": tiling32[0], "launch_form": tiling32[1],
                       "traffic": measured_traffic(32, tiling32[0], tiling32[1]) if kb32 == 2 else None,
                       "error_vs_fp64": fp32_error()}
        if not args.no_fp32_long:
            out["fp32"]["error_vs_fp64_full_length"] = fp32_error_full_length()
    if not args.no_adjoint:
        out["adjoint"] = time_adjoint()
    if not args.no_batched:
        out["batched"] = time_batched()
        out["inspiral_modes"] = time_inspiral_modes()
    if not args.no_others:
        out["other_workloads"] = time_small_and_mid()
    if not args.no_copy:
        cb = copy_bandwidth()
        out["hbm_copy"] = dict(cb, note="2 GiB read + 2 GiB write by a plain streaming kernel; context for the "
                                        "8 TB/s peak, which stays the roofline's",
                               lw_step_per_launch_frac_of_copy=achieved / (cb["GBs"] * 1e9))
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
