#!/usr/bin/env python3
"""Throughput of the coupled spin-torque-oscillator reservoir on one MI355X.

One benchmark step is one whole job over the workload's synthetic input
series, with every input already resident in HBM: all RK4 steps of every
input sample (coupling contraction, LLG + spin-torque right-hand side,
stage combination, one record per sample) followed by the FP64 ridge
readout of the records.  The metric is node-steps/s = N x RK4 steps per
second of wall time over the timed steps.

Default workload: 10,000 coupled oscillators in FP64, the paper's precision
(1,000 input samples x 20 RK4 steps, dt = 0.01), the largest configuration,
where the coupling matrix (800 MB) is streamed from HBM once per RK4 stage.
The JSON line also carries the same workload in FP32, 1,000 oscillators in
FP32 and FP64 (10,000 samples x 20 steps), 16 oscillators in FP64 (2,000 x
20), the parameter sweep, the multi-stream workload and the adjoints under
"also", the roofline of the dominant kernel, and the CPU oracle timed on
the host cores: a bounded prefix of the default workload, the whole
16-oscillator series and a stated prefix of the 1,000-oscillator series.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-steps/s at N=1e3,1e4 (FP32/FP64); batched-sweep & adjoint vs plain, % roofline"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {
    "k_sweep_stage": ("sto_device.hpp", "sto_internal.hpp", "sto_sweep.hpp", "sto_sweep.hip", "sweep_tune.hpp"),
    "k_multi": ("sto_device.hpp", "sto_internal.hpp", "sto_multi.hip"),
    "k_stage": ("sto_device.hpp", "sto_internal.hpp", "sto_kernels.hip"),
    "k_small": ("sto_device.hpp", "sto_internal.hpp", "sto_small.hip"),
    "k_resident": ("sto_device.hpp", "sto_internal.hpp", "sto_resident.hip"),
}


# Of the shared internal header only the structures a kernel takes as
# arguments enter its hash: the rest of it is host-side.
KERNEL_STRUCTS = {"k_sweep_stage": ("SweepRes", "SweepTask", "SweepDev")}
DEFAULT_STRUCTS = ("DevState",)


def _kernel_structs(text: str, names) -> bytes:
    import re
    parts = []
    for name in names:
        m = re.search(r"struct " + name + r" \{.*?\n\};", text, flags=re.S)
        parts.append(m.group(0) if m else "")
    return "\n".join(parts).encode()


def kernel_source_hash(kernel: str) -> str:
    """Hash of the sources a kernel is compiled from (stale counters are dropped)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2312_01121_amd", "csrc", f), "rb") as fh:
            data = fh.read()
        if f == "sto_internal.hpp":
            data = _kernel_structs(data.decode(), KERNEL_STRUCTS.get(kernel, DEFAULT_STRUCTS))
        h.update(data)
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str, dtype: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; otherwise None."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get(f"{kernel}/{workload}/{dtype}")
    if not rec or rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def washout_of(samples: int) -> int:
    """Records skipped before the readout fit: max(5, ceil(samples / 10))."""
    return max(5, int(math.ceil(0.1 * samples)))


def run_workload(stx, torch, name: str, dtype: str, steps: int, warmup: int, arrays=None, samples=None):
    from workloads import WORKLOADS, make_workload_arrays
    from paper_2312_01121_amd import params

    wl = WORKLOADS[name]
    if samples is not None:
        wl = wl.with_samples(samples)
        if arrays is not None:
            arrays = dict(arrays, u=arrays["u"][:samples].copy(), y=arrays["y"][:samples].copy())
    a = arrays if arrays is not None else make_workload_arrays(wl)
    prm = stx.make_params(**params.table1(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps),
                          dtype=dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    elem = 8 if dtype == "f64" else 4
    r = stx.Reservoir(a["W"], a["w_in"], a["m0"], prm)
    path = r.path
    u_d = torch.from_numpy(a["u"]).cuda()
    y = a["y"].copy()
    y[:5] = 0.0                                     # undefined targets lie inside the washout
    y_d = torch.from_numpy(y).cuda()
    states = torch.empty((wl.samples, wl.n, 3), dtype=tdt, device="cuda")
    w_out = torch.empty(wl.n + 1, dtype=torch.float64, device="cuda")
    wash = washout_of(wl.samples)
    stream = torch.cuda.current_stream()

    def one_step():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r.run_device(u_d, states, stream)
        e1.record(stream)
        _, nmse = stx.readout_fit_device(states, y_d, wash, wl.ridge, 0, w_out, stream)
        e2.record(stream)
        return e0, e1, e2, nmse

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [one_step() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_each = sorted(e0.elapsed_time(e1) for e0, e1, _, _ in evs)
    run_ms = sum(run_each) / steps
    fit_ms = sum(e1.elapsed_time(e2) for _, e1, e2, _ in evs) / steps
    nmse = evs[-1][3]
    r.close()
    wall_s = (t1 - t0) / steps
    # a path that runs the whole series in one launch, against one launch per
    # RK4 stage (the stream kernel) on the same inputs, outside the timed steps
    stream_us = None
    if path != "stream":
        k_samples = min(wl.samples, 1000)
        prm_s = stx.make_params(**params.table1(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps),
                                dtype=dtype, path="stream")
        with stx.Reservoir(a["W"], a["w_in"], a["m0"], prm_s) as rs:
            u_k = u_d[:k_samples].contiguous()
            rs.run_device(u_k[:1].contiguous(), states[:1], stream)
            rs.set_state(a["m0"])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rs.run_device(u_k, states[:k_samples], stream)
            e1.record(stream)
            torch.cuda.synchronize()
            stream_us = e0.elapsed_time(e1) * 1e3 / (k_samples * wl.substeps)
    node_steps = wl.n * wl.steps
    launches = 4 * wl.steps if path == "stream" else 1
    kernel = {"stream": "k_stage", "resident": "k_resident", "small": "k_small"}[path]
    algo_bytes = float(wl.n) * wl.n * elem * 4 * wl.steps / launches   # W read once per RK4 stage
    launch_s = run_ms * 1e-3 / launches
    achieved = algo_bytes / launch_s / 1e9
    return {
        "workload": name, "n": wl.n, "dtype": dtype, "path": path, "samples": wl.samples,
        "substeps": wl.substeps, "rk4_steps": wl.steps, "dt": wl.dt,
        "value": node_steps / wall_s, "ms_per_step": wall_s * 1e3,
        "run_ms": run_ms, "run_ms_median": run_each[len(run_each) // 2], "run_ms_min": run_each[0],
        "run_ms_max": run_each[-1], "readout_ms": fit_ms, "us_per_rk4_step": run_ms * 1e3 / wl.steps,
        "readout_nmse": nmse,
        "kernel": kernel, "launches_per_run": launches, "avg_launch_us": launch_s * 1e6,
        "algo_bytes_per_launch": algo_bytes, "achieved_gbs": achieved,
        "hbm_frac": achieved / HBM_PEAK_GBS,
        "stream_path_us_per_rk4_step": stream_us,
        "speedup_vs_stream_path": (stream_us / (run_ms * 1e3 / wl.steps)) if stream_us else None,
    }


def run_adjoint_workload(stx, torch, name: str, dtype: str, samples: int, steps: int, warmup: int):
    """Gradient of the ridge objective of a run with respect to W, w_in, m0
    and the four scalars: forward run, readout fit, readout gradient and the
    adjoint (reservoir_adjoint_device), over the first `samples` input
    samples of the workload; the plain forward run of the same inputs is
    timed beside it."""
    from workloads import WORKLOADS, make_workload_arrays
    from paper_2312_01121_amd import params

    wl = WORKLOADS[name].with_samples(samples)
    a = make_workload_arrays(wl)
    prm = stx.make_params(**params.table1(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps),
                          dtype=dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    elem = 8 if dtype == "f64" else 4
    r = stx.Reservoir(a["W"], a["w_in"], a["m0"], prm)
    u_d = torch.from_numpy(a["u"]).cuda()
    y = a["y"].copy()
    y[:5] = 0.0
    y_d = torch.from_numpy(y).cuda()
    m0_d = torch.from_numpy(a["m0"]).to("cuda", tdt).contiguous()
    states = torch.empty((wl.samples, wl.n, 3), dtype=tdt, device="cuda")
    wash = washout_of(wl.samples)
    stream = torch.cuda.current_stream()

    def one_step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        r.set_state(a["m0"])
        ev[0].record(stream)
        r.run_device(u_d, states, stream)
        ev[1].record(stream)
        w_d, _ = stx.readout_fit_device(states, y_d, wash, wl.ridge, 0, None, stream)
        g_d, loss = stx.readout_grad_device(states, y_d, wash, wl.ridge, w_d, 0, None, stream)
        ev[2].record(stream)
        out = r.adjoint_device(m0_d, u_d, grad_states_dev=g_d, stream=stream)
        ev[3].record(stream)
        return ev, loss, out

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [one_step() for _ in range(steps)]
    torch.cuda.synchronize()
    wall_s = (time.perf_counter() - t0) / steps
    fwd_ms = sum(ev[0].elapsed_time(ev[1]) for ev, _, _ in runs) / steps
    loss_ms = sum(ev[1].elapsed_time(ev[2]) for ev, _, _ in runs) / steps
    adj_ms = sum(ev[2].elapsed_time(ev[3]) for ev, _, _ in runs) / steps
    path = r.path
    out = runs[-1][2]
    finite = bool(torch.isfinite(out["W"]).all()) and bool(torch.isfinite(out["scalars"]).all())
    r.close()
    # passes over W (or its transpose) the adjoint makes: the forward with
    # checkpoints, the recompute of every segment but the last, the reverse
    ld = (wl.n + 63) // 64 * 64
    per_step = (4 * (3 + 2) + 1) * ld * elem
    seg = max(1, min(wl.steps, (4 << 30) // per_step))
    last = wl.steps - (wl.steps - 1) // seg * seg
    stage_passes = 4 * (wl.steps + (wl.steps - last) + wl.steps)
    algo = stage_passes * float(wl.n) * wl.n * elem
    return {
        "workload": f"adjoint/{name}", "n": wl.n, "dtype": dtype, "samples": wl.samples,
        "rk4_steps": wl.steps, "forward_path": path, "checkpoint_every": seg,
        "value": wl.n * wl.steps / (adj_ms * 1e-3), "unit": "node-steps/s (gradient)",
        "ms_per_step": wall_s * 1e3, "forward_ms": fwd_ms, "loss_ms": loss_ms, "adjoint_ms": adj_ms,
        "adjoint_over_forward": adj_ms / fwd_ms, "us_per_rk4_step": adj_ms * 1e3 / wl.steps,
        "stage_passes_over_W": stage_passes, "algo_bytes": algo,
        "effective_gbs": algo / (adj_ms * 1e-3) / 1e9, "hbm_frac": algo / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "ridge_objective": runs[-1][1], "gradients_finite": finite,
    }


def run_streams_workload(stx, torch, name: str, steps: int, warmup: int, coupling: str = "x", plain: bool = True):
    """S input streams share one reservoir (FP32 MFMA coupling on the
    multi-stream path, either coupling); one step is the run of every stream
    plus one readout per stream.  The same runs through the plain
    single-reservoir path, one stream after another over the whole series,
    are timed beside it (unless plain is False)."""
    from workloads import STREAMS, WORKLOADS, make_stream_arrays
    from paper_2312_01121_amd import params

    wl = WORKLOADS[name]
    S = STREAMS[name]
    a = make_stream_arrays(wl, S)
    prm = stx.make_params(**params.table1(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps), dtype="f32",
                          coupling=coupling)
    import numpy as np
    m0s = np.ascontiguousarray(np.broadcast_to(a["m0"], (S, wl.n, 3)))
    r = stx.Reservoir(a["W"], a["w_in"], m0s, prm, streams=S)
    u_d = torch.from_numpy(a["u"]).cuda()
    y = np.nan_to_num(a["y"], nan=0.0)
    y_d = [torch.from_numpy(np.ascontiguousarray(y[:, st])).cuda() for st in range(S)]
    states = torch.empty((wl.samples, S, wl.n, 3), dtype=torch.float32, device="cuda")
    w_outs = [torch.empty(wl.n + 1, dtype=torch.float64, device="cuda") for _ in range(S)]
    wash = washout_of(wl.samples)
    stream = torch.cuda.current_stream()

    def one_step():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r.run_device(u_d, states, stream)
        e1.record(stream)
        # one readout per stream, all fitted in one batched call
        _, nm = stx.readout_fit_batch_device([states[:, st] for st in range(S)], y_d, wash, wl.ridge, 0, w_outs,
                                             stream)
        return e0, e1, list(nm)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [one_step() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in evs) / steps
    nmse = evs[-1][2]
    path = r.path
    r.close()
    # plain path: every stream through the single-reservoir kernels, one
    # after another, each over the whole series (measured, not scaled)
    plain_path, plain_ms = None, None
    if plain:
        r1 = stx.Reservoir(a["W"], a["w_in"], a["m0"], prm)
        plain_path = r1.path
        st1 = torch.empty((wl.samples, wl.n, 3), dtype=torch.float32, device="cuda")
        u_all = [torch.from_numpy(np.ascontiguousarray(a["u"][:, st])).cuda() for st in range(S)]
        r1.run_device(u_all[0], st1, stream)                # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for st in range(S):
            r1.set_state(a["m0"])
            r1.run_device(u_all[st], st1, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1)
        r1.close()
    wall_s = (t1 - t0) / steps
    C = 3 if coupling == "xyz" else 1
    flops = 2.0 * wl.n * wl.n * S * C * 4 * wl.steps
    return {
        "workload": name, "n": wl.n, "streams": S, "coupling": coupling, "dtype": "f32", "path": path,
        "samples": wl.samples,
        "substeps": wl.substeps, "rk4_steps": wl.steps,
        "value": S * wl.n * wl.steps / wall_s, "ms_per_step": wall_s * 1e3, "run_ms": run_ms,
        "us_per_rk4_step": run_ms * 1e3 / wl.steps, "readout_nmse_mean": float(np.mean(nmse)),
        "kernel": "k_multi" if path == "multi" else "k_bfwd", "mfma_tflops": flops / (run_ms * 1e-3) / 1e12,
        "mfma_frac": flops / (run_ms * 1e-3) / 157.3e12,
        "plain_path": plain_path, "plain_run_ms_for_all_streams": plain_ms,
        "speedup_vs_plain": plain_ms / run_ms if plain_ms else None,
    }


def run_streams_adjoint_workload(stx, torch, name: str, coupling: str, steps: int, warmup: int,
                                 checkpoint_every: int = 100, own_checkpoints: bool = False):
    """The differentiation workload: S input streams share one reservoir;
    one step is the forward run of every stream, one ridge readout and its
    objective's gradient per stream, and the adjoint of all streams
    (gradients of the summed objective with respect to W, w_in, every
    stream's m0 and the four scalars), with a state checkpoint every
    `checkpoint_every` RK4 steps.  The checkpoints are the forward run's
    records (reservoir_adjoint_records_device: each segment is recomputed
    from its record and reversed), or with own_checkpoints the adjoint's own
    checkpointing forward pass (reservoir_adjoint_device).  The coupling is all three components (an
    N x N by N x 3S product per stage) or x only.  The coupling and input
    amplitudes are the paper's (A_cp = A_in = 1 Oe): at the workload's
    a_cp = 0.1, a_in = 1 the trajectory is chaotic (largest Lyapunov exponent
    about 0.5 per ns), and the adjoint of a 200 ns horizon grows by ~e^100,
    beyond the FP32 range."""
    import numpy as np
    from workloads import STREAMS, WORKLOADS, make_stream_arrays
    from paper_2312_01121_amd import params

    wl = WORKLOADS[name]
    S = STREAMS[name]
    a = make_stream_arrays(wl, S)
    amp = params.field_unit()          # 1 Oe in the dimensionless unit
    prm = stx.make_params(**params.table1(a_cp=amp, a_in=amp, dt=wl.dt, substeps=wl.substeps),
                          dtype="f32", coupling=coupling)
    m0s = np.ascontiguousarray(np.broadcast_to(a["m0"], (S, wl.n, 3)))
    r = stx.Reservoir(a["W"], a["w_in"], m0s, prm, streams=S)
    path = r.path
    u_d = torch.from_numpy(a["u"]).cuda()
    y = np.nan_to_num(a["y"], nan=0.0)
    y_d = [torch.from_numpy(np.ascontiguousarray(y[:, st])).cuda() for st in range(S)]
    m0_d = torch.from_numpy(m0s).to("cuda", torch.float32).contiguous()
    states = torch.empty((wl.samples, S, wl.n, 3), dtype=torch.float32, device="cuda")
    g_rec = torch.empty_like(states)
    wash = washout_of(wl.samples)
    stream = torch.cuda.current_stream()

    def one_step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        r.set_state(m0s)
        ev[0].record(stream)
        r.run_device(u_d, states, stream)
        ev[1].record(stream)
        loss = 0.0
        w_ds, _ = stx.readout_fit_batch_device([states[:, st] for st in range(S)], y_d, wash, wl.ridge, 0, None,
                                               stream)
        for st in range(S):
            rec = states[:, st].contiguous()
            g, j = stx.readout_grad_device(rec, y_d[st], wash, wl.ridge, w_ds[st], 0, None, stream)
            g_rec[:, st] = g
            loss += j
        ev[2].record(stream)
        out = r.adjoint_device(m0_d, u_d, grad_states_dev=g_rec, checkpoint_every=checkpoint_every, stream=stream,
                               records_dev=None if own_checkpoints else states)
        ev[3].record(stream)
        return ev, loss, out

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [one_step() for _ in range(steps)]
    torch.cuda.synchronize()
    wall_s = (time.perf_counter() - t0) / steps
    fwd_ms = sum(ev[0].elapsed_time(ev[1]) for ev, _, _ in runs) / steps
    loss_ms = sum(ev[1].elapsed_time(ev[2]) for ev, _, _ in runs) / steps
    adj_ms = sum(ev[2].elapsed_time(ev[3]) for ev, _, _ in runs) / steps
    out = runs[-1][2]
    finite = all(bool(torch.isfinite(t).all()) for t in out.values())
    r.close()
    C = 3 if coupling == "xyz" else 1
    segs = (wl.steps + checkpoint_every - 1) // checkpoint_every
    last = wl.steps - (segs - 1) * checkpoint_every
    # stage products of the adjoint: [checkpointing forward,] recompute, reverse
    if own_checkpoints:
        products = 4 * (wl.steps + (wl.steps - last) + wl.steps)
    else:
        products = 4 * (wl.steps + wl.steps)
    flops = products * 2.0 * wl.n * wl.n * S * C + 2.0 * wl.n * wl.n * 4 * wl.steps * S * C   # + dL/dW
    return {
        "workload": f"adjoint/{name}", "n": wl.n, "streams": S, "coupling": coupling, "dtype": "f32",
        "a_cp": amp, "a_in": amp,
        "forward_path": path, "samples": wl.samples, "rk4_steps": wl.steps, "checkpoint_every": checkpoint_every,
        "checkpoints": "own forward pass" if own_checkpoints else "the run's records",
        "value": S * wl.n * wl.steps / (adj_ms * 1e-3), "unit": "node-steps/s (gradient)",
        "ms_per_step": wall_s * 1e3, "forward_ms": fwd_ms, "loss_ms": loss_ms, "adjoint_ms": adj_ms,
        "adjoint_over_forward": adj_ms / fwd_ms, "us_per_rk4_step": adj_ms * 1e3 / wl.steps,
        "mfma_tflops": flops / (adj_ms * 1e-3) / 1e12, "mfma_frac": flops / (adj_ms * 1e-3) / 157.3e12,
        "ridge_objective_sum": runs[-1][1], "gradients_finite": finite,
    }


def run_sweep_workload(stx, torch, name: str, steps: int, warmup: int, plain_samples: int = 200,
                       samples=None, plain: bool = True):
    """Parameter sweep (SWEEP path): every reservoir's run plus one readout
    per reservoir is one step.  The plain single-reservoir path (each
    reservoir alone, its own auto-selected kernel, one after another) is
    timed on the first ``plain_samples`` samples (all of them with
    --plain-full) and scaled to the full series; the per-sample cost of
    every path is constant, so the scaling is linear."""
    import numpy as np
    from workloads import SWEEPS, make_sweep_arrays
    from paper_2312_01121_amd import params

    sw_def = SWEEPS[name]
    if samples is not None:
        import dataclasses
        sw_def = dataclasses.replace(sw_def, samples=samples)
    a = make_sweep_arrays(sw_def)
    res = a["reservoirs"]
    for r in res:
        r["prm"] = stx.make_params(**params.table1(a_cp=r["a_cp"], a_in=r["a_in"], dt=sw_def.dt,
                                                   substeps=sw_def.substeps, current_scale=r["current_scale"],
                                                   field_scale=r["field_scale"]), dtype="f32")
    sw = stx.Sweep(res)
    T = sw_def.samples
    u_d = torch.from_numpy(a["u"]).cuda()
    y_d = torch.from_numpy(np.nan_to_num(a["y"], nan=0.0)).cuda()
    states = torch.empty(T * sw.nodes * 3, dtype=torch.float32, device="cuda")
    w_outs = [torch.empty(n + 1, dtype=torch.float64, device="cuda") for n in sw.ns]
    wash = washout_of(T)
    stream = torch.cuda.current_stream()

    def one_step():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sw.run_device(u_d, states, stream)
        e1.record(stream)
        # one readout per reservoir, all fitted in one batched call
        recs = [states[T * 3 * int(sw.offsets[i]): T * 3 * int(sw.offsets[i + 1])].view(T, n, 3)
                for i, n in enumerate(sw.ns)]
        _, nm = stx.readout_fit_batch_device(recs, y_d, wash, sw_def.ridge, 0, w_outs, stream)
        return e0, e1, list(nm)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [one_step() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in evs) / steps
    nmse = np.array(evs[-1][2])
    sw.close()
    # plain path: each reservoir alone
    plain_samples = min(plain_samples, T)
    u_p = torch.from_numpy(np.ascontiguousarray(a["u"][:plain_samples])).cuda()
    plain_ms = 0.0
    paths = {}
    for r in (res if plain else []):
        one = stx.Reservoir(r["W"], r["w_in"], r["m0"], r["prm"])
        paths[one.path] = paths.get(one.path, 0) + 1
        st1 = torch.empty((plain_samples, r["n"], 3), dtype=torch.float32, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        one.run_device(u_p, st1, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms += e0.elapsed_time(e1) * T / plain_samples
        one.close()
    wall_s = (t1 - t0) / steps
    launches = 4 * sw_def.steps
    algo = float(sum(r["n"] ** 2 for r in res)) * 4
    achieved = algo / (run_ms * 1e-3 / launches) / 1e9
    return {
        "workload": name, "reservoirs": len(res), "nodes": int(sw.nodes), "n_min": int(min(sw.ns)),
        "n_max": int(max(sw.ns)), "dtype": "f32", "path": "sweep", "samples": T, "rk4_steps": sw_def.steps,
        "value": sw.nodes * sw_def.steps / wall_s, "ms_per_step": wall_s * 1e3, "run_ms": run_ms,
        "us_per_rk4_step": run_ms * 1e3 / sw_def.steps, "kernel": "k_sweep_stage", "launches_per_run": launches,
        "algo_bytes_per_launch": algo, "achieved_gbs": achieved, "hbm_frac": achieved / HBM_PEAK_GBS,
        "readout_nmse_median": float(np.median(nmse)), "readout_nmse_min": float(np.min(nmse)),
        "plain_paths": paths, "plain_run_ms_estimate": plain_ms if plain else None,
        "plain_samples_timed": plain_samples if plain else 0,
        "speedup_vs_plain": plain_ms / run_ms if plain else None,
    }


# Table 2 of the paper (wall time in seconds for its stated benchmark: u = 0,
# FP64, RK4 with a 1e-11 s step): its NumPy baseline and its GPU Torch code.
PAPER_N = [1, 10, 100, 1000, 2500, 5000, 10000]
PAPER_TABLE2_S = {
    "numpy_base": [0.81, 0.93, 1.12, 5.78, 36.38, 2.79 * 60, 13.40 * 60],
    "torch_gpu": [None, 7.47, 7.55, 7.14, 7.59, 0.22 * 60, 0.56 * 60],
}


def paper_table(stx, torch, steps: int, repeats: int = 3, chunk_steps: int = 50000, sizes=None):
    """The paper's benchmark on this GPU: u = 0, FP64, dt = 1e-11 s (0.01 in
    units of 1 ns), the paper's coupling generator (U[-1,1], zero diagonal,
    spectral radius 1), its identical initial tilt and A_cp = A_in = 1 Oe,
    for N = 1 ... 10^4, ``steps`` RK4 steps each, ``repeats`` times from the
    same initial state (the paper reports the mean of repeated runs, Sec. 4).
    A long run is issued in chunks of ``chunk_steps`` steps that continue
    the state (bitwise the same as one call), each writing its records into
    one reused buffer, so that progress can be printed."""
    import numpy as np
    from workloads import make_paper_arrays
    from paper_2312_01121_amd import params

    g = params.field_unit()
    substeps = 20
    samples = max(1, steps // substeps)
    chunk = max(1, min(samples, chunk_steps // substeps))
    rows = []
    for i, n in enumerate(PAPER_N):
        if sizes and n not in sizes:
            continue
        a = make_paper_arrays(n, 1)
        prm = stx.make_params(**params.table1(a_cp=g * 1.0, a_in=g * 1.0, substeps=substeps), dtype="f64")
        r = stx.Reservoir(a["W"], a["w_in"], a["m0"], prm)
        u_d = torch.zeros((chunk, 1), dtype=torch.float64, device="cuda")
        states = torch.empty((chunk, n, 3), dtype=torch.float64, device="cuda")
        r.run_device(u_d[:1].contiguous(), states[:1].contiguous())   # warm-up
        stream = torch.cuda.current_stream()
        secs, drift = [], 0.0
        for rep in range(repeats):
            r.set_state(a["m0"])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            done = 0
            while done < samples:
                k = min(chunk, samples - done)
                r.run_device(u_d[:k], states[:k], stream)
                done += k
                if done < samples:
                    # progress of a long run (the wait does not enter the event time)
                    torch.cuda.synchronize()
                    log(f"paper N={n} repeat {rep + 1}: {done * substeps} of {samples * substeps} steps")
                    drift = max(drift, float(torch.max(torch.abs(torch.linalg.norm(states[:k], dim=2) - 1.0))))
            e1.record(stream)
            torch.cuda.synchronize()
            secs.append(e0.elapsed_time(e1) * 1e-3)
            k = samples - (samples - 1) // chunk * chunk
            drift = max(drift, float(torch.max(torch.abs(torch.linalg.norm(states[:k], dim=2) - 1.0))))
        med = float(np.median(secs))
        base = PAPER_TABLE2_S["numpy_base"][i]
        rows.append({"n": n, "path": r.path, "rk4_steps": samples * substeps, "repeats": repeats,
                     "seconds": secs, "seconds_median": med, "seconds_min": min(secs), "seconds_max": max(secs),
                     "us_per_rk4_step": med * 1e6 / (samples * substeps),
                     "node_steps_per_s": n * samples * substeps / med, "max_norm_drift": drift,
                     "paper_numpy_base_s": base, "paper_torch_gpu_s": PAPER_TABLE2_S["torch_gpu"][i]})
        r.close()
        log(json.dumps(rows[-1]))
    return rows


def oracle_rate(name: str, arrays, budget_s: float, whole: bool = False):
    """The FP64 oracle (correctly rounded coupling sums) on the first input
    samples of a workload, sample by sample until the time budget would be
    exceeded (or over every sample with ``whole``).  Returns node-steps/s,
    the samples run, the seconds and the threads the coupling product used."""
    from oracle import _native, constants, sto
    from workloads import WORKLOADS

    wl = WORKLOADS[name]
    prm = constants.dimensionless(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps)
    samples = 0
    total = len(arrays["u"])
    t0 = time.perf_counter()
    m = arrays["m0"]
    while True:
        _, m = sto.run(arrays["W"], arrays["w_in"], m, arrays["u"][samples:samples + 1], prm)
        samples += 1
        el = time.perf_counter() - t0
        if samples >= total:
            break
        if not whole and (el >= budget_s * 0.5 or el / samples * (samples + 1) > budget_s):
            break
    # the product runs on one thread below 2^16 matrix entries, else on all
    threads = _native.exact_threads() if wl.n * wl.n >= (1 << 16) else 1
    return wl.n * samples * wl.substeps / el, samples, el, threads


def cpu_baseline(name: str, arrays, budget_s: float = 12.0):
    """The oracle on this host's cores: a bounded prefix of the benchmark's
    own workload (the reported value), the whole 16-oscillator series and a
    prefix of the 1,000-oscillator series, and the oracle's NumPy-BLAS form."""
    from oracle import constants
    from workloads import WORKLOADS, make_workload_arrays

    wl = WORKLOADS[name]
    value, samples, el, threads = oracle_rate(name, arrays, budget_s)
    others = []
    for other, whole, budget in (("sto16", True, 0.0), ("sto1k", False, 12.0)):
        if other == name:
            continue
        ow = WORKLOADS[other]
        a = make_workload_arrays(ow)
        v, smp, sec, thr = oracle_rate(other, a, budget, whole=whole)
        others.append({
            "workload": other, "n": ow.n, "value": v, "unit": "node-steps/s", "cores": thr,
            "samples": smp, "rk4_steps": smp * ow.substeps, "seconds": sec,
            "horizon": "whole series" if smp == ow.samples else f"first {smp} of {ow.samples} samples",
        })
        log(json.dumps(others[-1]))
    prm = constants.dimensionless(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps)
    return {
        "value": value, "unit": "node-steps/s", "cores": threads, "kind": "oracle",
        "sample": f"first {samples} input sample(s) = {samples * wl.substeps} RK4 steps of the {name} "
                  f"workload (N={wl.n}), FP64 oracle with correctly rounded coupling sums, {el:.1f} s",
        "other_workloads": others,
        "blas_form": cpu_blas_form(name, arrays, prm),
    }


def phase_breakdown(stx, torch, name: str, dtype: str, stages: int = 400, samples: int = 20, coupling: str = "x"):
    """Exchange phases of the persistent kernel a workload runs on
    (reservoir_trace_phases): wave 0 of every workgroup stamps the device's
    constant-rate clock at stage start, stage input gathered, own rows
    computed and own rows published, for the first `stages` RK4 stages of a
    run of `samples` samples.  Medians over workgroups and stages, in
    microseconds; `after_last_publish` is the time from the last workgroup's
    publish of a stage to a workgroup's completed gather of the next."""
    import numpy as np
    from workloads import STREAMS, WORKLOADS, make_stream_arrays, make_workload_arrays
    from paper_2312_01121_amd import params

    wl = WORKLOADS[name]
    S = STREAMS.get(name, 1)
    if S > 1:
        dtype = "f32"
        a = make_stream_arrays(wl, S, samples=samples)
        m0 = np.ascontiguousarray(np.broadcast_to(a["m0"], (S, wl.n, 3)))
    else:
        a = make_workload_arrays(wl, samples=samples)
        m0 = a["m0"]
    prm = stx.make_params(**params.table1(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps),
                          dtype=dtype, coupling=coupling)
    r = stx.Reservoir(a["W"], a["w_in"], m0, prm, streams=S)
    u = torch.from_numpy(a["u"]).cuda()
    r.run_device(u[:1].contiguous())                   # warm-up
    r.set_state(m0)
    r.trace_phases(stages)
    r.run_device(u)
    torch.cuda.synchronize()
    st, khz = r.phase_times()
    path = r.path
    r.trace_phases(0)
    r.close()
    t = st.astype(np.float64) * (1e3 / khz)           # microseconds
    ok = np.all(st > 0, axis=2)
    # the resident kernel's workgroups all wait for each other; those of the
    # multi-stream kernel only for their own stream group, so no time
    # relative to the last publish of the whole grid is reported there
    across = path == "resident"
    med = lambda x: float(np.median(x)) if np.size(x) else None  # noqa: E731
    last_pub = np.max(np.where(ok, t[:, :, 3], -np.inf), axis=0)
    return {
        "workload": name, "dtype": dtype, "coupling": coupling, "path": path, "workgroups": int(st.shape[0]),
        "stages": int(st.shape[1]),
        "clock_khz": khz,
        "gather_us": med((t[:, :, 1] - t[:, :, 0])[ok]), "compute_us": med((t[:, :, 2] - t[:, :, 1])[ok]),
        "publish_us": med((t[:, :, 3] - t[:, :, 2])[ok]),
        "stage_us": med(np.diff(t[:, :, 0], axis=1)[ok[:, 1:] & ok[:, :-1]]),
        "after_last_publish_us": med((t[:, 1:, 1] - last_pub[None, :-1])[ok[:, 1:]]) if across else None,
        "publish_spread_us": (med((last_pub - np.min(np.where(ok, t[:, :, 3], np.inf), axis=0))[1:])
                              if across else None),
    }


def cpu_blas_form(name: str, arrays, prm, budget_s: float = 4.0):
    """The oracle with its coupling as NumPy's matrix product (the analogue of
    the paper's NumPy baseline), timed on one input sample with BLAS pinned to
    one thread and then on all host cores; names the CPU and the BLAS."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import sto
    from workloads import WORKLOADS

    wl = WORKLOADS[name]

    def rate():
        t0 = time.perf_counter()
        samples = 0
        while True:
            sto.run(arrays["W"], arrays["w_in"], arrays["m0"], arrays["u"][samples:samples + 1], prm, dot="blas")
            samples += 1
            el = time.perf_counter() - t0
            if el >= budget_s or samples >= wl.samples:
                return wl.n * samples * wl.substeps / el, samples

    np.dot(np.ones(4), np.ones(4))   # load the BLAS before asking for its thread pool
    pools = [p for p in threadpool_info() if p.get("user_api") == "blas"]
    with threadpool_limits(limits=1, user_api="blas"):
        one, s1 = rate()
    allc, s2 = rate()
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(line.split(":", 1)[1].strip() for line in fh if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {
        "node_steps_per_s_1_thread": one, "node_steps_per_s_all_cores": allc,
        "threads_all_cores": pools[0]["num_threads"] if pools else None,
        "blas": f"{pools[0]['internal_api']} {pools[0]['version']}" if pools else "unknown",
        "cpu_model": cpu, "host_cpus": os.cpu_count(),
        "samples": [s1, s2],
    }


def finish(torch):
    """Drain the device and drop torch's cached blocks before the line is
    printed: every library handle is already closed, so nothing is left for
    interpreter exit to free on the device."""
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sto10k")
    ap.add_argument("--dtype", default="f64", choices=("f32", "f64"))
    ap.add_argument("--no-also", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--adjoint", default=None, metavar="WORKLOAD:DTYPE:SAMPLES",
                    help="time only the adjoint line for this workload (e.g. sto10k:f32:50; for the "
                         "multi-stream workload the second field is the coupling: streams64:xyz:0)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--own-checkpoints", action="store_true",
                    help="multi-stream adjoint: checkpoints from the adjoint's own forward pass, not the records")
    ap.add_argument("--samples", type=int, default=None,
                    help="run only the first SAMPLES input samples of the main workload (short profiled runs)")
    ap.add_argument("--paper-table", type=int, default=0, metavar="STEPS",
                    help="only run the paper's benchmark (u = 0, FP64, N = 1..1e4) for STEPS RK4 steps each")
    ap.add_argument("--paper-n", type=int, nargs="+", default=None, metavar="N",
                    help="paper benchmark: only these sizes (of 1, 10, 100, 1000, 2500, 5000, 10000)")
    ap.add_argument("--repeats", type=int, default=3, help="paper benchmark: runs per size (median and spread)")
    ap.add_argument("--no-plain", action="store_true",
                    help="sweep workload: skip timing the plain single-reservoir path")
    ap.add_argument("--plain-full", action="store_true",
                    help="sweep workload: time the plain path over the whole input series, not a prefix")
    ap.add_argument("--coupling", default="x", choices=("x", "xyz"),
                    help="multi-stream workload: the paper's m^x coupling or all three components")
    ap.add_argument("--phases", type=int, default=0, metavar="STAGES",
                    help="only print the exchange-phase breakdown of the workload's persistent kernel over STAGES stages")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device with a plain copy kernel (scales HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: every workload here fits one GPU; use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    import paper_2312_01121_amd as stx
    from workloads import WORKLOADS, make_workload_arrays

    if args.phases:
        res = phase_breakdown(stx, torch, args.workload, args.dtype, args.phases, coupling=args.coupling)
        finish(torch)
        print(json.dumps({"phases": res}), flush=True)
        return
    if args.paper_table:
        rows = paper_table(stx, torch, args.paper_table, args.repeats, sizes=args.paper_n)
        finish(torch)
        print(json.dumps({"paper_table": rows, "steps": args.paper_table}), flush=True)
        return
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst
    from workloads import STREAMS, SWEEPS
    if args.adjoint:
        name, dt, samples = args.adjoint.split(":")
        if name in STREAMS:
            res = run_streams_adjoint_workload(stx, torch, name, dt, args.steps, args.warmup,
                                               own_checkpoints=args.own_checkpoints)
        else:
            res = run_adjoint_workload(stx, torch, name, dt, int(samples), args.steps, args.warmup)
        finish(torch)
        print(json.dumps({"adjoint": res}), flush=True)
        return
    if args.workload in SWEEPS or args.workload in STREAMS:
        if args.workload in SWEEPS:
            res = run_sweep_workload(stx, torch, args.workload, args.steps, args.warmup, samples=args.samples,
                                     plain=not args.no_plain,
                                     plain_samples=10 ** 9 if args.plain_full else 200)
            roof = {"bound": "hbm", "kernel": res["kernel"], "achieved": res["achieved_gbs"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": res["hbm_frac"], "traffic": stored_traffic("k_sweep_stage", args.workload, "f32")}
            unit_nodes = res["nodes"]
        else:
            res = run_streams_workload(stx, torch, args.workload, args.steps, args.warmup, coupling=args.coupling,
                                       plain=not args.no_plain)
            roof = {"bound": "mfma", "kernel": res["kernel"], "achieved": res["mfma_tflops"], "peak": 157.3,
                    "unit": "TFLOP/s", "frac": res["mfma_frac"], "traffic": None}
            unit_nodes = res["n"] * res["streams"]
        finish(torch)
        print(json.dumps({
            "metric": METRIC, "value": res["value"], "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": args.workload, "nodes": unit_nodes, "rk4_steps": res["rk4_steps"],
                       "path": res["path"], "coupling": res.get("coupling", "x"), "parallelism": "single GPU"},
            "roofline": roof, "cpu_baseline": None, "detail": res, "also": []}), flush=True)
        return
    attainable = stx.sto_read_bandwidth(2 << 30, 5)
    log(f"attainable HBM read bandwidth (plain streaming kernel): {attainable:.0f} GB/s")
    arrays = make_workload_arrays(WORKLOADS[args.workload])
    log("main", args.workload, args.dtype)
    main_res = run_workload(stx, torch, args.workload, args.dtype, args.steps, args.warmup, arrays, args.samples)
    log(json.dumps(main_res))
    also = []
    if not args.no_also:
        plan = [(args.workload, "f64" if args.dtype == "f32" else "f32", 1, 1),
                ("sto1k", "f32", 5, 1), ("sto1k", "f64", 5, 1), ("sto16", "f64", 5, 1)]
        for name, dt, k, w in plan:
            log("also", name, dt)
            res = run_workload(stx, torch, name, dt, k, w, arrays if name == args.workload else None)
            log(json.dumps(res))
            also.append(res)
        log("also sweep256")
        res = run_sweep_workload(stx, torch, "sweep256", 1, 1)
        log(json.dumps(res))
        also.append(res)
        log("also streams64")
        res = run_streams_workload(stx, torch, "streams64", 1, 1)
        log(json.dumps(res))
        also.append(res)
        for name, dt, samples in (("sto10k", "f32", 50), ("sto1k", "f64", 200)):
            log("also adjoint", name, dt, samples)
            res = run_adjoint_workload(stx, torch, name, dt, samples, 1, 1)
            log(json.dumps(res))
            also.append(res)
        log("also streams64 xyz")
        res = run_streams_workload(stx, torch, "streams64", 1, 1, coupling="xyz")
        log(json.dumps(res))
        also.append(res)
        log("also adjoint streams64 xyz")
        res = run_streams_adjoint_workload(stx, torch, "streams64", "xyz", 1, 1)
        log(json.dumps(res))
        also.append(res)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(args.workload, arrays)
        # the GPU's rate over the oracle's, on each workload both ran
        cpu["gpu_over_oracle"] = main_res["value"] / cpu["value"]
        gpu_rate = {(a["workload"], a["dtype"]): a["value"] for a in also if "workload" in a}
        for o in cpu.get("other_workloads", []):
            g = gpu_rate.get((o["workload"], "f64"))
            o["gpu_over_oracle"] = g / o["value"] if g else None
        log(json.dumps(cpu))

    traffic = stored_traffic(main_res["kernel"], args.workload, args.dtype)
    out = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "n": main_res["n"], "samples": main_res["samples"],
                   "substeps": main_res["substeps"], "rk4_steps": main_res["rk4_steps"], "dt": main_res["dt"],
                   "path": main_res["path"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": main_res["kernel"], "achieved": main_res["achieved_gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": main_res["hbm_frac"], "traffic": traffic,
                     "attainable": attainable, "frac_attainable": main_res["achieved_gbs"] / attainable},
        "cpu_baseline": cpu,
        "detail": main_res,
        "also": also,
    }
    finish(torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
