"""Autotuners of the single-stream paths.

Default mode (the streaming kernels, STO_PATH_STREAM): times every compiled
launch shape (rows of W per wave x unroll of the column loop) of the stage
kernel on this GPU, for each element type and a ladder of sizes, and writes
the fastest shape per size bucket into ``csrc/stream_tune.hpp``.

``--sweep``: times candidate tables of the sweep kernel's rows per lane
group and row pitch (by reservoir size) on the 256-reservoir sweep workload
and writes the fastest into ``csrc/sweep_tune.hpp``.

``--paths``: times the three single-stream paths at a ladder of sizes for
each element type and coupling -- the one-workgroup kernel (small), the
cooperative kernel with W in the LDS of many workgroups (resident) in every
candidate launch shape (waves and rows per workgroup) that fits, and the
per-stage streaming kernel -- and writes the fastest path and shape per size
bucket into ``csrc/path_tune.hpp``, which sets the automatic path choice and
the resident launch shape.

Within 2 % of the fastest, the path table keeps the choice of the next
smaller size (run-to-run noise would otherwise alternate paths between
neighbouring sizes); ``--paths-from LOG`` rewrites the table from the
printed lines of an earlier ``--paths`` run, on the CPU.

Rebuild the library afterwards (``python paper_2312_01121_amd/_build.py``).

Usage (on the GPU): python -m paper_2312_01121_amd.autotune [--paths] [--write [PATH]] [--samples S]
"""

from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

VARIANTS = [(1, 4), (2, 2), (2, 4), (4, 1), (4, 2), (4, 4), (8, 1), (8, 2)]
SIZES = {"f32": [3200, 4096, 6144, 8192, 10000, 14000], "f64": [2200, 3072, 4096, 6144, 8192, 10000]}
HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "stream_tune.hpp")
PATH_HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "path_tune.hpp")
# sizes of the path ladder and the resident launch shapes tried (waves, rows
# per workgroup; 0 rows: ceil(n / CUs))
PATH_SIZES = {"f64": [16, 32, 48, 64, 80, 96, 128, 140, 192, 256, 384, 512, 768, 1000, 1280, 1536, 2048],
              "f32": [16, 32, 64, 96, 128, 160, 199, 256, 384, 512, 768, 1000, 1280, 1536, 2048, 2560, 3072]}
# (waves, rows per workgroup (0: ceil(n / CUs)), waves per row)
RESIDENT_SHAPES = [(4, 0, 1), (8, 0, 1), (16, 0, 1), (4, 4, 1), (8, 8, 1), (16, 16, 1), (8, 16, 1),
                   (4, 0, 2), (8, 0, 2), (16, 0, 2), (8, 4, 2), (8, 8, 2), (16, 8, 2),
                   (8, 0, 4), (16, 0, 4), (8, 8, 4)]
SPLIT_MIN_N = 256   # rows shorter than this are not worth two waves
SAME_AS_PREVIOUS = 0.02   # keep the next smaller size's choice within 2 % of the fastest
PATH_CODE = {"small": 1, "resident": 2, "stream": 3}


def measure(stx, torch, n: int, dtype: str, variants, samples: int):
    """Microseconds per stage launch for each variant (one reservoir of n nodes)."""
    rng = np.random.default_rng(n)
    w = rng.standard_normal((n, n)) / np.sqrt(n)
    np.fill_diagonal(w, 0.0)
    w_in = rng.uniform(-1, 1, (n, 1))
    v = rng.standard_normal((n, 3)) * 0.05
    v[:, 2] += 1.0
    m0 = v / np.linalg.norm(v, axis=1, keepdims=True)
    prm = stx.make_params(**stx.params.table1(), dtype=dtype, path="stream")
    r = stx.Reservoir(w, w_in, m0, prm)
    u = torch.from_numpy(rng.uniform(-1, 1, (samples, 1))).cuda()
    stream = torch.cuda.current_stream()
    out = {}
    for rows, unroll in variants:
        stx.sto_set_stream_variant(rows, unroll)
        r.set_state(m0)
        r.run_device(u[:1].contiguous(), None, stream)       # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r.run_device(u, None, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        out[(rows, unroll)] = e0.elapsed_time(e1) * 1e3 / (samples * prm.substeps * 4)
    stx.sto_set_stream_variant(0, 0)
    r.close()
    return out


def table(best):
    """Size buckets: each measured size covers n up to the midpoint to the next."""
    lines = []
    for dtype, elem in (("f32", 4), ("f64", 8)):
        sizes = sorted(best[dtype])
        for i, n in enumerate(sizes):
            n_max = (n + sizes[i + 1]) // 2 if i + 1 < len(sizes) else (1 << 30)
            rows, unroll = best[dtype][n]
            lines.append(f"    {{{elem}, {n_max}, {rows}, {unroll}}},")
    return "\n".join(lines)


def write_header(best, measured, path=HEADER):
    text = f"""// Launch shapes of the streaming kernels by element type and size, chosen
// by measurement.  Written by paper_2312_01121_amd/autotune.py; entries are
// scanned in order and the first with n <= n_max applies.
#pragma once

namespace sto {{

struct StreamTuneEntry {{
    int elem_bytes;
    int n_max;
    int rows;
    int unroll;
}};

// Fastest shape per size bucket (microseconds per stage launch measured for
// every compiled variant at the sizes below).
constexpr StreamTuneEntry kStreamTune[] = {{
{table(best)}
}};

// Measured (dtype, n): {{rows x unroll: us per launch}}
// {json.dumps(measured, sort_keys=True)}

}}  // namespace sto
"""
    with open(path, "w") as fh:
        fh.write(text)


def time_path(stx, torch, n, dtype, coupling, path, shape, samples, reps=3):
    """Best of ``reps`` runs, microseconds per RK4 step; None if the path or
    shape cannot hold n."""
    for k in ("STO_RESIDENT_WAVES", "STO_RESIDENT_RPB", "STO_RESIDENT_SPLIT"):
        os.environ.pop(k, None)
    if shape is not None:
        os.environ["STO_RESIDENT_WAVES"] = str(shape[0])
        if shape[1]:
            os.environ["STO_RESIDENT_RPB"] = str(shape[1])
        os.environ["STO_RESIDENT_SPLIT"] = str(shape[2])
    rng = np.random.default_rng(n)
    w = rng.standard_normal((n, n)) / np.sqrt(n)
    np.fill_diagonal(w, 0.0)
    w_in = rng.uniform(-1, 1, (n, 1))
    v = rng.standard_normal((n, 3)) * 0.05
    v[:, 2] += 1.0
    m0 = v / np.linalg.norm(v, axis=1, keepdims=True)
    prm = stx.make_params(**stx.params.table1(), dtype=dtype, coupling=coupling, path=path)
    try:
        r = stx.Reservoir(w, w_in, m0, prm)
    except stx.StoError:
        return None
    try:
        u = torch.from_numpy(rng.uniform(-1, 1, (samples, 1))).cuda()
        r.run_device(u[:2].contiguous())
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            r.run_device(u)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e3 / (samples * prm.substeps))
        return best
    except stx.StoError:
        return None
    finally:
        r.close()
        for k in ("STO_RESIDENT_WAVES", "STO_RESIDENT_RPB", "STO_RESIDENT_SPLIT"):
            os.environ.pop(k, None)


def path_table(best):
    lines = []
    for (dtype, coupling), per in sorted(best.items()):
        elem = 4 if dtype == "f32" else 8
        xyz = 1 if coupling == "xyz" else 0
        sizes = sorted(per)
        for i, n in enumerate(sizes):
            n_max = (n + sizes[i + 1]) // 2 if i + 1 < len(sizes) else (1 << 30)
            path, waves, rpb, split = per[n]
            lines.append(f"    {{{elem}, {xyz}, {n_max}, {PATH_CODE[path]}, {waves}, {rpb}, {split}}},   // {path}")
    return "\n".join(lines)


def write_path_header(best, measured, path=PATH_HEADER):
    text = f"""// Path and launch shape of a single-stream reservoir by element type,
// coupling and size, chosen by measurement.  Written by
// paper_2312_01121_amd/autotune.py --paths; entries are scanned in order and
// the first with matching element size and coupling and n <= n_max applies.
// Each measured size covers n up to the midpoint to the next; above the last
// one the entry's path holds while it can (the resident path falls back to
// the stream path where W no longer fits the CUs' LDS).
#pragma once

namespace sto {{

struct PathTuneEntry {{
    int elem_bytes;
    int xyz;        // 0: m^x coupling, 1: all three components
    int n_max;
    int path;       // 1 small, 2 resident, 3 stream (sto_path values)
    int waves;      // resident: waves per workgroup (4, 8 or 16)
    int rpb;        // resident: rows per workgroup (0: ceil(n / CUs))
    int split;      // resident: waves per row (1, 2 or 4: each sums its share of the columns)
}};

// Fastest path and shape per size bucket (microseconds per RK4 step measured
// for every path and resident shape that holds the size; listed below).
constexpr PathTuneEntry kPathTune[] = {{
{path_table(best)}
}};

// Measured (dtype/coupling/n): {{path or resident_WAVESxROWS[sSPLIT]: us per RK4 step}}
// {json.dumps(measured, sort_keys=True)}

}}  // namespace sto
"""
    with open(path, "w") as fh:
        fh.write(text)


def tune_paths(stx, torch, samples, write):
    best, measured = {}, {}
    for dtype, sizes in PATH_SIZES.items():
        for coupling in ("x", "xyz"):
            best[(dtype, coupling)] = {}
            for n in sizes:
                s = samples if n <= 1000 else max(10, samples // 3)
                times = {"small": time_path(stx, torch, n, dtype, coupling, "small", None, s),
                         "stream": time_path(stx, torch, n, dtype, coupling, "stream", None, s)}
                for shape in RESIDENT_SHAPES:
                    if shape[2] > 1 and n < SPLIT_MIN_N:
                        continue
                    name = f"resident_{shape[0]}x{shape[1]}" + (f"s{shape[2]}" if shape[2] > 1 else "")
                    times[name] = time_path(stx, torch, n, dtype, coupling, "resident", shape, s)
                ok = {k: v for k, v in times.items() if v is not None}
                measured[f"{dtype}/{coupling}/{n}"] = {k: round(v, 2) for k, v in ok.items()}
                key = min(ok, key=ok.get)
                print(json.dumps({"dtype": dtype, "coupling": coupling, "n": n, "best": key,
                                  "us": round(ok[key], 2), "all": measured[f"{dtype}/{coupling}/{n}"]}), flush=True)
    if write:
        write_path_header(choose(measured), measured, write)
        print(f"wrote {write}", file=sys.stderr)


def parse_choice(key):
    """(path, waves, rows, split) of a measured key."""
    if not key.startswith("resident_"):
        return (key, 0, 0, 1)
    spec = key[len("resident_"):]
    split = int(spec.split("s")[1]) if "s" in spec else 1
    waves, rpb = (int(x) for x in spec.split("s")[0].split("x"))
    return ("resident", waves, rpb, split)


def choose(measured, keep_within=SAME_AS_PREVIOUS):
    """Path and shape per size from the measured times.  The fastest, except
    that the choice of the next smaller size is kept while it is within
    ``keep_within`` (relative) of the fastest: differences that small are
    run-to-run noise, and would otherwise alternate the path between
    neighbouring sizes."""
    best = {}
    for dtype in PATH_SIZES:
        for coupling in ("x", "xyz"):
            per, prev = {}, None
            sizes = sorted(int(k.split("/")[2]) for k in measured if k.startswith(f"{dtype}/{coupling}/"))
            for n in sizes:
                ok = measured[f"{dtype}/{coupling}/{n}"]
                key = min(ok, key=ok.get)
                if prev in ok and ok[prev] <= ok[key] * (1 + keep_within):
                    key = prev
                per[n] = parse_choice(key)
                prev = key
            if per:
                best[(dtype, coupling)] = per
    return best


def measured_from_log(path):
    """The measured times of a ``--paths`` run, from its printed lines."""
    measured = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("{"):
                d = json.loads(line)
                measured[f"{d['dtype']}/{d['coupling']}/{d['n']}"] = d["all"]
    return measured


SWEEP_HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "sweep_tune.hpp")
# Candidate tables (n_max, rows per lane group, row pitch in elements) for
# FP32: uniform shapes, a short 64-byte pitch below a size threshold (less
# padding), 4 rows per group for the largest reservoirs.  They are timed on
# the 256-reservoir sweep workload itself, where the reservoirs compete for
# HBM and L2: optima measured per size on sweeps of equal reservoirs did not
# carry over to it.
SWEEP_CANDIDATES = [
    [(1 << 30, 8, 64)],
    [(1 << 30, 8, 32)],
    [(1 << 30, 8, 16)],
    [(1 << 30, 4, 64)],
    [(48, 8, 16), (1 << 30, 8, 64)],
    [(192, 8, 16), (1 << 30, 8, 64)],
    [(192, 8, 16), (1 << 30, 8, 32)],
    [(1792, 8, 32), (1 << 30, 4, 32)],
]


def table_env(cand):
    return ",".join(f"{n}:{r}:{p}" for n, r, p in cand)


def time_sweep_table(stx, torch, cand, samples=200, reps=3):
    """Microseconds per RK4 step of the 256-reservoir sweep workload with a
    candidate table."""
    from workloads import SWEEPS, make_sweep_arrays
    os.environ["STO_SWEEP_TABLE"] = table_env(cand)
    try:
        import dataclasses
        from paper_2312_01121_amd import params
        sw_def = dataclasses.replace(SWEEPS["sweep256"], samples=samples)
        a = make_sweep_arrays(sw_def)
        res = a["reservoirs"]
        for r in res:
            r["prm"] = stx.make_params(**params.table1(a_cp=r["a_cp"], a_in=r["a_in"], dt=sw_def.dt,
                                                       substeps=sw_def.substeps, current_scale=r["current_scale"],
                                                       field_scale=r["field_scale"]), dtype="f32")
        sw = stx.Sweep(res)
        u = torch.from_numpy(a["u"]).cuda()
        sw.run_device(u[:2].contiguous())
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sw.run_device(u)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e3 / (samples * sw_def.substeps))
        sw.close()
        return best
    finally:
        os.environ.pop("STO_SWEEP_TABLE", None)


def tune_sweep(stx, torch, write):
    measured = {}
    for cand in SWEEP_CANDIDATES:
        us = time_sweep_table(stx, torch, cand)
        measured[table_env(cand)] = round(us, 2)
        print(json.dumps({"table": table_env(cand), "us_per_rk4_step": round(us, 2)}), flush=True)
    best = min(SWEEP_CANDIDATES, key=lambda c: measured[table_env(c)])
    if write:
        lines = [f"    {{4, {n}, {r}, {p}}}," for n, r, p in best] + ["    {8, 1073741824, 8, 64},"]
        table = "\n".join(lines)
        text = f"""// Rows per lane group and row pitch of the sweep kernel by element type and
// reservoir size, chosen by measurement.  Written by
// paper_2312_01121_amd/autotune.py --sweep, which times candidate tables on
// the 256-reservoir FP32 sweep workload (N log-uniform in [32, 2048]) and
// keeps the fastest; FP64 sweeps keep 8 rows and a 64-element pitch.
// Entries are scanned in order and the first with n <= n_max applies.
#pragma once

namespace sto {{

struct SweepTuneEntry {{
    int elem_bytes;
    int n_max;
    int rows;    // rows of W per lane group (2, 4 or 8)
    int pitch;   // row pitch of W and the state, in elements (a multiple of 16 bytes)
}};

constexpr SweepTuneEntry kSweepTune[] = {{
{table}
}};

// Measured (candidate table n_max:rows:pitch,...): us per RK4 step of the sweep
// {json.dumps(measured, sort_keys=True)}

}}  // namespace sto
"""
        with open(write, "w") as fh:
            fh.write(text)
        print(f"wrote {write}", file=sys.stderr)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--samples", type=int, default=3)
    ap.add_argument("--paths", action="store_true", help="tune the path choice and resident shapes instead")
    ap.add_argument("--sweep", action="store_true", help="tune the sweep kernel's rows per group and row pitch")
    ap.add_argument("--write", nargs="?", const="default", default=None, metavar="PATH",
                    help="write the table header (default: csrc/stream_tune.hpp, or csrc/path_tune.hpp)")
    ap.add_argument("--paths-from", metavar="LOG",
                    help="write the path table from the printed lines of an earlier --paths run (no GPU)")
    args = ap.parse_args()
    if args.paths_from:
        measured = measured_from_log(args.paths_from)
        write = PATH_HEADER if args.write in (None, "default") else args.write
        write_path_header(choose(measured), measured, write)
        print(f"wrote {write}", file=sys.stderr)
        return
    import torch
    assert torch.cuda.is_available(), "the autotuner runs on the GPU"
    import paper_2312_01121_amd as stx

    if args.paths:
        write = PATH_HEADER if args.write == "default" else args.write
        tune_paths(stx, torch, max(args.samples, 60), write)
        return
    if args.sweep:
        tune_sweep(stx, torch, SWEEP_HEADER if args.write == "default" else args.write)
        return
    if args.write == "default":
        args.write = HEADER

    best, measured = {}, {}
    for dtype, sizes in SIZES.items():
        best[dtype] = {}
        for n in sizes:
            times = measure(stx, torch, n, dtype, VARIANTS, args.samples)
            (rows, unroll), us = min(times.items(), key=lambda kv: kv[1])
            best[dtype][n] = (rows, unroll)
            measured[f"{dtype}/{n}"] = {f"{r}x{u}": round(t, 2) for (r, u), t in times.items()}
            print(json.dumps({"dtype": dtype, "n": n, "best": f"{rows}x{unroll}", "us": round(us, 2),
                              "all": measured[f"{dtype}/{n}"]}), flush=True)
    if args.write:
        write_header(best, measured, args.write)
        print(f"wrote {args.write}", file=sys.stderr)


if __name__ == "__main__":
    main()
