"""Autotuner for the streaming kernels (STO_PATH_STREAM).

Times every compiled launch shape (rows of W per wave x unroll of the column
loop) of the stage kernel on this GPU, for each element type and a ladder of
sizes, and writes the fastest shape per size bucket into
``csrc/stream_tune.hpp`` (the table the library consults).  Rebuild the
library afterwards (``python paper_2312_01121_amd/_build.py``).

Usage (on the GPU): python -m paper_2312_01121_amd.autotune [--write [PATH]] [--samples S]
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--samples", type=int, default=3)
    ap.add_argument("--write", nargs="?", const=HEADER, default=None, metavar="PATH",
                    help="write the table header (default path: csrc/stream_tune.hpp)")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the autotuner runs on the GPU"
    import paper_2312_01121_amd as stx

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
