"""Write the full-horizon FP64 fixtures of the oracle (CPU only).

The GPU parity tests compare FP64 runs of the library over a workload's
whole input series with these files.  Each file holds, for one workload,
what the oracle (``oracle.sto.run``, correctly rounded coupling sums) gives
on the seeded inputs of ``workloads``:

* ``sums``: for every record (state after each input sample) the sum over
  nodes of each component m^x, m^y, m^z (shape samples x 3; each sum by
  math.fsum, so exactly rounded);
* ``idx`` and ``records``: the complete records at a few sample indices
  spread over the horizon, the last one included;
* ``final``: the state after the last sample (equal to the last record);
* ``meta``: a JSON string naming the workload, its sizes and a SHA-256 of
  the oracle and generator sources the file was made with.

Nothing here reads the HIP library.  Usage, from the repository root:

    python tests/golden/make_horizon.py [name ...]

with names from ``CASES`` (default: all).  The 1,000-node series takes
about 10 minutes on 8 cores, the 10,000-node series about 40.
"""

from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import constants, sto  # noqa: E402
from workloads import WORKLOADS, make_paper_arrays, make_workload_arrays  # noqa: E402

# name -> (how the inputs are made, number of full records kept)
CASES = {
    "sto1k": ("workload", 21),
    "sto10k": ("workload", 11),
    "paper2500": ("paper", 3),
    "paper5000": ("paper", 3),
    "paper10000": ("paper", 3),
}
PAPER_STEPS = 5000          # RK4 steps of the paper-setup fixtures (u = 0)


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in ("oracle/sto.py", "oracle/exactdot.c", "oracle/constants.py", "workloads/inputs.py"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def case_inputs(name: str):
    """(arrays, oracle constants, description) of one fixture case."""
    kind, _ = CASES[name]
    if kind == "workload":
        wl = WORKLOADS[name]
        a = make_workload_arrays(wl)
        prm = constants.dimensionless(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps)
        return a, prm, {"workload": name, "n": wl.n, "samples": wl.samples, "substeps": wl.substeps}
    n = int(name[len("paper"):])
    samples = PAPER_STEPS // 20
    a = make_paper_arrays(n, samples)
    g = constants.GAMMA * constants.T0          # 1 Oe in the dimensionless field unit
    prm = constants.dimensionless(a_cp=g, a_in=g, dt=0.01, substeps=20)
    return a, prm, {"workload": name, "n": n, "samples": samples, "substeps": 20,
                    "setup": "paper benchmark: u = 0, A_cp = A_in = 1 Oe"}


def record_indices(samples: int, keep: int):
    return sorted({int(round(k * (samples - 1) / (keep - 1))) for k in range(keep)})


def make(name: str) -> str:
    a, prm, meta = case_inputs(name)
    samples = len(a["u"])
    idx = record_indices(samples, CASES[name][1])
    sums = np.empty((samples, 3))
    kept = {}
    t0 = time.time()

    def on_sample(s, m):
        sums[s] = [math.fsum(c) for c in m]
        if s in idx:
            kept[s] = sto.to_aos(m).copy()
        if s % max(1, samples // 20) == 0:
            print(f"{name}: sample {s + 1}/{samples}, {time.time() - t0:.0f} s", flush=True)

    # records are not kept in memory beyond the ones stored
    _, final = run_streaming(a, prm, on_sample)
    meta.update({"oracle_sha256": source_hash(), "seconds": round(time.time() - t0, 1),
                 "dot": "exact"})
    out = os.path.join(HERE, f"horizon_{name}.npz")
    np.savez_compressed(out, sums=sums, idx=np.array(idx), records=np.stack([kept[i] for i in idx]),
                        final=final, meta=np.array(json.dumps(meta)))
    return out


def run_streaming(a, prm, on_sample):
    """sto.run over the whole series in chunks, so that the records of a long
    series are never all held at once."""
    m = a["m0"]
    u = a["u"]
    chunk = 200
    for start in range(0, len(u), chunk):
        part = u[start:start + chunk]
        _, m = sto.run(a["W"], a["w_in"], m, part, prm,
                       on_sample=lambda s, st, base=start: on_sample(base + s, st))
    return None, m


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        print("wrote", make(nm), flush=True)
