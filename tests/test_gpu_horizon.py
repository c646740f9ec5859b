"""FP64 parity over the configurations' whole input series.

The oracle's full-horizon trajectories are stored in ``tests/golden`` by
``tests/golden/make_horizon.py`` (which calls only the oracle; see its
header for what each file holds).  Each test runs the library over the
same seeded inputs, from the same initial state, for every sample of the
series, and compares

* every record's sum over nodes of m^x, m^y and m^z with the oracle's
  (all 10,000 records at N = 1,000; all 1,000 at N = 10,000), and
* the complete records the file keeps (21 or 11 spread over the series,
  the last one included) element by element,

at the FP64 bar: every element within 1e-10 (so each sum within n * 1e-10).
The trajectories are chaotic (largest Lyapunov exponent about 0.6 per ns),
so this bar holds only if the library computes the oracle's bits at every
step.  The paper's own benchmark setup (u = 0, the paper's generator and
amplitudes, 5,000 RK4 steps) is checked the same way at N = 2,500, 5,000
and 10,000.
"""

import json
import os
import sys

import numpy as np
import pytest

from common import lib_params
from oracle import constants
from workloads import WORKLOADS, make_paper_arrays, make_workload_arrays

pytestmark = pytest.mark.gpu
F64_TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def stx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_01121_amd
    return paper_2312_01121_amd


def load(name):
    path = os.path.join(GOLDEN, f"horizon_{name}.npz")
    if not os.path.exists(path):
        # the CPU suite requires every fixture (test_oracle_pins.py)
        pytest.skip(f"{path} has not been written")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files} | {"meta": json.loads(str(z["meta"]))}


def run_and_compare(stx, a, prm, fix, dtype="f64", path="auto"):
    """Whole series on the device; returns (max sum error, max record error)."""
    import torch
    n = a["W"].shape[0]
    samples = len(a["u"])
    with stx.Reservoir(a["W"], a["w_in"], a["m0"], lib_params(prm, dtype, path)) as r:
        used = r.path
        u_d = torch.from_numpy(np.ascontiguousarray(a["u"])).cuda()
        st = torch.empty((samples, n, 3), dtype=torch.float64, device="cuda")
        r.run_device(u_d, st)
        torch.cuda.synchronize()
        final = r.get_state()
    sums = st.sum(dim=1).cpu().numpy()
    kept = st[torch.from_numpy(fix["idx"]).cuda()].cpu().numpy()
    d_sum = float(np.max(np.abs(sums - fix["sums"])))
    d_rec = float(np.max(np.abs(kept - fix["records"])))
    d_fin = float(np.max(np.abs(final - fix["final"])))
    worst = int(np.argmax(np.max(np.abs(sums - fix["sums"]), axis=1)))
    say(f"  path {used}: max |sum diff| {d_sum:.3g} (worst record {worst}), max |record diff| {d_rec:.3g}, "
        f"final {d_fin:.3g}")
    return used, d_sum, max(d_rec, d_fin)


@pytest.mark.parametrize("path", ["resident", "stream"])
def test_sto1k_f64_whole_series(stx, path):
    """N = 1,000: 10,000 samples x 20 steps (200,000 RK4 steps) on the
    resident kernel (the default at this size) and on the stream kernel."""
    wl = WORKLOADS["sto1k"]
    fix = load("sto1k")
    assert fix["sums"].shape == (wl.samples, 3)
    a = make_workload_arrays(wl)
    prm = constants.dimensionless(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps)
    say(f"sto1k f64 whole series ({wl.steps} RK4 steps), {path}")
    used, d_sum, d_rec = run_and_compare(stx, a, prm, fix, path=path)
    assert used == path
    assert d_rec <= F64_TOL and d_sum <= wl.n * F64_TOL


def test_sto10k_f64_whole_series(stx):
    """N = 10,000: 1,000 samples x 20 steps on the stream kernel, in the
    launch configuration the benchmark times."""
    wl = WORKLOADS["sto10k"]
    fix = load("sto10k")
    assert fix["sums"].shape == (wl.samples, 3)
    a = make_workload_arrays(wl)
    prm = constants.dimensionless(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps)
    say(f"sto10k f64 whole series ({wl.steps} RK4 steps)")
    used, d_sum, d_rec = run_and_compare(stx, a, prm, fix)
    assert used == "stream"
    assert d_rec <= F64_TOL and d_sum <= wl.n * F64_TOL


@pytest.mark.parametrize("n", [2500, 5000, 10000])
def test_paper_setup_f64_whole_series(stx, n):
    """The paper's benchmark (Sec. 3.2) at its three largest sizes: u = 0,
    A_cp = A_in = 1 Oe, the paper's generator and initial tilt, 5,000 RK4
    steps (250 records)."""
    fix = load(f"paper{n}")
    samples = fix["meta"]["samples"]
    a = make_paper_arrays(n, samples)
    g = constants.GAMMA * constants.T0
    prm = constants.dimensionless(a_cp=g, a_in=g, dt=0.01, substeps=20)
    say(f"paper setup n={n}, {samples * 20} RK4 steps")
    used, d_sum, d_rec = run_and_compare(stx, a, prm, fix)
    assert d_rec <= F64_TOL and d_sum <= n * F64_TOL
