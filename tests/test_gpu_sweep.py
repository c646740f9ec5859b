"""GPU parity of the parameter-sweep path (many reservoirs of uneven size and
their own constants, one shared input, one launch per RK4 stage over all of
them) against the CPU oracle run once per reservoir."""

import sys

import numpy as np
import pytest

from common import lib_params
from oracle import constants, sto
from workloads import SWEEPS, make_sweep_arrays

pytestmark = pytest.mark.gpu
F64_TOL = 1e-10
F32_TOL = 1e-5


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def stx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_01121_amd
    return paper_2312_01121_amd


def oracle_prm(r, substeps=20):
    return constants.dimensionless(a_cp=r["a_cp"], a_in=r["a_in"], current_scale=r["current_scale"],
                                   field_scale=r["field_scale"], substeps=substeps)


def small_sweep(sizes, seed=7):
    rng = np.random.default_rng(seed)
    res = []
    for n in sizes:
        w = rng.standard_normal((n, n)) / np.sqrt(n)
        np.fill_diagonal(w, 0.0)
        v = rng.standard_normal((n, 3)) * 0.05
        v[:, 2] += 1.0
        res.append({"n": n, "W": w, "w_in": rng.uniform(-1, 1, (n, 1)),
                    "m0": v / np.linalg.norm(v, axis=1, keepdims=True),
                    "current_scale": rng.uniform(0.5, 1.5), "field_scale": rng.uniform(0.5, 1.5),
                    "a_cp": rng.uniform(0.01, 0.5), "a_in": rng.uniform(0.1, 2.0)})
    return res


SIZES = [1, 5, 33, 64, 65, 100, 129, 200, 257, 300, 513]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sweep_matches_oracle(stx, dtype):
    res = small_sweep(SIZES)
    u = np.random.default_rng(8).uniform(-1, 1, (6, 1))
    substeps = 20 if dtype == "f64" else 1
    samples = 6 if dtype == "f64" else 1
    say("sweep", dtype, SIZES)
    for r in res:
        r["prm"] = lib_params(oracle_prm(r, substeps), dtype=dtype)
    with stx.Sweep(res) as sw:
        recs = sw.run(u[:samples])
    worst = 0.0
    f32 = (lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)) if dtype == "f32" else (lambda x: x)
    for r, rec in zip(res, recs):
        rec_o, _ = sto.run(f32(r["W"]), f32(r["w_in"]), f32(r["m0"]), u[:samples], oracle_prm(r, substeps))
        worst = max(worst, float(np.max(np.abs(rec - rec_o))))
    say("  max diff", worst)
    assert worst <= (F64_TOL if dtype == "f64" else F32_TOL)


def test_sweep_equals_single_runs_and_continues(stx):
    res = small_sweep([17, 90, 301], seed=9)
    u = np.random.default_rng(10).uniform(-1, 1, (5, 1))
    for r in res:
        r["prm"] = lib_params(oracle_prm(r), dtype="f64")
    with stx.Sweep(res) as sw:
        whole = sw.run(u)
        fin = sw.get_state()
    with stx.Sweep(res) as sw:
        a = sw.run(u[:2])
        b = sw.run(u[2:])
        assert all(np.array_equal(x, y) for x, y in zip(sw.get_state(), fin))
    for r, wr, ar, br in zip(res, whole, a, b):
        assert np.array_equal(np.concatenate([ar, br]), wr)
        with stx.Reservoir(r["W"], r["w_in"], r["m0"], r["prm"]) as one:
            assert np.array_equal(one.run(u), wr)


def test_sweep256_every_reservoir_matches_oracle(stx):
    """The 256-reservoir sweep (N from 33 to 2042, FP32, each reservoir with
    its own constants) in the launch configuration the benchmark times: one
    input sample (20 steps, well inside the Lyapunov time) of every
    reservoir against the FP64 oracle run on the same (FP32-rounded) inputs."""
    sw_def = SWEEPS["sweep256"]
    a = make_sweep_arrays(sw_def, samples=1)
    res = a["reservoirs"]
    for r in res:
        r["prm"] = lib_params(oracle_prm(r), dtype="f32")
    say("sweep256, every reservoir, one sample")
    with stx.Sweep(res) as sw:
        recs = sw.run(a["u"])
    f32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)  # noqa: E731
    errs = []
    for i, r in enumerate(res):
        rec_o, _ = sto.run(f32(r["W"]), f32(r["w_in"]), f32(r["m0"]), a["u"], oracle_prm(r))
        errs.append(float(np.max(np.abs(recs[i] - rec_o))))
    worst = int(np.argmax(errs))
    say(f"  max diff {errs[worst]:.3g} (reservoir {worst}, n = {res[worst]['n']}), median {np.median(errs):.3g}")
    assert max(errs) <= F32_TOL


def test_sweep256_largest_f64_match_oracle(stx):
    """The 8 largest reservoirs of the 256-reservoir sweep (N = 1,733 to
    2,042, their own constants) run together in FP64 over 3 input samples
    (60 RK4 steps): every record within 1e-10 of the oracle."""
    sw_def = SWEEPS["sweep256"]
    samples = 3
    a = make_sweep_arrays(sw_def, samples=samples)
    res = sorted(a["reservoirs"], key=lambda r: -r["n"])[:8]
    for r in res:
        r["prm"] = lib_params(oracle_prm(r), dtype="f64")
    say("sweep256, 8 largest, f64", [r["n"] for r in res])
    with stx.Sweep(res) as sw:
        recs = sw.run(a["u"])
    worst = 0.0
    for r, rec in zip(res, recs):
        rec_o, _ = sto.run(r["W"], r["w_in"], r["m0"], a["u"], oracle_prm(r))
        worst = max(worst, float(np.max(np.abs(rec - rec_o))))
    say("  max diff", worst)
    assert worst <= F64_TOL


def test_sweep_graph_replay_equals_direct_launches(stx, monkeypatch):
    """The stage launches of a few samples captured into a HIP graph and
    replayed (the default) give the bits of the same launches issued one by
    one: runs of 11 samples with 2-sample graphs (5 replays and one sample
    issued directly), repeated three times with other sweep work and
    synchronisations between them, each against the direct run; and the
    FP64 records against the oracle."""
    res = small_sweep([33, 70, 129, 300], seed=12)
    u = np.random.default_rng(13).uniform(-1, 1, (11, 1))
    for r in res:
        r["prm"] = lib_params(oracle_prm(r, 4), dtype="f64")
    monkeypatch.setenv("STO_SWEEP_GRAPH", "0")
    with stx.Sweep(res) as sw:
        direct = sw.run(u)
    monkeypatch.setenv("STO_SWEEP_GRAPH", "1")
    monkeypatch.setenv("STO_SWEEP_GRAPH_SAMPLES", "2")
    other = small_sweep([50, 90], seed=14)
    for r in other:
        r["prm"] = lib_params(oracle_prm(r, 4), dtype="f64")
    for rep in range(3):
        say("sweep graph replay", rep)
        with stx.Sweep(res) as sw:
            got = sw.run(u)
        assert all(np.array_equal(a, b) for a, b in zip(got, direct)), rep
        with stx.Sweep(other) as sw2:          # other work between the replays
            sw2.run(u[:3])
    for r, rec in zip(res, direct):
        rec_o, _ = sto.run(r["W"], r["w_in"], r["m0"], u, oracle_prm(r, 4))
        assert float(np.max(np.abs(rec - rec_o))) <= F64_TOL


@pytest.mark.parametrize("rows,pitch", [(2, 4), (4, 16), (8, 64), (2, 2), (8, 2), (8, 8), (4, 4)])
def test_sweep_shapes_match_oracle(stx, rows, pitch, monkeypatch):
    """Every rows-per-group and row pitch the tuner may choose gives the
    oracle's trajectory (FP64, bitwise-level bar; FP32 pitch 2 is rounded up
    to the 16-byte minimum)."""
    monkeypatch.setenv("STO_SWEEP_ROWS", str(rows))
    monkeypatch.setenv("STO_SWEEP_PITCH", str(pitch))
    # sizes of a few nodes: a short pitch then holds fewer vectors than a
    # group has rows, and the pitch is widened to keep one lane per row
    res = small_sweep([1, 2, 3, 5, 7, 9, 33, 64, 65, 130, 257], seed=15)
    u = np.random.default_rng(16).uniform(-1, 1, (3, 1))
    for dtype in ("f64", "f32"):
        sub = 20 if dtype == "f64" else 1
        for r in res:
            r["prm"] = lib_params(oracle_prm(r, sub), dtype=dtype)
        say("sweep shape", rows, pitch, dtype)
        with stx.Sweep(res) as sw:
            recs = sw.run(u)
        f32 = (lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)) if dtype == "f32" else (lambda x: x)
        worst = max(float(np.max(np.abs(rec - sto.run(f32(r["W"]), f32(r["w_in"]), f32(r["m0"]), u,
                                                      oracle_prm(r, sub))[0])))
                    for r, rec in zip(res, recs))
        assert worst <= (F64_TOL if dtype == "f64" else F32_TOL), (dtype, worst)
