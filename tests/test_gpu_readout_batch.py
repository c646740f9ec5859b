"""GPU parity of the batched readout (readout_fit_batch_device): every item
against the oracle's ridge readout and against readout_fit_device on the
same records, in both forms (primal and dual), both feature sets and both
record types; strided record sets with their own targets (the streams of a
multi-stream run); errors naming the item concerned."""

import sys

import numpy as np
import pytest

from oracle import readout

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def stx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_01121_amd
    return paper_2312_01121_amd


def predictions(rec, w, washout, features):
    phi = readout.features(rec, washout, "xyz" if features else "x")
    return phi @ w


@pytest.mark.parametrize("features", [0, 1])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_readout_matches_oracle_and_single(stx, features, dtype):
    """Items of 3 to 400 nodes over 270 fitted rows: primal and dual forms,
    the primal/dual boundary (270 columns) and several 32-column panels and
    16 x 16 tiles with ragged edges."""
    import torch
    rng = np.random.default_rng(21 + features)
    T, wash, lam = 300, 30, 1e-4
    ns = [3, 17, 64, 100, 269, 400]
    y = np.tanh(rng.standard_normal(T))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    states = [torch.from_numpy(rng.standard_normal((T, n, 3)) * 0.5).to(tdt).cuda() for n in ns]
    y_d = torch.from_numpy(y).cuda()
    say("batch readout", dtype, "features", features)
    ws, nm = stx.readout_fit_batch_device(states, y_d, wash, lam, features)
    for q, n in enumerate(ns):
        rec = states[q].double().cpu().numpy()   # the records as the GPU read them
        w_o, e_o = readout.readout_fit(rec, y, wash, lam, components="xyz" if features else "x")
        w_s, e_s = stx.readout_fit_device(states[q], y_d, wash, lam, features)
        w_b = ws[q].cpu().numpy()
        p_b = predictions(rec, w_b, wash, features)
        p_o = predictions(rec, w_o, wash, features)
        say("  n", n, "nmse", nm[q], "oracle", e_o, "single", e_s)
        assert abs(nm[q] - e_o) <= 1e-9 * max(1.0, e_o)
        assert abs(nm[q] - e_s) <= 1e-9 * max(1.0, e_s)
        assert float(np.max(np.abs(p_b - p_o))) <= 1e-7
        assert float(np.max(np.abs(w_b - w_s.cpu().numpy()))) <= 1e-6 * max(1.0, float(np.max(np.abs(w_o))))


def test_batch_readout_strided_streams(stx):
    """Stream q of a (T, S, n, 3) record tensor, passed as a strided view
    with its own target series, fits as its contiguous copy does."""
    import torch
    rng = np.random.default_rng(5)
    T, S, n, wash, lam = 200, 5, 50, 20, 1e-5
    states = torch.from_numpy(rng.standard_normal((T, S, n, 3)) * 0.3).float().cuda()
    y_d = [torch.from_numpy(np.tanh(rng.standard_normal(T))).cuda() for _ in range(S)]
    ws, nm = stx.readout_fit_batch_device([states[:, q] for q in range(S)], y_d, wash, lam)
    for q in range(S):
        w_s, e_s = stx.readout_fit_device(states[:, q].contiguous(), y_d[q], wash, lam)
        assert abs(nm[q] - e_s) <= 1e-10 * max(1.0, e_s)
        assert float(torch.max(torch.abs(ws[q] - w_s))) <= 1e-8


def test_batch_readout_streams64_shape(stx):
    """64 items of 512 nodes (the multi-stream workload's readouts), a few
    of them against the oracle."""
    import torch
    rng = np.random.default_rng(64)
    T, S, n, wash, lam = 1000, 64, 512, 100, 1e-6
    states = torch.from_numpy(np.tanh(rng.standard_normal((T, S, n, 3)))).float().cuda()
    y = np.tanh(rng.standard_normal(T))
    y_d = torch.from_numpy(y).cuda()
    ws, nm = stx.readout_fit_batch_device([states[:, q] for q in range(S)], y_d, wash, lam)
    for q in (0, 31, 63):
        rec = states[:, q].double().cpu().numpy()
        w_o, e_o = readout.readout_fit(rec, y, wash, lam)
        say("  stream", q, "nmse", nm[q], "oracle", e_o)
        assert abs(nm[q] - e_o) <= 1e-9 * max(1.0, e_o)
        p_b = predictions(rec, ws[q].cpu().numpy(), wash, 0)
        assert float(np.max(np.abs(p_b - predictions(rec, w_o, wash, 0)))) <= 1e-6


def test_batch_readout_errors_name_the_item(stx):
    import torch
    rng = np.random.default_rng(3)
    T, wash = 60, 6
    y_d = torch.from_numpy(np.tanh(rng.standard_normal(T))).cuda()
    states = [torch.from_numpy(rng.standard_normal((T, n, 3))).cuda() for n in (4, 9, 12)]
    bad = states[1].clone()
    bad[20, 3, 0] = float("nan")
    with pytest.raises(stx.StoError) as ei:
        stx.readout_fit_batch_device([states[0], bad, states[2]], y_d, wash, 1e-3)
    assert ei.value.status == stx.STO_E_NONFINITE and "item 1" in str(ei.value)
    zero = torch.zeros((T, 5, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(stx.StoError) as ei:
        stx.readout_fit_batch_device([states[0], states[1], zero], y_d, wash, 0.0)
    assert ei.value.status == stx.STO_E_INVALID and "item 2" in str(ei.value)
