"""The allocation-free readout (readout_fit_device_noalloc) against the
allocating one (readout_fit_device): same weights and NMSE, bit for bit (the
same kernels on the same inputs), on two calls in a row, the second smaller,
and a clear refusal when the workspace would exceed the static array."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def stx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_01121_amd
    return paper_2312_01121_amd


def records(rng, T, n, dtype):
    import torch
    rec = rng.standard_normal((T, n, 3)) * 0.5
    y = np.tanh(rng.standard_normal(T))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    return torch.from_numpy(rec).to("cuda", tdt).contiguous(), torch.from_numpy(y).cuda()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_readout_equals_allocating_one(stx, dtype):
    import torch
    rng = np.random.default_rng(71)
    # primal (rows >= cols), then a smaller dual fit (rows < cols) in a row:
    # the second call reuses the array the first one filled
    for T, n, washout, lam, features in ((1200, 300, 100, 1e-6, 0), (160, 200, 16, 1e-4, 1), (90, 40, 9, 1e-3, 0)):
        say(f"noalloc readout {dtype} T={T} n={n} features={features}")
        st, y = records(rng, T, n, dtype)
        cols = (3 * n if features else n) + 1
        w_ref, e_ref = stx.readout_fit_device(st, y, washout, lam, features)
        w = torch.full((cols,), float("nan"), dtype=torch.float64, device="cuda")
        e = stx.readout_fit_device_noalloc(st, y, washout, lam, w, features)
        torch.cuda.synchronize()
        assert torch.equal(w, w_ref), (T, n)
        assert e == e_ref, (e, e_ref)


def test_noalloc_readout_refuses_oversized_workspace(stx):
    import torch
    # 20,000 fitted rows x 1,001 columns: 160 MB of design matrix
    st = torch.zeros((20001, 1000, 3), dtype=torch.float32, device="cuda")
    y = torch.zeros(20001, dtype=torch.float64, device="cuda")
    w = torch.empty(1001, dtype=torch.float64, device="cuda")
    with pytest.raises(stx.StoError) as ei:
        stx.readout_fit_device_noalloc(st, y, 1, 1e-6, w)
    assert ei.value.status == stx.STO_E_UNSUPPORTED
    assert "allocation-free" in str(ei.value)
