"""GPU parity of the multi-stream path (S input streams share one W; the
coupling of all streams is one FP32 MFMA product per stage) against the
CPU oracle run once per stream."""

import sys

import numpy as np
import pytest

from common import lib_params, oracle_params, random_case
from oracle import sto
from workloads import STREAMS, WORKLOADS, make_stream_arrays

pytestmark = pytest.mark.gpu
F32_TOL = 1e-5


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def stx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_01121_amd
    return paper_2312_01121_amd


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def stream_case(n, streams, seed, samples):
    w, w_in, m0, _ = random_case(n, seed=seed, samples=1)
    rng = np.random.default_rng(seed + 100)
    u = rng.uniform(-1, 1, (samples, streams, 1))
    return w, w_in, m0, u


def distinct_states(rng, streams, n):
    m0s = np.empty((streams, n, 3))
    for s in range(streams):
        v = rng.standard_normal((n, 3)) * 0.05
        v[:, 2] += 1.0
        m0s[s] = v / np.linalg.norm(v, axis=1, keepdims=True)
    return m0s


@pytest.mark.parametrize("n,streams,coupling", [(16, 2, "x"), (100, 5, "x"), (257, 17, "x"), (512, 64, "x"),
                                                (16, 2, "xyz"), (100, 5, "xyz"), (257, 17, "xyz"),
                                                (512, 64, "xyz"), (700, 20, "xyz"), (1000, 7, "xyz"),
                                                (1024, 33, "x")])
def test_multi_one_step_matches_oracle(stx, n, streams, coupling):
    """One RK4 step per stream from the same FP32-representable state (every
    stream its own initial state), both couplings; several tiles and ragged
    node and stream tails."""
    w, w_in, m0, u = stream_case(n, streams, seed=n, samples=1)
    prm = oracle_params(a_cp=0.3, substeps=1, coupling=coupling)
    say("multi one step", n, streams, coupling)
    m0s = distinct_states(np.random.default_rng(n + 7), streams, n)
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32"), streams=streams) as r:
        assert r.path == "multi"
        rec = r.run(u)
    worst = 0.0
    for s in (range(streams) if streams <= 8 else (0, 1, streams // 2, streams - 1)):
        rec_o, _ = sto.run(f32(w), f32(w_in), f32(m0s[s]), u[:, s], prm)
        worst = max(worst, float(np.max(np.abs(rec[:, s] - rec_o))))
    say("  max diff", worst)
    assert worst <= F32_TOL


@pytest.mark.parametrize("n,streams,coupling", [(300, 7, "xyz"), (257, 17, "x"), (512, 64, "xyz")])
def test_multi_row_tiles_agree(stx, n, streams, coupling, monkeypatch):
    """One and two 16-node row tiles per workgroup (STO_MULTI_TILES) give
    the same bits (each tile's products and wave sums are the same), and
    both match the oracle; ragged last row tile and stream group."""
    w, w_in, m0, u = stream_case(n, streams, seed=n + 1, samples=2)
    prm = oracle_params(a_cp=0.3, substeps=3, coupling=coupling)
    m0s = distinct_states(np.random.default_rng(n + 9), streams, n)
    recs = {}
    for tiles in ("1", "2"):
        monkeypatch.setenv("STO_MULTI_TILES", tiles)
        say("multi row tiles", tiles, n, streams, coupling)
        with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32"), streams=streams) as r:
            assert r.path == "multi"
            recs[tiles] = r.run(u)
    assert np.array_equal(recs["1"], recs["2"])
    worst = 0.0
    for s in (range(streams) if streams <= 8 else (0, streams // 2, streams - 1)):
        rec_o, _ = sto.run(f32(w), f32(w_in), f32(m0s[s]), u[:, s], prm)
        worst = max(worst, float(np.max(np.abs(recs["2"][:, s] - rec_o))))
    say("  max diff", worst)
    assert worst <= F32_TOL


@pytest.mark.parametrize("path", ["multi", "batch"])
@pytest.mark.parametrize("coupling", ["x", "xyz"])
def test_streams_renormalize_and_several_inputs(stx, path, coupling):
    """Renormalisation after every step and three inputs per stream, over
    two samples of 4 RK4 steps, per stream against the oracle on the same
    FP32-representable inputs."""
    n, S, n_in = 100, 7, 3
    w, w_in, m0, _ = random_case(n, n_in=n_in, seed=11, samples=1)
    u = np.random.default_rng(12).uniform(-1, 1, (2, S, n_in))
    prm = oracle_params(a_cp=0.3, substeps=4, coupling=coupling, renormalize=True)
    m0s = distinct_states(np.random.default_rng(13), S, n)
    say("streams renorm + inputs", path, coupling)
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32", path=path), streams=S) as r:
        assert r.path == path
        rec = r.run(u)
    worst = 0.0
    for s in range(S):
        rec_o, _ = sto.run(f32(w), f32(w_in), f32(m0s[s]), u[:, s], prm)
        worst = max(worst, float(np.max(np.abs(rec[:, s] - rec_o))))
        # renormalised records have unit norm to FP32 rounding
        assert float(np.max(np.abs(np.linalg.norm(rec[:, s], axis=-1) - 1.0))) <= 1e-6
    say("  max diff", worst)
    assert worst <= F32_TOL


@pytest.mark.parametrize("coupling", ["x", "xyz"])
def test_multi_streams64_lyapunov_horizon(stx, coupling):
    """The 64-stream, 512-node workload over ~one Lyapunov time (8 samples =
    160 steps), checked per stream against the FP64 oracle, for the paper's
    coupling and the isotropic one (the N x 192 product)."""
    wl = WORKLOADS["streams64"]
    S = STREAMS["streams64"]
    a = make_stream_arrays(wl, S, samples=8)
    prm = oracle_params(a_cp=wl.a_cp, a_in=wl.a_in, coupling=coupling)
    m0s = np.broadcast_to(a["m0"], (S, wl.n, 3)).copy()
    say("streams64 horizon", coupling)
    with stx.Reservoir(a["W"], a["w_in"], m0s, lib_params(prm, dtype="f32"), streams=S) as r:
        assert r.path == "multi"
        rec = r.run(a["u"])
    worst = 0.0
    for s in (0, 7, 31, 63):
        rec_o, _ = sto.run(a["W"], a["w_in"], a["m0"], a["u"][:, s], prm)
        worst = max(worst, float(np.max(np.abs(rec[:, s] - rec_o))))
    say("  max diff", worst)
    assert worst <= F32_TOL


@pytest.mark.parametrize("coupling", ["x", "xyz"])
def test_multi_continuation_and_state(stx, coupling):
    n, S = 70, 9
    w, w_in, m0, u = stream_case(n, S, seed=3, samples=6)
    prm = oracle_params(a_cp=0.3, coupling=coupling)
    rng = np.random.default_rng(4)
    m0s = np.empty((S, n, 3))
    for s in range(S):
        v = rng.standard_normal((n, 3)) * 0.05
        v[:, 2] += 1.0
        m0s[s] = v / np.linalg.norm(v, axis=1, keepdims=True)
    lp = lib_params(prm, dtype="f32")
    with stx.Reservoir(w, w_in, m0s, lp, streams=S) as r:
        whole = r.run(u)
        fin = r.get_state()
    with stx.Reservoir(w, w_in, m0s, lp, streams=S) as r:
        a = r.run(u[:2])
        b = r.run(u[2:])
        assert np.array_equal(r.get_state(), fin)
        r.set_state(m0s)
        again = r.run(u)
    assert np.array_equal(np.concatenate([a, b]), whole)
    assert np.array_equal(again, whole)
    # each stream evolves on its own: stream 3 alone (FP32, single-stream path)
    with stx.Reservoir(w, w_in, m0s[3], lp) as r1:
        one = r1.run(u[:, 3])
    assert np.max(np.abs(one - whole[:, 3])) <= 1e-4


def test_multi_rejects_unsupported(stx):
    w, w_in, m0, _ = random_case(20, seed=5, samples=1)
    m0s = np.broadcast_to(m0, (3, 20, 3)).copy()
    with pytest.raises(stx.StoError) as ei:
        stx.Reservoir(w, w_in, m0s, lib_params(oracle_params(), dtype="f64"), streams=3)
    assert ei.value.status == stx.STO_E_UNSUPPORTED
    # beyond the persistent kernel (N > 1024: its W slice no longer fits the
    # registers): path="multi" is refused, the automatic choice is the
    # per-stage batch path
    for n, coupling in ((1100, "x"), (1100, "xyz")):
        w, w_in, m0, _ = random_case(n, seed=5, samples=1)
        m0s = np.broadcast_to(m0, (3, n, 3)).copy()
        prm = oracle_params(coupling=coupling)
        with pytest.raises(stx.StoError) as ei:
            stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32", path="multi"), streams=3)
        assert ei.value.status == stx.STO_E_UNSUPPORTED
        with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32"), streams=3) as r:
            assert r.path == "batch"


# ---------------------------------------------------------------------------
# BATCH path: the same product, one launch per RK4 stage, both couplings
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,streams,coupling", [(16, 2, "x"), (100, 5, "xyz"), (257, 17, "x"), (512, 64, "xyz"),
                                                (1100, 3, "x")])
def test_batch_one_step_matches_oracle(stx, n, streams, coupling):
    """One RK4 step per stream from the same FP32-representable state."""
    w, w_in, m0, u = stream_case(n, streams, seed=n + 1, samples=1)
    prm = oracle_params(a_cp=0.3, substeps=1, coupling=coupling)
    say("batch one step", n, streams, coupling)
    rng = np.random.default_rng(n)
    m0s = np.empty((streams, n, 3))
    for s in range(streams):
        v = rng.standard_normal((n, 3)) * 0.05
        v[:, 2] += 1.0
        m0s[s] = v / np.linalg.norm(v, axis=1, keepdims=True)
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32", path="batch"), streams=streams) as r:
        assert r.path == "batch"
        rec = r.run(u)
    worst = 0.0
    for s in (range(streams) if streams <= 8 else (0, 1, streams // 2, streams - 1)):
        rec_o, _ = sto.run(f32(w), f32(w_in), f32(m0s[s]), u[:, s], prm)
        worst = max(worst, float(np.max(np.abs(rec[:, s] - rec_o))))
    say("  max diff", worst)
    assert worst <= F32_TOL


def test_batch_streams64_xyz_lyapunov_horizon(stx):
    """The 64-stream, 512-node workload with all three components coupled
    (the N x 3S product), over ~one Lyapunov time (8 samples = 160 steps),
    per stream against the FP64 oracle."""
    wl = WORKLOADS["streams64"]
    S = STREAMS["streams64"]
    a = make_stream_arrays(wl, S, samples=8)
    prm = oracle_params(a_cp=wl.a_cp, a_in=wl.a_in, coupling="xyz")
    m0s = np.broadcast_to(a["m0"], (S, wl.n, 3)).copy()
    say("streams64 xyz horizon")
    with stx.Reservoir(a["W"], a["w_in"], m0s, lib_params(prm, dtype="f32", path="batch"), streams=S) as r:
        assert r.path == "batch"
        rec = r.run(a["u"])
    worst = 0.0
    for s in (0, 7, 31, 63):
        rec_o, _ = sto.run(a["W"], a["w_in"], a["m0"], a["u"][:, s], prm)
        worst = max(worst, float(np.max(np.abs(rec[:, s] - rec_o))))
    say("  max diff", worst)
    assert worst <= F32_TOL


@pytest.mark.parametrize("coupling", ["x", "xyz"])
def test_batch_continuation_and_agreement(stx, coupling):
    """Split runs equal the whole run bitwise; the batch and the persistent
    multi-stream paths agree to FP32 rounding."""
    n, S = 70, 9
    w, w_in, m0, u = stream_case(n, S, seed=3, samples=6)
    prm = oracle_params(a_cp=0.3, coupling=coupling)
    m0s = np.broadcast_to(m0, (S, n, 3)).copy()
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32", path="batch"), streams=S) as r:
        whole = r.run(u)
        fin = r.get_state()
        r.set_state(m0s)
        a = r.run(u[:2])
        b = r.run(u[2:])
        assert np.array_equal(r.get_state(), fin)
    assert np.array_equal(np.concatenate([a, b]), whole)
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype="f32", path="multi"), streams=S) as r:
        multi = r.run(u)
    say("batch vs multi", float(np.max(np.abs(multi - whole))))
    assert np.max(np.abs(multi - whole)) <= 1e-5


@pytest.mark.parametrize("S,n,coupling,path", [(64, 512, "x", "multi"), (8, 200, "xyz", "multi"), (1, 1000, "x", "resident")])
def test_phase_trace_leaves_results_unchanged(stx, S, n, coupling, path):
    """A run with the phase trace armed (the stamping instance of the
    persistent kernel) writes the same records as a plain run, bitwise, and
    every stamped stage has start <= gathered <= computed <= published."""
    import torch
    say("phase trace", S, n, coupling, path)
    rng = np.random.default_rng(21)
    w = rng.standard_normal((n, n)) / np.sqrt(n)
    w_in = rng.uniform(-1, 1, (n, 1))
    v = rng.standard_normal((S, n, 3)) * 0.3
    v[..., 2] += 1.0
    m0 = v / np.linalg.norm(v, axis=-1, keepdims=True)
    samples, stages = 6, 12
    u = torch.from_numpy(rng.uniform(-1, 1, (samples, S, 1))).cuda()
    prm = lib_params(oracle_params(a_cp=0.3, a_in=0.7, substeps=2, coupling=coupling), "f32", path)
    with stx.Reservoir(w, w_in, m0 if S > 1 else m0[0], prm, streams=S) as r:
        assert r.path == path
        plain = torch.empty((samples, S, n, 3) if S > 1 else (samples, n, 3), dtype=torch.float32, device="cuda")
        r.run_device(u.reshape(samples, -1).contiguous(), plain)
        r.set_state(m0 if S > 1 else m0[0])
        r.trace_phases(stages)
        traced = torch.empty_like(plain)
        r.run_device(u.reshape(samples, -1).contiguous(), traced)
        torch.cuda.synchronize()
        st, khz = r.phase_times()
        r.trace_phases(0)
    assert torch.equal(plain, traced)
    assert khz > 0 and st.shape[1] == stages and st.shape[2] == 4
    stamped = np.all(st > 0, axis=2)
    assert stamped.any()
    t = st[stamped].astype(np.int64)
    assert np.all(np.diff(t, axis=1) >= 0)
