"""GPU parity of the adjoint (reservoir_adjoint*) and the readout gradient
(readout_grad_device) against the oracle's discrete adjoint, and the
torch.autograd wrappers end to end.

Tolerances.  In FP64 the forward trajectory the adjoint differentiates is
bitwise the oracle's (exactly rounded coupling sums); the adjoint's own sums
(W^T bbar, the dL/dW product, the scalar sums) are plain FP64 in an order
of their own.  Each of them carries a relative rounding error of a few
units of 2^-53 times the number of terms, amplified along the reversed
trajectory by at most the growth of the tangent dynamics over the horizon
(a factor e^(lambda_max t) < 2 over the 20-60 steps used here), so the
bound written below, 1e-9 of the largest gradient entry, leaves a margin of
more than 10^3.  FP32 computes the whole adjoint in FP32 (scalar sums in
FP64): relative error ~ 1e-7 per operation, grown over the horizon, hence
2e-4 of the largest entry.
"""

import sys

import numpy as np
import pytest

from common import lib_params, oracle_params, oracle_streams_adjoint, random_case
from oracle import adjoint, readout, sto

pytestmark = pytest.mark.gpu
F64_TOL = 1e-9
F32_TOL = 2e-4
SCALARS = ("a_cp", "a_in", "h_s", "h_appl")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def stx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2312_01121_amd
    return paper_2312_01121_amd


def rel_err(got, ref):
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def compare(got, ref, tol, label):
    """Each array against its largest entry, each scalar gradient against
    its own magnitude."""
    errs = {k: rel_err(got[k], ref[k]) for k in ("W", "w_in", "m0")}
    for k in SCALARS:
        errs[k] = abs(float(got[k]) - float(ref[k])) / max(abs(float(ref[k])), 1e-300)
    say(label, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= tol, (label, k, v)


def case(n, n_in=1, samples=4, substeps=5, seed=0, coupling="x", renormalize=False, a_cp=0.3, a_in=0.7):
    w, w_in, m0, u = random_case(n, n_in=n_in, seed=seed, samples=samples, spread=0.3)
    prm = oracle_params(a_cp=a_cp, a_in=a_in, substeps=substeps, coupling=coupling, renormalize=renormalize)
    rng = np.random.default_rng(seed + 100)
    g_rec = rng.standard_normal((samples, n, 3))
    g_fin = rng.standard_normal((n, 3))
    return w, w_in, m0, u, prm, g_rec, g_fin


F64_CASES = [
    # n, n_in, coupling, renormalize, checkpoint_every
    (1, 1, "x", False, 0),
    (16, 1, "x", False, 7),
    (16, 2, "x", False, 1),
    (37, 1, "xyz", False, 3),
    (130, 1, "x", True, 0),
    (130, 2, "xyz", True, 7),
    (257, 1, "x", False, 6),
]


@pytest.mark.parametrize("n,n_in,coupling,renorm,seg", F64_CASES)
def test_adjoint_matches_oracle_f64(stx, n, n_in, coupling, renorm, seg):
    w, w_in, m0, u, prm, g_rec, g_fin = case(n, n_in=n_in, coupling=coupling, renormalize=renorm)
    say(f"adjoint f64 n={n} n_in={n_in} coupling={coupling} renorm={renorm} seg={seg}")
    ref = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, g_fin)
    with stx.Reservoir(w, w_in, m0, lib_params(prm, "f64")) as r:
        got = r.adjoint(m0, u, g_rec, g_fin, checkpoint_every=seg)
        # the handle's own state is neither used nor changed
        assert np.array_equal(r.get_state(), m0)
    compare(got, ref, F64_TOL, f"n={n}")


@pytest.mark.parametrize("n,coupling,renorm", [(16, "x", False), (100, "xyz", True), (300, "x", False)])
def test_adjoint_matches_oracle_f32(stx, n, coupling, renorm):
    w, w_in, m0, u, prm, g_rec, g_fin = case(n, coupling=coupling, renormalize=renorm)
    # the oracle differentiates the inputs as the FP32 library holds them
    # (the library rounds m0 itself: it requires a unit-norm m0 on creation)
    w, w_in = (np.float32(a).astype(np.float64) for a in (w, w_in))
    g_rec, g_fin = np.float32(g_rec).astype(np.float64), np.float32(g_fin).astype(np.float64)
    say(f"adjoint f32 n={n} coupling={coupling} renorm={renorm}")
    ref = adjoint.run_adjoint(w, w_in, np.float32(m0).astype(np.float64), u, prm, g_rec, g_fin, dot="blas")
    with stx.Reservoir(w, w_in, m0, lib_params(prm, "f32")) as r:
        got = r.adjoint(m0, u, g_rec, g_fin, checkpoint_every=5)
    compare(got, ref, F32_TOL, f"f32 n={n}")


@pytest.mark.parametrize("n,dtype", [(1000, "f64"), (2500, "f32")])
def test_adjoint_large_n(stx, n, dtype):
    """Several tiles of the streaming and product kernels and a ragged tail
    (2500 = 39 x 64 + 4), over a short horizon the oracle finishes quickly."""
    w, w_in, m0, u, prm, g_rec, g_fin = case(n, samples=1, substeps=3, seed=5)
    m0_ref = m0
    if dtype == "f32":
        w, w_in = (np.float32(a).astype(np.float64) for a in (w, w_in))
        m0_ref = np.float32(m0).astype(np.float64)
        g_rec, g_fin = np.float32(g_rec).astype(np.float64), np.float32(g_fin).astype(np.float64)
    say(f"adjoint large n={n} {dtype}")
    ref = adjoint.run_adjoint(w, w_in, m0_ref, u, prm, g_rec, g_fin, dot="blas")
    with stx.Reservoir(w, w_in, m0, lib_params(prm, dtype)) as r:
        got = r.adjoint(m0, u, g_rec, g_fin, checkpoint_every=2)
    compare(got, ref, F64_TOL if dtype == "f64" else F32_TOL, f"large n={n}")


def test_adjoint_segments_agree(stx):
    """Segment length only changes where the forward is recomputed.  On the
    per-stage kernels (segments that are not whole samples) dL/dm0, dL/dw_in
    and the scalars are bitwise the same for every length, dL/dW equal up to
    the product's order; segments of whole samples run on the persistent
    resident kernels, whose sums take another order (1e-13)."""
    w, w_in, m0, u, prm, g_rec, g_fin = case(64, samples=3, substeps=5, seed=2)
    say("adjoint segments 64")
    outs, kern = {}, {}
    with stx.Reservoir(w, w_in, m0, lib_params(prm, "f64")) as r:
        for seg in (1, 4, 7, 0, 5, 15):
            outs[seg] = r.adjoint(m0, u, g_rec, g_fin, checkpoint_every=seg)
            kern[seg] = r.adjoint_kernels
    for seg in (1, 4, 7):
        assert kern[seg] == {"forward": "stage", "reverse": "stage"}, (seg, kern[seg])
    for seg in (0, 5, 15):
        assert kern[seg] == {"forward": "persistent", "reverse": "persistent"}, (seg, kern[seg])
    for group in ((1, 4, 7), (0, 5, 15)):
        ref = outs[group[0]]
        for seg in group[1:]:
            o = outs[seg]
            assert np.array_equal(o["m0"], ref["m0"]), seg
            if group[0] == 1:
                assert np.array_equal(o["w_in"], ref["w_in"]), seg
                for k in SCALARS:
                    assert o[k] == ref[k], (seg, k)
            assert rel_err(o["W"], ref["W"]) <= 1e-13
    compare(outs[0], outs[1], 1e-13, "persistent vs per-stage")


# The persistent single-stream adjoint (one cooperative launch for the
# recompute and one for the reversed stages of every segment): both
# precisions and couplings, renormalisation, 1 to 5 input channels (5 runs
# on the per-stage kernels), several segments, the launch shapes of the
# path table (4 waves, 8 waves x 8 rows; 16 waves x 16 rows in FP32, whose
# reverse runs with 8 waves), against the oracle and against the per-stage
# kernels (STO_RES_ADJOINT=0).
RES_CASES = [
    # dtype, n, n_in, coupling, renorm, samples, checkpoint samples
    ("f64", 40, 1, "x", False, 4, 2),
    ("f64", 300, 2, "xyz", True, 3, 0),
    ("f64", 1000, 1, "x", False, 2, 1),
    ("f64", 1500, 4, "x", True, 2, 0),
    ("f64", 2048, 1, "x", False, 1, 0),
    ("f64", 1000, 1, "xyz", False, 1, 0),
    ("f32", 200, 3, "x", False, 4, 2),
    ("f32", 700, 1, "xyz", True, 3, 1),
    ("f32", 1000, 1, "x", False, 2, 0),
    ("f32", 90, 5, "x", False, 3, 0),
]


@pytest.mark.parametrize("dtype,n,n_in,coupling,renorm,samples,cps", RES_CASES,
                         ids=[f"{c[0]}-n{c[1]}-in{c[2]}-{c[3]}" + ("-renorm" if c[4] else "") for c in RES_CASES])
def test_adjoint_resident_reverse(stx, dtype, n, n_in, coupling, renorm, samples, cps, monkeypatch):
    sub = 5
    w, w_in, m0, u, prm, g_rec, g_fin = case(n, n_in=n_in, samples=samples, substeps=sub, seed=n + n_in,
                                             coupling=coupling, renormalize=renorm)
    m0_ref = m0
    if dtype == "f32":
        w, w_in, g_rec, g_fin = (np.float32(a).astype(np.float64) for a in (w, w_in, g_rec, g_fin))
        m0_ref = np.float32(m0).astype(np.float64)
    say(f"adjoint resident reverse {dtype} n={n} n_in={n_in} {coupling} renorm={renorm}")
    ref = adjoint.run_adjoint(w, w_in, m0_ref, u, prm, g_rec, g_fin, dot="blas")
    got = {}
    for res in ("1", "0"):
        monkeypatch.setenv("STO_RES_ADJOINT", res)
        with stx.Reservoir(w, w_in, m0, lib_params(prm, dtype)) as r:
            got[res] = r.adjoint(m0, u, g_rec, g_fin, checkpoint_every=cps * sub)
            persistent = res == "1" and n_in <= 4
            assert r.adjoint_kernels == ({"forward": "persistent", "reverse": "persistent"} if persistent
                                         else {"forward": "stage", "reverse": "stage"}), (res, r.adjoint_kernels)
        compare(got[res], ref, F64_TOL if dtype == "f64" else F32_TOL, f"resident={res}")
    compare(got["1"], got["0"], F64_TOL if dtype == "f64" else F32_TOL, "persistent vs per-stage")


# The traced recompute runs the forward's launch shape, four waves per row
# included (forced through the environment); the reverse keeps one wave per
# row.  Against the oracle's adjoint.
SPLIT_CASES = [("f64", 1000, "x", 16, 0), ("f64", 600, "xyz", 8, 8), ("f32", 700, "xyz", 8, 8)]


@pytest.mark.parametrize("dtype,n,coupling,waves,rpb", SPLIT_CASES,
                         ids=[f"{c[0]}-n{c[1]}-{c[2]}-{c[3]}x{c[4]}s4" for c in SPLIT_CASES])
def test_adjoint_four_waves_per_row(stx, dtype, n, coupling, waves, rpb, monkeypatch):
    sub = 5
    w, w_in, m0, u, prm, g_rec, g_fin = case(n, samples=2, substeps=sub, seed=n + 11, coupling=coupling)
    m0_ref = m0
    if dtype == "f32":
        w, w_in, g_rec, g_fin = (np.float32(a).astype(np.float64) for a in (w, w_in, g_rec, g_fin))
        m0_ref = np.float32(m0).astype(np.float64)
    monkeypatch.setenv("STO_RESIDENT_WAVES", str(waves))
    monkeypatch.setenv("STO_RESIDENT_SPLIT", "4")
    if rpb:
        monkeypatch.setenv("STO_RESIDENT_RPB", str(rpb))
    say(f"adjoint four waves per row {dtype} n={n} {coupling} {waves}x{rpb}")
    ref = adjoint.run_adjoint(w, w_in, m0_ref, u, prm, g_rec, g_fin, dot="blas")
    with stx.Reservoir(w, w_in, m0, lib_params(prm, dtype)) as r:
        assert r.path == "resident"
        got = r.adjoint(m0, u, g_rec, g_fin, checkpoint_every=sub)
        assert r.adjoint_kernels == {"forward": "persistent", "reverse": "persistent"}, r.adjoint_kernels
    compare(got, ref, F64_TOL if dtype == "f64" else F32_TOL, "four waves per row")


def test_adjoint_device_api(stx):
    import torch
    w, w_in, m0, u, prm, g_rec, g_fin = case(40, samples=3, substeps=4, seed=9)
    say("adjoint device api 40")
    ref = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, None)
    dev = torch.device("cuda")
    with stx.Reservoir(w, w_in, m0, lib_params(prm, "f64")) as r:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
        out = r.adjoint_device(t(m0), t(u), grad_states_dev=t(g_rec))
        torch.cuda.synchronize()
        got = {"W": out["W"].cpu().numpy(), "w_in": out["w_in"].cpu().numpy(), "m0": out["m0"].cpu().numpy()}
        got.update({k: float(v) for k, v in zip(SCALARS, out["scalars"].cpu().numpy())})
        compare(got, ref, F64_TOL, "device api")
        # only the scalars requested
        only = r.adjoint_device(t(m0), t(u), grad_states_dev=t(g_rec), want=("scalars",))
        assert np.array_equal(only["scalars"].cpu().numpy(), out["scalars"].cpu().numpy())


@pytest.mark.parametrize("dtype,S,coupling,renorm,seg", [("f64", 1, "x", False, 10), ("f64", 1, "xyz", True, 0),
                                                         ("f32", 1, "x", False, 15), ("f32", 5, "xyz", True, 10),
                                                         ("f32", 3, "x", False, 0)])
def test_adjoint_records_as_checkpoints(stx, dtype, S, coupling, renorm, seg):
    """reservoir_adjoint_records_device takes its checkpoints from the run's
    records instead of a forward pass of its own: the same gradients as
    reservoir_adjoint_device (bitwise in FP64, where every path rounds the
    stage sums exactly), and the oracle's."""
    import torch
    dev = torch.device("cuda")
    n, samples, sub = 40, 6, 5
    rng = np.random.default_rng(41)
    w, w_in, m0, _ = random_case(n, seed=43, samples=1, spread=0.3)
    m0s = m0 if S == 1 else unit_states(rng, S, n)
    lead = (samples,) if S == 1 else (samples, S)
    u = rng.uniform(-1, 1, lead + (1,))
    prm = oracle_params(a_cp=0.3, a_in=0.7, substeps=sub, coupling=coupling, renormalize=renorm)
    g_rec = rng.standard_normal(lead + (n, 3))
    g_fin = rng.standard_normal(m0s.shape)
    m0_ref = m0s
    if dtype == "f32":
        w, w_in, g_rec, g_fin, m0_ref = (np.float32(a).astype(np.float64) for a in (w, w_in, g_rec, g_fin, m0s))
    say(f"adjoint records {dtype} S={S} {coupling} renorm={renorm} seg={seg}")
    if S == 1:
        ref = adjoint.run_adjoint(w, w_in, m0_ref, u, prm, g_rec, g_fin, dot="blas")
    else:
        ref = oracle_streams_adjoint(w, w_in, m0_ref, u, prm, g_rec, g_fin)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    t = lambda a, dt=tdt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    host = lambda o: {**{k: o[k].cpu().numpy() for k in ("W", "w_in", "m0")},  # noqa: E731
                      **{k: float(v) for k, v in zip(SCALARS, o["scalars"].cpu().numpy())}}
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, dtype), streams=S) as r:
        u_d = t(u, torch.float64)
        records = torch.empty(lead + (n, 3), dtype=tdt, device=dev)
        r.run_device(u_d, records)
        args = dict(grad_states_dev=t(g_rec), grad_final_dev=t(g_fin), checkpoint_every=seg)
        own = host(r.adjoint_device(t(m0s), u_d, **args))
        from_rec = host(r.adjoint_device(t(m0s), u_d, records_dev=records, **args))
        torch.cuda.synchronize()
        if dtype == "f64":
            for k in ("W", "w_in", "m0"):
                assert np.array_equal(from_rec[k], own[k]), k
            for k in SCALARS:
                assert from_rec[k] == own[k], k
        else:
            compare(from_rec, own, F32_TOL, "records vs own checkpoints")
        compare(from_rec, ref, F64_TOL if dtype == "f64" else F32_TOL, "records vs oracle")
        # segments must be whole samples when the records are the checkpoints
        with pytest.raises(stx.StoError) as ei:
            r.adjoint_device(t(m0s), u_d, records_dev=records, grad_states_dev=t(g_rec), checkpoint_every=sub + 2)
        assert ei.value.status == stx.STO_E_INVALID


def test_adjoint_zero_steps(stx):
    w, w_in, m0, u, prm, g_rec, g_fin = case(8, seed=4)
    with stx.Reservoir(w, w_in, m0, lib_params(prm, "f64")) as r:
        got = r.adjoint(m0, u[:0], None, g_fin)
    assert np.array_equal(got["m0"], g_fin)
    assert not np.any(got["W"]) and not np.any(got["w_in"])
    assert all(got[k] == 0.0 for k in SCALARS)


def test_adjoint_rejects_and_reports(stx):
    w, w_in, m0, u, prm, g_rec, g_fin = case(8, seed=4)
    with stx.Reservoir(w, w_in, m0, lib_params(prm, "f64")) as r:
        with pytest.raises(stx.StoError) as e:
            stx.reservoir_adjoint(r.h, 8, 1, prm.substeps, m0, u, 7, None, None)   # not a multiple of substeps
        assert e.value.status == stx.STO_E_INVALID
        with pytest.raises(stx.StoError) as e:
            r.adjoint(m0, u, checkpoint_every=-1)
        assert e.value.status == stx.STO_E_INVALID
    # a state that becomes non-finite (lambda = -1 and m along p: 1 + lambda m.p = 0)
    prm_bad = oracle_params(substeps=2).replace(lam=-1.0)
    m_p = np.tile(np.array([[1.0, 0.0, 0.0]]), (8, 1))
    with stx.Reservoir(np.zeros((8, 8)), w_in, m_p, lib_params(prm_bad, "f64")) as r3:
        with pytest.raises(stx.StoError) as e:
            r3.adjoint(m_p, u[:2], g_rec[:2])
        assert e.value.status == stx.STO_E_NONFINITE


@pytest.mark.parametrize("dtype,features", [("f64", 0), ("f32", 0), ("f64", 1)])
def test_readout_grad_matches_oracle(stx, dtype, features):
    import torch
    rng = np.random.default_rng(3)
    T, n, washout, lam = 60, 12, 6, 1e-4
    rec = rng.standard_normal((T, n, 3))
    if dtype == "f32":
        rec = np.float32(rec).astype(np.float64)
    y = rng.standard_normal(T)
    comps = "xyz" if features else "x"
    j_ref, w_ref, g_ref = readout.ridge_objective_grad(rec, y, washout, lam, comps)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rec_d = torch.from_numpy(rec).to("cuda", tdt).contiguous()
    y_d = torch.from_numpy(y).cuda()
    w_d, _ = stx.readout_fit_device(rec_d, y_d, washout, lam, features)
    g_d, j = stx.readout_grad_device(rec_d, y_d, washout, lam, w_d, features)
    g = g_d.double().cpu().numpy()
    tol = 1e-10 if dtype == "f64" else 1e-5
    say(f"readout grad {dtype} features={features}", rel_err(g, g_ref), abs(j - j_ref) / j_ref)
    assert rel_err(g, g_ref) <= tol and abs(j - j_ref) <= tol * j_ref


def test_autograd_end_to_end(stx):
    """loss.backward() through the ridge loss and the run equals the oracle's
    adjoint driven by the oracle's ridge gradient."""
    import torch
    from paper_2312_01121_amd import autograd
    n, samples, sub, washout, lam = 16, 30, 5, 5, 1e-3
    w, w_in, m0, u = random_case(n, seed=8, samples=samples, spread=0.3)
    prm = oracle_params(a_cp=0.3, a_in=0.7, substeps=sub)
    y = np.tanh(np.convolve(u[:, 0], np.ones(5))[:samples])
    say("autograd end to end 16")
    rec, _ = sto.run(w, w_in, m0, u, prm)
    j_ref, _, g_rec = readout.ridge_objective_grad(rec, y, washout, lam)
    ref = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, None)

    leaf = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)  # noqa: E731
    W, WIN, M0 = leaf(w), leaf(w_in), leaf(m0)
    sc = [leaf(getattr(prm, k)) for k in SCALARS]
    records = autograd.reservoir_records(W, WIN, M0, *sc, torch.from_numpy(u).cuda(), lib_params(prm, "f64"))
    assert np.array_equal(records.detach().cpu().numpy(), rec)
    loss = autograd.ridge_loss(records, torch.from_numpy(y).cuda(), washout, lam)
    assert abs(float(loss) - j_ref) <= 1e-10 * j_ref
    loss.backward()
    got = {"W": W.grad.numpy(), "w_in": WIN.grad.numpy(), "m0": M0.grad.numpy()}
    got.update({k: float(t.grad) for k, t in zip(SCALARS, sc)})
    compare(got, ref, 1e-8, "autograd")


# ---------------------------------------------------------------------------
# S input streams sharing W (the batched FP32 adjoint)
# ---------------------------------------------------------------------------
def unit_states(rng, streams, n, spread=0.3):
    v = rng.standard_normal((streams, n, 3)) * spread
    v[..., 2] += 1.0
    return v / np.linalg.norm(v, axis=2, keepdims=True)


# Segments of whole samples (0: the whole run, 4, 8) run the forward on the
# persistent multi-stream kernel; a 3-step segment on the per-stage kernels.
@pytest.mark.parametrize("coupling,seg,renorm", [("x", 0, False), ("xyz", 3, False), ("xyz", 4, False),
                                                 ("x", 8, False), ("xyz", 4, True), ("x", 3, True)])
def test_adjoint_streams_matches_oracle(stx, coupling, seg, renorm):
    n, S, samples, sub = 40, 3, 3, 4
    w, w_in, _, _ = random_case(n, seed=21, samples=1, spread=0.3)
    rng = np.random.default_rng(22)
    m0s = unit_states(rng, S, n)
    u = rng.uniform(-1, 1, (samples, S, 1))
    prm = oracle_params(a_cp=0.3, a_in=0.7, substeps=sub, coupling=coupling, renormalize=renorm)
    g_rec = np.float32(rng.standard_normal((samples, S, n, 3))).astype(np.float64)
    g_fin = np.float32(rng.standard_normal((S, n, 3))).astype(np.float64)
    w, w_in = (np.float32(a).astype(np.float64) for a in (w, w_in))
    say(f"adjoint streams S={S} n={n} {coupling} seg={seg} renorm={renorm}")
    ref = oracle_streams_adjoint(w, w_in, np.float32(m0s).astype(np.float64), u, prm, g_rec, g_fin)
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, "f32"), streams=S) as r:
        got = r.adjoint(m0s, u, g_rec, g_fin, checkpoint_every=seg)
        # segments of whole samples run on the persistent kernels
        kern = r.adjoint_kernels
        whole = seg == 0 or seg % sub == 0
        assert kern == ({"forward": "persistent", "reverse": "persistent"} if whole
                        else {"forward": "stage", "reverse": "stage"}), kern
    compare(got, ref, F32_TOL, f"streams {coupling}")


@pytest.mark.parametrize("coupling,n,S,seg,renorm", [("xyz", 300, 7, 0, True), ("x", 130, 20, 8, False),
                                                     ("xyz", 40, 3, 4, False), ("xyz", 700, 6, 4, False),
                                                     ("x", 1000, 3, 0, True)])
def test_adjoint_streams_reverse_kernels_agree(stx, coupling, n, S, seg, renorm, monkeypatch):
    """The reversed stages on the persistent kernel (several 16-node tiles
    and stream groups with a ragged last group; every register-slice size of
    W, up to N = 1,000; one and two row tiles per workgroup) and on the
    per-stage kernels (STO_MULTI_REVERSE=0), against the oracle and against
    each other."""
    samples, sub = 2, 4
    w, w_in, _, _ = random_case(n, seed=31, samples=1, spread=0.3)
    rng = np.random.default_rng(32)
    m0s = unit_states(rng, S, n)
    u = rng.uniform(-1, 1, (samples, S, 1))
    prm = oracle_params(a_cp=0.3, a_in=0.7, substeps=sub, coupling=coupling, renormalize=renorm)
    g_rec = np.float32(rng.standard_normal((samples, S, n, 3))).astype(np.float64)
    g_fin = np.float32(rng.standard_normal((S, n, 3))).astype(np.float64)
    w, w_in = (np.float32(a).astype(np.float64) for a in (w, w_in))
    ref = oracle_streams_adjoint(w, w_in, np.float32(m0s).astype(np.float64), u, prm, g_rec, g_fin)
    got = {}
    # persistent reverse with the library's choice of row tiles, with two
    # row tiles per workgroup forced, and the per-stage reverse
    for key, rev, tiles in (("auto", "1", None), ("two", "1", "2"), ("stage", "0", None)):
        monkeypatch.setenv("STO_MULTI_REVERSE", rev)
        if tiles:
            monkeypatch.setenv("STO_MULTI_TILES", tiles)
        else:
            monkeypatch.delenv("STO_MULTI_TILES", raising=False)
        say(f"adjoint streams {key} S={S} n={n} {coupling} seg={seg} renorm={renorm}")
        with stx.Reservoir(w, w_in, m0s, lib_params(prm, "f32"), streams=S) as r:
            assert r.path == "multi"
            got[key] = r.adjoint(m0s, u, g_rec, g_fin, checkpoint_every=seg)
            assert r.adjoint_kernels["reverse"] == ("persistent" if rev == "1" else "stage"), key
        compare(got[key], ref, F32_TOL, f"streams {key} {coupling}")
    compare(got["auto"], got["stage"], F32_TOL, "persistent vs per-stage reverse")
    compare(got["two"], got["stage"], F32_TOL, "two row tiles vs per-stage reverse")


@pytest.mark.parametrize("n_in,coupling", [(3, "xyz"), (4, "x"), (5, "xyz")])
def test_adjoint_streams_several_inputs(stx, n_in, coupling, monkeypatch):
    """Several input channels: dL/dw_in of every channel (summed in
    registers over a segment by the persistent reverse for up to 4 channels;
    5 channels reverse on the per-stage kernels), against the oracle and
    against the per-stage reverse."""
    n, S, samples, sub = 60, 6, 2, 4
    w, w_in, _, _ = random_case(n, n_in=n_in, seed=51, samples=1, spread=0.3)
    rng = np.random.default_rng(52)
    m0s = unit_states(rng, S, n)
    u = rng.uniform(-1, 1, (samples, S, n_in))
    prm = oracle_params(a_cp=0.3, a_in=0.7, substeps=sub, coupling=coupling, renormalize=False)
    g_rec = np.float32(rng.standard_normal((samples, S, n, 3))).astype(np.float64)
    g_fin = np.float32(rng.standard_normal((S, n, 3))).astype(np.float64)
    w, w_in = (np.float32(a).astype(np.float64) for a in (w, w_in))
    ref = oracle_streams_adjoint(w, w_in, np.float32(m0s).astype(np.float64), u, prm, g_rec, g_fin)
    got = {}
    for rev in ("1", "0"):
        monkeypatch.setenv("STO_MULTI_REVERSE", rev)
        say(f"adjoint streams n_in={n_in} {coupling} reverse={rev}")
        with stx.Reservoir(w, w_in, m0s, lib_params(prm, "f32"), streams=S) as r:
            assert r.path == "multi"
            got[rev] = r.adjoint(m0s, u, g_rec, g_fin, checkpoint_every=sub)
            persistent = rev == "1" and n_in <= 4
            assert r.adjoint_kernels["reverse"] == ("persistent" if persistent else "stage"), (rev, n_in)
        compare(got[rev], ref, F32_TOL, f"streams n_in={n_in} reverse={rev}")
    compare(got["1"], got["0"], F32_TOL, "persistent vs per-stage reverse")


def test_adjoint_streams64_xyz_oracle_and_central_fd(stx):
    """The differentiation workload's shape: N = 512, 64 input streams sharing
    W, all three components coupled (the N x 192 product), one input sample
    of 5 RK4 steps.  The GPU adjoint (FP32) against the oracle's adjoint, and
    the oracle's adjoint against FP64 central differences (h = 1e-6) of the
    oracle's forward for the four scalars and a random direction of W."""
    from workloads import STREAMS, WORKLOADS, make_stream_arrays
    wl = WORKLOADS["streams64"]
    S = STREAMS["streams64"]
    a = make_stream_arrays(wl, S, samples=1)
    prm = oracle_params(a_cp=wl.a_cp, a_in=wl.a_in, coupling="xyz", substeps=5)
    rng = np.random.default_rng(64)
    m0s = unit_states(rng, S, wl.n, spread=0.05)
    g_rec = np.float32(rng.standard_normal((1, S, wl.n, 3))).astype(np.float64)
    w, w_in = (np.float32(x).astype(np.float64) for x in (a["W"], a["w_in"]))
    m0_ref = np.float32(m0s).astype(np.float64)
    say("adjoint streams64 xyz")
    ref = oracle_streams_adjoint(w, w_in, m0_ref, a["u"], prm, g_rec, None, workers=16)
    with stx.Reservoir(w, w_in, m0s, lib_params(prm, "f32"), streams=S) as r:
        assert r.path == "multi"
        # a segment of the whole sample: the persistent forward and reverse
        got = r.adjoint(m0s, a["u"], g_rec, checkpoint_every=5)
        assert r.adjoint_kernels == {"forward": "persistent", "reverse": "persistent"}, r.adjoint_kernels
    compare(got, ref, F32_TOL, "streams64 xyz")

    def loss(p, ww):
        tot = 0.0
        for s in range(S):
            rec, _ = sto.run(ww, w_in, m0_ref[s], a["u"][:, s], p, dot="blas")
            tot += float(np.sum(rec * g_rec[:, s]))
        return tot

    h = 1e-6
    errs = {}
    for name in SCALARS:
        v = getattr(prm, name)
        fd = (loss(prm.replace(**{name: v + h}), w) - loss(prm.replace(**{name: v - h}), w)) / (2 * h)
        errs[name] = abs(fd - ref[name]) / max(abs(ref[name]), 1e-30)
    d_w = rng.standard_normal(w.shape)
    fd = (loss(prm, w + h * d_w) - loss(prm, w - h * d_w)) / (2 * h)
    mine = float(np.sum(ref["W"] * d_w))
    errs["W"] = abs(fd - mine) / abs(mine)
    say("  oracle adjoint vs central differences", {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-6


@pytest.mark.parametrize("coupling", ["xyz", "x"])
def test_adjoint_streams64_paper_amplitudes_records(stx, coupling, monkeypatch):
    """The differentiation workload in the configuration the benchmark times:
    N = 512, 64 streams, the paper's amplitudes (A_cp = A_in = 1 Oe), 10
    input samples of 20 RK4 steps, a checkpoint every 100 steps taken from
    the run's records (reservoir_adjoint_records_device), the library's
    choice of row tiles and stream groups (13 groups with a ragged last one
    for isotropic coupling).  The persistent reverse and the per-stage
    reverse against the oracle's adjoint (FP64, every stream)."""
    import torch
    from workloads import STREAMS, WORKLOADS, make_stream_arrays
    wl = WORKLOADS["streams64"]
    S = STREAMS["streams64"]
    samples = 10
    a = make_stream_arrays(wl, S, samples=samples)
    amp = 1.764e7 * 1e-9                      # 1 Oe in the dimensionless field unit
    prm = oracle_params(a_cp=amp, a_in=amp, coupling=coupling, substeps=wl.substeps)
    rng = np.random.default_rng(65)
    m0s = np.ascontiguousarray(np.broadcast_to(a["m0"], (S, wl.n, 3)))
    g_rec = np.float32(rng.standard_normal((samples, S, wl.n, 3))).astype(np.float64)
    w, w_in = (np.float32(x).astype(np.float64) for x in (a["W"], a["w_in"]))
    say(f"adjoint streams64 paper amplitudes {coupling}: oracle over {S} streams")
    ref = oracle_streams_adjoint(w, w_in, np.float32(m0s).astype(np.float64), a["u"], prm, g_rec, None,
                                 workers=16)
    dev = torch.device("cuda")
    got = {}
    for rev in ("1", "0"):
        monkeypatch.setenv("STO_MULTI_REVERSE", rev)
        say(f"  reverse={rev}")
        with stx.Reservoir(w, w_in, m0s, lib_params(prm, "f32"), streams=S) as r:
            assert r.path == "multi"
            u_d = torch.from_numpy(a["u"]).to(dev)
            records = torch.empty((samples, S, wl.n, 3), dtype=torch.float32, device=dev)
            r.run_device(u_d, records)
            out = r.adjoint_device(torch.from_numpy(m0s).to(dev, torch.float32), u_d,
                                   grad_states_dev=torch.from_numpy(g_rec).to(dev, torch.float32),
                                   checkpoint_every=100, records_dev=records)
            torch.cuda.synchronize()
            assert r.adjoint_kernels == {"forward": "persistent",
                                         "reverse": "persistent" if rev == "1" else "stage"}, r.adjoint_kernels
        got[rev] = {**{k: out[k].double().cpu().numpy() for k in ("W", "w_in", "m0")},
                    **{k: float(v) for k, v in zip(SCALARS, out["scalars"].cpu().numpy())}}
        compare(got[rev], ref, F32_TOL, f"streams64 paper amplitudes {coupling} reverse={rev}")
    compare(got["1"], got["0"], F32_TOL, "persistent vs per-stage reverse")


def test_adjoint_matches_central_fd_f64(stx):
    """dJ of the ridge objective of a GPU run (FP64, 12 samples x 20 steps)
    by the adjoint against central differences (h = 1e-6) of GPU runs."""
    import torch
    n, samples, washout, lam = 64, 12, 2, 1e-4
    w, w_in, m0, u = random_case(n, seed=31, samples=samples, spread=0.3)
    prm = oracle_params(a_cp=0.3, a_in=0.7)
    y = np.tanh(np.convolve(u[:, 0], np.ones(5))[:samples])
    u_d = torch.from_numpy(u).cuda()
    y_d = torch.from_numpy(y).cuda()

    def objective(p, ww, grad=False):
        with stx.Reservoir(ww, w_in, m0, lib_params(p, "f64")) as r:
            st = torch.empty((samples, n, 3), dtype=torch.float64, device="cuda")
            r.run_device(u_d, st)
            w_d, _ = stx.readout_fit_device(st, y_d, washout, lam)
            g, j = stx.readout_grad_device(st, y_d, washout, lam, w_d)
            if not grad:
                return j
            out = r.adjoint_device(torch.from_numpy(m0).cuda(), u_d, grad_states_dev=g)
            torch.cuda.synchronize()
            return j, out

    say("adjoint vs central differences (GPU, f64)")
    _, out = objective(prm, w, grad=True)
    scal = out["scalars"].cpu().numpy()
    gw = out["W"].cpu().numpy()
    h = 1e-6
    errs = {}
    for q, name in enumerate(SCALARS):
        v = getattr(prm, name)
        fd = (objective(prm.replace(**{name: v + h}), w) - objective(prm.replace(**{name: v - h}), w)) / (2 * h)
        errs[name] = abs(fd - scal[q]) / max(abs(scal[q]), 1e-30)
    d_w = np.random.default_rng(32).standard_normal(w.shape)
    fd = (objective(prm, w + h * d_w) - objective(prm, w - h * d_w)) / (2 * h)
    mine = float(np.sum(gw * d_w))
    errs["W"] = abs(fd - mine) / abs(mine)
    say("  ", {k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-6
