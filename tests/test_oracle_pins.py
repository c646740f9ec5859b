"""The CPU oracle against closed forms, invariants and brute force (no GPU)."""

import math
from fractions import Fraction

import numpy as np
import pytest

import pins
from oracle import constants, readout, sto
from oracle import exact_dot, exact_matvec, exact_sum


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


# ----------------------------------------------------------------------------
# Correctly rounded dot products
# ----------------------------------------------------------------------------
def _exact(x, y):
    return float(sum((Fraction(a) * Fraction(b) for a, b in zip(x, y)), Fraction(0)))


def test_exact_dot_matches_rational_arithmetic():
    rng = np.random.default_rng(1)
    for trial in range(600):
        n = int(rng.integers(1, 40))
        x = rng.standard_normal(n) * np.exp2(rng.integers(-300, 300, n))
        y = rng.standard_normal(n) * np.exp2(rng.integers(-300, 300, n))
        if trial % 3 == 0 and n > 1:
            y[-1] = -(x[0] * y[0]) / x[-1]        # heavy cancellation
        assert exact_dot(x, y) == _exact(x, y)


def test_exact_dot_ties_and_extremes():
    # 1 + 2^-53 lies halfway between 1 and 1 + 2^-52: ties go to the even one
    assert exact_dot([1.0, 2.0 ** -53], [1.0, 1.0]) == 1.0
    assert exact_dot([1.0 + 2.0 ** -52, 2.0 ** -53], [1.0, 1.0]) == 1.0 + 2.0 ** -51
    # a sticky bit below the halfway point breaks the tie upwards
    assert exact_dot([1.0, 2.0 ** -53, 2.0 ** -200], [1.0, 1.0, 1.0]) == 1.0 + 2.0 ** -52
    # subnormal results and products below the subnormal range
    assert exact_dot([5e-324], [0.5]) == 0.0
    assert exact_dot([5e-324, 5e-324], [0.5, 0.5]) == 5e-324
    assert exact_dot([3e-200], [3e-200]) == 0.0
    # catastrophic cancellation is exact
    assert exact_dot([1e308, 1e308, 1.0], [1e10, -1e10, 3.0]) == 3.0
    big = [1e300, 1e-300]
    assert exact_dot(big, [1e8, 1.0]) == _exact(big, [1e8, 1.0])
    assert exact_dot([1.0], [0.0]) == 0.0
    assert exact_dot([], []) == 0.0


def test_exact_sum_equals_fsum():
    rng = np.random.default_rng(2)
    for _ in range(200):
        x = rng.standard_normal(50) * np.exp2(rng.integers(-80, 80, 50))
        assert exact_sum(x) == math.fsum(x)


def test_exact_matvec_rows():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((9, 31))
    x = rng.standard_normal(31)
    out = exact_matvec(a, x)
    assert all(out[k] == _exact(a[k], x) for k in range(9))
    np.testing.assert_allclose(out, a @ x, rtol=1e-13)


def test_exact_matvec_fast_path_against_rational_arithmetic():
    """Rows decided by the certified enclosure and rows sent to the
    superaccumulator both equal the rational-arithmetic result: ordinary
    rows, heavy cancellation, wide exponent ranges, products below 2^-960
    and above 2^960, zero rows, exact ties and results one sticky bit away
    from a tie."""
    from oracle._native import exact_fallbacks, exact_matvec_reference
    rng = np.random.default_rng(31)
    rows = []
    for trial in range(400):
        n = int(rng.integers(1, 70))
        kind = trial % 8
        x = rng.standard_normal(n)
        if kind == 1:
            x *= np.exp2(rng.integers(-300, 300, n))
        if kind == 2 and n > 1:
            x[-1] = -x[0]                                   # cancellation
        if kind == 3:
            x *= np.exp2(-700.0)                            # tiny products
        if kind == 4:
            x *= np.exp2(600.0)                             # huge products
        if kind == 5:
            x[:] = 0.0
        rows.append(x)
    width = max(len(r) for r in rows)
    a = np.zeros((len(rows) + 3, width + 2))
    for k, r in enumerate(rows):
        a[k, :len(r)] = r
    v = rng.standard_normal(width + 2) * np.exp2(rng.integers(-40, 40, width + 2))
    v[:3] = 1.0
    # a tie (1 + 2^-53 lies halfway between two doubles), a tie broken by a
    # sticky bit far below, and a result just below a power of two
    a[-3, :2] = [1.0, 2.0 ** -53]
    a[-2, :3] = [1.0, 2.0 ** -53, 2.0 ** -300]
    a[-1, :2] = [2.0, -(2.0 ** -60)]
    ref = [float(sum((Fraction(a[k, i]) * Fraction(v[i]) for i in range(a.shape[1])),
                     Fraction(0))) for k in range(a.shape[0])]
    f0 = exact_fallbacks()
    got = exact_matvec(a, v)
    sent = exact_fallbacks() - f0
    assert [float(g) for g in got] == ref
    assert np.array_equal(exact_matvec_reference(a, v), got)
    # the ties, the tiny, huge and zero rows went to the superaccumulator;
    # most ordinary rows were certified
    assert 3 <= sent < a.shape[0] // 2, sent


def test_exact_matvec_fast_path_on_workload_shapes():
    """On the coupling matrices of the sized workloads the fast product equals
    the superaccumulator bit for bit, and certifies (nearly) every row."""
    from oracle._native import exact_fallbacks, exact_matvec_reference
    rng = np.random.default_rng(32)
    for n in (16, 257, 1000, 3000):
        a = rng.standard_normal((n, n)) / math.sqrt(n)
        np.fill_diagonal(a, 0.0)
        x = np.cos(rng.uniform(0, math.pi, n))
        f0 = exact_fallbacks()
        got = exact_matvec(a, x)
        assert np.array_equal(got, exact_matvec_reference(a, x))
        assert exact_fallbacks() - f0 <= 1


def test_matvec_rules_agree_on_exact_data():
    """Small integers times dyadic values: every rounding rule is exact."""
    rng = np.random.default_rng(4)
    a = rng.integers(-9, 10, (6, 6)).astype(float)
    x = rng.integers(-16, 17, 6) / 8.0
    ref = np.array([float(sum(Fraction(a[k, i]) * Fraction(x[i]) for i in range(6)))
                    for k in range(6)])
    for rule in ("exact", "blas", "loop"):
        assert np.array_equal(sto.matvec(a, x, rule), ref)


# ----------------------------------------------------------------------------
# Constants
# ----------------------------------------------------------------------------
def test_dimensionless_constants():
    """Table 1 in the unit t0 = 1 ns, h = gamma t0 H."""
    prm = constants.dimensionless()
    assert math.isclose(prm.h_appl, 3.528, rel_tol=1e-15)
    assert math.isclose(constants.demag_oe(), 18199.87456077639, rel_tol=1e-14)
    assert math.isclose(prm.h_k, 0.01764 * (18616.0 - 18199.87456077639), rel_tol=1e-13)
    assert math.isclose(constants.spin_torque_field_oe(), 134.868, rel_tol=1e-5)
    assert math.isclose(prm.h_s, 0.01764 * constants.spin_torque_field_oe(), rel_tol=1e-15)
    assert prm.p == (1.0, 0.0, 6.123233995736766e-17)      # Table 1 prints 6.123234e-17
    assert prm.dt == 0.01 and prm.alpha == 0.005 and prm.lam == 0.288
    # the paper's 1e-11 s step is 0.01 in units of 1 ns
    assert math.isclose(1e-11 / constants.T0, prm.dt, rel_tol=1e-15)


# ----------------------------------------------------------------------------
# Readout (ridge regression)
# ----------------------------------------------------------------------------
def _records(rng, t=60, n=7):
    return rng.standard_normal((t, n, 3))


def test_ridge_equals_augmented_least_squares():
    """(Phi^T Phi + lam I) w = Phi^T y is the least-squares solution of the
    stacked system [Phi; sqrt(lam) I] w = [y; 0] (textbook reduction)."""
    rng = np.random.default_rng(5)
    rec = _records(rng)
    y = rng.standard_normal(60)
    for lam in (1e-6, 1e-2, 3.0):
        phi = readout.features(rec, 6, "x")
        w = readout.ridge(phi, y[6:], lam)
        aug = np.vstack([phi, math.sqrt(lam) * np.eye(phi.shape[1])])
        rhs = np.concatenate([y[6:], np.zeros(phi.shape[1])])
        w_ls = np.linalg.lstsq(aug, rhs, rcond=None)[0]
        np.testing.assert_allclose(w, w_ls, rtol=1e-8, atol=1e-10)


def test_ridge_primal_equals_dual():
    rng = np.random.default_rng(6)
    for rows, cols in ((40, 12), (12, 40)):
        phi = rng.standard_normal((rows, cols))
        y = rng.standard_normal(rows)
        wp = readout.ridge(phi, y, 0.1, "primal")
        wd = readout.ridge(phi, y, 0.1, "dual")
        np.testing.assert_allclose(wp, wd, rtol=1e-10, atol=1e-12)


def test_readout_perfect_feature_and_bias_only():
    rng = np.random.default_rng(7)
    rec = _records(rng, t=80, n=5)
    y = rng.standard_normal(80)
    rec[:, 3, 0] = y                         # one node's m^x is the target
    w, e = readout.readout_fit(rec, y, 8, 1e-10)
    assert e < 1e-12 and abs(w[3] - 1.0) < 1e-6
    rec0 = np.zeros_like(rec)
    _, e0 = readout.readout_fit(rec0, y, 8, 1e-10)   # constant features: NMSE 1
    assert abs(e0 - 1.0) < 1e-9
    phi = readout.features(rec, 8, "xyz")
    assert phi.shape == (72, 16) and np.all(phi[:, -1] == 1.0)


def test_default_washout():
    assert readout.default_washout(2000) == 200
    assert readout.default_washout(10) == 5
    assert readout.default_washout(1001) == 101


# ----------------------------------------------------------------------------
# Failure handling
# ----------------------------------------------------------------------------
def test_oracle_raises_on_nonfinite_state():
    """lambda = -1 with m = p makes 1 + lambda m.p vanish: H_s is infinite."""
    prm = constants.dimensionless().replace(lam=-1.0, p=(1.0, 0.0, 0.0))
    m0 = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    with np.errstate(all="ignore"), pytest.raises(FloatingPointError):
        sto.run(np.zeros((2, 2)), np.zeros((2, 1)), m0, np.zeros((3, 1)), prm)


def test_norm_drift_bounded_on_sto16_prefix():
    """On the 16-node workload the |m|-1 drift stays at integrator level."""
    from workloads import WORKLOADS, make_workload_arrays
    wl = WORKLOADS["sto16"]
    a = make_workload_arrays(wl, samples=50)
    prm = constants.dimensionless(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps)
    rec, _ = sto.run(a["W"], a["w_in"], a["m0"], a["u"], prm)
    assert 0.0 < sto.norm_drift(rec) < 1e-5


# ----------------------------------------------------------------------------
# Stored full-horizon fixtures: made by the current oracle from the current
# generators (tests/golden/make_horizon.py)
# ----------------------------------------------------------------------------
def _fixture(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"horizon_{name}.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files} | {"meta": json.loads(str(z["meta"]))}


@pytest.mark.parametrize("name", ["sto1k", "sto10k", "paper2500", "paper5000", "paper10000"])
def test_horizon_fixture_is_current(name):
    """Each fixture records a hash of the oracle and generator sources it was
    written with: it must be the current one, and its first records must be
    what the oracle computes now (the first sample, or the first two)."""
    import sys
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_horizon
    fix = _fixture(name)
    assert fix["meta"]["oracle_sha256"] == make_horizon.source_hash(), name
    a, prm, meta = make_horizon.case_inputs(name)
    assert meta["n"] == fix["meta"]["n"] and meta["samples"] == fix["meta"]["samples"] == len(fix["sums"])
    k = 2 if meta["n"] <= 1000 else 1
    rec, _ = sto.run(a["W"], a["w_in"], a["m0"], a["u"][:k], prm)
    assert np.array_equal(np.array([[math.fsum(rec[s, :, c]) for c in range(3)] for s in range(k)]),
                          fix["sums"][:k])
    assert fix["idx"][0] == 0 and np.array_equal(fix["records"][0], rec[0])
    assert fix["idx"][-1] == meta["samples"] - 1 and np.array_equal(fix["records"][-1], fix["final"])
