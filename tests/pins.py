"""Pins of the CPU oracle: results fixed by the paper and by mathematics.

Each ``pin_*`` function checks the oracle (or a variant of it handed in as
``rhs`` / ``step`` / ``runner``) against something other than itself:
closed forms of special cases, conservation laws, convergence order, brute
force on tiny inputs and structural symmetries.  Each raises
AssertionError on failure.  ``tests/test_oracle_pins.py`` runs them on the
oracle; ``tests/test_oracle_mutants.py`` runs them on oracle copies with a
planted mistake and checks that every mistake is caught.
"""

from __future__ import annotations

import cmath
import math
from fractions import Fraction

import numpy as np

from oracle import constants, sto


def _prm(**kw):
    return constants.dimensionless().replace(**kw)


def default_runner(w, w_in, m0, u, prm, rhs=sto.field, step=None, dot="exact"):
    return sto.run(w, w_in, m0, u, prm, dot=dot, rhs=rhs, step=step)


def _unit_random(rng, n, spread=1.0):
    v = rng.standard_normal((n, 3))
    v[:, 2] += 1.0 / max(spread, 1e-9)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# Field at m = e_z: closed form (Eq. (gov) with b evaluated by hand)
# --------------------------------------------------------------------------
def ez_closed_form(bx, by, alpha):
    """F at m = e_z for transverse field (bx, by): m x b = (-by, bx, 0) and
    m x (m x b) = (-bx, -by, 0), so F = (by + a bx, -bx + a by, 0)/(1+a^2)."""
    d = 1.0 + alpha * alpha
    return ((by + alpha * bx) / d, (-bx + alpha * by) / d, np.zeros_like(bx))


def pin_field_at_ez(rhs=sto.field, **_):
    """P1: STT term, spin-torque amplitude and input field at m = e_z, W = 0."""
    for p in [constants.P_VEC, (0.6, 0.0, 0.8), (0.48, 0.6, 0.64)]:
        for alpha in (0.005, 0.3):
            prm = _prm(p=p, alpha=alpha, lam=0.288)
            n = 4
            m = (np.zeros(n), np.zeros(n), np.ones(n))
            h_in = np.array([0.0, 0.3, -1.1, 2.0])
            k = rhs(m, np.zeros((n, n)), h_in, prm, "exact")
            hs = prm.h_s / (1.0 + prm.lam * p[2])
            # p x e_z = (p_y, -p_x, 0)
            bx = h_in + hs * p[1]
            by = -hs * p[0]
            ex = ez_closed_form(bx, by, alpha)
            for j in range(3):
                np.testing.assert_allclose(k[j], ex[j], rtol=1e-13, atol=1e-15)


def pin_coupling_brute_force(rhs=sto.field, **_):
    """P6: coupling index, factor and direction against a brute-force sum.

    Target nodes sit at e_z, so their m^x is zero and their field has the
    closed form above with b_x = a_cp sum_i w_ki m_i^x + h_in; the sum is
    evaluated exactly with fractions over an asymmetric integer matrix and
    dyadic source states.
    """
    n_t, n_s = 4, 4
    n = n_t + n_s
    rng = np.random.default_rng(7)
    w = rng.integers(-5, 6, size=(n, n)).astype(float)
    np.fill_diagonal(w, 0.0)
    src = np.array([[0.75, 0.5, math.sqrt(1 - 0.75**2 - 0.25)],
                    [-0.5, 0.5, math.sqrt(0.5)],
                    [0.25, -0.75, math.sqrt(1 - 0.0625 - 0.5625)],
                    [-0.875, 0.0, math.sqrt(1 - 0.765625)]])
    m_aos = np.zeros((n, 3))
    m_aos[:n_t, 2] = 1.0
    m_aos[n_t:] = src
    m = sto.to_soa(m_aos)
    for coupling in ("x", "xyz"):
        prm = _prm(a_cp=0.125, alpha=0.05, coupling=coupling, p=(0.6, 0.0, 0.8))
        h_in = np.array([0.5, -0.25, 0.0, 1.0] + [0.0] * n_s)
        k = rhs(m, w, h_in, prm, "exact")
        hs = prm.h_s / (1.0 + prm.lam * prm.p[2])
        for t in range(n_t):
            cx = float(Fraction(prm.a_cp) * sum(Fraction(w[t, i]) * Fraction(m_aos[i, 0])
                                                 for i in range(n)))
            cy = float(Fraction(prm.a_cp) * sum(Fraction(w[t, i]) * Fraction(m_aos[i, 1])
                                                 for i in range(n)))
            bx = cx + h_in[t] + hs * prm.p[1]
            by = (cy if coupling == "xyz" else 0.0) - hs * prm.p[0]
            ex = ez_closed_form(np.array(bx), np.array(by), prm.alpha)
            got = (k[0][t], k[1][t], k[2][t])
            for j in range(3):
                assert abs(got[j] - float(ex[j])) <= 1e-13 * (1 + abs(float(ex[j]))), \
                    (coupling, t, j, got[j], float(ex[j]))


def pin_gilbert_form(rhs=sto.field, **_):
    """The explicit form of Eq. (gov) solves the implicit Gilbert equation
    dm/dt = -g m x b + alpha m x dm/dt, and dm/dt is orthogonal to m.

    b is rebuilt from its definition in the paper (Eq. (gov) and the field
    list that follows it); W = 0 so only the local terms enter.
    """
    rng = np.random.default_rng(3)
    n = 16
    m_aos = _unit_random(rng, n, spread=2.0)
    m = sto.to_soa(m_aos)
    prm = _prm(alpha=0.2, p=(0.48, 0.6, 0.64))
    h_in = rng.uniform(-1, 1, n)
    k = np.stack(rhs(m, np.zeros((n, n)), h_in, prm, "exact"), axis=1)
    p = np.array(prm.p)
    hs = prm.h_s / (1.0 + prm.lam * (m_aos @ p))
    b = np.zeros((n, 3))
    b[:, 0] = h_in
    b[:, 2] = prm.h_appl + prm.h_k * m_aos[:, 2]
    b += hs[:, None] * np.cross(p[None, :], m_aos)
    gilbert = -prm.g * np.cross(m_aos, b) + prm.alpha * np.cross(m_aos, k)
    np.testing.assert_allclose(k, gilbert, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(np.einsum("nc,nc->n", m_aos, k), 0.0, atol=1e-12)


# --------------------------------------------------------------------------
# Pure precession: exact discrete rotation map of RK4
# --------------------------------------------------------------------------
def rk4_amplification(x):
    """RK4 applied to y' = lambda y multiplies y by R(lambda dt) each step."""
    return 1 + x + x * x / 2 + x ** 3 / 6 + x ** 4 / 24


def pin_precession_map(rhs=sto.field, step=None, runner=default_runner, **_):
    """P2/P3: alpha = 0, no current, W = 0, u = 0.

    m_z is then bitwise constant and z = m_x + i m_y obeys z' = i w z with
    w = h_appl + h_k m_z, so RK4 gives exactly z_n = R(i w dt)^n z_0 and
    |z_n| = |R(i w dt)|^n |z_0| with |R(ix)|^2 = 1 - x^6/72 + x^8/576.
    """
    rng = np.random.default_rng(11)
    n = 5
    m0 = _unit_random(rng, n, spread=0.3)
    prm = _prm(alpha=0.0, h_s=0.0, a_in=0.0, a_cp=0.0)
    samples = 250
    u = np.zeros((samples, 1))
    rec, _ = runner(np.zeros((n, n)), np.zeros((n, 1)), m0, u, prm, rhs=rhs, step=step)
    assert np.array_equal(rec[:, :, 2], np.broadcast_to(m0[:, 2], (samples, n))), "m_z moved"
    z0 = m0[:, 0] + 1j * m0[:, 1]
    for s in (0, 9, 99, samples - 1):
        steps = (s + 1) * prm.substeps
        x = 1j * (prm.h_appl + prm.h_k * m0[:, 2]) * prm.dt
        ex = rk4_amplification(x) ** steps * z0
        got = rec[s, :, 0] + 1j * rec[s, :, 1]
        assert np.max(np.abs(got - ex)) < 1e-12, (s, np.max(np.abs(got - ex)))
        xr = (prm.h_appl + prm.h_k * m0[:, 2]) * prm.dt
        mod = (1 - xr ** 6 / 72 + xr ** 8 / 576) ** (steps / 2) * np.abs(z0)
        assert np.max(np.abs(np.abs(got) - mod)) < 1e-12


def pin_precession_tilted_field(rhs=sto.field, step=None, runner=default_runner, **_):
    """Constant field b = (a_in w_in u, 0, h_appl) with h_k = 0, alpha = 0 and
    no current: Eq. (gov) reduces to the linear ODE dm/dt = b x m = B m with
    B the cross-product matrix of b.  Classic RK4 then maps m exactly by the
    matrix polynomial R(B dt) = I + B dt + (B dt)^2/2 + (B dt)^3/6 + (B dt)^4/24
    per step, and the exact flow is Rodrigues' rotation about b by |b| t.
    Pins the input field path (Eq. (in)), its direction e_x and the sense of
    precession.
    """
    rng = np.random.default_rng(5)
    n = 3
    m0 = _unit_random(rng, n, spread=0.5)
    w_in = np.array([[0.5], [-1.0], [0.25]])
    prm = _prm(alpha=0.0, h_s=0.0, h_k=0.0, a_cp=0.0, a_in=1.5, substeps=40)
    u0 = 0.8
    u = np.full((5, 1), u0)
    rec, _ = runner(np.zeros((n, n)), w_in, m0, u, prm, rhs=rhs, step=step)
    for s in (0, 4):
        steps = (s + 1) * prm.substeps
        t = steps * prm.dt
        for k in range(n):
            b = np.array([prm.a_in * (w_in[k, 0] * u0), 0.0, prm.h_appl])
            bm = np.array([[0.0, -b[2], b[1]], [b[2], 0.0, -b[0]], [-b[1], b[0], 0.0]]) * prm.dt
            r = np.eye(3) + bm + bm @ bm / 2 + bm @ bm @ bm / 6 + bm @ bm @ bm @ bm / 24
            ex = np.linalg.matrix_power(r, steps) @ m0[k]
            assert np.max(np.abs(rec[s, k] - ex)) < 1e-13, (s, k, rec[s, k], ex)
            kk = b / np.linalg.norm(b)
            th = np.linalg.norm(b) * t
            v = m0[k]
            rot = (v * math.cos(th) + np.cross(kk, v) * math.sin(th)
                   + kk * (kk @ v) * (1 - math.cos(th)))
            assert np.max(np.abs(rec[s, k] - rot)) < 1e-6, (s, k, rec[s, k], rot)


# --------------------------------------------------------------------------
# Damping: closed forms and fourth-order convergence
# --------------------------------------------------------------------------
def pin_damping_closed_form(rhs=sto.field, step=None, runner=default_runner, **_):
    """P4: alpha > 0, h_k = 0, no current, W = 0, u = 0.

    m_z(t) = tanh(alpha h_appl t/(1+alpha^2) + atanh m_z(0)) and the azimuth
    advances at h_appl/(1+alpha^2).  The RK4 error must shrink 16-fold per
    halving of dt (classic RK4 is fourth order).
    """
    n = 3
    th0 = np.array([0.3, 1.2, 2.5])
    m0 = np.stack([np.sin(th0), np.zeros(n), np.cos(th0)], axis=1)
    alpha = 0.1
    t_end = 4.0
    errs = []
    for dt in (0.08, 0.04, 0.02):
        sub = int(round(t_end / dt))
        prm = _prm(alpha=alpha, h_s=0.0, h_k=0.0, a_cp=0.0, a_in=0.0, dt=dt, substeps=sub)
        rec, _ = runner(np.zeros((n, n)), np.zeros((n, 1)), m0, np.zeros((1, 1)), prm,
                        rhs=rhs, step=step)
        d = 1 + alpha * alpha
        mz = np.tanh(alpha * prm.h_appl * t_end / d + np.arctanh(m0[:, 2]))
        phi = prm.h_appl * t_end / d
        sin_th = np.sqrt(1 - mz * mz)
        ex = np.stack([sin_th * np.cos(phi), sin_th * np.sin(phi), mz], axis=1)
        errs.append(np.max(np.abs(rec[0] - ex)))
    assert errs[-1] < 1e-5, errs
    for a, b in zip(errs, errs[1:]):
        assert 13.0 < a / b < 19.0, errs


def _relax_G(z, a, b):
    """Antiderivative of 1/((a + b z)(1 - z^2)) by partial fractions."""
    ca = b * b / (b * b - a * a)
    cb = 1.0 / (2.0 * (a + b))
    cc = 1.0 / (2.0 * (a - b))
    return (ca / b) * np.log(np.abs(a + b * z)) - cb * np.log1p(-z) + cc * np.log1p(z)


def pin_relaxation(rhs=sto.field, step=None, runner=default_runner, **_):
    """Uncoupled, undriven, current-free macrospin with Table 1 constants:
    dm_z/dt = alpha (h_appl + h_k m_z)(1 - m_z^2)/(1+alpha^2), so
    G(m_z(t)) - G(m_z(0)) = alpha t/(1+alpha^2) for the antiderivative G of
    1/((h_appl + h_k z)(1 - z^2)).  The exact m_z(t) is found by inverting G;
    the RK4 error of the direction m/|m| against it shrinks at least 16-fold
    per halving of dt, and m relaxes to the field-aligned fixed point +e_z.
    """
    from scipy.optimize import brentq

    th0 = 0.5
    m0 = np.array([[math.sin(th0), 0.0, math.cos(th0)]])
    t_end = 100.0
    probes = (10.0, 40.0, 100.0)
    errs = []
    for dt in (0.02, 0.01):
        sub = int(round(10.0 / dt))
        prm = _prm(h_s=0.0, a_cp=0.0, a_in=0.0, dt=dt, substeps=sub)
        samples = int(round(t_end / 10.0))
        rec, _ = runner(np.zeros((1, 1)), np.zeros((1, 1)), m0, np.zeros((samples, 1)), prm,
                        rhs=rhs, step=step)
        a, b = prm.h_appl, prm.h_k
        d = 1 + prm.alpha * prm.alpha
        g0 = _relax_G(m0[0, 2], a, b)
        e = 0.0
        for t in probes:
            target = prm.alpha * t / d
            z = brentq(lambda z: _relax_G(z, a, b) - g0 - target, m0[0, 2], 1.0 - 1e-15,
                       xtol=1e-16, rtol=1e-15)
            r = rec[int(round(t / 10.0)) - 1, 0]
            e = max(e, abs(r[2] / np.linalg.norm(r) - z))
        errs.append(e)
        assert 1.0 - rec[-1, 0, 2] / np.linalg.norm(rec[-1, 0]) < 1e-5, rec[-1, 0]
    assert errs[-1] < 1e-6 and 12.0 < errs[0] / errs[1] < 40.0, errs


# --------------------------------------------------------------------------
# Energy: conservation without damping, decay with damping
# --------------------------------------------------------------------------
def energy(m_aos, w, w_in, u, prm):
    """E = -sum(h_appl m_z + h_k m_z^2/2) - a_cp/2 x^T W x - a_in u sum(w_in x),
    whose negative gradient is the field b of Eq. (gov) without spin torque
    (W symmetric)."""
    x = m_aos[:, 0]
    mz = m_aos[:, 2]
    return (-np.sum(prm.h_appl * mz + prm.h_k * mz * mz / 2.0)
            - prm.a_cp / 2.0 * (x @ w @ x) - prm.a_in * u * np.sum(w_in[:, 0] * x))


def pin_energy(rhs=sto.field, step=None, runner=default_runner, **_):
    """P5: symmetric W, no current, constant input.  alpha = 0 conserves E up
    to the RK4 error; alpha > 0 makes E non-increasing."""
    rng = np.random.default_rng(2)
    n = 8
    a = rng.standard_normal((n, n))
    w = (a + a.T) / 2.0
    np.fill_diagonal(w, 0.0)
    w_in = rng.uniform(-1, 1, (n, 1))
    m0 = _unit_random(rng, n, spread=1.0)
    u0 = 0.7
    prm = _prm(alpha=0.0, h_s=0.0, a_cp=0.5, a_in=0.8, substeps=20)
    rec, _ = runner(w, w_in, m0, np.full((100, 1), u0), prm, rhs=rhs, step=step)
    e0 = energy(m0, w, w_in, u0, prm)
    es = np.array([energy(r, w, w_in, u0, prm) for r in rec])
    assert np.max(np.abs(es - e0)) < 1e-6 * max(1.0, abs(e0)), np.max(np.abs(es - e0))
    prm = prm.replace(alpha=0.05)
    rec, _ = runner(w, w_in, m0, np.full((100, 1), u0), prm, rhs=rhs, step=step)
    es = np.array([energy(m0, w, w_in, u0, prm)] + [energy(r, w, w_in, u0, prm) for r in rec])
    assert np.all(np.diff(es) <= 1e-9), np.max(np.diff(es))
    assert es[-1] < es[0] - 1e-3


# --------------------------------------------------------------------------
# Whole coupled, driven system: order, norm drift, structure, units
# --------------------------------------------------------------------------
def _coupled_case(n=6, seed=4):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n)) / math.sqrt(n)
    np.fill_diagonal(w, 0.0)
    w_in = rng.uniform(-1, 1, (n, 1))
    m0 = _unit_random(rng, n, spread=0.05)
    u = rng.uniform(-1, 1, (4, 1))
    return w, w_in, m0, u


def pin_global_order(rhs=sto.field, step=None, runner=default_runner, **_):
    """P7: the full coupled, driven system converges at fourth order, and the
    drift of |m_k| from 1 (exactly conserved by Eq. (gov)) shrinks at least
    at fourth order (16 to 32-fold) per halving of dt: it is integrator
    error, not a defect of the field."""
    w, w_in, m0, u = _coupled_case()
    finals, drifts = [], []
    for dt, sub in ((0.04, 10), (0.02, 20), (0.01, 40)):
        prm = _prm(dt=dt, substeps=sub, a_cp=0.3, alpha=0.02)
        rec, fin = runner(w, w_in, m0, u, prm, rhs=rhs, step=step)
        finals.append(fin)
        drifts.append(sto.norm_drift(rec))
    e1 = np.max(np.abs(finals[0] - finals[1]))
    e2 = np.max(np.abs(finals[1] - finals[2]))
    assert 12.0 < e1 / e2 < 20.0, (e1, e2)
    assert 12.0 < drifts[0] / drifts[1] < 40.0 and 12.0 < drifts[1] / drifts[2] < 40.0, drifts


def pin_structure(rhs=sto.field, step=None, runner=default_runner, **_):
    """P8: relabelling nodes permutes the output exactly (the coupling sums
    are rounded once, so their order does not matter); a block-diagonal
    coupling matrix gives exactly the separate runs of its blocks."""
    w, w_in, m0, u = _coupled_case(n=7, seed=9)
    prm = _prm(a_cp=0.4)
    rec, _ = runner(w, w_in, m0, u, prm, rhs=rhs, step=step)
    perm = np.random.default_rng(1).permutation(7)
    rec_p, _ = runner(w[perm][:, perm], w_in[perm], m0[perm], u, prm, rhs=rhs, step=step)
    assert np.array_equal(rec_p, rec[:, perm])
    w2, w_in2, m02, _ = _coupled_case(n=4, seed=10)
    big = np.zeros((11, 11))
    big[:7, :7] = w
    big[7:, 7:] = w2
    rec_b, _ = runner(big, np.vstack([w_in, w_in2]), np.vstack([m0, m02]), u, prm,
                      rhs=rhs, step=step)
    rec_2, _ = runner(w2, w_in2, m02, u, prm, rhs=rhs, step=step)
    assert np.array_equal(rec_b[:, :7], rec) and np.array_equal(rec_b[:, 7:], rec_2)


def pin_units(rhs=sto.field, step=None, runner=default_runner, **_):
    """P9: Eq. (gov) in CGS units with gamma explicit and dt = 1e-11 s gives
    the dimensionless trajectory (t0 = 1 ns, h = gamma t0 H) to round-off."""
    w, w_in, m0, u = _coupled_case(n=5, seed=12)
    phys = constants.physical(a_cp_oe=20.0, a_in_oe=40.0)
    g = constants.GAMMA * constants.T0
    dim = constants.dimensionless(a_cp=g * 20.0, a_in=g * 40.0)
    rec_p, _ = runner(w, w_in, m0, u, phys, rhs=rhs, step=step)
    rec_d, _ = runner(w, w_in, m0, u, dim, rhs=rhs, step=step)
    assert np.max(np.abs(rec_p - rec_d)) < 1e-11, np.max(np.abs(rec_p - rec_d))


def pin_continuation(runner=default_runner, rhs=sto.field, step=None, **_):
    """P10: running u[:a] then u[a:] from the state reached equals one run."""
    w, w_in, m0, u = _coupled_case(n=5, seed=13)
    prm = _prm()
    rec, fin = runner(w, w_in, m0, u, prm, rhs=rhs, step=step)
    r1, f1 = runner(w, w_in, m0, u[:1], prm, rhs=rhs, step=step)
    r2, f2 = runner(w, w_in, f1, u[1:], prm, rhs=rhs, step=step)
    assert np.array_equal(np.concatenate([r1, r2]), rec) and np.array_equal(f2, fin)


# --------------------------------------------------------------------------
# Renormalisation: projected precession in closed form
# --------------------------------------------------------------------------
def pin_renormalize(rhs=sto.field, step=None, runner=default_runner, **_):
    """Optional projection after each step (off by default).

    With alpha = 0, h_k = 0, no current, W = 0 and u = 0 one RK4 step maps
    z = m_x + i m_y to R(i h_appl dt) z and keeps m_z; the projection then
    divides the whole vector by its length.  Projection keeps the ratio
    z/m_z, so after n steps z/m_z = R^n z_0/m_z0, and the unit length fixes
    m_z = sign(m_z0)/sqrt(1 + |R^n z_0/m_z0|^2).  Every record must have unit
    length to round-off, and the projected run must differ from the plain
    one (whose length shrinks by |R| per step in the transverse part).
    """
    rng = np.random.default_rng(21)
    n = 4
    m0 = _unit_random(rng, n, spread=0.8)
    m0[3] *= -1.0                       # one node in the lower hemisphere
    prm = _prm(alpha=0.0, h_s=0.0, h_k=0.0, a_cp=0.0, a_in=0.0, dt=0.05, substeps=30,
               renormalize=True)
    samples = 40
    rec, _ = runner(np.zeros((n, n)), np.zeros((n, 1)), m0, np.zeros((samples, 1)), prm,
                    rhs=rhs, step=step)
    ratio0 = (m0[:, 0] + 1j * m0[:, 1]) / m0[:, 2]
    amp = rk4_amplification(1j * prm.h_appl * prm.dt)
    for s in (0, 7, samples - 1):
        steps = (s + 1) * prm.substeps
        r = amp ** steps * ratio0
        mz = np.sign(m0[:, 2]) / np.sqrt(1.0 + np.abs(r) ** 2)
        z = r * mz
        got = rec[s]
        assert np.max(np.abs(got[:, 2] - mz)) < 1e-13, (s, got[:, 2], mz)
        assert np.max(np.abs(got[:, 0] + 1j * got[:, 1] - z)) < 1e-13, s
    lengths = np.sqrt(np.sum(rec * rec, axis=2))
    assert np.max(np.abs(lengths - 1.0)) < 1e-15, np.max(np.abs(lengths - 1.0))
    plain, _ = runner(np.zeros((n, n)), np.zeros((n, 1)), m0, np.zeros((samples, 1)),
                      prm.replace(renormalize=False), rhs=rhs, step=step)
    assert np.max(np.abs(np.sqrt(np.sum(plain[-1] ** 2, axis=1)) - 1.0)) > 1e-9
    # the coupled, driven system: unit records, close to the unprojected run
    w, w_in, m0c, u = _coupled_case(n=6, seed=22)
    prm = _prm(a_cp=0.3, alpha=0.02, dt=0.01, substeps=20, renormalize=True)
    rec, _ = runner(w, w_in, m0c, u, prm, rhs=rhs, step=step)
    plain, _ = runner(w, w_in, m0c, u, prm.replace(renormalize=False), rhs=rhs, step=step)
    assert np.max(np.abs(np.sqrt(np.sum(rec * rec, axis=2)) - 1.0)) < 1e-15
    d = np.max(np.abs(rec - plain))
    assert 0.0 < d < 1e-5, d


# --------------------------------------------------------------------------
# Largest Lyapunov exponent: fixed points with known linearisation
# --------------------------------------------------------------------------
def pin_lyapunov(rhs=sto.field, step=None, lyap=sto.lyapunov_max, **_):
    """Benettin's estimate on an uncoupled, undriven, current-free macrospin.

    At m = s e_z (s = +-1) the field is b = (h_appl + s h_k) e_z =: B e_z and
    the transverse part z = m_x + i m_y of a nearby state obeys, to first
    order, dz/dt = mu z with mu = B (i - s alpha)/(1 + alpha^2).  The RK4 map
    multiplies z by R(mu dt) per step, so the transverse exponent of the
    discrete map is log|R(mu dt)|/dt.  A perturbation along m itself changes
    only |m|, which Eq. (gov) conserves, and m stays a fixed point: that
    direction has exponent 0.  Hence

    * at -e_z with h_appl > h_k the largest exponent is log|R(mu dt)|/dt > 0;
    * at +e_z it is 0 (the transverse mode decays, at the relaxation rate).

    The initial direction of the twin is random, so the accumulated log
    growth has a transient; it cancels in the increment between two
    horizons run from the same seed, which must equal the exponent.  dt and
    substeps differ from 0.01 and 20 so that a wrong time normalisation
    shows.
    """
    base = _prm(alpha=0.1, h_s=0.0, a_cp=0.0, a_in=0.0, dt=0.02, substeps=7)
    t1, t2 = 150, 400
    zero = np.zeros((1, 1))
    for sgn, h_k, tol in ((-1.0, 0.0, 1e-7), (-1.0, 1.5, 3e-6), (1.0, base.h_k, 2e-5)):
        prm = base.replace(h_k=h_k)
        m0 = np.array([[0.0, 0.0, sgn]])
        l1 = lyap(zero, zero, m0, np.zeros((t1, 1)), prm, rhs=rhs, step=step)
        l2 = lyap(zero, zero, m0, np.zeros((t2, 1)), prm, rhs=rhs, step=step)
        span = prm.substeps * prm.dt
        inc = (l2 * t2 * span - l1 * t1 * span) / ((t2 - t1) * span)
        big_b = prm.h_appl + prm.h_k * sgn
        mu = big_b * (1j - sgn * prm.alpha) / (1.0 + prm.alpha ** 2)
        ex = max(0.0, math.log(abs(rk4_amplification(mu * prm.dt))) / prm.dt)
        assert abs(inc - ex) < tol, (sgn, h_k, inc, ex)
    # two uncoupled spins: the unstable one sets the exponent of the pair
    prm = base.replace(h_k=0.0)
    m0 = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    z2 = np.zeros((2, 2))
    l1 = lyap(z2, np.zeros((2, 1)), m0, np.zeros((t1, 1)), prm, rhs=rhs, step=step)
    l2 = lyap(z2, np.zeros((2, 1)), m0, np.zeros((t2, 1)), prm, rhs=rhs, step=step)
    inc = (l2 * t2 - l1 * t1) / (t2 - t1)
    mu = prm.h_appl * (1j + prm.alpha) / (1.0 + prm.alpha ** 2)
    ex = math.log(abs(rk4_amplification(mu * prm.dt))) / prm.dt
    assert abs(inc - ex) < 1e-7, (inc, ex)


ALL_PINS = [
    pin_field_at_ez,
    pin_coupling_brute_force,
    pin_gilbert_form,
    pin_precession_map,
    pin_precession_tilted_field,
    pin_damping_closed_form,
    pin_relaxation,
    pin_energy,
    pin_global_order,
    pin_structure,
    pin_units,
    pin_continuation,
    pin_renormalize,
    pin_lyapunov,
]
