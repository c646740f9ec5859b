"""Pins for the oracle's discrete adjoint and readout gradient (no GPU).

None of these re-types the adjoint.  Each derivative is obtained a second,
independent way:

* central finite differences (h = 1e-6) of the forward oracle in FP64;
* complex-step differentiation of the forward oracle: the forward RK4 map
  is evaluated with one input moved by i*h (h = 1e-20), and Im L / h is the
  exact directional derivative up to rounding (no cancellation, unlike
  finite differences).  The forward oracle is itself pinned in ``pins.py``;
* a closed form for pure precession (alpha = 0, no current, no coupling,
  no input): z = m_x + i m_y follows z_n = R(i w dt)^n z_0 exactly, with
  R the RK4 amplification polynomial and w = h_appl + h_k m_z, so the
  derivatives with respect to h_appl and to the initial state are
  polynomials in R;
* the ridge objective at its optimum, differentiated by complex step
  through a plain linear solve of the normal equations.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from oracle import adjoint, constants, readout, sto

H_CS = 1e-20
SCALARS = ("a_cp", "a_in", "h_s", "h_appl")


def adjoint_case(coupling="x", renormalize=False, n=5, samples=3, substeps=4, n_in=1, seed=3):
    """A small coupled, driven, asymmetric case with every constant away from 1."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n)) / np.sqrt(n)
    np.fill_diagonal(w, 0.0)
    w_in = rng.uniform(-1, 1, (n, n_in))
    v = rng.standard_normal((n, 3)) * 0.3
    v[:, 2] += 1.0
    m0 = v / np.linalg.norm(v, axis=1, keepdims=True)
    u = rng.uniform(-1, 1, (samples, n_in))
    prm = constants.dimensionless(a_cp=0.3, a_in=0.7, dt=0.01, substeps=substeps,
                                  renormalize=renormalize, coupling=coupling)
    g_rec = rng.standard_normal((samples, n, 3))
    g_fin = rng.standard_normal((n, 3))
    return w, w_in, m0, u, prm, g_rec, g_fin


def complex_loss(w, w_in, m0, u, prm, g_rec, g_fin):
    """L = sum_n <G_n, record n> + <G_final, final> by the forward oracle, in
    complex arithmetic (every input may carry an imaginary perturbation)."""
    m = tuple(np.asarray(m0[:, c], dtype=complex) for c in range(3))
    total = 0.0
    for s in range(len(u)):
        h_in = prm.a_in * (w_in @ u[s])
        for _ in range(prm.substeps):
            m = sto.rk4_step(m, w, h_in, prm, "blas")
        total = total + sum(np.sum(g_rec[s][:, c] * m[c]) for c in range(3))
    return total + sum(np.sum(g_fin[:, c] * m[c]) for c in range(3))


def complex_step_derivatives(w, w_in, m0, u, prm, g_rec, g_fin, seed=7):
    """Directional derivatives of L by complex step: the four scalars, and W,
    w_in, m0 along random directions (returned with the directions)."""
    rng = np.random.default_rng(seed)
    out = {}
    for name in SCALARS:
        p2 = dataclasses.replace(prm, **{name: getattr(prm, name) + 1j * H_CS})
        out[name] = complex_loss(w, w_in, m0, u, p2, g_rec, g_fin).imag / H_CS
    d_w = rng.standard_normal(w.shape)
    d_win = rng.standard_normal(w_in.shape)
    d_m0 = rng.standard_normal(m0.shape)
    out["W"] = (complex_loss(w + 1j * H_CS * d_w, w_in, m0, u, prm, g_rec, g_fin).imag / H_CS, d_w)
    out["w_in"] = (complex_loss(w, w_in + 1j * H_CS * d_win, m0, u, prm, g_rec, g_fin).imag / H_CS, d_win)
    out["m0"] = (complex_loss(w, w_in, m0 + 1j * H_CS * d_m0, u, prm, g_rec, g_fin).imag / H_CS, d_m0)
    return out


def pin_adjoint_complex_step(vjp=None, reverse=None, tol=1e-10, **_):
    """Every gradient of the adjoint equals the complex-step derivative of the
    forward oracle, for both couplings, with and without renormalisation."""
    for coupling in ("x", "xyz"):
        for renorm in (False, True):
            w, w_in, m0, u, prm, g_rec, g_fin = adjoint_case(coupling, renorm)
            got = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, g_fin, dot="blas", vjp=vjp, reverse=reverse)
            ref = complex_step_derivatives(w, w_in, m0, u, prm, g_rec, g_fin)
            for name in SCALARS:
                assert abs(got[name] - ref[name]) <= tol * max(1.0, abs(ref[name])), \
                    (coupling, renorm, name, got[name], ref[name])
            for name in ("W", "w_in", "m0"):
                val, d = ref[name]
                mine = float(np.sum(np.asarray(got[name]) * d))
                assert abs(mine - val) <= tol * max(1.0, abs(val)), (coupling, renorm, name, mine, val)


def rk4_amplification(x):
    return 1 + x + x * x / 2 + x ** 3 / 6 + x ** 4 / 24


def rk4_amplification_prime(x):
    return 1 + x + x * x / 2 + x ** 3 / 6


def pin_adjoint_precession(vjp=None, reverse=None, **_):
    """alpha = 0, h_s = 0, W = 0, u = 0: closed-form derivatives of a linear
    loss on the final record with respect to h_appl and the initial state."""
    rng = np.random.default_rng(11)
    n, samples, sub = 6, 3, 7
    prm = constants.dimensionless(a_cp=0.3, a_in=0.7, dt=0.01, substeps=sub).replace(alpha=0.0, h_s=0.0)
    w = np.zeros((n, n))
    w_in = rng.uniform(-1, 1, (n, 1))
    u = np.zeros((samples, 1))
    v = rng.standard_normal((n, 3)) * 0.4
    v[:, 2] += 1.0
    m0 = v / np.linalg.norm(v, axis=1, keepdims=True)
    g_rec = np.zeros((samples, n, 3))
    g_rec[-1] = rng.standard_normal((n, 3))
    got = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, None, dot="blas", vjp=vjp, reverse=reverse)

    steps = samples * sub
    om = prm.h_appl + prm.h_k * m0[:, 2]
    x = 1j * om * prm.dt
    r = rk4_amplification(x)
    z0 = m0[:, 0] + 1j * m0[:, 1]
    dz_dom = steps * r ** (steps - 1) * rk4_amplification_prime(x) * (1j * prm.dt) * z0
    gam = g_rec[-1][:, 0] + 1j * g_rec[-1][:, 1]
    d_happl = float(np.sum(np.real(np.conj(gam) * dz_dom)))
    d_m0 = np.stack([np.real(np.conj(gam) * r ** steps),
                     np.real(np.conj(gam) * 1j * r ** steps),
                     g_rec[-1][:, 2] + np.real(np.conj(gam) * dz_dom) * prm.h_k], axis=1)
    assert abs(got["h_appl"] - d_happl) <= 1e-12 * max(1.0, abs(d_happl)), (got["h_appl"], d_happl)
    assert np.max(np.abs(got["m0"] - d_m0)) <= 1e-12 * max(1.0, np.max(np.abs(d_m0))), \
        np.max(np.abs(got["m0"] - d_m0))
    # no coupling field and no input: their scalar derivatives vanish exactly
    assert got["a_cp"] == 0.0 and got["a_in"] == 0.0


def ridge_objective_plain(records, y, washout, lam, components="x"):
    """The ridge objective at its optimum through a plain solve of the normal
    equations (valid in complex arithmetic: no conjugates are taken)."""
    t, n, _ = records.shape
    rows = records[washout:]
    f = rows[:, :, 0] if components == "x" else rows.reshape(t - washout, 3 * n)
    phi = np.concatenate([f, np.ones((t - washout, 1))], axis=1)
    yy = y[washout:]
    w = np.linalg.solve(phi.T @ phi + lam * np.eye(phi.shape[1]), phi.T @ yy)
    r = phi @ w - yy
    return (r @ r + lam * (w @ w)) / (t - washout)


def pin_ridge_envelope(**_):
    """The readout gradient equals the complex-step derivative of the ridge
    objective, for both feature sets and both solve forms."""
    rng = np.random.default_rng(5)
    for comps, t, n in (("x", 40, 6), ("xyz", 40, 5), ("x", 12, 20)):
        rec = rng.standard_normal((t, n, 3))
        y = rng.standard_normal(t)
        washout, lam = 6, 1e-3
        j, _, grad = readout.ridge_objective_grad(rec, y, washout, lam, comps)
        assert abs(j - ridge_objective_plain(rec, y, washout, lam, comps)) <= 1e-12 * max(1.0, j)
        d = rng.standard_normal(rec.shape)
        cs = ridge_objective_plain(rec + 1j * H_CS * d, y, washout, lam, comps).imag / H_CS
        mine = float(np.sum(grad * d))
        assert abs(mine - cs) <= 1e-9 * max(1.0, abs(cs)), (comps, mine, cs)


def pin_adjoint_central_fd(vjp=None, reverse=None, **_):
    """Central finite differences (h = 1e-6) of the forward oracle in FP64
    agree with the adjoint to 1e-7 relative (truncation ~h^2, rounding
    ~1e-16/h), for the four scalars and a random direction of W."""
    w, w_in, m0, u, prm, g_rec, g_fin = adjoint_case("xyz", True)
    got = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, g_fin, dot="blas", vjp=vjp, reverse=reverse)

    def loss(p, ww):
        rec, fin = sto.run(ww, w_in, m0, u, p, dot="blas")
        return float(np.sum(rec * g_rec) + np.sum(fin * g_fin))

    h = 1e-6
    for name in SCALARS:
        v = getattr(prm, name)
        fd = (loss(prm.replace(**{name: v + h}), w) - loss(prm.replace(**{name: v - h}), w)) / (2 * h)
        assert abs(fd - got[name]) <= 1e-7 * max(1.0, abs(fd)), (name, fd, got[name])
    d_w = np.random.default_rng(9).standard_normal(w.shape)
    fd = (loss(prm, w + h * d_w) - loss(prm, w - h * d_w)) / (2 * h)
    mine = float(np.sum(got["W"] * d_w))
    assert abs(fd - mine) <= 1e-7 * max(1.0, abs(fd)), (fd, mine)


ADJOINT_PINS = [pin_adjoint_complex_step, pin_adjoint_precession, pin_adjoint_central_fd]
ALL = ADJOINT_PINS + [pin_ridge_envelope]
