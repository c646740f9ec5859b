"""Discrete adjoint of the RK4 trajectory (plain FP64 reverse mode).

Oracle (test infrastructure): this module is the reference the HIP adjoint
is checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may use it.

What it computes.  The forward map is the oracle's own trajectory: classic
RK4 on Eq. (gov) with the coupling of Eq. (coup) and the input field of
Eq. (in), one record after the last step of every input sample (paper,
Sec. 3.1 and 3.2; ``sto.run``).  A loss L is given through its gradient
with respect to the records, G[n] = dL/d(record n), and optionally with
respect to the final state.  Reverse-mode differentiation of every step,
stage by stage in the opposite order of the forward, gives the exact
derivative of the discrete map (not of the continuous ODE):

* dL/dW      = a_cp * sum over all stages of outer(bbar_x, x^x)
               (x-only coupling; with the isotropic variant the sum also
               runs over the y and z components);
* dL/dw_in   = a_in * sum over all stages of outer(bbar_x, u_n);
* dL/dm0     = the adjoint state after the first step has been reversed;
* dL/da_cp   = sum over all stages of bbar . (W x);
* dL/da_in   = sum over all stages of bbar_x (w_in u_n);
* dL/dh_s    = sum over all stages of (bbar . (p x m)) / (1 + lambda m.p);
* dL/dh_appl = sum over all stages of bbar_z;

where x is a stage input, u_n the input sample the stage sees, and bbar the
adjoint of the effective field b of Eq. (gov) at that stage.  The paper has
no adjoint: this is the chain rule applied to its integrator, written out
below with the same names as ``sto.field``.

Reverse step.  A forward step from m takes stage inputs x1 = m,
x2 = m + (dt/2) k1, x3 = m + (dt/2) k2, x4 = m + dt k3, with k_i = F(x_i),
and returns m' = m + (dt/6)(k1 + 2 k2 + 2 k3 + k4), optionally divided by
its norm.  Given a = dL/dm' (after the projection has been reversed):
kbar4 = (dt/6) a; xbar4 = dF(x4)^T kbar4;
kbar3 = (dt/3) a + dt xbar4; xbar3 = dF(x3)^T kbar3;
kbar2 = (dt/3) a + (dt/2) xbar3; xbar2 = dF(x2)^T kbar2;
kbar1 = (dt/6) a + (dt/2) xbar2; xbar1 = dF(x1)^T kbar1;
dL/dm = a + xbar1 + xbar2 + xbar3 + xbar4.
dF(x)^T v has a pointwise part (the derivative of F through x_k with the
coupling held fixed) and the coupling part a_cp W^T bbar_x along e_x.
"""

from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from . import sto
from .constants import Params


def _dot3(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def field_vjp(m, c, h_in, v, prm: Params):
    """Reverse-mode derivative of the pointwise right-hand side of Eq. (gov).

    F(m) = -c1 m x b - c2 m x (m x b), with c1 = g/(1+alpha^2),
    c2 = alpha g/(1+alpha^2) and
    b = (c_x + h_in + hs q_x, c_y + hs q_y, h_appl + h_k m_z + c_z + hs q_z),
    q = p x m, hs = h_s / (1 + lambda m.p).

    Arguments: m the stage input (3 arrays), c the coupling field a_cp W m
    (3 arrays; y and z zero for the x-only coupling), h_in the input field,
    v the adjoint of F.  Returns (mbar, bbar, hs_partial):
    mbar = v^T dF/dm with c held fixed, bbar = v^T dF/db, and
    hs_partial = v^T dF/dh_s.
    """
    mx, my, mz = m
    px, py, pz = prm.p
    cx, cy, cz = c
    mp = (mx * px + my * py) + mz * pz
    den = 1.0 + prm.lam * mp
    hs = prm.h_s / den
    q = sto.cross((px, py, pz), m)
    b = ((cx + h_in) + hs * q[0], cy + hs * q[1], (prm.h_appl + prm.h_k * mz + cz) + hs * q[2])
    mb = sto.cross(m, b)
    d = 1.0 + prm.alpha * prm.alpha
    c1 = prm.g / d
    c2 = prm.alpha * prm.g / d
    # F = -c1 mb - c2 (m x mb):  v.(m x dmb) = dmb.(v x m),  v.(dm x mb) = dm.(mb x v)
    vm = sto.cross(v, m)
    mbbar = tuple(-c1 * v[j] - c2 * vm[j] for j in range(3))
    t1 = sto.cross(mb, v)
    # mb = m x b:  mbbar.(dm x b) = dm.(b x mbbar),  mbbar.(m x db) = db.(mbbar x m)
    t2 = sto.cross(b, mbbar)
    bbar = sto.cross(mbbar, m)
    mbar = [-c2 * t1[j] + t2[j] for j in range(3)]
    # b through m: h_k m_z, hs q with q = p x m, and hs(m.p)
    mbar[2] = mbar[2] + prm.h_k * bbar[2]
    qbar_p = sto.cross(bbar, (px, py, pz))          # (hs bbar) x p, hs applied below
    hsbar = _dot3(bbar, q)
    dhs_dmp = -prm.lam * hs / den
    p = (px, py, pz)
    for j in range(3):
        mbar[j] = mbar[j] + hs * qbar_p[j] + hsbar * dhs_dmp * p[j]
    return tuple(mbar), bbar, hsbar / den


def rk4_stages(m, w, h_in, prm: Params, dot: str):
    """One forward RK4 step (the arithmetic of ``sto.rk4_step``) that also
    returns the four stage inputs and the state before the optional projection."""
    dt = prm.dt
    k1 = sto.field(m, w, h_in, prm, dot)
    x2 = sto.axpy(m, dt / 2.0, k1)
    k2 = sto.field(x2, w, h_in, prm, dot)
    x3 = sto.axpy(m, dt / 2.0, k2)
    k3 = sto.field(x3, w, h_in, prm, dot)
    x4 = sto.axpy(m, dt, k3)
    k4 = sto.field(x4, w, h_in, prm, dot)
    pre = tuple(m[j] + (dt / 6.0) * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]) for j in range(3))
    out = pre
    if prm.renormalize:
        nrm = np.sqrt((pre[0] * pre[0] + pre[1] * pre[1]) + pre[2] * pre[2])
        out = tuple(pre[j] / nrm for j in range(3))
    return (m, x2, x3, x4), pre, out


def reverse_step(stages, pre, out, abar, w, wt, u_s, raw_in, prm: Params, dot: str,
                 grads: Dict[str, object], vjp=None):
    """Reverse one forward step: from abar = dL/dm' return dL/dm, and add
    this step's contributions to ``grads`` ("W", "w_in", and the scalars)."""
    vjp = field_vjp if vjp is None else vjp
    dt = prm.dt
    weight = (dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0)   # weight of k_i in m'
    hstage = (0.0, dt / 2.0, dt / 2.0, dt)              # x_i = m + hstage[i] k_{i-1}
    comps = (0, 1, 2) if prm.coupling == "xyz" else (0,)
    zero = np.zeros_like(abar[0])
    a = tuple(abar)
    if prm.renormalize:
        nrm = np.sqrt((pre[0] * pre[0] + pre[1] * pre[1]) + pre[2] * pre[2])
        ao = _dot3(a, out)
        a = tuple((a[c] - ao * out[c]) / nrm for c in range(3))
    h_in = prm.a_in * raw_in
    mbar = list(a)
    xbar_next = None
    for i in (3, 2, 1, 0):
        v = tuple(weight[i] * a[c] + (hstage[i + 1] * xbar_next[c] if i < 3 else 0.0)
                  for c in range(3))
        x = stages[i]
        wx = [sto.matvec(w, x[c], dot) for c in comps]
        cfield = [prm.a_cp * wxc for wxc in wx] + [zero] * (3 - len(comps))
        mloc, bbar, hs_partial = vjp(x, tuple(cfield), h_in, v, prm)
        xbar = list(mloc)
        for k, c in enumerate(comps):
            xbar[c] = xbar[c] + prm.a_cp * (wt @ bbar[c])
            grads["W"] += prm.a_cp * np.outer(bbar[c], x[c])
            grads["a_cp"] += float(bbar[c] @ wx[k])
        grads["w_in"] += prm.a_in * np.outer(bbar[0], u_s)
        grads["a_in"] += float(bbar[0] @ raw_in)
        grads["h_s"] += float(np.sum(hs_partial))
        grads["h_appl"] += float(np.sum(bbar[2]))
        for c in range(3):
            mbar[c] = mbar[c] + xbar[c]
        xbar_next = xbar
    return mbar


def run_adjoint(w, w_in, m0, u, prm: Params, grad_records: Optional[np.ndarray] = None,
                grad_final: Optional[np.ndarray] = None, dot: str = "exact",
                vjp=None, reverse=None) -> Dict[str, object]:
    """Gradients of L with dL/d(records) = grad_records (samples, N, 3) and
    dL/d(final state) = grad_final (N, 3); either may be None (zero).

    Returns a dict with "W" (N, N), "w_in" (N, n_in), "m0" (N, 3), the
    scalars "a_cp", "a_in", "h_s", "h_appl", and "records" and "final", the
    forward trajectory (identical to ``sto.run``).
    """
    reverse = reverse_step if reverse is None else reverse
    w = np.ascontiguousarray(w, dtype=np.float64)
    w_in = np.ascontiguousarray(w_in, dtype=np.float64)
    if w_in.ndim == 1:
        w_in = w_in[:, None]
    u = np.asarray(u, dtype=np.float64).reshape(len(u), -1)
    n = w.shape[0]
    samples, sub = len(u), prm.substeps
    wt = np.ascontiguousarray(w.T)

    # forward, keeping every step's stage inputs and pre-projection state
    m = sto.to_soa(m0)
    trace = []
    records = np.empty((samples, n, 3))
    for s in range(samples):
        h_in = sto.input_field(w_in, u[s], prm, dot)
        for _ in range(sub):
            stages, pre, m = rk4_stages(m, w, h_in, prm, dot)
            trace.append((stages, pre, m))
        records[s] = sto.to_aos(m)
    final = sto.to_aos(m)

    grads = {"W": np.zeros((n, n)), "w_in": np.zeros_like(w_in),
             "a_cp": 0.0, "a_in": 0.0, "h_s": 0.0, "h_appl": 0.0}
    abar = [np.zeros(n) for _ in range(3)]              # dL/dm_{j+1}
    if grad_final is not None:
        abar = [abar[c] + grad_final[:, c] for c in range(3)]
    for j in reversed(range(samples * sub)):
        s = j // sub
        if (j + 1) % sub == 0 and grad_records is not None:
            abar = [abar[c] + grad_records[s][:, c] for c in range(3)]
        stages, pre, out = trace[j]
        raw_in = sto.matvec(w_in, u[s], dot)
        abar = reverse(stages, pre, out, abar, w, wt, u[s], raw_in, prm, dot, grads, vjp)
    res = dict(grads)
    res.update({"m0": sto.to_aos(tuple(abar)), "records": records, "final": final})
    return res


def linear_loss(records: np.ndarray, grad_records: np.ndarray, final: Optional[np.ndarray] = None,
                grad_final: Optional[np.ndarray] = None):
    """L = sum <G_n, record n> (+ <G_final, final>): the loss whose gradient
    with respect to the records is G; used to check the adjoint."""
    val = np.sum(records * grad_records)
    if grad_final is not None:
        val = val + np.sum(final * grad_final)
    return val
