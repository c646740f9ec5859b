"""Pins of the oracle's adjoint and readout gradient, and planted mistakes
in copies of the adjoint that the pins must reject (no GPU)."""

import numpy as np
import pytest

import pins_adjoint
from oracle import adjoint, sto


@pytest.mark.parametrize("pin", pins_adjoint.ALL, ids=lambda f: f.__name__)
def test_adjoint_pin(pin):
    pin()


VJP_MUTANTS = ["mbbar_sign", "t1_dropped", "bbar_order", "no_hk", "qbar_sign", "no_dhs",
               "hs_partial_den", "t2_order", "no_c1"]
REVERSE_MUTANTS = ["weight", "hstage", "coupling_untransposed", "no_direct", "renorm_skipped",
                   "acp_grad_scaled", "win_grad_unscaled", "stage_order"]


def vjp_variant(mut):
    """A copy of the pointwise adjoint with one planted mistake."""
    def vjp(m, c, h_in, v, prm):
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
        if mut == "no_c1":
            c1 = prm.g
        vm = sto.cross(v, m)
        sgn = 1.0 if mut == "mbbar_sign" else -1.0
        mbbar = tuple(-c1 * v[j] + sgn * c2 * vm[j] for j in range(3))
        t1 = sto.cross(mb, v)
        t2 = sto.cross(mbbar, b) if mut == "t2_order" else sto.cross(b, mbbar)
        bbar = sto.cross(m, mbbar) if mut == "bbar_order" else sto.cross(mbbar, m)
        mbar = [(0.0 if mut == "t1_dropped" else -c2 * t1[j]) + t2[j] for j in range(3)]
        if mut != "no_hk":
            mbar[2] = mbar[2] + prm.h_k * bbar[2]
        qbar_p = sto.cross(bbar, (px, py, pz))
        hsbar = (bbar[0] * q[0] + bbar[1] * q[1]) + bbar[2] * q[2]
        dhs_dmp = 0.0 if mut == "no_dhs" else -prm.lam * hs / den
        qs = -1.0 if mut == "qbar_sign" else 1.0
        p = (px, py, pz)
        for j in range(3):
            mbar[j] = mbar[j] + qs * hs * qbar_p[j] + hsbar * dhs_dmp * p[j]
        return tuple(mbar), bbar, (hsbar if mut == "hs_partial_den" else hsbar / den)
    return vjp


def reverse_variant(mut):
    """A copy of the reverse RK4 step with one planted mistake."""
    def reverse(stages, pre, out, abar, w, wt, u_s, raw_in, prm, dot, grads, vjp=None):
        vjp = adjoint.field_vjp
        dt = prm.dt
        weight = (dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0)
        if mut == "weight":
            weight = (dt / 6.0, dt / 6.0, dt / 3.0, dt / 3.0)
        hstage = (0.0, dt / 2.0, dt, dt / 2.0) if mut == "hstage" else (0.0, dt / 2.0, dt / 2.0, dt)
        comps = (0, 1, 2) if prm.coupling == "xyz" else (0,)
        zero = np.zeros_like(abar[0])
        a = tuple(abar)
        if prm.renormalize and mut != "renorm_skipped":
            nrm = np.sqrt((pre[0] * pre[0] + pre[1] * pre[1]) + pre[2] * pre[2])
            ao = (a[0] * out[0] + a[1] * out[1]) + a[2] * out[2]
            a = tuple((a[c] - ao * out[c]) / nrm for c in range(3))
        h_in = prm.a_in * raw_in
        mbar = [zero.copy() for _ in range(3)] if mut == "no_direct" else list(a)
        xbar_next = None
        order = (0, 1, 2, 3) if mut == "stage_order" else (3, 2, 1, 0)
        for idx, i in enumerate(order):
            nxt = order[idx - 1] if idx > 0 else None
            v = tuple(weight[i] * a[c] + (hstage[nxt] * xbar_next[c] if nxt is not None else 0.0)
                      for c in range(3))
            x = stages[i]
            wx = [sto.matvec(w, x[c], dot) for c in comps]
            cfield = [prm.a_cp * wxc for wxc in wx] + [zero] * (3 - len(comps))
            mloc, bbar, hs_partial = vjp(x, tuple(cfield), h_in, v, prm)
            xbar = list(mloc)
            for k, c in enumerate(comps):
                mat = w if mut == "coupling_untransposed" else wt
                xbar[c] = xbar[c] + prm.a_cp * (mat @ bbar[c])
                grads["W"] += prm.a_cp * np.outer(bbar[c], x[c])
                scale = prm.a_cp if mut == "acp_grad_scaled" else 1.0
                grads["a_cp"] += float(bbar[c] @ wx[k]) * scale
            grads["w_in"] += (1.0 if mut == "win_grad_unscaled" else prm.a_in) * np.outer(bbar[0], u_s)
            grads["a_in"] += float(bbar[0] @ raw_in)
            grads["h_s"] += float(np.sum(hs_partial))
            grads["h_appl"] += float(np.sum(bbar[2]))
            for c in range(3):
                mbar[c] = mbar[c] + xbar[c]
            xbar_next = xbar
        return mbar
    return reverse


def _rejected(**kw):
    for pin in pins_adjoint.ADJOINT_PINS:
        try:
            pin(**kw)
        except AssertionError:
            return True
    return False


@pytest.mark.parametrize("mut", VJP_MUTANTS)
def test_vjp_mutant_rejected(mut):
    assert _rejected(vjp=vjp_variant(mut)), f"no pin rejects the pointwise-adjoint mutant {mut}"


@pytest.mark.parametrize("mut", REVERSE_MUTANTS)
def test_reverse_mutant_rejected(mut):
    assert _rejected(reverse=reverse_variant(mut)), f"no pin rejects the reverse-step mutant {mut}"


def test_unmutated_copies_pass():
    """The copies above, without a mistake, pass every pin (so a rejection
    is caused by the planted mistake alone)."""
    assert not _rejected(vjp=vjp_variant("none"))
    assert not _rejected(reverse=reverse_variant("none"))


def test_adjoint_forward_is_the_oracle_trajectory():
    w, w_in, m0, u, prm, g_rec, g_fin = pins_adjoint.adjoint_case()
    rec, fin = sto.run(w, w_in, m0, u, prm)
    got = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, g_fin)
    assert np.array_equal(got["records"], rec) and np.array_equal(got["final"], fin)
