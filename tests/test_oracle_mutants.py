"""Planted mistakes in the oracle must each fail at least one pin (no GPU).

Every mutant below is a copy of the oracle's right-hand side, RK4 step or
driver with one plausible mistake: a flipped sign, a dropped term or factor,
a wrong index or a transposed operand, a wrong stage or weight, an
off-by-one in the records.  The pins in ``pins.py`` must reject every one,
which shows that they constrain each part of the oracle.
"""

import numpy as np
import pytest

import pins
from oracle import sto

FIELD_MUTANTS = [
    "stt_sign", "no_lambda", "lambda_sign", "damping_sign", "no_llg_factor",
    "coupling_self", "coupling_transposed", "coupling_into_y", "no_hk",
    "input_sign", "mmb_order", "no_acp", "mp_component", "bz_no_stt",
    "half_precession", "hk_sign", "input_into_z",
]
STEP_MUTANTS = ["rk4_weight", "rk4_stage3_input", "rk4_stage4_half", "rk4_dt3", "euler",
                "renorm_xy_only", "renorm_squared", "renorm_input", "renorm_skipped"]
RUN_MUTANTS = ["record_before", "input_lag"]


def field_variant(mut):
    def rhs(m, w, h_in, prm, dot="exact"):
        mx, my, mz = m
        px, py, pz = prm.p
        a_cp = 1.0 if mut == "no_acp" else prm.a_cp
        if mut == "coupling_self":
            c = a_cp * (w.sum(axis=1) * mx)
        elif mut == "coupling_transposed":
            c = a_cp * sto.matvec(np.ascontiguousarray(w.T), mx, dot)
        else:
            c = a_cp * sto.matvec(w, mx, dot)
        cy = cz = 0.0
        if prm.coupling == "xyz":
            cy = a_cp * sto.matvec(w, my, dot)
            cz = a_cp * sto.matvec(w, mz, dot)
        if mut == "mp_component":
            mp = (mx * px + my * py) + my * pz
        else:
            mp = (mx * px + my * py) + mz * pz
        if mut == "no_lambda":
            hs = prm.h_s / 1.0 + 0.0 * mp
        elif mut == "lambda_sign":
            hs = prm.h_s / (1.0 - prm.lam * mp)
        else:
            hs = prm.h_s / (1.0 + prm.lam * mp)
        q = sto.cross((px, py, pz), m)
        if mut == "stt_sign":
            q = sto.cross(m, (px, py, pz))
        qx, qy, qz = q
        if mut == "no_hk":
            hz = prm.h_appl + 0.0 * mz
        elif mut == "hk_sign":
            hz = prm.h_appl - prm.h_k * mz
        else:
            hz = prm.h_appl + prm.h_k * mz
        hin = -h_in if mut == "input_sign" else h_in
        if mut == "coupling_into_y":
            bx, by = hin + hs * qx, c + cy + hs * qy
        elif mut == "input_into_z":
            bx, by = c + hs * qx, cy + hs * qy
        else:
            bx, by = (c + hin) + hs * qx, cy + hs * qy
        bz = (hz + cz) + (0.0 if mut == "bz_no_stt" else hs * qz)
        if mut == "input_into_z":
            bz = bz + hin
        mb = sto.cross(m, (bx, by, bz))
        mmb = sto.cross(mb, m) if mut == "mmb_order" else sto.cross(m, mb)
        d = 1.0 + prm.alpha * prm.alpha
        c1 = prm.g / d
        c2 = prm.alpha * prm.g / d
        if mut == "no_llg_factor":
            c1, c2 = prm.g, prm.alpha * prm.g
        if mut == "half_precession":
            c1 = 0.5 * c1
        sgn = 1.0 if mut == "damping_sign" else -1.0
        return tuple((-c1) * mb[j] + sgn * c2 * mmb[j] for j in range(3))
    return rhs


def step_variant(mut):
    def project(v):
        nrm = np.sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])
        if mut == "renorm_squared":
            nrm = nrm * nrm
        if mut == "renorm_xy_only":
            return (v[0] / nrm, v[1] / nrm, v[2])
        return tuple(v[j] / nrm for j in range(3))

    def step(m, w, h_in, prm, dot="exact", rhs=sto.field):
        dt = prm.dt
        if prm.renormalize and mut == "renorm_input":
            m = project(m)
        k1 = rhs(m, w, h_in, prm, dot)
        if mut == "euler":
            return sto.axpy(m, dt, k1)
        k2 = rhs(sto.axpy(m, dt / 2.0, k1), w, h_in, prm, dot)
        k3 = rhs(sto.axpy(m, dt / 2.0, k1 if mut == "rk4_stage3_input" else k2),
                 w, h_in, prm, dot)
        k4 = rhs(sto.axpy(m, dt / 2.0 if mut == "rk4_stage4_half" else dt, k3),
                 w, h_in, prm, dot)
        c2 = 1.0 if mut == "rk4_weight" else 2.0
        h6 = dt / 3.0 if mut == "rk4_dt3" else dt / 6.0
        out = tuple(m[j] + h6 * (k1[j] + c2 * k2[j] + 2.0 * k3[j] + k4[j]) for j in range(3))
        if prm.renormalize and mut not in ("renorm_input", "renorm_skipped"):
            out = project(out)
        return out
    return step


def lyapunov_variant(mut):
    """Copies of Benettin's twin-trajectory estimate with one mistake."""
    import math

    def lyap(w, w_in, m0, u, prm, d0=1e-10, seed=1, dot="blas", rhs=sto.field, step=None):
        rng = np.random.default_rng(seed)
        n = w.shape[0]
        u = np.asarray(u, dtype=np.float64).reshape(len(u), -1)
        a = sto.to_soa(m0)
        d = rng.standard_normal((n, 3))
        d *= d0 / np.linalg.norm(d)
        b = sto.to_soa(np.asarray(m0) + d)
        total = 0.0
        for s in range(len(u)):
            h_in = sto.input_field(w_in, u[s], prm, dot)
            for _ in range(prm.substeps):
                a = sto.rk4_step(a, w, h_in, prm, dot)
                b = sto.rk4_step(b, w, h_in, prm, dot)
            diff = np.stack([b[j] - a[j] for j in range(3)], axis=1)
            if mut == "x_only":
                dist = float(np.linalg.norm(diff[:, 0]))
            else:
                dist = float(np.linalg.norm(diff))
            growth = math.log10(dist / d0) if mut == "log10" else math.log(dist / d0)
            total += -growth if mut == "log_sign" else growth
            if mut != "no_rescale":
                b = sto.to_soa(sto.to_aos(a) + diff * (d0 / dist))
        if mut == "per_sample":
            return total / len(u)
        if mut == "per_step":
            return total / (len(u) * prm.substeps)
        return total / (len(u) * prm.substeps * prm.dt)
    return lyap


LYAP_MUTANTS = ["no_rescale", "per_sample", "per_step", "log10", "log_sign", "x_only"]


def runner_variant(mut):
    def runner(w, w_in, m0, u, prm, rhs=sto.field, step=None, dot="exact"):
        u = np.asarray(u, dtype=np.float64).reshape(len(u), -1)
        m = sto.to_soa(m0)
        rec = np.empty((len(u), w.shape[0], 3))
        for s in range(len(u)):
            us = u[s - 1] if (mut == "input_lag" and s > 0) else u[s]
            h_in = sto.input_field(np.asarray(w_in).reshape(w.shape[0], -1), us, prm, dot)
            before = sto.to_aos(m)
            for _ in range(prm.substeps):
                m = sto.rk4_step(m, w, h_in, prm, dot)
            rec[s] = before if mut == "record_before" else sto.to_aos(m)
        return rec, sto.to_aos(m)
    return runner


# cheapest pins first: each mutant stops at the first pin that rejects it
_ORDER = sorted(pins.ALL_PINS, key=lambda f: [
    "pin_field_at_ez", "pin_coupling_brute_force", "pin_gilbert_form",
    "pin_precession_tilted_field", "pin_damping_closed_form", "pin_global_order",
    "pin_units", "pin_structure", "pin_continuation", "pin_energy",
    "pin_precession_map", "pin_relaxation", "pin_renormalize",
    "pin_lyapunov"].index(f.__name__))


def _caught(**kw):
    for pin in _ORDER:
        try:
            with np.errstate(all="ignore"):
                pin(**kw)
        except (AssertionError, FloatingPointError, ValueError, np.linalg.LinAlgError):
            return pin.__name__
    return None


def test_unmutated_oracle_passes_every_pin():
    assert _caught() is None


@pytest.mark.parametrize("mut", FIELD_MUTANTS)
def test_field_mutant_is_caught(mut):
    assert _caught(rhs=field_variant(mut)) is not None, mut


def test_field_variant_without_mutation_is_the_oracle():
    """The mutant template itself (no mistake planted) reproduces the oracle
    bitwise, so every failure above comes from the planted mistake."""
    assert _caught(rhs=field_variant("none")) is None


@pytest.mark.parametrize("mut", STEP_MUTANTS)
def test_step_mutant_is_caught(mut):
    assert _caught(step=step_variant(mut)) is not None, mut


@pytest.mark.parametrize("mut", RUN_MUTANTS)
def test_runner_mutant_is_caught(mut):
    assert _caught(runner=runner_variant(mut)) is not None, mut


def test_step_variant_without_mutation_is_the_oracle():
    """The RK4 template with no mistake planted passes every pin, with and
    without renormalisation."""
    assert _caught(step=step_variant("none")) is None


@pytest.mark.parametrize("mut", LYAP_MUTANTS)
def test_lyapunov_mutant_is_caught(mut):
    # only the Lyapunov pin calls the estimate, so it is the one to run
    with np.errstate(all="ignore"), pytest.raises((AssertionError, FloatingPointError, ValueError)):
        pins.pin_lyapunov(lyap=lyapunov_variant(mut))


def test_lyapunov_variant_without_mutation_is_the_oracle():
    pins.pin_lyapunov(lyap=lyapunov_variant("none"))
