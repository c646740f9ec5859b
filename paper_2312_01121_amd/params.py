"""Dimensionless constants for the library's ``sto_params``.

Table 1 of the paper lists the constants of Eq. (gov) in CGS units.  The
library works in the unit t0 = 1 ns for time and 1/(gamma t0) for fields,
so a field H in Oe becomes h = gamma * t0 * H and the paper's step of
1e-11 s becomes dt = 0.01.  The spin-torque amplitude is
hbar * eta * I / (2 e M V) in Oe (hbar in erg s, V in cm^3).
"""

from __future__ import annotations

import math

# Table 1 (gamma in rad/(Oe s), M in emu/cm^3, fields in Oe, I in A,
# V = pi * 60^2 * 2 nm^3, e in C, hbar in J s)
GAMMA = 1.764e7
ALPHA = 0.005
M_S = 1448.3
H_K = 18616.0
H_APPL = 200.0
ETA = 0.537
LAMBDA = 0.288
I_CURRENT = 2.5e-3
VOLUME_NM3 = math.pi * 60.0 ** 2 * 2.0
E_CHARGE = 1.60217733e-19
HBAR_JS = 1.05457266e-34
T_UNIT = 1e-9


def field_unit() -> float:
    """gamma * t0: multiplies a field in Oe to give the dimensionless field."""
    return GAMMA * T_UNIT


def spin_torque_oe(current: float = I_CURRENT) -> float:
    hbar_cgs = HBAR_JS * 1e7
    volume_cm3 = VOLUME_NM3 * 1e-21
    return hbar_cgs * ETA * current / (2.0 * E_CHARGE * M_S * volume_cm3)


def table1(a_cp: float = 0.1, a_in: float = 1.0, dt: float = 0.01, substeps: int = 20,
           current_scale: float = 1.0, field_scale: float = 1.0) -> dict:
    """Keyword arguments for ``sto_params`` at the paper's Table 1 values.

    a_cp, a_in: coupling and input amplitudes in the dimensionless unit.
    current_scale, field_scale: multipliers of I and H_appl.
    """
    g = field_unit()
    return dict(
        alpha=ALPHA,
        h_appl=g * (H_APPL * field_scale),
        h_k=g * (H_K - 4.0 * math.pi * M_S),
        h_s=g * spin_torque_oe(I_CURRENT * current_scale),
        lambda_stt=LAMBDA,
        p=(math.sin(math.pi / 2.0), 0.0, math.cos(math.pi / 2.0)),
        a_cp=a_cp,
        a_in=a_in,
        dt=dt,
        substeps=substeps,
    )
