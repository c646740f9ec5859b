"""Physical constants of the oracle and their dimensionless form.

Table 1 of the paper lists the constants in CGS-Gaussian units with the
current in amperes and the volume in nm^3.  The oracle works in a
dimensionless form of Eq. (gov): time in units of t0 = 1 ns and fields in
units of 1 / (gamma * t0) = 56.689 Oe, so that every field h = gamma * t0 * H
and the equation reads

    dm/dtau = -1/(1+alpha^2) m x b - alpha/(1+alpha^2) m x (m x b).

With that unit the paper's step of 1e-11 s is dt = 0.01.  The oracle keeps
the physical-unit constants too, so a test can integrate Eq. (gov) with
gamma explicit and compare.

This module belongs to the oracle (test infrastructure); the HIP library
derives its own constants independently.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Tuple

# Table 1, converted to CGS where needed.
GAMMA = 1.764e7                  # rad / (Oe s)
ALPHA = 0.005
M_SAT = 1448.3                   # emu / cm^3
H_K = 18.616e3                   # Oe
H_APPL = 200.0                   # Oe
ETA = 0.537
LAMBDA_STT = 0.288
CURRENT = 2.5e-3                 # A
VOLUME = math.pi * 60.0 ** 2 * 2.0 * 1e-21   # nm^3 -> cm^3
E_CHARGE = 1.60217733e-19        # C
HBAR = 1.05457266e-34 * 1e7      # J s -> erg s
P_VEC = (math.sin(math.pi / 2.0), 0.0, math.cos(math.pi / 2.0))  # (1, 0, 6.1e-17)
A_CP_OE = 1.0                    # Oe
A_IN_OE = 1.0                    # Oe

T0 = 1e-9                        # s, the time unit of the dimensionless form


def spin_torque_field_oe(current: float = CURRENT) -> float:
    """hbar eta I / (2 e M V) in Oe: the numerator of H_s in Eq. (gov)."""
    return HBAR * ETA * current / (2.0 * E_CHARGE * M_SAT * VOLUME)


def demag_oe() -> float:
    """4 pi M in Oe."""
    return 4.0 * math.pi * M_SAT


@dataclasses.dataclass(frozen=True)
class Params:
    """Constants of Eq. (gov) in one consistent unit system.

    ``g`` is the prefactor that turns a field into an angular rate: gamma in
    physical units, 1 in the dimensionless form.  ``coupling`` is "x" for the
    paper's Eq. (coup) (only m^x couples, into e_x) or "xyz" for the
    isotropic variant in which all three components couple.
    """

    alpha: float
    h_appl: float
    h_k: float          # H_K - 4 pi M, times g t0 in the dimensionless form
    h_s: float          # hbar eta I / (2 e M V)
    lam: float
    p: Tuple[float, float, float]
    a_cp: float
    a_in: float
    dt: float
    substeps: int = 20
    g: float = 1.0
    renormalize: bool = False
    coupling: str = "x"

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


def dimensionless(a_cp: float = 0.1, a_in: float = 1.0, dt: float = 0.01,
                  substeps: int = 20, current_scale: float = 1.0,
                  field_scale: float = 1.0, coupling: str = "x",
                  renormalize: bool = False) -> Params:
    """Table 1 in the dimensionless unit (t0 = 1 ns, h = gamma t0 H).

    ``a_cp`` and ``a_in`` are given directly in the dimensionless field unit
    (the paper's 1 Oe is 0.01764).  ``current_scale`` and ``field_scale``
    multiply I and H_appl.
    """
    u = GAMMA * T0
    return Params(
        alpha=ALPHA,
        h_appl=u * (H_APPL * field_scale),
        h_k=u * (H_K - demag_oe()),
        h_s=u * spin_torque_field_oe(CURRENT * current_scale),
        lam=LAMBDA_STT,
        p=P_VEC,
        a_cp=a_cp,
        a_in=a_in,
        dt=dt,
        substeps=substeps,
        g=1.0,
        renormalize=renormalize,
        coupling=coupling,
    )


def physical(a_cp_oe: float = A_CP_OE, a_in_oe: float = A_IN_OE,
             dt_s: float = 1e-11, substeps: int = 20,
             coupling: str = "x") -> Params:
    """Table 1 in CGS units with seconds; gamma enters through ``g``."""
    return Params(
        alpha=ALPHA,
        h_appl=H_APPL,
        h_k=H_K - demag_oe(),
        h_s=spin_torque_field_oe(),
        lam=LAMBDA_STT,
        p=P_VEC,
        a_cp=a_cp_oe,
        a_in=a_in_oe,
        dt=dt_s,
        substeps=substeps,
        g=GAMMA,
        coupling=coupling,
    )
