"""Plain FP64 classic-RK4 integration of N coupled spin-torque oscillators.

Oracle (test infrastructure): this module is the reference the HIP library
is checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may use it.

What it computes (paper, Sec. 3.1 and 3.2):

* Eq. (gov): dm_k/dt = -g/(1+a^2) m_k x b_k - a g/(1+a^2) m_k x (m_k x b_k),
  with g = gamma (physical units) or 1 (dimensionless form);
* b_k = H_k^total + H_s(m_k) p x m_k, with the spin-torque amplitude
  H_s(m_k) = h_s / (1 + lambda m_k . p);
* H_k^total = H(m_k) + H_k^cp + H_k^in, where
  H(m_k) = (h_appl + h_k m_k^z) e_z,
  Eq. (coup): H_k^cp = a_cp sum_i w_ki m_i^x e_x (the summand is read as
  m_i^x: with m_k^x the sum would not be the O(N^2) matrix product the paper
  describes), and
  Eq. (in):   H_k^in = a_in sum_j w^in_kj u_j e_x;
* classic fourth-order Runge-Kutta with a fixed step (Sec. 3.2); the input
  is a discrete series held constant for ``substeps`` steps per sample, so
  all four stages of a step see the same input value;
* one record of the state after the last step of each sample.

Fixed evaluation order.  The model is chaotic for coupled, driven
configurations, so any change in rounding grows along the trajectory (the
paper notes exactly this growth, Sec. 3.3).  The oracle therefore fixes the
arithmetic completely:

* each coupling and input sum is the exact sum rounded once to the nearest
  double (``dot="exact"``; ``"blas"`` uses NumPy's matrix product in
  whatever order BLAS chooses);
* every other operation is one IEEE double operation, evaluated in the
  grouping written in ``field`` and ``rk4_step`` (no fused multiply-add).

The optional renormalisation (off by default; the paper relies on the
conservation law |m_k| = 1 instead) divides each m_k by
sqrt((m^x)^2 + (m^y)^2 + (m^z)^2) after every full step.
"""

from __future__ import annotations

import math
from typing import Callable, Optional, Tuple

import numpy as np

from . import _native
from .constants import Params

Vec3 = Tuple[np.ndarray, np.ndarray, np.ndarray]


def matvec(a: np.ndarray, x: np.ndarray, dot: str) -> np.ndarray:
    """Row sums sum_i a[k, i] x[i] under the chosen rounding rule."""
    if dot == "exact":
        return _native.exact_matvec(a, x)
    if dot == "blas":
        return np.ascontiguousarray(a) @ np.ascontiguousarray(x)
    if dot == "loop":
        rows, cols = a.shape
        out = np.empty(rows)
        for k in range(rows):
            s = 0.0
            for i in range(cols):
                s += float(a[k, i]) * float(x[i])
            out[k] = s
        return out
    raise ValueError(f"unknown dot rule {dot!r}")


def cross(a: Vec3, b: Vec3) -> Vec3:
    """a x b, component by component; each product and difference rounded once."""
    ax, ay, az = a
    bx, by, bz = b
    return (ay * bz - az * by, az * bx - ax * bz, ax * by - ay * bx)


def coupling_field(w: np.ndarray, m: Vec3, prm: Params, dot: str):
    """Eq. (coup): a_cp * W m^x (x-only), or a_cp * W m for all three components."""
    mx, my, mz = m
    if prm.coupling == "x":
        return (prm.a_cp * matvec(w, mx, dot), None, None)
    if prm.coupling == "xyz":
        return (prm.a_cp * matvec(w, mx, dot), prm.a_cp * matvec(w, my, dot),
                prm.a_cp * matvec(w, mz, dot))
    raise ValueError(f"unknown coupling {prm.coupling!r}")


def input_field(w_in: np.ndarray, u_n: np.ndarray, prm: Params, dot: str) -> np.ndarray:
    """Eq. (in): a_in * sum_j w^in_kj u_j, the x-component of H^in."""
    return prm.a_in * matvec(w_in, np.atleast_1d(u_n), dot)


def field(m: Vec3, w: np.ndarray, h_in: np.ndarray, prm: Params, dot: str = "exact") -> Vec3:
    """Right-hand side of Eq. (gov) for all nodes at state m."""
    mx, my, mz = m
    px, py, pz = prm.p
    cx, cy, cz = coupling_field(w, m, prm, dot)
    # spin-torque amplitude H_s(m) = h_s / (1 + lambda m.p)
    mp = (mx * px + my * py) + mz * pz
    hs = prm.h_s / (1.0 + prm.lam * mp)
    qx, qy, qz = cross((px, py, pz), m)                 # p x m
    # b = (H + H^cp + H^in) + H_s p x m; H is along e_z, H^in along e_x
    hz = prm.h_appl + prm.h_k * mz
    if cy is None:
        bx = (cx + h_in) + hs * qx
        by = hs * qy
        bz = hz + hs * qz
    else:
        bx = (cx + h_in) + hs * qx
        by = cy + hs * qy
        bz = (hz + cz) + hs * qz
    mb = cross(m, (bx, by, bz))                          # m x b
    mmb = cross(m, mb)                                   # m x (m x b)
    c1 = prm.g / (1.0 + prm.alpha * prm.alpha)
    c2 = (prm.alpha * prm.g) / (1.0 + prm.alpha * prm.alpha)
    return tuple((-c1) * mb[j] - c2 * mmb[j] for j in range(3))


def axpy(m: Vec3, h: float, k: Vec3) -> Vec3:
    """m + h k, component-wise."""
    return tuple(m[j] + h * k[j] for j in range(3))


def rk4_step(m: Vec3, w: np.ndarray, h_in: np.ndarray, prm: Params,
             dot: str = "exact", rhs: Callable = field) -> Vec3:
    """One classic RK4 step of size prm.dt."""
    dt = prm.dt
    k1 = rhs(m, w, h_in, prm, dot)
    k2 = rhs(axpy(m, dt / 2.0, k1), w, h_in, prm, dot)
    k3 = rhs(axpy(m, dt / 2.0, k2), w, h_in, prm, dot)
    k4 = rhs(axpy(m, dt, k3), w, h_in, prm, dot)
    out = tuple(m[j] + (dt / 6.0) * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j])
                for j in range(3))
    if prm.renormalize:
        nrm = np.sqrt((out[0] * out[0] + out[1] * out[1]) + out[2] * out[2])
        out = tuple(out[j] / nrm for j in range(3))
    return out


def to_soa(m_aos: np.ndarray) -> Vec3:
    m_aos = np.asarray(m_aos, dtype=np.float64)
    return (m_aos[:, 0].copy(), m_aos[:, 1].copy(), m_aos[:, 2].copy())


def to_aos(m: Vec3) -> np.ndarray:
    return np.stack(m, axis=1)


def run(w: np.ndarray, w_in: np.ndarray, m0: np.ndarray, u: np.ndarray, prm: Params,
        dot: str = "exact", rhs: Callable = field, step: Callable = None,
        on_sample: Optional[Callable[[int, Vec3], None]] = None):
    """Integrate over every input sample; return (records, final state).

    records[n] is the (N, 3) state after the ``substeps`` steps that hold
    input sample u[n]; the initial state is not recorded.
    """
    w = np.ascontiguousarray(w, dtype=np.float64)
    w_in = np.ascontiguousarray(w_in, dtype=np.float64)
    if w_in.ndim == 1:
        w_in = w_in[:, None]
    u = np.asarray(u, dtype=np.float64).reshape(len(u), -1)
    n = w.shape[0]
    if w.shape != (n, n) or w_in.shape[0] != n or u.shape[1] != w_in.shape[1]:
        raise ValueError("inconsistent shapes")
    step = rk4_step if step is None else step
    m = to_soa(m0)
    records = np.empty((len(u), n, 3))
    for s in range(len(u)):
        h_in = input_field(w_in, u[s], prm, dot)
        for _ in range(prm.substeps):
            m = step(m, w, h_in, prm, dot, rhs)
        if not all(np.all(np.isfinite(c)) for c in m):
            raise FloatingPointError(f"non-finite state after sample {s}")
        records[s] = to_aos(m)
        if on_sample is not None:
            on_sample(s, m)
    return records, to_aos(m)


def norm_drift(records: np.ndarray) -> float:
    """max over records and nodes of | |m_k| - 1 |."""
    nrm = np.sqrt(np.einsum("tnc,tnc->tn", records, records))
    return float(np.max(np.abs(nrm - 1.0))) if nrm.size else 0.0


def lyapunov_max(w, w_in, m0, u, prm: Params, d0: float = 1e-10, seed: int = 1,
                 dot: str = "blas", rhs: Callable = field, step: Callable = None) -> float:
    """Largest Lyapunov exponent (per unit time) by Benettin's twin method.

    A copy of the state perturbed by d0 in a random direction is integrated
    beside the reference; after each sample the separation is measured and
    rescaled back to d0.  The exponent is the sum of the log growth factors
    divided by the time integrated.  ``rhs`` and ``step`` are the hooks that
    ``run`` takes.
    """
    step = rk4_step if step is None else step
    rng = np.random.default_rng(seed)
    n = w.shape[0]
    w_in2 = w_in[:, None] if np.ndim(w_in) == 1 else w_in
    u = np.asarray(u, dtype=np.float64).reshape(len(u), -1)
    a = to_soa(m0)
    d = rng.standard_normal((n, 3))
    d *= d0 / np.linalg.norm(d)
    b = to_soa(np.asarray(m0) + d)
    total = 0.0
    for s in range(len(u)):
        h_in = input_field(w_in2, u[s], prm, dot)
        for _ in range(prm.substeps):
            a = step(a, w, h_in, prm, dot, rhs)
            b = step(b, w, h_in, prm, dot, rhs)
        diff = np.stack([b[j] - a[j] for j in range(3)], axis=1)
        dist = float(np.linalg.norm(diff))
        total += math.log(dist / d0)
        b = to_soa(to_aos(a) + diff * (d0 / dist))
    return total / (len(u) * prm.substeps * prm.dt)
