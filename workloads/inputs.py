"""Seeded generators for the synthetic coupled-oscillator workloads.

Every array is drawn from NumPy's PCG64 through ``SeedSequence`` so that the
oracle, the tests and the benchmark see bit-identical inputs.  The random
streams are split as ``SeedSequence(seed).spawn(4)`` -> [coupling matrix,
input weights, initial state, input series].

Distributions (paper, Sec. 3.1, the paragraph after Eq. (in), and the
initial condition Eq. (initial)):

* coupling matrix: zero diagonal; either i.i.d. N(0,1)/sqrt(N) entries
  ("normal", used by every sized workload below) or the paper's U[-1,1]
  entries rescaled to spectral radius 1 ("paper");
* input weights: U[-1,1];
* initial state: a random unit vector within 2 degrees of +z ("random"),
  or the paper's identical tilt of one degree for every node ("paper");
* input series: u ~ U[-1,1], one value per sample, held for ``substeps``
  integrator steps;
* readout target: y_n = tanh(u_{n-1} + ... + u_{n-5}), undefined (NaN) for
  n < 5.

No field evaluation, integration, readout solve or physical constant lives
here.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """Sizes and knobs of one synthetic workload.

    ``a_cp`` is the coupling strength multiplying the N(0,1)/sqrt(N) matrix
    and ``a_in`` the input amplitude, both in the dimensionless field unit.
    ``dtypes`` lists the arithmetic types the workload is run in.
    """

    name: str
    n: int
    samples: int
    substeps: int = 20
    dt: float = 0.01
    a_cp: float = 0.1
    a_in: float = 1.0
    n_in: int = 1
    dtypes: tuple = ("f64",)
    seed: int = 0
    coupling_kind: str = "normal"
    init_kind: str = "random"
    ridge: float = 1e-6

    @property
    def steps(self) -> int:
        return self.samples * self.substeps

    def with_samples(self, samples: int) -> "Workload":
        return dataclasses.replace(self, samples=samples)


# The sized workloads: 16, 1,000 and 10,000 coupled oscillators, and 64
# input streams driving one 512-node reservoir.
WORKLOADS: Dict[str, Workload] = {
    "sto16": Workload("sto16", n=16, samples=2000, dtypes=("f64",)),
    "sto1k": Workload("sto1k", n=1000, samples=10000, dtypes=("f32", "f64")),
    "sto10k": Workload("sto10k", n=10000, samples=1000, dtypes=("f32", "f64")),
    "streams64": Workload("streams64", n=512, samples=1000, dtypes=("f32",)),
}
STREAMS: Dict[str, int] = {"streams64": 64}


def seed_streams(seed: int, key: Optional[int] = None):
    """Four independent generators [coupling, input weights, initial, input].

    ``key`` selects a sub-experiment (one reservoir of a sweep, one input
    stream); ``None`` is the plain single-reservoir stream.
    """
    ss = np.random.SeedSequence(seed if key is None else [seed, key])
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]


def draw_coupling(rng: np.random.Generator, n: int, kind: str = "normal") -> np.ndarray:
    """Dense n x n coupling matrix with zero diagonal (float64, C order).

    "paper": U[-1,1] entries rescaled to spectral radius 1.  The radius is
    computed from the eigenvalues for n <= 2000; above that it is taken from
    the circular law, rho = sqrt(n / 3) for i.i.d. entries of variance 1/3
    (relative error O(n^-1/2); a full eigendecomposition of a 10^4 matrix
    would take minutes and only rescales W)."""
    if kind == "normal":
        w = rng.standard_normal((n, n))
        w *= 1.0 / math.sqrt(n)
    elif kind == "paper":
        w = rng.uniform(-1.0, 1.0, size=(n, n))
        np.fill_diagonal(w, 0.0)
        if n <= 1:
            rho = 0.0
        elif n <= 2000:
            rho = float(np.max(np.abs(np.linalg.eigvals(w))))
        else:
            rho = math.sqrt(n / 3.0)
        if rho > 0.0:
            w /= rho
    else:
        raise ValueError(f"unknown coupling kind {kind!r}")
    np.fill_diagonal(w, 0.0)
    return np.ascontiguousarray(w)


def draw_input_weights(rng: np.random.Generator, n: int, n_in: int = 1) -> np.ndarray:
    """Input weights w_in, U[-1,1], shape (n, n_in)."""
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(n, n_in)))


def draw_initial(rng: np.random.Generator, n: int, kind: str = "random") -> np.ndarray:
    """Initial unit magnetisations, shape (n, 3), AoS.

    "random": polar angle U[0, 2 deg], azimuth U[0, 2 pi).
    "paper":  every node tilted by phi0 = 2 pi / 360 in polar angle and in
              azimuth, as in Eq. (initial).
    """
    phi0 = 2.0 * math.pi / 360.0
    if kind == "random":
        theta = rng.uniform(0.0, 2.0 * phi0, size=n)
        psi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    elif kind == "paper":
        theta = np.full(n, phi0)
        psi = np.full(n, phi0)
    else:
        raise ValueError(f"unknown initial kind {kind!r}")
    m = np.empty((n, 3))
    m[:, 0] = np.sin(theta) * np.cos(psi)
    m[:, 1] = np.sin(theta) * np.sin(psi)
    m[:, 2] = np.cos(theta)
    return m


def draw_inputs(rng: np.random.Generator, samples: int, n_in: int = 1) -> np.ndarray:
    """Input series u ~ U[-1,1], shape (samples, n_in)."""
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(samples, n_in)))


def draw_target(u: np.ndarray, delay: int = 5) -> np.ndarray:
    """Synthetic readout target y_n = tanh(sum_{k=1..delay} u_{n-k}).

    Uses the first input channel; entries n < delay are NaN.
    """
    u0 = np.asarray(u, dtype=np.float64).reshape(len(u), -1)[:, 0]
    y = np.full(len(u0), np.nan)
    for n in range(delay, len(u0)):
        y[n] = math.tanh(math.fsum(u0[n - delay:n]))
    return y


def make_workload_arrays(wl: Workload, samples: Optional[int] = None,
                         key: Optional[int] = None) -> Dict[str, np.ndarray]:
    """All arrays of one workload, drawn from ``wl.seed``.

    ``samples`` truncates the input series to a prefix (the first samples of
    the full series, so a prefix run sees exactly the inputs of the full
    run).
    """
    g_w, g_in, g_m0, g_u = seed_streams(wl.seed, key)
    w = draw_coupling(g_w, wl.n, wl.coupling_kind)
    w_in = draw_input_weights(g_in, wl.n, wl.n_in)
    m0 = draw_initial(g_m0, wl.n, wl.init_kind)
    u = draw_inputs(g_u, wl.samples, wl.n_in)
    if samples is not None:
        u = np.ascontiguousarray(u[:samples])
    y = draw_target(u)
    return {"W": w, "w_in": w_in, "m0": m0, "u": u, "y": y}


def make_stream_arrays(wl: Workload, streams: int, samples: Optional[int] = None) -> Dict[str, np.ndarray]:
    """One reservoir (W, w_in, m0 from ``wl.seed``) driven by ``streams``
    independent input series: stream s draws u from SeedSequence([seed, 1000 + s]).

    u has shape (samples, streams, n_in) and y (samples, streams); every
    stream starts from the same m0.
    """
    base = make_workload_arrays(wl, samples=1)
    t = wl.samples if samples is None else samples
    us = []
    for st in range(streams):
        g_u = seed_streams(wl.seed, 1000 + st)[3]
        us.append(draw_inputs(g_u, wl.samples, wl.n_in)[:t])
    u = np.ascontiguousarray(np.stack(us, axis=1))
    y = np.stack([draw_target(u[:, st]) for st in range(streams)], axis=1)
    return {"W": base["W"], "w_in": base["w_in"], "m0": base["m0"], "u": u, "y": y}


def make_paper_arrays(n: int, samples: int) -> Dict[str, np.ndarray]:
    """The paper's benchmark setup at size n (Sec. 3.2): u = 0, the paper's
    coupling generator (U[-1,1], zero diagonal, spectral radius 1), U[-1,1]
    input weights and the identical initial tilt of Eq. (initial).  The
    arrays of size n come from SeedSequence([0, 5000 + n])."""
    g_w, g_in, g_m0, _ = seed_streams(0, 5000 + n)
    return {"W": draw_coupling(g_w, n, "paper"), "w_in": draw_input_weights(g_in, n, 1),
            "m0": draw_initial(g_m0, n, "paper"), "u": np.zeros((samples, 1))}


@dataclasses.dataclass(frozen=True)
class Sweep:
    """A parameter sweep: ``count`` reservoirs of log-uniform size in
    [n_lo, n_hi], each with its own coupling matrix, input weights, initial
    state and constants, driven by one shared input series."""

    name: str
    count: int
    n_lo: int
    n_hi: int
    samples: int
    substeps: int = 20
    dt: float = 0.01
    seed: int = 0
    ridge: float = 1e-6

    @property
    def steps(self) -> int:
        return self.samples * self.substeps


SWEEPS: Dict[str, Sweep] = {
    "sweep256": Sweep("sweep256", count=256, n_lo=32, n_hi=2048, samples=2000),
}


def make_sweep_arrays(sw: Sweep, samples: Optional[int] = None, count: Optional[int] = None):
    """Per-reservoir arrays and draws of a sweep.

    Reservoir r uses SeedSequence([seed, r]) for [W, w_in, m0, constants];
    its size comes from the sweep's own stream (SeedSequence(seed) spawn[0]).
    The draws per reservoir are plain random numbers: ``current_scale`` and
    ``field_scale`` ~ U[0.5, 1.5] (multipliers of I and H_appl), ``a_cp`` ~
    U[0.01, 0.5] and ``a_in`` ~ U[0.1, 2] in the dimensionless field unit.
    The shared input u ~ U[-1, 1] and the target come from the sweep's
    input stream (spawn[3]).
    """
    count = sw.count if count is None else count
    g_size, _, _, g_u = seed_streams(sw.seed)
    sizes = np.rint(np.exp(g_size.uniform(math.log(sw.n_lo), math.log(sw.n_hi), size=sw.count))).astype(int)
    u = draw_inputs(g_u, sw.samples, 1)
    if samples is not None:
        u = np.ascontiguousarray(u[:samples])
    res = []
    for r in range(count):
        g_w, g_in, g_m0, g_p = seed_streams(sw.seed, r)
        n = int(sizes[r])
        res.append({
            "n": n,
            "W": draw_coupling(g_w, n, "normal"),
            "w_in": draw_input_weights(g_in, n, 1),
            "m0": draw_initial(g_m0, n, "random"),
            "current_scale": float(g_p.uniform(0.5, 1.5)),
            "field_scale": float(g_p.uniform(0.5, 1.5)),
            "a_cp": float(g_p.uniform(0.01, 0.5)),
            "a_in": float(g_p.uniform(0.1, 2.0)),
        })
    return {"reservoirs": res, "u": u, "y": draw_target(u)}
