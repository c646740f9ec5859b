"""Helpers shared by the GPU tests: one set of constants fed to both sides.

The oracle and the library each derive the dimensionless constants of
Table 1 on their own; the parity tests hand both sides the same numbers
(the oracle's) so that a comparison tests the integration, not the unit
conversion.  ``test_library_host.py`` checks separately that the library's
own presets equal the oracle's constants bit for bit.
"""

from __future__ import annotations

import functools

import numpy as np

from oracle import constants, sto
from workloads import WORKLOADS, make_workload_arrays


def oracle_params(a_cp=0.1, a_in=1.0, dt=0.01, substeps=20, coupling="x", renormalize=False, **kw):
    prm = constants.dimensionless(a_cp=a_cp, a_in=a_in, dt=dt, substeps=substeps, coupling=coupling,
                                  renormalize=renormalize)
    return prm.replace(**kw) if kw else prm


def lib_params(prm, dtype="f64", path="auto"):
    import paper_2312_01121_amd as stx
    return stx.make_params(prm.alpha, prm.h_appl, prm.h_k, prm.h_s, prm.lam, prm.p, prm.a_cp, prm.a_in,
                           prm.dt, substeps=prm.substeps, renormalize=prm.renormalize, dtype=dtype,
                           coupling=prm.coupling, path=path)


def workload_case(name, samples=None):
    wl = WORKLOADS[name]
    arrays = make_workload_arrays(wl, samples=samples)
    prm = oracle_params(a_cp=wl.a_cp, a_in=wl.a_in, dt=wl.dt, substeps=wl.substeps)
    return wl, arrays, prm


@functools.lru_cache(maxsize=None)
def oracle_run_cached(name, samples):
    wl, a, prm = workload_case(name, samples)
    rec, fin = sto.run(a["W"], a["w_in"], a["m0"], a["u"], prm)
    return rec, fin


def random_case(n, n_in=1, seed=0, samples=10, spread=0.05):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n)) / np.sqrt(n)
    np.fill_diagonal(w, 0.0)
    w_in = rng.uniform(-1, 1, (n, n_in))
    v = rng.standard_normal((n, 3)) * spread
    v[:, 2] += 1.0
    m0 = v / np.linalg.norm(v, axis=1, keepdims=True)
    u = rng.uniform(-1, 1, (samples, n_in))
    return w, w_in, m0, u


def _one_stream_adjoint(args):
    """Worker: the oracle's adjoint of one input stream (BLAS on one thread)."""
    from threadpoolctl import threadpool_limits
    from oracle import adjoint
    w, w_in, m0, u, prm, g_rec, g_fin, dot = args
    with threadpool_limits(limits=1):
        r = adjoint.run_adjoint(w, w_in, m0, u, prm, g_rec, g_fin, dot=dot)
    return {k: r[k] for k in ("W", "w_in", "m0", "a_cp", "a_in", "h_s", "h_appl")}


def oracle_streams_adjoint(w, w_in, m0s, u, prm, g_rec, g_fin, dot="blas", workers=1):
    """The oracle's adjoint run once per stream: dL/dW, dL/dw_in and the
    scalars of the shared reservoir sum over the streams (in stream order).
    workers > 1 runs the streams in that many spawned CPU processes (they
    never touch the GPU)."""
    S = m0s.shape[0]
    jobs = [(w, w_in, m0s[s], u[:, s], prm, g_rec[:, s], None if g_fin is None else g_fin[s], dot)
            for s in range(S)]
    if workers > 1:
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, S),
                                 mp_context=multiprocessing.get_context("spawn")) as ex:
            parts = list(ex.map(_one_stream_adjoint, jobs))
    else:
        parts = [_one_stream_adjoint(j) for j in jobs]
    tot = {}
    for r in parts:
        for k in ("W", "w_in", "a_cp", "a_in", "h_s", "h_appl"):
            tot[k] = tot.get(k, 0.0) + r[k]
    tot["m0"] = np.stack([r["m0"] for r in parts])
    return tot
