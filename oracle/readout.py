"""Ridge-regression readout of the reservoir states (FP64 oracle).

Oracle (test infrastructure).  The paper trains only the readout of the
reservoir (Sec. 1) and uses the N node states as its features (Sec. 3.1,
after Table 1); it does not fix the algorithm.  The readout here is ridge
regression:

* features: the x-component of every node at each record (or all three
  components), plus a constant 1 for the bias, for records n >= washout;
* weights: w = argmin |Phi w - y|^2 + lambda |w|^2 over all coefficients,
  bias included, solved through the normal equations
  (Phi^T Phi + lambda I) w = Phi^T y with a Cholesky factorisation (primal),
  or, when there are fewer rows than columns, through the equivalent dual
  form w = Phi^T (Phi Phi^T + lambda I)^{-1} y;
* score: NMSE = sum (y - Phi w)^2 / sum (y - mean y)^2 on the fitted rows.
"""

from __future__ import annotations

import math

import numpy as np


def default_washout(samples: int) -> int:
    """max(5, ceil(0.1 * samples)): skips the transient and the undefined targets."""
    return max(5, int(math.ceil(0.1 * samples)))


def features(records: np.ndarray, washout: int, components: str = "x") -> np.ndarray:
    """Design matrix Phi = [state features, 1] for records n >= washout."""
    records = np.asarray(records, dtype=np.float64)
    t, n, _ = records.shape
    rows = records[washout:]
    if components == "x":
        f = rows[:, :, 0]
    elif components == "xyz":
        f = rows.reshape(t - washout, 3 * n)
    else:
        raise ValueError(components)
    return np.concatenate([f, np.ones((t - washout, 1))], axis=1)


def _cholesky_solve(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    ell = np.linalg.cholesky(a)
    z = np.linalg.solve(ell, b)          # forward substitution (L lower)
    return np.linalg.solve(ell.T, z)     # back substitution


def ridge(phi: np.ndarray, y: np.ndarray, lam: float, form: str = "auto") -> np.ndarray:
    """Ridge weights for design Phi and targets y; penalty lam on every weight."""
    rows, cols = phi.shape
    if form == "auto":
        form = "primal" if rows >= cols else "dual"
    if form == "primal":
        g = phi.T @ phi + lam * np.eye(cols)
        return _cholesky_solve(g, phi.T @ y)
    if form == "dual":
        k = phi @ phi.T + lam * np.eye(rows)
        return phi.T @ _cholesky_solve(k, y)
    raise ValueError(form)


def nmse(phi: np.ndarray, y: np.ndarray, w: np.ndarray) -> float:
    r = y - phi @ w
    d = y - np.mean(y)
    return float((r @ r) / (d @ d))


def readout_fit(records: np.ndarray, y: np.ndarray, washout: int, lam: float,
                components: str = "x", form: str = "auto"):
    """Fit the readout; return (weights with the bias last, NMSE)."""
    phi = features(records, washout, components)
    yy = np.asarray(y, dtype=np.float64)[washout:]
    w = ridge(phi, yy, lam, form)
    return w, nmse(phi, yy, w)


def ridge_objective_grad(records: np.ndarray, y: np.ndarray, washout: int, lam: float,
                         components: str = "x", form: str = "auto"):
    """Ridge objective at its optimum and its gradient with respect to the records.

    J = (|Phi w* - y|^2 + lambda |w*|^2) / T' with T' the number of fitted
    rows and w* the ridge weights.  The objective is stationary in w at w*,
    so the total derivative with respect to Phi equals the partial one
    (envelope theorem): dJ/dPhi = (2/T') (Phi w* - y) w*^T.  The bias column
    is constant and rows before the washout do not enter, so their gradient
    is zero.  Returns (J, w*, dJ/d(records) with the records' shape).
    """
    records = np.asarray(records, dtype=np.float64)
    t, n, _ = records.shape
    phi = features(records, washout, components)
    yy = np.asarray(y, dtype=np.float64)[washout:]
    w = ridge(phi, yy, lam, form)
    r = phi @ w - yy
    rows = t - washout
    j = float((r @ r + lam * (w @ w)) / rows)
    dphi = (2.0 / rows) * np.outer(r, w)
    grad = np.zeros_like(records)
    if components == "x":
        grad[washout:, :, 0] = dphi[:, :n]
    else:
        grad[washout:] = dphi[:, :3 * n].reshape(rows, n, 3)
    return j, w, grad
