"""torch.autograd wrappers over the library's forward run, ridge readout and
adjoint.  Argument marshalling only: the forward is ``reservoir_run_device``,
the loss is ``readout_fit_device`` + ``readout_grad_device`` and the
backward is ``reservoir_adjoint_records_device`` (the forward's records are
the checkpoints of its segments; ``reservoir_adjoint_device`` when the
segments are not whole samples).

    records = reservoir_records(W, w_in, m0, a_cp, a_in, h_s, h_appl, u, prm)
    loss = ridge_loss(records, y, washout, lam)
    loss.backward()          # W.grad, w_in.grad, m0.grad, a_cp.grad, ...

W (n, n), w_in (n, n_in), m0 (n, 3) and the four scalars are tensors (any
device, any float dtype); u is a CUDA float64 tensor (samples, n_in); prm is
an ``sto_params`` whose a_cp, a_in, h_s and h_appl are replaced by the
tensors' values.  The run computes in prm's dtype on the current CUDA device.
"""

from __future__ import annotations

import ctypes

import torch

from . import Reservoir, readout_fit_device, readout_grad_device, sto_params

_FIELDS = ("a_cp", "a_in", "h_s", "h_appl")


def _with_scalars(prm: sto_params, values) -> sto_params:
    out = sto_params()
    ctypes.memmove(ctypes.byref(out), ctypes.byref(prm), ctypes.sizeof(sto_params))
    for name, v in zip(_FIELDS, values):
        setattr(out, name, float(v))
    return out


class ReservoirRecords(torch.autograd.Function):
    """Records of a run (samples, n, 3); backward by the discrete adjoint."""

    @staticmethod
    def forward(ctx, W, w_in, m0, a_cp, a_in, h_s, h_appl, u, prm, checkpoint_every):
        vals = [float(t) for t in (a_cp, a_in, h_s, h_appl)]
        p = _with_scalars(prm, vals)
        host = lambda t: t.detach().to("cpu", torch.float64).numpy()
        res = Reservoir(host(W), host(w_in), host(m0), p)
        dt = torch.float64 if res.dtype == "f64" else torch.float32
        dev = u.device
        samples = u.shape[0]
        records = torch.empty((samples, res.n, 3), dtype=dt, device=dev)
        res.run_device(u, records)
        ctx.res = res
        ctx.save_for_backward(records)   # the checkpoints of the backward (segments of whole samples)
        ctx.m_start = m0.detach().to(dev, dt).contiguous()
        ctx.u = u
        ctx.checkpoint_every = checkpoint_every
        ctx.like = (W, w_in, m0, a_cp, a_in, h_s, h_appl)
        return records

    @staticmethod
    def backward(ctx, grad_records):
        res = ctx.res
        dt = torch.float64 if res.dtype == "f64" else torch.float32
        g = grad_records.to(dt).contiguous()
        records, = ctx.saved_tensors
        out = res.adjoint_device(ctx.m_start, ctx.u, grad_states_dev=g, checkpoint_every=ctx.checkpoint_every,
                                 records_dev=records if ctx.checkpoint_every % res.substeps == 0 else None)
        W, w_in, m0, a_cp, a_in, h_s, h_appl = ctx.like
        cast = lambda x, like: x.to(like.device, like.dtype).reshape(like.shape)
        sc = out["scalars"]
        grads = (cast(out["W"], W), cast(out["w_in"], w_in), cast(out["m0"], m0),
                 cast(sc[0], a_cp), cast(sc[1], a_in), cast(sc[2], h_s), cast(sc[3], h_appl))
        return grads + (None, None, None)


class RidgeLoss(torch.autograd.Function):
    """Ridge objective at its optimum, J = (|Phi w* - y|^2 + lam |w*|^2) / T'."""

    @staticmethod
    def forward(ctx, records, y, washout, lam, features):
        rec = records.detach().contiguous()
        w, _ = readout_fit_device(rec, y, washout, lam, features)
        grad, loss = readout_grad_device(rec, y, washout, lam, w, features)
        ctx.save_for_backward(grad)
        ctx.w = w
        return torch.tensor(loss, dtype=torch.float64, device=records.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return (grad_out.to(grad.dtype) * grad, None, None, None, None)


def reservoir_records(W, w_in, m0, a_cp, a_in, h_s, h_appl, u, prm: sto_params, checkpoint_every: int = 0):
    return ReservoirRecords.apply(W, w_in, m0, a_cp, a_in, h_s, h_appl, u, prm, checkpoint_every)


def ridge_loss(records, y, washout: int, lam: float, features: int = 0):
    return RidgeLoss.apply(records, y, washout, lam, features)
