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

Handles are kept between calls, one per device and configuration (sizes,
dtype, coupling, substeps, renormalisation, path; at most four, the oldest
dropped first): W, w_in and the constants are loaded into it from device
buffers (``reservoir_load_device``) only when they differ from what it
holds, a tensor being the same when it is the same object at the same
in-place version.  A tuning loop that updates W in place therefore moves no
W through host memory; only the four scalars are read as host numbers.
``release()`` frees the kept handles.
"""

from __future__ import annotations

import atexit
import ctypes
import weakref
from collections import OrderedDict

import torch

from . import Reservoir, readout_fit_device, readout_grad_device, sto_params

_FIELDS = ("a_cp", "a_in", "h_s", "h_appl")
_MAX_HANDLES = 4


def _with_scalars(prm: sto_params, values) -> sto_params:
    out = sto_params()
    ctypes.memmove(ctypes.byref(out), ctypes.byref(prm), ctypes.sizeof(sto_params))
    for name, v in zip(_FIELDS, values):
        setattr(out, name, float(v))
    return out


class _Held:
    """What a kept handle holds: the tensors its W and w_in came from (object
    and in-place version) and its constants."""

    def __init__(self, res: Reservoir):
        self.res = res
        self.W = self.w_in = None
        self.prm = b""

    @staticmethod
    def token(t):
        return (weakref.ref(t), t._version)

    @staticmethod
    def same(tok, t) -> bool:
        return tok is not None and tok[0]() is t and tok[1] == t._version


_HANDLES: "OrderedDict[tuple, _Held]" = OrderedDict()


def release():
    """Free the handles kept between calls."""
    while _HANDLES:
        _, held = _HANDLES.popitem()
        held.res.close()


# kept handles are freed while the HIP runtime is still up, not by the
# garbage collector at interpreter teardown
atexit.register(release)


def _dev64(t, dev):
    return t.detach().to(dev, torch.float64).contiguous()


def _handle(W, w_in, m0, p: sto_params, dev, m_init=None) -> Reservoir:
    """A handle holding W, w_in and the constants p, with m0 (None: keep) as
    its state; loads from the device only what changed.  A new handle starts
    from m0, else from m_init."""
    n = int(W.shape[0])
    n_in = int(w_in.numel() // n)
    key = (dev.index, n, n_in, p.dtype, p.coupling, p.substeps, p.renormalize, p.path)
    held = _HANDLES.get(key)
    pb = bytes(p)
    if held is None:
        while len(_HANDLES) >= _MAX_HANDLES:
            _HANDLES.popitem(last=False)[1].res.close()
        with torch.cuda.device(dev):
            m = m0 if m0 is not None else m_init
            held = _Held(Reservoir.from_device(_dev64(W, dev), _dev64(w_in, dev), _dev64(m, dev), p))
        _HANDLES[key] = held
    else:
        _HANDLES.move_to_end(key)
        load_W = not _Held.same(held.W, W)
        load_win = not _Held.same(held.w_in, w_in)
        if load_W or load_win or m0 is not None or held.prm != pb:
            with torch.cuda.device(dev):
                held.res.load_device(_dev64(W, dev) if load_W else None, _dev64(w_in, dev) if load_win else None,
                                     _dev64(m0, dev) if m0 is not None else None, p if held.prm != pb else None)
    held.W, held.w_in, held.prm = _Held.token(W), _Held.token(w_in), pb
    return held.res


class ReservoirRecords(torch.autograd.Function):
    """Records of a run (samples, n, 3); backward by the discrete adjoint."""

    @staticmethod
    def forward(ctx, W, w_in, m0, a_cp, a_in, h_s, h_appl, u, prm, checkpoint_every):
        vals = [float(t) for t in (a_cp, a_in, h_s, h_appl)]
        p = _with_scalars(prm, vals)
        dev = u.device
        res = _handle(W, w_in, m0, p, dev)
        dt = torch.float64 if res.dtype == "f64" else torch.float32
        samples = u.shape[0]
        records = torch.empty((samples, res.n, 3), dtype=dt, device=dev)
        res.run_device(u, records)
        ctx.prm = p
        # the records are the checkpoints of the backward (segments of whole
        # samples); W and w_in are saved so that autograd rejects their
        # in-place change before the backward
        ctx.save_for_backward(records, W, w_in)
        ctx.m_start = m0.detach().to(dev, dt).contiguous()
        ctx.u = u
        ctx.checkpoint_every = checkpoint_every
        ctx.like = (W, w_in, m0, a_cp, a_in, h_s, h_appl)
        return records

    @staticmethod
    def backward(ctx, grad_records):
        W, w_in, m0, a_cp, a_in, h_s, h_appl = ctx.like
        # the handle may have been loaded with other arrays since the forward
        res = _handle(W, w_in, None, ctx.prm, ctx.u.device, m_init=m0)
        dt = torch.float64 if res.dtype == "f64" else torch.float32
        g = grad_records.to(dt).contiguous()
        records = ctx.saved_tensors[0]
        out = res.adjoint_device(ctx.m_start, ctx.u, grad_states_dev=g, checkpoint_every=ctx.checkpoint_every,
                                 records_dev=records if ctx.checkpoint_every % res.substeps == 0 else None)
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
