"""Python binding of libsto_reservoir.so (the MI355X coupled-STO reservoir).

A thin ctypes layer over ``include/sto_reservoir.h``: the functions below
carry the C entry points' names and only marshal arguments; every step of
the computation runs in the library's HIP kernels.  PyTorch is used only
for device buffers and streams (``run_device``).  Importing this package
fails loudly if the shared library has not been built
(``python paper_2312_01121_amd/_build.py``).
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

from . import params  # noqa: F401

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsto_reservoir.so")

STO_OK, STO_E_INVALID, STO_E_NOMEM, STO_E_DEVICE, STO_E_NONFINITE, STO_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
STO_F64, STO_F32 = 0, 1
STO_COUPLE_X, STO_COUPLE_XYZ = 0, 1
PATH_AUTO, PATH_SMALL, PATH_RESIDENT, PATH_STREAM, PATH_MULTI, PATH_BATCH = 0, 1, 2, 3, 4, 5
PATH_NAMES = {PATH_SMALL: "small", PATH_RESIDENT: "resident", PATH_STREAM: "stream", PATH_MULTI: "multi",
              PATH_BATCH: "batch"}
_STATUS_NAMES = {STO_E_INVALID: "invalid", STO_E_NOMEM: "nomem", STO_E_DEVICE: "device",
                 STO_E_NONFINITE: "nonfinite", STO_E_UNSUPPORTED: "unsupported"}


class StoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{_STATUS_NAMES.get(status, status)}] {message}")
        self.status = status


class sto_params(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double), ("h_appl", ctypes.c_double), ("h_k", ctypes.c_double),
        ("h_s", ctypes.c_double), ("lambda_stt", ctypes.c_double), ("p", ctypes.c_double * 3),
        ("a_cp", ctypes.c_double), ("a_in", ctypes.c_double), ("dt", ctypes.c_double),
        ("substeps", ctypes.c_int32), ("renormalize", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("coupling", ctypes.c_int32), ("path", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


def make_params(alpha, h_appl, h_k, h_s, lambda_stt, p, a_cp, a_in, dt, substeps=20,
                renormalize=False, dtype="f64", coupling="x", path="auto") -> sto_params:
    pr = sto_params()
    pr.alpha, pr.h_appl, pr.h_k, pr.h_s, pr.lambda_stt = alpha, h_appl, h_k, h_s, lambda_stt
    pr.p[0], pr.p[1], pr.p[2] = p
    pr.a_cp, pr.a_in, pr.dt = a_cp, a_in, dt
    pr.substeps = int(substeps)
    pr.renormalize = int(bool(renormalize))
    pr.dtype = {"f64": STO_F64, "f32": STO_F32}[dtype]
    pr.coupling = {"x": STO_COUPLE_X, "xyz": STO_COUPLE_XYZ}[coupling]
    pr.path = {"auto": PATH_AUTO, "small": PATH_SMALL, "resident": PATH_RESIDENT, "stream": PATH_STREAM,
               "multi": PATH_MULTI, "batch": PATH_BATCH}[path]
    pr.reserved = 0
    return pr


def _load():
    # torch's HIP libraries load their own bundled HIP runtime under the
    # unversioned name libamdhip64.so; loading it first makes this library's
    # libamdhip64.so.7 resolve to that same runtime instead of a second copy
    # (two runtimes in one process cannot share the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2312_01121_amd/_build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    H = ctypes.c_void_p
    lib.reservoir_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(sto_params), dp, dp, dp,
                                     ctypes.POINTER(H)]
    lib.reservoir_create_streams.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.POINTER(sto_params), dp, dp, dp, ctypes.POINTER(H)]
    lib.reservoir_create_device.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.POINTER(sto_params), vp, vp, vp, vp, ctypes.POINTER(H)]
    lib.reservoir_create_device.restype = ctypes.c_int
    lib.reservoir_load_device.argtypes = [H, vp, vp, vp, ctypes.POINTER(sto_params), vp]
    lib.reservoir_load_device.restype = ctypes.c_int
    lib.reservoir_streams.argtypes = [H]
    lib.reservoir_streams.restype = ctypes.c_int64
    lib.reservoir_run.argtypes = [H, dp, ctypes.c_int64, dp]
    lib.reservoir_run_device.argtypes = [H, vp, ctypes.c_int64, vp, vp]
    lib.reservoir_get_state.argtypes = [H, dp]
    lib.reservoir_set_state.argtypes = [H, dp]
    lib.reservoir_path.argtypes = [H]
    lib.reservoir_path.restype = ctypes.c_int32
    lib.reservoir_destroy.argtypes = [H]
    lib.reservoir_destroy.restype = None
    lib.readout_fit.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_int32, dp, dp]
    lib.readout_fit_device.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, vp, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_int32, vp, dp, vp]
    lib.readout_fit_device.restype = ctypes.c_int
    lib.readout_fit_device_noalloc.argtypes = lib.readout_fit_device.argtypes
    lib.readout_fit_device_noalloc.restype = ctypes.c_int
    lib.readout_fit_batch_device.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(vp), ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                             ctypes.POINTER(vp), dp, vp]
    lib.readout_fit_batch_device.restype = ctypes.c_int
    pp = ctypes.POINTER(dp)
    lib.sweep_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                 ctypes.POINTER(sto_params), pp, pp, pp, ctypes.POINTER(H)]
    lib.sweep_create.restype = ctypes.c_int
    lib.sweep_nodes.argtypes = [H]
    lib.sweep_nodes.restype = ctypes.c_int64
    lib.sweep_run.argtypes = [H, dp, ctypes.c_int64, dp]
    lib.sweep_run.restype = ctypes.c_int
    lib.sweep_run_device.argtypes = [H, vp, ctypes.c_int64, vp, vp]
    lib.sweep_run_device.restype = ctypes.c_int
    lib.sweep_get_state.argtypes = [H, dp]
    lib.sweep_get_state.restype = ctypes.c_int
    lib.sweep_destroy.argtypes = [H]
    lib.sweep_destroy.restype = None
    lib.sto_set_stream_variant.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.sto_set_stream_variant.restype = ctypes.c_int
    lib.sto_read_bandwidth.argtypes = [ctypes.c_int64, ctypes.c_int32, dp]
    lib.sto_read_bandwidth.restype = ctypes.c_int
    lib.reservoir_adjoint.argtypes = [H, dp, dp, ctypes.c_int64, dp, dp, dp, dp, dp, dp, ctypes.c_int64]
    lib.reservoir_adjoint.restype = ctypes.c_int
    lib.reservoir_adjoint_device.argtypes = [H, vp, vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.c_int64, vp]
    lib.reservoir_adjoint_device.restype = ctypes.c_int
    lib.reservoir_adjoint_records_device.argtypes = [H, vp, vp, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp,
                                                     ctypes.c_int64, vp]
    lib.reservoir_adjoint_records_device.restype = ctypes.c_int
    lib.readout_grad_device.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, vp, ctypes.c_int64,
                                        ctypes.c_double, ctypes.c_int32, vp, vp, dp, vp]
    lib.readout_grad_device.restype = ctypes.c_int
    lib.reservoir_adjoint_kernels.argtypes = [H]
    lib.reservoir_adjoint_kernels.restype = ctypes.c_int32
    lib.reservoir_trace_phases.argtypes = [H, ctypes.c_int64]
    lib.reservoir_trace_phases.restype = ctypes.c_int
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.reservoir_phase_times.argtypes = [H, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64, i64p, i64p, i64p]
    lib.reservoir_phase_times.restype = ctypes.c_int
    lib.sto_last_error.restype = ctypes.c_char_p
    for name in ("reservoir_create", "reservoir_create_streams", "reservoir_run", "reservoir_run_device", "reservoir_get_state",
                 "reservoir_set_state", "readout_fit"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()

EXPORTED = ("reservoir_create", "reservoir_create_streams", "reservoir_create_device", "reservoir_load_device", "reservoir_streams", "reservoir_run", "reservoir_run_device", "reservoir_get_state",
            "reservoir_set_state", "reservoir_path", "reservoir_destroy", "readout_fit", "readout_fit_device",
            "readout_fit_device_noalloc",
            "readout_fit_batch_device", "sweep_create", "sweep_nodes", "sweep_run", "sweep_run_device", "sweep_get_state", "sweep_destroy",
            "reservoir_adjoint", "reservoir_adjoint_device", "reservoir_adjoint_records_device", "readout_grad_device",
            "reservoir_trace_phases", "reservoir_phase_times", "reservoir_adjoint_kernels",
            "sto_read_bandwidth", "sto_set_stream_variant", "sto_last_error")

SCALAR_NAMES = ("a_cp", "a_in", "h_s", "h_appl")


def lib():
    return _lib


def sto_last_error() -> str:
    return _lib.sto_last_error().decode()


def _check(status: int):
    if status != STO_OK:
        raise StoError(status, sto_last_error())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def reservoir_create(n: int, n_in: int, prm: sto_params, W, w_in, m0) -> ctypes.c_void_p:
    W = _f64(W, (n, n))
    w_in = _f64(w_in, (n, n_in))
    m0 = _f64(m0, (n, 3))
    h = ctypes.c_void_p()
    _check(_lib.reservoir_create(n, n_in, ctypes.byref(prm), _dptr(W), _dptr(w_in), _dptr(m0), ctypes.byref(h)))
    return h


def reservoir_create_streams(n: int, n_in: int, streams: int, prm: sto_params, W, w_in, m0) -> ctypes.c_void_p:
    W = _f64(W, (n, n))
    w_in = _f64(w_in, (n, n_in))
    m0 = _f64(m0, (streams, n, 3))
    h = ctypes.c_void_p()
    _check(_lib.reservoir_create_streams(n, n_in, streams, ctypes.byref(prm), _dptr(W), _dptr(w_in), _dptr(m0),
                                         ctypes.byref(h)))
    return h


def _addr(ptr: Optional[int]):
    """A device address (an int) as a void pointer; None or 0 is NULL."""
    return ctypes.c_void_p(ptr) if ptr else None


def reservoir_create_device(n: int, n_in: int, streams: int, prm: sto_params, W_ptr: int, w_in_ptr: int,
                            m0_ptr: int, stream_ptr: Optional[int]) -> ctypes.c_void_p:
    """Device pointers of doubles: W (n, n), w_in (n, n_in), m0 (streams, n, 3)."""
    h = ctypes.c_void_p()
    _check(_lib.reservoir_create_device(n, n_in, streams, ctypes.byref(prm), _addr(W_ptr), _addr(w_in_ptr), _addr(m0_ptr),
                                        _addr(stream_ptr), ctypes.byref(h)))
    return h


def reservoir_load_device(h, W_ptr: Optional[int], w_in_ptr: Optional[int], m_ptr: Optional[int],
                          prm: Optional[sto_params], stream_ptr: Optional[int]):
    _check(_lib.reservoir_load_device(h, _addr(W_ptr), _addr(w_in_ptr), _addr(m_ptr),
                                      ctypes.byref(prm) if prm is not None else None, _addr(stream_ptr)))


def reservoir_streams(h) -> int:
    return int(_lib.reservoir_streams(h))


def reservoir_run(h, u, steps: int, states: Optional[np.ndarray] = None):
    """u: (samples, n_in) float64; states: None or a C-contiguous float64
    array of (samples, n, 3) that receives the records."""
    u = _f64(u)
    if states is not None:
        assert states.dtype == np.float64 and states.flags.c_contiguous
    _check(_lib.reservoir_run(h, _dptr(u), steps, _dptr(states) if states is not None else None))


def reservoir_run_device(h, u_dev_ptr: int, steps: int, states_dev_ptr: Optional[int], stream_ptr: Optional[int]):
    _check(_lib.reservoir_run_device(h, ctypes.c_void_p(u_dev_ptr), steps,
                                     ctypes.c_void_p(states_dev_ptr) if states_dev_ptr else None,
                                     ctypes.c_void_p(stream_ptr) if stream_ptr else None))


def reservoir_get_state(h, n: int) -> np.ndarray:
    m = np.empty((n, 3))
    _check(_lib.reservoir_get_state(h, _dptr(m)))
    return m


def reservoir_set_state(h, m):
    m = _f64(m)
    _check(_lib.reservoir_set_state(h, _dptr(m)))


def reservoir_path(h) -> int:
    return int(_lib.reservoir_path(h))


ADJ_FWD_STAGE, ADJ_FWD_PERSISTENT, ADJ_REV_STAGE, ADJ_REV_PERSISTENT = 1, 2, 4, 8


def reservoir_adjoint_kernels(h) -> int:
    return int(_lib.reservoir_adjoint_kernels(h))


def reservoir_trace_phases(h, stages: int):
    _check(_lib.reservoir_trace_phases(h, stages))


def reservoir_phase_times(h):
    """(stamps [group][stage][point] as uint64, clock rate in kHz)."""
    g, st, khz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.reservoir_phase_times(h, None, 0, ctypes.byref(g), ctypes.byref(st), ctypes.byref(khz)))
    out = np.zeros((g.value, st.value, 4), dtype=np.uint64)
    if out.size:
        _check(_lib.reservoir_phase_times(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), out.size,
                                          ctypes.byref(g), ctypes.byref(st), ctypes.byref(khz)))
    return out, int(khz.value)


def reservoir_destroy(h):
    if h:
        _lib.reservoir_destroy(h)


def readout_fit(states, y, washout: int, lam: float, features: int = 0) -> Tuple[np.ndarray, float]:
    states = _f64(states)
    T, n, _ = states.shape
    y = _f64(y).ravel()
    cols = (3 * n if features else n) + 1
    w = np.empty(cols)
    nmse = np.empty(1)
    _check(_lib.readout_fit(_dptr(states), T, n, _dptr(y), washout, lam, features, _dptr(w), _dptr(nmse)))
    return w, float(nmse[0])


def readout_fit_device(states_dev, y_dev, washout: int, lam: float, features: int = 0, w_out_dev=None,
                       stream=None) -> float:
    """states_dev: CUDA float32/float64 tensor (T, n, 3); y_dev: CUDA float64
    tensor (T,); w_out_dev: CUDA float64 tensor of F + 1 weights (allocated
    if None).  Returns (w_out_dev, nmse)."""
    import torch
    assert states_dev.is_cuda and states_dev.is_contiguous() and states_dev.dim() == 3
    assert y_dev.is_cuda and y_dev.dtype == torch.float64 and y_dev.is_contiguous()
    T, n, _ = states_dev.shape
    cols = (3 * n if features else n) + 1
    if w_out_dev is None:
        w_out_dev = torch.empty(cols, dtype=torch.float64, device=states_dev.device)
    assert w_out_dev.dtype == torch.float64 and w_out_dev.numel() == cols
    dtype = {torch.float64: STO_F64, torch.float32: STO_F32}[states_dev.dtype]
    nmse = np.empty(1)
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(_lib.readout_fit_device(ctypes.c_void_p(states_dev.data_ptr()), dtype, T, n,
                                   ctypes.c_void_p(y_dev.data_ptr()), washout, lam, features,
                                   ctypes.c_void_p(w_out_dev.data_ptr()), _dptr(nmse), ctypes.c_void_p(s)))
    return w_out_dev, float(nmse[0])


def readout_fit_device_noalloc(states_dev, y_dev, washout: int, lam: float, w_out_dev, features: int = 0,
                               stream=None) -> float:
    """readout_fit_device with its workspace in the library's static device
    array (no device allocation; w_out_dev must be given).  Returns nmse."""
    import torch
    assert states_dev.is_cuda and states_dev.is_contiguous() and states_dev.dim() == 3
    assert y_dev.is_cuda and y_dev.dtype == torch.float64 and y_dev.is_contiguous()
    T, n, _ = states_dev.shape
    cols = (3 * n if features else n) + 1
    assert w_out_dev.is_cuda and w_out_dev.dtype == torch.float64 and w_out_dev.numel() == cols
    dtype = {torch.float64: STO_F64, torch.float32: STO_F32}[states_dev.dtype]
    nmse = np.empty(1)
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(_lib.readout_fit_device_noalloc(ctypes.c_void_p(states_dev.data_ptr()), dtype, T, n,
                                           ctypes.c_void_p(y_dev.data_ptr()), washout, lam, features,
                                           ctypes.c_void_p(w_out_dev.data_ptr()), _dptr(nmse), ctypes.c_void_p(s)))
    return float(nmse[0])


def readout_fit_batch_device(states_list, y_dev, washout: int, lam: float, features: int = 0, w_list=None,
                             stream=None):
    """Fit one readout per record set, all at once.  states_list: CUDA
    float32/float64 tensors of shape (T, n_q, 3) with contiguous records
    (strides (r, 3, 1) for any row stride r, e.g. states[:, q] of a
    (T, S, n, 3) multi-stream record tensor); y_dev: one CUDA float64 (T,)
    target tensor shared by all, or a list of one per record set; w_list:
    CUDA float64 tensors of F_q + 1 weights (allocated if None).  Returns
    (w_list, nmse array)."""
    import torch
    assert len(states_list) >= 1
    y_list = list(y_dev) if isinstance(y_dev, (list, tuple)) else [y_dev] * len(states_list)
    assert len(y_list) == len(states_list)
    T = states_list[0].shape[0]
    dt = states_list[0].dtype
    count = len(states_list)
    ptrs = (ctypes.c_void_p * count)()
    strides = (ctypes.c_int64 * count)()
    ns = (ctypes.c_int64 * count)()
    if w_list is None:
        w_list = [None] * count
    w_list = list(w_list)
    wptrs = (ctypes.c_void_p * count)()
    yptrs = (ctypes.c_void_p * count)()
    for q, st in enumerate(states_list):
        yq = y_list[q]
        assert yq.is_cuda and yq.dtype == torch.float64 and yq.is_contiguous() and yq.numel() == T
        yptrs[q] = yq.data_ptr()
        assert st.is_cuda and st.dim() == 3 and st.shape[0] == T and st.shape[2] == 3 and st.dtype == dt
        assert st.stride(2) == 1 and st.stride(1) == 3, "records of one row must be contiguous (n, 3)"
        n = st.shape[1]
        cols = (3 * n if features else n) + 1
        if w_list[q] is None:
            w_list[q] = torch.empty(cols, dtype=torch.float64, device=st.device)
        assert w_list[q].dtype == torch.float64 and w_list[q].numel() == cols and w_list[q].is_contiguous()
        ptrs[q] = st.data_ptr()
        strides[q] = st.stride(0)
        ns[q] = n
        wptrs[q] = w_list[q].data_ptr()
    dtype = {torch.float64: STO_F64, torch.float32: STO_F32}[dt]
    nmse = np.empty(count)
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(_lib.readout_fit_batch_device(count, ptrs, strides, dtype, T, ns, yptrs, washout, lam, features, wptrs,
                                         _dptr(nmse), ctypes.c_void_p(s)))
    return w_list, nmse


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def reservoir_adjoint(h, n: int, n_in: int, substeps: int, m_start, u, steps: int, grad_states=None,
                      grad_final=None, checkpoint_every: int = 0) -> dict:
    """Host arrays in and out (float64).  Returns {"W", "w_in", "m0", "a_cp",
    "a_in", "h_s", "h_appl"}: the gradients of the loss whose gradient with
    respect to the records is grad_states (and to the final state grad_final).
    For a handle of S > 1 streams, m_start, grad_final and "m0" are
    (S, n, 3), u is (samples, S, n_in) and grad_states (samples, S, n, 3).
    Every array is sized from the handle's own S before the call."""
    streams = reservoir_streams(h)
    if streams < 1:
        raise StoError(STO_E_INVALID, "invalid handle")
    samples = max(0, steps) // substeps
    m_start = _f64(m_start, (streams * n, 3))
    u = _f64(u)
    if u.size < samples * streams * n_in:
        raise ValueError("u holds fewer than steps/substeps * streams * n_in values")
    gs = _f64(grad_states, (samples * streams * n, 3)) if grad_states is not None else None
    gf = _f64(grad_final, (streams * n, 3)) if grad_final is not None else None
    m0_shape = (n, 3) if streams == 1 else (streams, n, 3)
    out = {"W": np.empty((n, n)), "w_in": np.empty((n, n_in)), "m0": np.empty(m0_shape)}
    scal = np.empty(4)
    _check(_lib.reservoir_adjoint(h, _dptr(m_start), _dptr(u), steps, _dptr(gs) if gs is not None else None,
                                  _dptr(gf) if gf is not None else None, _dptr(out["W"]), _dptr(out["w_in"]),
                                  _dptr(out["m0"]), _dptr(scal), checkpoint_every))
    out.update({k: float(v) for k, v in zip(SCALAR_NAMES, scal)})
    return out


def reservoir_adjoint_device(h, m_start_dev, u_dev, steps: int, grad_states_dev=None, grad_final_dev=None,
                             grad_W_dev=None, grad_w_in_dev=None, grad_m0_dev=None, grad_scalars_dev=None,
                             checkpoint_every: int = 0, stream=None, records_dev=None):
    """CUDA tensors of the handle's dtype (u and the scalars float64); every
    output tensor may be None to skip it.  With records_dev (the run's
    records) the call is reservoir_adjoint_records_device."""
    import torch
    s = (stream or torch.cuda.current_stream()).cuda_stream
    if records_dev is None:
        _check(_lib.reservoir_adjoint_device(h, _vp(m_start_dev), _vp(u_dev), steps, _vp(grad_states_dev),
                                             _vp(grad_final_dev), _vp(grad_W_dev), _vp(grad_w_in_dev),
                                             _vp(grad_m0_dev), _vp(grad_scalars_dev), checkpoint_every,
                                             ctypes.c_void_p(s)))
    else:
        _check(_lib.reservoir_adjoint_records_device(h, _vp(m_start_dev), _vp(u_dev), steps, _vp(records_dev),
                                                     _vp(grad_states_dev), _vp(grad_final_dev), _vp(grad_W_dev),
                                                     _vp(grad_w_in_dev), _vp(grad_m0_dev), _vp(grad_scalars_dev),
                                                     checkpoint_every, ctypes.c_void_p(s)))


def readout_grad_device(states_dev, y_dev, washout: int, lam: float, w_dev, features: int = 0, grad_dev=None,
                        stream=None):
    """Ridge objective at its optimum J and dJ/d(records) (CUDA tensor like
    states_dev).  Returns (grad_dev, J)."""
    import torch
    assert states_dev.is_cuda and states_dev.is_contiguous() and states_dev.dim() == 3
    assert y_dev.is_cuda and y_dev.dtype == torch.float64 and y_dev.is_contiguous()
    assert w_dev.is_cuda and w_dev.dtype == torch.float64 and w_dev.is_contiguous()
    T, n, _ = states_dev.shape
    if grad_dev is None:
        grad_dev = torch.empty_like(states_dev)
    assert grad_dev.dtype == states_dev.dtype and grad_dev.shape == states_dev.shape and grad_dev.is_contiguous()
    dtype = {torch.float64: STO_F64, torch.float32: STO_F32}[states_dev.dtype]
    loss = np.empty(1)
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(_lib.readout_grad_device(_vp(states_dev), dtype, T, n, _vp(y_dev), washout, lam, features, _vp(w_dev),
                                    _vp(grad_dev), _dptr(loss), ctypes.c_void_p(s)))
    return grad_dev, float(loss[0])


def sto_set_stream_variant(rows: int, unroll: int):
    """Launch shape of the stream kernels for this process ((0, 0): table)."""
    _check(_lib.sto_set_stream_variant(rows, unroll))


def sto_read_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Attainable HBM read bandwidth (GB/s) of a plain streaming kernel."""
    out = np.empty(1)
    _check(_lib.sto_read_bandwidth(nbytes, reps, _dptr(out)))
    return float(out[0])


class Reservoir:
    """Owns one library handle; every method calls the C entry point of the same name.

    With streams > 1, m0 is (streams, n, 3), u is (samples, streams, n_in)
    and the records are (samples, streams, n, 3)."""

    def __init__(self, W, w_in, m0, prm: sto_params, streams: int = 1):
        W = np.asarray(W)
        self.n = W.shape[0]
        w_in = np.asarray(w_in, dtype=np.float64).reshape(self.n, -1)
        self.n_in = w_in.shape[1]
        self.streams = int(streams)
        self.substeps = prm.substeps
        self.dtype = "f64" if prm.dtype == STO_F64 else "f32"
        if self.streams == 1:
            self.h = reservoir_create(self.n, self.n_in, prm, W, w_in, m0)
        else:
            self.h = reservoir_create_streams(self.n, self.n_in, self.streams, prm, W, w_in, m0)

    @classmethod
    def from_device(cls, W_dev, w_in_dev, m0_dev, prm: sto_params, streams: int = 1, stream=None) -> "Reservoir":
        """A handle built from CUDA float64 tensors (reservoir_create_device):
        W (n, n), w_in (n, n_in), m0 ([streams,] n, 3)."""
        import torch
        self = cls.__new__(cls)
        self.n = int(W_dev.shape[0])
        self.n_in = int(w_in_dev.numel() // self.n)
        self.streams = int(streams)
        self.substeps = prm.substeps
        self.dtype = "f64" if prm.dtype == STO_F64 else "f32"
        self._check_device(W_dev, (self.n, self.n))
        self._check_device(w_in_dev, (self.n * self.n_in,))
        self._check_device(m0_dev, (self.streams * self.n * 3,))
        s = (stream or torch.cuda.current_stream()).cuda_stream
        self.h = reservoir_create_device(self.n, self.n_in, self.streams, prm, W_dev.data_ptr(), w_in_dev.data_ptr(),
                                         m0_dev.data_ptr(), s)
        return self

    @staticmethod
    def _check_device(t, shape):
        import torch
        assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "a contiguous CUDA float64 tensor"
        assert t.numel() == int(np.prod(shape)), f"{tuple(t.shape)} does not hold {shape}"

    def load_device(self, W_dev=None, w_in_dev=None, m_dev=None, prm: Optional[sto_params] = None, stream=None):
        """Replace W, w_in, the state and/or the constants from CUDA float64
        tensors (reservoir_load_device); None keeps the current one."""
        import torch
        if W_dev is not None:
            self._check_device(W_dev, (self.n, self.n))
        if w_in_dev is not None:
            self._check_device(w_in_dev, (self.n * self.n_in,))
        if m_dev is not None:
            self._check_device(m_dev, (self.streams * self.n * 3,))
        s = (stream or torch.cuda.current_stream()).cuda_stream
        ptr = lambda t: t.data_ptr() if t is not None else None
        reservoir_load_device(self.h, ptr(W_dev), ptr(w_in_dev), ptr(m_dev), prm, s)
        if prm is not None:
            self.substeps = prm.substeps

    @property
    def path(self) -> str:
        return PATH_NAMES[reservoir_path(self.h)]

    def _record_shape(self, samples):
        return (samples, self.n, 3) if self.streams == 1 else (samples, self.streams, self.n, 3)

    def run(self, u, record: bool = True) -> Optional[np.ndarray]:
        u = _f64(u).reshape(-1, self.streams * self.n_in)
        steps = len(u) * self.substeps
        states = np.empty(self._record_shape(len(u))) if record else None
        reservoir_run(self.h, u, steps, states)
        return states

    def run_device(self, u_dev, states_dev=None, stream=None):
        """u_dev: CUDA float64 tensor (samples, [streams,] n_in); states_dev:
        CUDA tensor (samples, [streams,] n, 3) of the handle's dtype, or None;
        stream: a torch.cuda.Stream (default: the current stream)."""
        import torch
        assert u_dev.is_cuda and u_dev.dtype == torch.float64 and u_dev.is_contiguous()
        samples = u_dev.numel() // (self.n_in * self.streams)
        if states_dev is not None:
            want = torch.float64 if self.dtype == "f64" else torch.float32
            assert states_dev.is_cuda and states_dev.dtype == want and states_dev.is_contiguous()
            assert states_dev.numel() == samples * self.streams * self.n * 3
        s = (stream or torch.cuda.current_stream()).cuda_stream
        reservoir_run_device(self.h, u_dev.data_ptr(), samples * self.substeps,
                             states_dev.data_ptr() if states_dev is not None else None, s)

    def adjoint(self, m_start, u, grad_states=None, grad_final=None, checkpoint_every: int = 0) -> dict:
        """Gradients (host, float64) of the run from m_start over u; see reservoir_adjoint."""
        u = _f64(u).reshape(-1, self.streams * self.n_in)
        return reservoir_adjoint(self.h, self.n, self.n_in, self.substeps, m_start, u, len(u) * self.substeps,
                                 grad_states, grad_final, checkpoint_every)

    def adjoint_device(self, m_start_dev, u_dev, grad_states_dev=None, grad_final_dev=None, want=("W", "w_in", "m0",
                       "scalars"), checkpoint_every: int = 0, stream=None, records_dev=None) -> dict:
        """Gradients as CUDA tensors of the handle's dtype (scalars: float64 (4,)).
        records_dev: the records of the run from m_start_dev over u_dev, used
        as the checkpoints (checkpoint_every a multiple of substeps)."""
        import torch
        dt = torch.float64 if self.dtype == "f64" else torch.float32
        dev = u_dev.device
        out = {}
        if "W" in want:
            out["W"] = torch.empty((self.n, self.n), dtype=dt, device=dev)
        if "w_in" in want:
            out["w_in"] = torch.empty((self.n, self.n_in), dtype=dt, device=dev)
        if "m0" in want:
            out["m0"] = torch.empty(((self.n, 3) if self.streams == 1 else (self.streams, self.n, 3)), dtype=dt,
                                    device=dev)
        if "scalars" in want:
            out["scalars"] = torch.empty(4, dtype=torch.float64, device=dev)
        samples = u_dev.numel() // (self.n_in * self.streams)
        # every buffer is checked against the handle's shape before the call
        per = self.streams * self.n
        assert u_dev.is_cuda and u_dev.dtype == torch.float64 and u_dev.is_contiguous()
        assert u_dev.numel() == samples * self.streams * self.n_in
        for t, count in ((m_start_dev, per * 3), (grad_states_dev, samples * per * 3), (grad_final_dev, per * 3),
                         (records_dev, samples * per * 3)):
            if t is not None:
                assert t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == count
        reservoir_adjoint_device(self.h, m_start_dev, u_dev, samples * self.substeps, grad_states_dev,
                                 grad_final_dev, out.get("W"), out.get("w_in"), out.get("m0"), out.get("scalars"),
                                 checkpoint_every, stream, records_dev)
        return out

    @property
    def adjoint_kernels(self) -> dict:
        """Kernel families of the last adjoint call on this handle."""
        m = reservoir_adjoint_kernels(self.h)
        return {"forward": ("persistent" if m & ADJ_FWD_PERSISTENT else "stage" if m & ADJ_FWD_STAGE else None),
                "reverse": ("persistent" if m & ADJ_REV_PERSISTENT else "stage" if m & ADJ_REV_STAGE else None)}

    def trace_phases(self, stages: int):
        """Arm (stages > 0) or free (0) the phase trace of the persistent paths."""
        reservoir_trace_phases(self.h, stages)

    def phase_times(self):
        """Stamps of the last run: (uint64 [group][stage][point], clock kHz)."""
        return reservoir_phase_times(self.h)

    def get_state(self) -> np.ndarray:
        m = reservoir_get_state(self.h, self.n * self.streams)
        return m if self.streams == 1 else m.reshape(self.streams, self.n, 3)

    def set_state(self, m):
        reservoir_set_state(self.h, np.asarray(m, dtype=np.float64).reshape(self.streams * self.n, 3))

    def close(self):
        if getattr(self, "h", None):
            reservoir_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sweep:
    """Many independent reservoirs stepped together (calls the sweep_* entry points).

    reservoirs: list of dicts with "W", "w_in", "m0" and a ``sto_params`` under
    "prm".  Records come back as a list with one (samples, n_r, 3) array per
    reservoir (host run), or as one device tensor laid out
    [reservoir][sample][node][xyz] (device run)."""

    def __init__(self, reservoirs):
        self.count = len(reservoirs)
        self.ns = [int(np.asarray(r["W"]).shape[0]) for r in reservoirs]
        self.n_in = int(np.asarray(reservoirs[0]["w_in"], dtype=np.float64).reshape(self.ns[0], -1).shape[1])
        self._keep = []
        dp = ctypes.POINTER(ctypes.c_double)

        def arr(key, shape_fn):
            ptrs = (dp * self.count)()
            for i, r in enumerate(reservoirs):
                a = _f64(r[key], shape_fn(i))
                self._keep.append(a)
                ptrs[i] = _dptr(a)
            return ptrs

        W = arr("W", lambda i: (self.ns[i], self.ns[i]))
        w_in = arr("w_in", lambda i: (self.ns[i], self.n_in))
        m0 = arr("m0", lambda i: (self.ns[i], 3))
        prms = (sto_params * self.count)(*[r["prm"] for r in reservoirs])
        nn = (ctypes.c_int64 * self.count)(*self.ns)
        self.substeps = prms[0].substeps
        self.dtype = "f64" if prms[0].dtype == STO_F64 else "f32"
        self.h = ctypes.c_void_p()
        _check(_lib.sweep_create(self.count, nn, self.n_in, prms, W, w_in, m0, ctypes.byref(self.h)))
        self._keep = []
        self.nodes = int(_lib.sweep_nodes(self.h))
        self.offsets = np.concatenate([[0], np.cumsum(self.ns)])

    def run(self, u, record: bool = True):
        u = _f64(u).reshape(-1, self.n_in)
        samples = len(u)
        states = np.empty(samples * self.nodes * 3) if record else None
        _check(_lib.sweep_run(self.h, _dptr(u), samples * self.substeps, _dptr(states) if record else None))
        if not record:
            return None
        return [states[samples * 3 * self.offsets[i]: samples * 3 * self.offsets[i + 1]].reshape(samples, n, 3)
                for i, n in enumerate(self.ns)]

    def run_device(self, u_dev, states_dev=None, stream=None):
        import torch
        assert u_dev.is_cuda and u_dev.dtype == torch.float64 and u_dev.is_contiguous()
        samples = u_dev.numel() // self.n_in
        if states_dev is not None:
            assert states_dev.is_cuda and states_dev.is_contiguous() and states_dev.numel() == samples * self.nodes * 3
        s = (stream or torch.cuda.current_stream()).cuda_stream
        _check(_lib.sweep_run_device(self.h, ctypes.c_void_p(u_dev.data_ptr()), samples * self.substeps,
                                     ctypes.c_void_p(states_dev.data_ptr()) if states_dev is not None else None,
                                     ctypes.c_void_p(s)))

    def get_state(self):
        m = np.empty((self.nodes, 3))
        _check(_lib.sweep_get_state(self.h, _dptr(m)))
        return [m[self.offsets[i]:self.offsets[i + 1]] for i in range(self.count)]

    def close(self):
        if getattr(self, "h", None):
            _lib.sweep_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
