"""Host-side checks of the HIP library that need no GPU.

* the shared library loads and exports every function include/*.h declares;
* invalid arguments are rejected before any device work;
* the library's own Table 1 presets equal the oracle's constants bit for bit.
"""

import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def stx():
    if not os.path.exists(os.path.join(ROOT, "paper_2312_01121_amd", "libsto_reservoir.so")):
        import __graft_entry__
        __graft_entry__.build()   # loads the build script by path, not through the package
    import paper_2312_01121_amd
    return paper_2312_01121_amd


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("reservoir_create", "reservoir_run", "reservoir_run_device", "reservoir_get_state",
               "reservoir_set_state", "reservoir_path", "reservoir_destroy", "readout_fit", "sto_last_error"):
        assert fn in names


def test_library_exports_every_declared_symbol(stx):
    lib = ctypes.CDLL(stx.LIB_PATH)
    for fn in declared_functions():
        assert hasattr(lib, fn), fn
    assert set(stx.EXPORTED) <= set(declared_functions())


def _ok_params(stx, **kw):
    from paper_2312_01121_amd import params
    p = params.table1()
    p.update(kw)
    return stx.make_params(**p)


def test_create_rejects_bad_arguments(stx):
    n = 4
    w = np.zeros((n, n))
    w_in = np.zeros((n, 1))
    m0 = np.tile([0.0, 0.0, 1.0], (n, 1))
    h = ctypes.c_void_p()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    lib = stx.lib()
    prm = _ok_params(stx)

    def create(nn=n, nin=1, pr=prm, W=w, m=m0):
        return lib.reservoir_create(nn, nin, ctypes.byref(pr), dp(W), dp(w_in), dp(m), ctypes.byref(h))

    assert create(nn=0) == stx.STO_E_INVALID
    assert create(nin=0) == stx.STO_E_INVALID
    assert create(pr=_ok_params(stx, dt=0.0)) == stx.STO_E_INVALID
    assert create(pr=_ok_params(stx, substeps=0)) == stx.STO_E_INVALID
    bad = _ok_params(stx)
    bad.dtype = 7
    assert create(pr=bad) == stx.STO_E_INVALID
    bad = _ok_params(stx)
    bad.reserved = 1
    assert create(pr=bad) == stx.STO_E_INVALID
    m_bad = m0.copy()
    m_bad[1] = [0.0, 0.0, 1.0 + 1e-9]
    assert create(m=m_bad) == stx.STO_E_INVALID
    assert "m0[1]" in stx.sto_last_error()
    w_nan = w.copy()
    w_nan[0, 1] = np.nan
    assert create(W=w_nan) == stx.STO_E_NONFINITE
    assert lib.reservoir_create(n, 1, ctypes.byref(prm), None, dp(w_in), dp(m0), ctypes.byref(h)) == stx.STO_E_INVALID
    big = _ok_params(stx, path="small")
    wb = np.zeros((400, 400))
    assert lib.reservoir_create(400, 1, ctypes.byref(big), dp(wb), dp(np.zeros((400, 1))),
                                dp(np.tile([0.0, 0.0, 1.0], (400, 1))), ctypes.byref(h)) == stx.STO_E_UNSUPPORTED


def test_readout_rejects_bad_arguments(stx):
    lib = stx.lib()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    rec = np.zeros((10, 3, 3))
    y = np.zeros(10)
    w = np.zeros(4)
    e = np.zeros(1)
    assert lib.readout_fit(dp(rec), 10, 3, dp(y), 10, 1e-6, 0, dp(w), dp(e)) == stx.STO_E_INVALID
    assert lib.readout_fit(dp(rec), 10, 3, dp(y), 2, -1.0, 0, dp(w), dp(e)) == stx.STO_E_INVALID
    assert lib.readout_fit(dp(rec), 10, 3, dp(y), 2, 1e-6, 2, dp(w), dp(e)) == stx.STO_E_INVALID
    y[4] = np.nan
    assert lib.readout_fit(dp(rec), 10, 3, dp(y), 2, 1e-6, 0, dp(w), dp(e)) == stx.STO_E_NONFINITE


def test_null_handle_is_rejected(stx):
    lib = stx.lib()
    u = np.zeros(4)
    assert lib.reservoir_run(None, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 20, None) == stx.STO_E_INVALID
    assert lib.reservoir_path(None) == -1
    lib.reservoir_destroy(None)


def test_presets_equal_oracle_constants(stx):
    """The library's Table 1 conversion and the oracle's give identical bits."""
    from oracle import constants
    from paper_2312_01121_amd import params
    for cs, fs in ((1.0, 1.0), (0.7, 1.3)):
        a = params.table1(current_scale=cs, field_scale=fs)
        b = constants.dimensionless(current_scale=cs, field_scale=fs)
        assert a["alpha"] == b.alpha and a["lambda_stt"] == b.lam and a["dt"] == b.dt
        assert a["h_appl"] == b.h_appl and a["h_k"] == b.h_k and a["h_s"] == b.h_s
        assert tuple(a["p"]) == tuple(b.p)


def test_adjoint_rejects_bad_arguments(stx):
    """Argument errors of the adjoint and the readout gradient come back
    before any device work."""
    lib = stx.lib()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    m = np.zeros((4, 3))
    u = np.zeros(4)
    assert lib.reservoir_adjoint(None, dp(m), dp(u), 20, None, None, None, None, None, None, 0) == stx.STO_E_INVALID
    assert lib.reservoir_adjoint_device(None, None, None, 20, None, None, None, None, None, None, 0,
                                        None) == stx.STO_E_INVALID
    # the records variant: records NULL, then a NULL handle
    assert lib.reservoir_adjoint_records_device(None, None, None, 20, None, None, None, None, None, None, None, 0,
                                                None) == stx.STO_E_INVALID
    assert lib.reservoir_adjoint_records_device(None, None, None, 20, m.ctypes.data, None, None, None, None, None,
                                                None, 0, None) == stx.STO_E_INVALID
    assert lib.readout_grad_device(None, 0, 10, 3, None, 2, 1e-6, 0, None, None, None, None) == stx.STO_E_INVALID



def test_readout_batch_rejects_bad_arguments(stx):
    """Argument errors of the batched readout come back before any device
    work: no items, NULL arrays, a stride below 3 n, a bad washout."""
    lib = stx.lib()
    vp = ctypes.c_void_p
    one = (vp * 1)(vp(16))
    n = (ctypes.c_int64 * 1)(4)
    w = (vp * 1)(vp(16))
    nmse = np.zeros(1)
    nm = nmse.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    y = (vp * 1)(vp(16))
    assert lib.readout_fit_batch_device(0, one, None, 0, 10, n, y, 2, 1e-6, 0, w, nm, None) == stx.STO_E_INVALID
    assert lib.readout_fit_batch_device(1, None, None, 0, 10, n, y, 2, 1e-6, 0, w, nm, None) == stx.STO_E_INVALID
    assert lib.readout_fit_batch_device(1, one, None, 0, 10, n, None, 2, 1e-6, 0, w, nm, None) == stx.STO_E_INVALID
    short = (ctypes.c_int64 * 1)(11)
    assert lib.readout_fit_batch_device(1, one, short, 0, 10, n, y, 2, 1e-6, 0, w, nm, None) == stx.STO_E_INVALID
    assert lib.readout_fit_batch_device(1, one, None, 0, 10, n, y, 10, 1e-6, 0, w, nm, None) == stx.STO_E_INVALID
    assert lib.readout_fit_batch_device(65536, one, None, 0, 10, n, y, 2, 1e-6, 0, w, nm, None) == stx.STO_E_INVALID


# ----------------------------------------------------------------------------
# Host buffers the binding hands to the library are as large as the header says
# ----------------------------------------------------------------------------
class _FakeLib:
    """Stands in for the shared library: every entry point checks that each
    host buffer it receives holds at least the number of doubles the header
    (include/sto_reservoir.h) says the library reads or writes there, and
    then writes its full extent, as the real library does.  The sizes come
    from a registry of the arrays the binding converted to pointers."""

    def __init__(self, registry, n, n_in, streams):
        self.reg, self.n, self.n_in, self.S = registry, n, n_in, streams
        self.substeps = None
        self.calls = []

    def _need(self, p, count, name, write=False):
        if p is None:
            return
        addr = ctypes.cast(p, ctypes.c_void_p).value
        have = self.reg.get(addr)
        assert have is not None, f"{name}: pointer not from a registered array"
        assert have >= 8 * count, f"{name}: {have} bytes, the library uses {8 * count}"
        if write:
            np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_double)), shape=(count,))[:] = 0.5

    def reservoir_create(self, n, n_in, prm, W, w_in, m0, hp):
        self.substeps = prm._obj.substeps
        self._need(W, n * n, "W"), self._need(w_in, n * n_in, "w_in"), self._need(m0, n * 3, "m0")
        hp._obj.value = 1
        return 0

    def reservoir_create_streams(self, n, n_in, S, prm, W, w_in, m0, hp):
        self.substeps = prm._obj.substeps
        self._need(W, n * n, "W"), self._need(w_in, n * n_in, "w_in"), self._need(m0, S * n * 3, "m0")
        hp._obj.value = 1
        return 0

    def reservoir_streams(self, h):
        return self.S

    def reservoir_path(self, h):
        return 2

    def reservoir_run(self, h, u, steps, states):
        samples = steps // self.substeps
        self._need(u, samples * self.S * self.n_in, "u")
        self._need(states, samples * self.S * self.n * 3, "states", write=True)
        self.calls.append("run")
        return 0

    def reservoir_get_state(self, h, m):
        self._need(m, self.S * self.n * 3, "m", write=True)
        self.calls.append("get_state")
        return 0

    def reservoir_set_state(self, h, m):
        self._need(m, self.S * self.n * 3, "m")
        return 0

    def reservoir_adjoint(self, h, m_start, u, steps, gs, gf, gW, gwin, gm0, gsc, ce):
        samples = steps // self.substeps
        per = self.S * self.n
        self._need(m_start, per * 3, "m_start"), self._need(u, samples * self.S * self.n_in, "u")
        self._need(gs, samples * per * 3, "grad_states"), self._need(gf, per * 3, "grad_final")
        self._need(gW, self.n * self.n, "grad_W", True), self._need(gwin, self.n * self.n_in, "grad_w_in", True)
        self._need(gm0, per * 3, "grad_m0", True), self._need(gsc, 4, "grad_scalars", True)
        self.calls.append("adjoint")
        return 0

    def reservoir_destroy(self, h):
        pass

    def sto_last_error(self):
        return b""


@pytest.mark.parametrize("streams", [1, 3])
def test_binding_host_buffers_have_the_header_sizes(stx, monkeypatch, streams):
    """Guards the host arrays of reservoir_run, reservoir_get_state and
    reservoir_adjoint for one stream and several: a binding that sized an
    output for one stream while the library writes S of them overran the
    heap (glibc reported the corruption later, in an unrelated free)."""
    registry = {}
    real_dptr = stx._dptr

    def dptr(a):
        registry[a.ctypes.data] = a.nbytes
        return real_dptr(a)

    n, n_in, samples = 6, 2, 4
    fake = _FakeLib(registry, n, n_in, streams)
    monkeypatch.setattr(stx, "_dptr", dptr)
    monkeypatch.setattr(stx, "_lib", fake)
    rng = np.random.default_rng(0)
    m0 = rng.standard_normal((n, 3)) if streams == 1 else rng.standard_normal((streams, n, 3))
    r = stx.Reservoir(rng.standard_normal((n, n)), rng.standard_normal((n, n_in)), m0,
                      _ok_params(stx, substeps=5), streams=streams)
    u = rng.standard_normal((samples, streams, n_in))
    rec = r.run(u)
    assert rec.size == samples * streams * n * 3 and np.all(rec == 0.5)
    st = r.get_state()
    assert st.size == streams * n * 3 and np.all(st == 0.5)
    r.set_state(st)
    g = rng.standard_normal(rec.shape)
    out = r.adjoint(m0, u, grad_states=g, grad_final=st)
    assert out["m0"].size == streams * n * 3 and np.all(out["m0"] == 0.5)
    assert out["W"].shape == (n, n) and out["w_in"].shape == (n, n_in)
    assert fake.calls == ["run", "get_state", "adjoint"]
    r.close()


def test_fake_library_catches_an_undersized_output(stx, monkeypatch):
    """The check above fails for a buffer one stream short (the mistake it guards)."""
    registry = {}
    fake = _FakeLib(registry, 4, 1, 2)
    buf = np.empty((4, 3))                       # room for one stream only
    registry[buf.ctypes.data] = buf.nbytes
    with pytest.raises(AssertionError, match="grad_m0"):
        fake._need(stx._dptr(buf), 2 * 4 * 3, "grad_m0", write=True)


def test_device_load_bindings_pass_addresses(stx, monkeypatch):
    """reservoir_create_device / reservoir_load_device hand the device
    addresses through unchanged, NULL for an absent array or parameter set."""
    seen = []

    class Fake:
        def reservoir_create_device(self, n, n_in, S, prm, W, w_in, m0, stream, hp):
            seen.append(("create", n, n_in, S, prm._obj.substeps, W.value, w_in.value, m0.value,
                         stream.value if stream is not None else None))
            hp._obj.value = 7
            return 0

        def reservoir_load_device(self, h, W, w_in, m, prm, stream):
            val = lambda p: p.value if p is not None else None  # noqa: E731
            seen.append(("load", h.value, val(W), val(w_in), val(m), prm._obj.a_cp if prm is not None else None,
                         val(stream)))
            return 0

    monkeypatch.setattr(stx, "_lib", Fake())
    h = stx.reservoir_create_device(5, 2, 3, _ok_params(stx, substeps=4), 0x1000, 0x2000, 0x3000, 0x4000)
    assert h.value == 7
    stx.reservoir_load_device(h, 0x5000, None, 0x6000, None, None)
    q = _ok_params(stx, substeps=4)
    q.a_cp = 0.25
    stx.reservoir_load_device(h, None, 0x7000, None, q, 0x8000)
    assert seen == [("create", 5, 2, 3, 4, 0x1000, 0x2000, 0x3000, 0x4000),
                    ("load", 7, 0x5000, None, 0x6000, None, None),
                    ("load", 7, None, 0x7000, None, 0.25, 0x8000)]


def test_device_entry_points_reject_bad_arguments(stx):
    """The checks that precede any device work: NULL handle, output or array
    pointers, sizes and constants out of range.  The addresses passed are
    never dereferenced because every case fails its checks first."""
    lib = stx.lib()
    h = ctypes.c_void_p()
    addr = ctypes.c_void_p(0x1000)
    prm = _ok_params(stx)

    def create(n=4, n_in=1, S=1, pr=prm, W=addr, w_in=addr, m0=addr, out=True):
        return lib.reservoir_create_device(n, n_in, S, ctypes.byref(pr), W, w_in, m0, None,
                                           ctypes.byref(h) if out else None)

    assert create(W=None) == stx.STO_E_INVALID
    assert create(m0=None) == stx.STO_E_INVALID
    assert create(out=False) == stx.STO_E_INVALID
    assert create(n=0) == stx.STO_E_INVALID
    assert create(n_in=0) == stx.STO_E_INVALID
    assert create(S=0) == stx.STO_E_INVALID
    assert create(pr=_ok_params(stx, dt=-1.0)) == stx.STO_E_INVALID
    assert lib.reservoir_load_device(None, addr, None, None, None, None) == stx.STO_E_INVALID
    assert "handle" in stx.sto_last_error()
