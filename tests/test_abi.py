"""C ABI of libfv on the CPU: the library loads, exports every symbol its header declares,
and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1604_03498_amd as fv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "fv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fv_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = fv.load()
    syms = header_symbols()
    assert set(syms) == set(fv.EXPORTED_SYMBOLS), syms
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_constants_match_header():
    """Every FV_* #define of the header has the same value in the Python binding."""
    txt = open(os.path.join(ROOT, "include", "fv.h")).read()
    defs = dict(re.findall(r"#define FV_([A-Z0-9_]+) \(?(-?[0-9.e+-]+)u?\)?", txt))
    assert len(defs) > 20
    for name, val in defs.items():
        assert hasattr(fv, name), name
        assert float(getattr(fv, name)) == float(val), name


def test_strerror_and_limits():
    assert fv.strerror(fv.OK) == "ok"
    assert fv.strerror(fv.E_INVAL) == "invalid argument"
    assert fv.strerror(12345) == "unknown status"
    K, D = fv.limits()
    assert K >= 256 and D >= 80


def _load_raw(K, D, w, mu, var, device=0):
    lib = fv.load()
    h = ctypes.c_void_p(123)
    pw = w.ctypes.data if w is not None else None
    pm = mu.ctypes.data if mu is not None else None
    pv = var.ctypes.data if var is not None else None
    rc = lib.fv_gmm_load(K, D, pw, pm, pv, device, ctypes.byref(h))
    return rc, h.value


def test_gmm_load_validation():
    K, D = 4, 3
    w = np.full(K, 0.25, np.float32)
    mu = np.zeros((K, D), np.float32)
    var = np.ones((K, D), np.float32)
    assert _load_raw(0, D, w, mu, var) == (fv.E_INVAL, None)
    assert _load_raw(K, 0, w, mu, var) == (fv.E_INVAL, None)
    assert _load_raw(K, D, None, mu, var)[0] == fv.E_INVAL
    assert _load_raw(K, D, w, None, var)[0] == fv.E_INVAL
    assert _load_raw(K, D, w, mu, None)[0] == fv.E_INVAL
    for bad in (0.0, -0.1, np.nan, np.inf):
        w2 = w.copy(); w2[1] = bad
        assert _load_raw(K, D, w2, mu, var)[0] == fv.E_INVAL
        v2 = var.copy(); v2[2, 1] = bad
        assert _load_raw(K, D, w, mu, v2)[0] == fv.E_INVAL
    m2 = mu.copy(); m2[0, 0] = np.nan
    assert _load_raw(K, D, w, m2, var)[0] == fv.E_INVAL
    big = 2048
    assert _load_raw(big, D, np.full(big, 1 / big, np.float32), np.zeros((big, D), np.float32),
                     np.ones((big, D), np.float32))[0] == fv.E_UNSUPPORTED
    assert fv.load().fv_gmm_load(K, D, w.ctypes.data, mu.ctypes.data, var.ctypes.data, 0, None) \
        == fv.E_INVAL


def test_encode_validation_without_device():
    lib = fv.load()
    out = np.zeros(8, np.float32)
    X = np.zeros((2, 2), np.float32)
    assert lib.fv_encode(None, X.ctypes.data, 2, out.ctypes.data, 0, 0, None) == fv.E_INVAL
    off = np.array([0, 2], np.int64)
    assert lib.fv_encode_batch(None, X.ctypes.data, off.ctypes.data, 1, out.ctypes.data, 0, 0,
                               None) == fv.E_INVAL
    assert lib.fv_gmm_free(None) == fv.OK
    assert lib.fv_gmm_info(None, None, None, None) == fv.E_INVAL


def test_pca_validation_without_device():
    lib = fv.load()
    h = ctypes.c_void_p(123)
    A = np.zeros((4, 6), np.float32)
    m = np.zeros(6, np.float32)
    assert lib.fv_pca_load(6, 4, A.ctypes.data, m.ctypes.data, 0, None) == fv.E_INVAL
    assert lib.fv_pca_load(0, 4, A.ctypes.data, m.ctypes.data, 0, ctypes.byref(h)) == fv.E_INVAL
    assert h.value is None
    assert lib.fv_pca_load(6, 0, A.ctypes.data, m.ctypes.data, 0, ctypes.byref(h)) == fv.E_INVAL
    assert lib.fv_pca_load(6, 4, None, m.ctypes.data, 0, ctypes.byref(h)) == fv.E_INVAL
    assert lib.fv_pca_load(6, 4, A.ctypes.data, None, 0, ctypes.byref(h)) == fv.E_INVAL
    A2 = A.copy(); A2[1, 2] = np.inf
    assert lib.fv_pca_load(6, 4, A2.ctypes.data, m.ctypes.data, 0, ctypes.byref(h)) == fv.E_INVAL
    m2 = m.copy(); m2[3] = np.nan
    assert lib.fv_pca_load(6, 4, A.ctypes.data, m2.ctypes.data, 0, ctypes.byref(h)) == fv.E_INVAL
    Ab = np.zeros((4, 257), np.float32); mb = np.zeros(257, np.float32)
    assert lib.fv_pca_load(257, 4, Ab.ctypes.data, mb.ctypes.data, 0, ctypes.byref(h)) \
        == fv.E_UNSUPPORTED
    Ad = np.zeros((97, 6), np.float32)
    assert lib.fv_pca_load(6, 97, Ad.ctypes.data, m.ctypes.data, 0, ctypes.byref(h)) \
        == fv.E_UNSUPPORTED
    assert lib.fv_pca_free(None) == fv.OK
    assert lib.fv_pca_info(None, None, None, None) == fv.E_INVAL
    X = np.zeros((2, 6), np.float32)
    out = np.zeros(8, np.float32)
    assert lib.fv_project(None, X.ctypes.data, 2, out.ctypes.data, 0, None) == fv.E_INVAL
    assert lib.fv_encode_projected(None, None, X.ctypes.data, 2, out.ctypes.data, 0, 0, None) \
        == fv.E_INVAL
    off = np.array([0, 2], np.int64)
    assert lib.fv_encode_batch_projected(None, None, X.ctypes.data, off.ctypes.data, 1,
                                         out.ctypes.data, 0, 0, None) == fv.E_INVAL


def test_em_step_validation_without_device():
    lib = fv.load()
    X = np.zeros((2, 2), np.float32)
    o = np.zeros(8, np.float32)
    ll = ctypes.c_double()
    assert lib.fv_em_step(None, X.ctypes.data, 2, 0, 1e-3, 0, None, o.ctypes.data, o.ctypes.data,
                          o.ctypes.data, ctypes.byref(ll)) == fv.E_INVAL


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    import paper_1604_03498_amd.fv as mod
    monkeypatch.setattr(mod, "_lib", None)
    monkeypatch.setattr(mod, "_LIB_PATH", str(tmp_path / "libfv.so"))
    with pytest.raises(RuntimeError):
        mod.load()
