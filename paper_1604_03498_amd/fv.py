"""ctypes binding of the libfv C ABI (include/fv.h).  Argument marshalling only.

Names mirror the C entry points without the ``fv_`` prefix.  Host arrays are numpy
arrays; device arrays and streams are torch tensors / ``torch.cuda.Stream`` objects (torch
is used for device memory and streams, nothing else).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

OK, PENDING = 0, 1
E_INVAL, E_NOMEM, E_DEVICE, E_BUDGET = -1, -2, -3, -4
E_AGAIN, E_NOTFOUND, E_TIMEOUT, E_UNSUPPORTED = -5, -6, -7, -8
PREC_FP32, PREC_BF16_SPLIT, PREC_FP16_SPLIT, PREC_BF16 = 0, 1, 2, 3
X_DEVICE, OUT_DEVICE, NO_POWER_NORM, NO_L2_NORM, ASYNC, THRESHOLD = 1, 2, 4, 8, 16, 32
PROJ_SPLIT16 = 64  # fv_project: the split-bf16 contraction of the 16-bit encoder forms
THRESHOLD_TAU = 1e-6  # posteriors at or below it are left out under THRESHOLD
DSIFT_DIM = 130  # dense-SIFT row: 128 values + the centre's normalised x and y

EXPORTED_SYMBOLS = ("fv_limits", "fv_gmm_load", "fv_gmm_free", "fv_gmm_info", "fv_encode",
                    "fv_encode_batch", "fv_gmm_set_tuning", "fv_gmm_get_tuning",
                    "fv_kernel_timing", "fv_kernel_timing_read", "fv_server_config_default", "fv_server_create", "fv_server_destroy",
                    "fv_server_submit", "fv_server_submit_device", "fv_server_poll",
                    "fv_server_next_done", "fv_server_cancel",
                    "fv_server_get_stats", "fv_strerror", "fv_last_device_error",
                    "fv_pca_load", "fv_pca_free", "fv_pca_info", "fv_project",
                    "fv_encode_projected", "fv_encode_batch_projected", "fv_em_step",
                    "fv_stream_release", "fv_dsift_rows", "fv_dsift", "fv_encode_images",
                    "fv_encode_noalloc", "fv_graph_counters")
EXEC_HIP, EXEC_FAKE = 0, 1


class Tuning(ctypes.Structure):
    _fields_ = [("batch_chunk", ctypes.c_int), ("batch_path", ctypes.c_int),
                ("single_split_below", ctypes.c_int64), ("batch_grid", ctypes.c_int),
                ("fused16_variant", ctypes.c_int)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("precision", ctypes.c_int),
                ("flags", ctypes.c_uint), ("max_queue", ctypes.c_int), ("n_streams", ctypes.c_int),
                ("max_batch_frames", ctypes.c_int), ("max_batch_rows", ctypes.c_int64),
                ("deadline_ms", ctypes.c_double), ("batch_window_us", ctypes.c_double),
                ("executor", ctypes.c_int),
                ("fake_K", ctypes.c_int), ("fake_D", ctypes.c_int),
                ("fake_us_per_krow", ctypes.c_double), ("fake_fail_every", ctypes.c_int),
                ("copy_threads", ctypes.c_int)]


class ReqStats(ctypes.Structure):
    _fields_ = [("t_submit_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_start_us", ctypes.c_double), ("t_done_us", ctypes.c_double),
                ("rows", ctypes.c_int64), ("batch_frames", ctypes.c_int), ("status", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("rows_done", ctypes.c_int64),
                ("queued", ctypes.c_int), ("in_flight", ctypes.c_int),
                ("admitted_bytes", ctypes.c_size_t), ("peak_admitted_bytes", ctypes.c_size_t),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("cancelled", ctypes.c_int64),
                ("graph_captures", ctypes.c_int64), ("graph_replays", ctypes.c_int64)]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfv.so")
_lib = None


class FvError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = strerror(code) if _lib is not None else str(code)
        if code == E_DEVICE and _lib is not None:
            msg += f" (hip error {last_device_error()})"
        super().__init__(f"{what}: {msg} [{code}]" if what else f"{msg} [{code}]")


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load libfv.so (built in-tree by paper_1604_03498_amd.build).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"libfv.so not built ({_LIB_PATH}); run python -m paper_1604_03498_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint
    lib.fv_limits.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fv_limits.restype = None
    lib.fv_gmm_load.argtypes = [i32, i32, vp, vp, vp, i32, ctypes.POINTER(vp)]
    lib.fv_gmm_free.argtypes = [vp]
    lib.fv_gmm_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fv_encode.argtypes = [vp, vp, i64, vp, i32, u32, vp]
    lib.fv_encode_batch.argtypes = [vp, vp, vp, i32, vp, i32, u32, vp]
    lib.fv_encode_noalloc.argtypes = [vp, vp, i64, vp, i32, u32, vp]
    lib.fv_encode_noalloc.restype = i32
    lib.fv_pca_load.argtypes = [i32, i32, vp, vp, i32, ctypes.POINTER(vp)]
    lib.fv_pca_free.argtypes = [vp]
    lib.fv_pca_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fv_project.argtypes = [vp, vp, i64, vp, u32, vp]
    lib.fv_encode_projected.argtypes = [vp, vp, vp, i64, vp, i32, u32, vp]
    lib.fv_encode_batch_projected.argtypes = [vp, vp, vp, vp, i32, vp, i32, u32, vp]
    lib.fv_gmm_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.fv_gmm_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.fv_gmm_set_tuning.restype = i32
    lib.fv_gmm_get_tuning.restype = i32
    lib.fv_kernel_timing.argtypes = [i32]
    lib.fv_kernel_timing_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.fv_server_config_default.argtypes = [ctypes.POINTER(ServerConfig)]
    lib.fv_server_config_default.restype = None
    lib.fv_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.fv_server_destroy.argtypes = [vp]
    lib.fv_server_submit.argtypes = [vp, vp, i64, ctypes.POINTER(ctypes.c_uint64)]
    lib.fv_server_submit_device.argtypes = [vp, vp, i64, ctypes.POINTER(ctypes.c_uint64)]
    lib.fv_server_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(ReqStats)]
    lib.fv_server_next_done.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
    lib.fv_server_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.fv_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats), i32]
    for f in (lib.fv_server_create, lib.fv_server_destroy, lib.fv_server_submit,
              lib.fv_server_submit_device, lib.fv_server_poll, lib.fv_server_next_done,
              lib.fv_server_cancel,
              lib.fv_server_get_stats):
        f.restype = i32
    lib.fv_strerror.argtypes = [i32]
    lib.fv_strerror.restype = ctypes.c_char_p
    lib.fv_last_device_error.argtypes = []
    lib.fv_em_step.argtypes = [vp, vp, i64, i32, ctypes.c_float, u32, vp, vp, vp, vp,
                               ctypes.POINTER(ctypes.c_double)]
    lib.fv_stream_release.argtypes = [i32, vp]
    lib.fv_graph_counters.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.fv_graph_counters.restype = i32
    lib.fv_dsift_rows.argtypes = [i32, i32, i32, vp, i32, i32, ctypes.POINTER(i64)]
    lib.fv_dsift.argtypes = [vp, i32, i32, i32, i32, vp, i32, i32, vp, u32, i32, vp]
    lib.fv_encode_images.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, i32, i32, vp, i32, u32,
                                     vp]
    for f in (lib.fv_pca_load, lib.fv_pca_free, lib.fv_pca_info, lib.fv_project,
              lib.fv_encode_projected, lib.fv_encode_batch_projected, lib.fv_em_step,
              lib.fv_stream_release, lib.fv_dsift_rows, lib.fv_dsift, lib.fv_encode_images):
        f.restype = i32
    for f in (lib.fv_gmm_load, lib.fv_gmm_free, lib.fv_gmm_info, lib.fv_encode,
              lib.fv_encode_batch, lib.fv_kernel_timing, lib.fv_kernel_timing_read,
              lib.fv_last_device_error):
        f.restype = i32
    _lib = lib
    return lib


def graph_counters():
    """fv_graph_counters: (captures, replays) of the library's launch graphs so far."""
    c, r = ctypes.c_int64(), ctypes.c_int64()
    _check(load().fv_graph_counters(ctypes.byref(c), ctypes.byref(r)), "fv_graph_counters")
    return int(c.value), int(r.value)


def strerror(code: int) -> str:
    return load().fv_strerror(int(code)).decode()


def last_device_error() -> int:
    return int(load().fv_last_device_error())


def limits():
    k, d = ctypes.c_int(), ctypes.c_int()
    load().fv_limits(ctypes.byref(k), ctypes.byref(d))
    return k.value, d.value


def kernel_timing(enable: bool):
    """Start (and reset) or stop event timing of libfv's kernel launches."""
    _check(load().fv_kernel_timing(1 if enable else 0), "fv_kernel_timing")


def kernel_timing_read(which: int = 0):
    """(total_ms, launches) of kernel class `which` (0 statistics, 1 finalize) since reset."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(load().fv_kernel_timing_read(int(which), ctypes.byref(ms), ctypes.byref(n)),
           "fv_kernel_timing_read")
    return ms.value, n.value


def _check(rc: int, what: str):
    if rc != OK:
        raise FvError(rc, what)


class Gmm:
    """Owning wrapper of an ``fv_gmm*`` handle."""

    def __init__(self, handle: int, K: int, D: int, device: int):
        self.handle, self.K, self.D, self.device = handle, K, D, device

    @property
    def out_len(self) -> int:
        return 2 * self.K * self.D

    def free(self):
        if self.handle:
            _check(load().fv_gmm_free(ctypes.c_void_p(self.handle)), "fv_gmm_free")
            self.handle = 0

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.fv_gmm_free(ctypes.c_void_p(self.handle))
                self.handle = 0
        except Exception:
            pass


def _host_f32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def gmm_load(weights, means, variances, device: int = 0) -> Gmm:
    mu = _host_f32(means)
    if mu.ndim != 2:
        raise ValueError("means must be [K, D]")
    K, D = mu.shape
    w = _host_f32(weights, (K,))
    var = _host_f32(variances, (K, D))
    h = ctypes.c_void_p()
    rc = load().fv_gmm_load(K, D, w.ctypes.data, mu.ctypes.data, var.ctypes.data, int(device),
                            ctypes.byref(h))
    _check(rc, "fv_gmm_load")
    return Gmm(h.value, K, D, int(device))


def gmm_free(g: Gmm):
    g.free()


def gmm_info(g: Gmm):
    K, D, dev = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().fv_gmm_info(ctypes.c_void_p(g.handle), ctypes.byref(K), ctypes.byref(D),
                              ctypes.byref(dev)), "fv_gmm_info")
    return K.value, D.value, dev.value


def set_tuning(g: Gmm, batch_chunk: int = 0, batch_path: int = 0, single_split_below: int = 0,
               batch_grid: int = 0, fused16_variant: int = 0):
    """fv_gmm_set_tuning (all zero = automatic)."""
    t = Tuning(int(batch_chunk), int(batch_path), int(single_split_below), int(batch_grid),
               int(fused16_variant))
    _check(load().fv_gmm_set_tuning(ctypes.c_void_p(g.handle), ctypes.byref(t)), "fv_gmm_set_tuning")


def get_tuning(g: Gmm) -> dict:
    t = Tuning()
    _check(load().fv_gmm_get_tuning(ctypes.c_void_p(g.handle), ctypes.byref(t)), "fv_gmm_get_tuning")
    return {"batch_chunk": t.batch_chunk, "batch_path": t.batch_path,
            "single_split_below": t.single_split_below, "batch_grid": t.batch_grid,
            "fused16_variant": t.fused16_variant}


def _is_torch(x) -> bool:
    return type(x).__module__.split(".")[0] == "torch"


def _stream_handle(stream, device: int):
    if stream is None:
        import torch
        return torch.cuda.current_stream(device).cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def stream_release(stream, device: int = 0) -> None:
    """fv_stream_release: free the library's cached scratch, staging and graphs for `stream`
    (a torch stream or a raw hipStream_t) on `device`; call before the stream is destroyed."""
    _check(load().fv_stream_release(device, ctypes.c_void_p(_stream_handle(stream, device))),
           "fv_stream_release")


def _marshal_x(g, X, width: int | None = None):
    """Returns (pointer, rows, is_device, keepalive).  Rows have `width` values (g.D by
    default)."""
    width = g.D if width is None else width
    if _is_torch(X):
        import torch
        if X.dtype != torch.float32 or X.dim() != 2 or X.shape[1] != width:
            raise ValueError(f"X must be a float32 [N, {width}] tensor")
        if not X.is_contiguous():
            raise ValueError("X must be contiguous")
        if X.is_cuda:
            if X.device.index != g.device:
                raise ValueError("X is on another device than the GMM")
            return X.data_ptr(), X.shape[0], True, X
        Xc = X.numpy()
        return Xc.ctypes.data, Xc.shape[0], False, Xc
    Xn = _host_f32(X)
    if Xn.ndim != 2 or Xn.shape[1] != width:
        raise ValueError(f"X must be [N, {width}]")
    return Xn.ctypes.data, Xn.shape[0], False, Xn


def _marshal_out(g: Gmm, out, n_vec: int, x_is_device: bool):
    shape = (g.out_len,) if n_vec is None else (n_vec, g.out_len)
    if out is None:
        if x_is_device:
            import torch
            out = torch.empty(shape, dtype=torch.float32, device=f"cuda:{g.device}")
        else:
            out = np.empty(shape, dtype=np.float32)
    if _is_torch(out):
        import torch
        if out.dtype != torch.float32 or tuple(out.shape) != shape or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 tensor of shape {shape}")
        if out.is_cuda:
            return out, out.data_ptr(), True
        return out, out.numpy().ctypes.data, False
    if not isinstance(out, np.ndarray) or out.dtype != np.float32 or out.shape != shape \
            or not out.flags.c_contiguous:
        raise ValueError(f"out must be a contiguous float32 array of shape {shape}")
    return out, out.ctypes.data, False


def encode(g: Gmm, X, out=None, precision: int = PREC_FP32, flags: int = 0, stream=None):
    """Fisher vector of one frame (fv_encode).  Returns `out` ([2KD] float32)."""
    xp, n, xdev, _keep = _marshal_x(g, X)
    out, op, odev = _marshal_out(g, out, None, xdev)
    f = int(flags) & ~(X_DEVICE | OUT_DEVICE)
    f |= (X_DEVICE if xdev else 0) | (OUT_DEVICE if odev else 0)
    s = _stream_handle(stream, g.device) if (xdev or odev or stream is not None) else 0
    rc = load().fv_encode(ctypes.c_void_p(g.handle), ctypes.c_void_p(xp), int(n),
                          ctypes.c_void_p(op), int(precision), f, ctypes.c_void_p(s))
    _check(rc, "fv_encode")
    return out


def encode_noalloc(g: Gmm, X, out=None, precision: int = PREC_FP32, flags: int = 0,
                   stream=None):
    """fv_encode_noalloc: fv_encode on the library's fixed per-GPU scratch (no allocation);
    X and out must be device tensors."""
    xp, n, xdev, _keep = _marshal_x(g, X)
    if not xdev:
        raise ValueError("encode_noalloc needs X in device memory")
    out, op, odev = _marshal_out(g, out, None, True)
    if not odev:
        raise ValueError("encode_noalloc needs out in device memory")
    f = (int(flags) & ~(X_DEVICE | OUT_DEVICE)) | X_DEVICE | OUT_DEVICE
    s = _stream_handle(stream, g.device)
    _check(load().fv_encode_noalloc(ctypes.c_void_p(g.handle), ctypes.c_void_p(xp), int(n),
                                    ctypes.c_void_p(op), int(precision), f, ctypes.c_void_p(s)),
           "fv_encode_noalloc")
    return out


def encode_batch(g: Gmm, X, offsets, out=None, precision: int = PREC_FP32, flags: int = 0,
                 stream=None):
    """Fisher vectors of B frames (fv_encode_batch); offsets is a host int64 array [B+1]."""
    xp, n, xdev, _keep = _marshal_x(g, X)
    if _is_torch(offsets):
        offsets = offsets.cpu().numpy()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or off.size < 1:
        raise ValueError("offsets must be a 1-D int64 array of B+1 entries")
    B = off.size - 1
    if B > 0 and off[-1] != n:
        raise ValueError("offsets[-1] must equal the number of rows of X")
    out, op, odev = _marshal_out(g, out, B, xdev)
    f = int(flags) & ~(X_DEVICE | OUT_DEVICE)
    f |= (X_DEVICE if xdev else 0) | (OUT_DEVICE if odev else 0)
    s = _stream_handle(stream, g.device) if (xdev or odev or stream is not None) else 0
    rc = load().fv_encode_batch(ctypes.c_void_p(g.handle), ctypes.c_void_p(xp),
                                ctypes.c_void_p(off.ctypes.data), int(B), ctypes.c_void_p(op),
                                int(precision), f, ctypes.c_void_p(s))
    _check(rc, "fv_encode_batch")
    return out


class Pca:
    """Owning wrapper of an ``fv_pca*`` (projection prologue y = A (x - m))."""

    def __init__(self, handle: int, Din: int, D: int, device: int):
        self.handle, self.Din, self.D, self.device = handle, Din, D, device

    def free(self):
        if self.handle:
            _check(load().fv_pca_free(ctypes.c_void_p(self.handle)), "fv_pca_free")
            self.handle = 0

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.fv_pca_free(ctypes.c_void_p(self.handle))
                self.handle = 0
        except Exception:
            pass


def pca_load(A, mean, device: int = 0) -> Pca:
    """fv_pca_load: A [D, Din], mean [Din] (host arrays)."""
    A = _host_f32(A)
    if A.ndim != 2:
        raise ValueError("A must be [D, Din]")
    D, Din = A.shape
    m = _host_f32(mean, (Din,))
    h = ctypes.c_void_p()
    _check(load().fv_pca_load(Din, D, A.ctypes.data, m.ctypes.data, int(device), ctypes.byref(h)),
           "fv_pca_load")
    return Pca(h.value, Din, D, int(device))


def project(p: Pca, X, out=None, stream=None, split16: bool = False):
    """fv_project: [N, Din] -> [N, D] (device tensors in, device tensor out; host arrays in,
    host array out).  split16: the split-bf16 contraction (as inside the 16-bit forms)."""
    xp, n, xdev, _keep = _marshal_x(p, X, p.Din)
    shape = (n, p.D)
    if out is None:
        if xdev:
            import torch
            out = torch.empty(shape, dtype=torch.float32, device=f"cuda:{p.device}")
        else:
            out = np.empty(shape, dtype=np.float32)
    if _is_torch(out):
        if tuple(out.shape) != shape or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 tensor of shape {shape}")
        op, odev = out.data_ptr(), out.is_cuda
        if not odev:
            op = out.numpy().ctypes.data
    else:
        if out.dtype != np.float32 or out.shape != shape or not out.flags.c_contiguous:
            raise ValueError(f"out must be a contiguous float32 array of shape {shape}")
        op, odev = out.ctypes.data, False
    f = (X_DEVICE if xdev else 0) | (OUT_DEVICE if odev else 0) | (PROJ_SPLIT16 if split16 else 0)
    s = _stream_handle(stream, p.device) if (xdev or odev or stream is not None) else 0
    _check(load().fv_project(ctypes.c_void_p(p.handle), ctypes.c_void_p(xp), int(n),
                             ctypes.c_void_p(op), f, ctypes.c_void_p(s)), "fv_project")
    return out


def encode_projected(g: Gmm, p: Pca, X, out=None, precision: int = PREC_FP32, flags: int = 0,
                     stream=None):
    """fv_encode_projected: X holds raw [N, Din] descriptors."""
    xp, n, xdev, _keep = _marshal_x(p, X, p.Din)
    out, op, odev = _marshal_out(g, out, None, xdev)
    f = int(flags) & ~(X_DEVICE | OUT_DEVICE)
    f |= (X_DEVICE if xdev else 0) | (OUT_DEVICE if odev else 0)
    s = _stream_handle(stream, g.device) if (xdev or odev or stream is not None) else 0
    _check(load().fv_encode_projected(ctypes.c_void_p(g.handle), ctypes.c_void_p(p.handle),
                                      ctypes.c_void_p(xp), int(n), ctypes.c_void_p(op),
                                      int(precision), f, ctypes.c_void_p(s)),
           "fv_encode_projected")
    return out


def encode_batch_projected(g: Gmm, p: Pca, X, offsets, out=None, precision: int = PREC_FP32,
                           flags: int = 0, stream=None):
    """fv_encode_batch_projected: X holds raw [sum N, Din] descriptors."""
    xp, n, xdev, _keep = _marshal_x(p, X, p.Din)
    if _is_torch(offsets):
        offsets = offsets.cpu().numpy()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or off.size < 1:
        raise ValueError("offsets must be a 1-D int64 array of B+1 entries")
    B = off.size - 1
    if B > 0 and off[-1] != n:
        raise ValueError("offsets[-1] must equal the number of rows of X")
    out, op, odev = _marshal_out(g, out, B, xdev)
    f = int(flags) & ~(X_DEVICE | OUT_DEVICE)
    f |= (X_DEVICE if xdev else 0) | (OUT_DEVICE if odev else 0)
    s = _stream_handle(stream, g.device) if (xdev or odev or stream is not None) else 0
    _check(load().fv_encode_batch_projected(ctypes.c_void_p(g.handle), ctypes.c_void_p(p.handle),
                                            ctypes.c_void_p(xp), ctypes.c_void_p(off.ctypes.data),
                                            int(B), ctypes.c_void_p(op), int(precision), f,
                                            ctypes.c_void_p(s)), "fv_encode_batch_projected")
    return out


def _scales_arg(scales, n_scales):
    """(count, pointer, keepalive) of a scale list; None asks for the n_scales smallest of the
    paper's nine scales (2 down to 1/8)."""
    if scales is None:
        return int(n_scales), None, None
    sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64).reshape(-1))
    return int(sc.size), sc.ctypes.data, sc


def dsift_rows(H: int, W: int, scales=None, n_scales: int = 8, bin: int = 4,
               step: int = 4) -> int:
    """fv_dsift_rows: descriptors per H x W image."""
    n, sp, _keep = _scales_arg(scales, n_scales)
    r = ctypes.c_int64()
    _check(load().fv_dsift_rows(int(H), int(W), n, ctypes.c_void_p(sp), int(bin), int(step),
                                ctypes.byref(r)), "fv_dsift_rows")
    return int(r.value)


def _marshal_images(images, device: int):
    """(pointer, n_images, H, W, is_device, keepalive) of [n, H, W] (or [H, W]) float32."""
    if _is_torch(images):
        import torch
        if images.dtype != torch.float32 or images.dim() not in (2, 3) or not images.is_contiguous():
            raise ValueError("images must be a contiguous float32 [n, H, W] or [H, W] tensor")
        im = images.unsqueeze(0) if images.dim() == 2 else images
        if im.is_cuda:
            if im.device.index != device:
                raise ValueError("images are on another device")
            return im.data_ptr(), im.shape[0], im.shape[1], im.shape[2], True, im
        a = im.numpy()
        return a.ctypes.data, a.shape[0], a.shape[1], a.shape[2], False, a
    a = _host_f32(images)
    if a.ndim == 2:
        a = a[None]
    if a.ndim != 3:
        raise ValueError("images must be [n, H, W] or [H, W]")
    return a.ctypes.data, a.shape[0], a.shape[1], a.shape[2], False, a


def dsift(images, scales=None, n_scales: int = 8, bin: int = 4, step: int = 4, device: int = 0,
          out=None, stream=None, flags: int = 0):
    """fv_dsift: [n, H, W] (or [H, W]) float32 images -> [n, rows, 130] descriptors (a device
    tensor for device images, a host array for host images); flags may add ASYNC."""
    ip, n, H, W, idev, _ki = _marshal_images(images, device)
    ns, sp, _ks = _scales_arg(scales, n_scales)
    rows = dsift_rows(H, W, scales, n_scales, bin, step)
    shape = (n, rows, DSIFT_DIM)
    if out is None:
        if idev:
            import torch
            out = torch.empty(shape, dtype=torch.float32, device=f"cuda:{device}")
        else:
            out = np.empty(shape, dtype=np.float32)
    if _is_torch(out):
        if tuple(out.shape) != shape or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 tensor of shape {shape}")
        op, odev = (out.data_ptr(), True) if out.is_cuda else (out.numpy().ctypes.data, False)
    else:
        if out.dtype != np.float32 or out.shape != shape or not out.flags.c_contiguous:
            raise ValueError(f"out must be a contiguous float32 array of shape {shape}")
        op, odev = out.ctypes.data, False
    f = (X_DEVICE if idev else 0) | (OUT_DEVICE if odev else 0) | (int(flags) & ASYNC)
    s = _stream_handle(stream, device) if (idev or odev or stream is not None) else 0
    _check(load().fv_dsift(ctypes.c_void_p(ip), int(n), int(H), int(W), ns, ctypes.c_void_p(sp),
                           int(bin), int(step), ctypes.c_void_p(op), f, int(device),
                           ctypes.c_void_p(s)), "fv_dsift")
    return out


def encode_images(g: Gmm, p: Pca, images, scales=None, n_scales: int = 8, bin: int = 4,
                  step: int = 4, out=None, precision: int = PREC_FP32, flags: int = 0,
                  stream=None):
    """fv_encode_images: one Fisher vector per image, [n, 2KD]."""
    ip, n, H, W, idev, _ki = _marshal_images(images, g.device)
    ns, sp, _ks = _scales_arg(scales, n_scales)
    out, op, odev = _marshal_out(g, out, n, idev)
    f = int(flags) & ~(X_DEVICE | OUT_DEVICE)
    f |= (X_DEVICE if idev else 0) | (OUT_DEVICE if odev else 0)
    s = _stream_handle(stream, g.device) if (idev or odev or stream is not None) else 0
    _check(load().fv_encode_images(ctypes.c_void_p(g.handle), ctypes.c_void_p(p.handle),
                                   ctypes.c_void_p(ip), int(n), int(H), int(W), ns,
                                   ctypes.c_void_p(sp), int(bin), int(step), ctypes.c_void_p(op),
                                   int(precision), f, ctypes.c_void_p(s)), "fv_encode_images")
    return out


def em_step(g: Gmm, X, precision: int = PREC_FP32, var_floor: float = 1e-6, stream=None):
    """fv_em_step: one EM iteration of the model g on X.  Returns (weights [K], means [K, D],
    variances [K, D], loglik) as host arrays and a float."""
    xp, n, xdev, _keep = _marshal_x(g, X)
    w = np.empty(g.K, np.float32)
    mu = np.empty((g.K, g.D), np.float32)
    var = np.empty((g.K, g.D), np.float32)
    ll = ctypes.c_double()
    s = _stream_handle(stream, g.device) if (xdev or stream is not None) else 0
    _check(load().fv_em_step(ctypes.c_void_p(g.handle), ctypes.c_void_p(xp), int(n),
                             int(precision), float(var_floor), X_DEVICE if xdev else 0,
                             ctypes.c_void_p(s), w.ctypes.data, mu.ctypes.data, var.ctypes.data,
                             ctypes.byref(ll)), "fv_em_step")
    return w, mu, var, ll.value


def em_fit(X, weights, means, variances, iters: int, precision: int = PREC_FP32,
           var_floor: float = 1e-6, device: int = 0, stream=None):
    """EM iterations from the given model (each step on the device, the new model loaded for
    the next).  Returns (weights, means, variances, [loglik of each step's input model])."""
    w, mu, var = (np.asarray(a, np.float32) for a in (weights, means, variances))
    lls = []
    for _ in range(int(iters)):
        g = gmm_load(w, mu, var, device)
        try:
            w, mu, var, ll = em_step(g, X, precision, var_floor, stream)
        finally:
            g.free()
        lls.append(ll)
    return w, mu, var, lls


def server_config(**kw) -> ServerConfig:
    """fv_server_config_default(), then the given fields."""
    c = ServerConfig()
    load().fv_server_config_default(ctypes.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


class Server:
    """Owning wrapper of an ``fv_server*`` (continuous-batching encoder)."""

    def __init__(self, g: Gmm | None, cfg: ServerConfig, out_len: int | None = None, D: int | None = None):
        h = ctypes.c_void_p()
        _check(load().fv_server_create(ctypes.c_void_p(g.handle) if g else None, ctypes.byref(cfg),
                                       ctypes.byref(h)), "fv_server_create")
        self.handle = h.value
        self.gmm = g
        self.out_len = g.out_len if g else 2 * cfg.fake_K * cfg.fake_D
        self.D = g.D if g else cfg.fake_D
        self._device_inputs = {}  # ticket -> frame kept alive until the ticket finishes

    def submit(self, X) -> int:
        Xn = _host_f32(X)
        if Xn.ndim != 2 or Xn.shape[1] != self.D:
            raise ValueError("X must be [N, D]")
        t = ctypes.c_uint64()
        rc = load().fv_server_submit(ctypes.c_void_p(self.handle), ctypes.c_void_p(Xn.ctypes.data),
                                     int(Xn.shape[0]), ctypes.byref(t))
        if rc != OK:
            raise FvError(rc, "fv_server_submit")
        return t.value

    def try_submit(self, X):
        """(code, ticket or None) without raising."""
        Xn = _host_f32(X)
        t = ctypes.c_uint64()
        rc = load().fv_server_submit(ctypes.c_void_p(self.handle), ctypes.c_void_p(Xn.ctypes.data),
                                     int(Xn.shape[0]), ctypes.byref(t))
        return rc, (t.value if rc == OK else None)

    def try_submit_device(self, X):
        """fv_server_submit_device for a contiguous float32 [N, D] tensor in device memory (a
        torch CUDA tensor; the fake executor also takes a numpy array).  (code, ticket or None);
        the tensor is kept referenced until the ticket finishes."""
        if _is_torch(X):
            if X.dtype.itemsize != 4 or not X.is_contiguous() or X.dim() != 2:
                raise ValueError("X must be a contiguous float32 [N, D] tensor")
            n, d, ptr = int(X.shape[0]), int(X.shape[1]), X.data_ptr()
        else:
            Xn = np.ascontiguousarray(X, dtype=np.float32)
            if Xn is not X:
                X = Xn
            n, d, ptr = int(Xn.shape[0]), int(Xn.shape[1]), Xn.ctypes.data
        if d != self.D:
            raise ValueError("X must be [N, D]")
        t = ctypes.c_uint64()
        rc = load().fv_server_submit_device(ctypes.c_void_p(self.handle), ctypes.c_void_p(ptr), n,
                                            ctypes.byref(t))
        if rc != OK:
            return rc, None
        self._device_inputs[t.value] = X
        return rc, t.value

    def submit_device(self, X) -> int:
        rc, t = self.try_submit_device(X)
        if rc != OK:
            raise FvError(rc, "fv_server_submit_device")
        return t

    def poll(self, ticket: int, want_out: bool = True):
        """(code, out or None, stats dict or None)."""
        out = np.empty(self.out_len, np.float32) if want_out else None
        st = ReqStats()
        rc = load().fv_server_poll(ctypes.c_void_p(self.handle), ctypes.c_uint64(ticket),
                                   ctypes.c_void_p(out.ctypes.data) if want_out else None,
                                   ctypes.byref(st))
        if rc == PENDING or rc == E_NOTFOUND:
            return rc, None, None
        self._device_inputs.pop(ticket, None)
        stats = {f: getattr(st, f) for f, _ in ReqStats._fields_}
        return rc, (out if rc == OK else None), stats

    def cancel(self, ticket: int) -> int:
        """fv_server_cancel: OK (withdrawn), PENDING (already in a launch) or E_NOTFOUND."""
        rc = load().fv_server_cancel(ctypes.c_void_p(self.handle), ctypes.c_uint64(ticket))
        if rc == OK:
            self._device_inputs.pop(ticket, None)
        elif rc not in (PENDING, E_NOTFOUND):
            _check(rc, "fv_server_cancel")
        return rc

    def next_done(self, timeout_ms: float = -1.0):
        t = ctypes.c_uint64()
        rc = load().fv_server_next_done(ctypes.c_void_p(self.handle), float(timeout_ms), ctypes.byref(t))
        if rc == PENDING:
            return None
        _check(rc, "fv_server_next_done")
        return t.value

    def stats(self, reset: bool = False) -> dict:
        st = ServerStats()
        _check(load().fv_server_get_stats(ctypes.c_void_p(self.handle), ctypes.byref(st), int(reset)),
               "fv_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            _check(load().fv_server_destroy(ctypes.c_void_p(self.handle)), "fv_server_destroy")
            self.handle = 0
            self._device_inputs.clear()  # destroy has waited for every launch

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.fv_server_destroy(ctypes.c_void_p(self.handle))
                self.handle = 0
        except Exception:
            pass
