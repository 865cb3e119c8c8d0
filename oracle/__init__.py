"""FP64 CPU oracle for Fisher-vector encoding -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The GPU library (``paper_1604_03498_amd``) never imports it, and the
two share no code: the only common dependency is the seeded data generator ``fvsynth``.

* ``fv_oracle.c`` -- plain sequential double-precision encoder (Algorithm 1 of the paper
  plus the improved-FV normalisation), built with gcc into ``liboracle.so``.
* ``brute.py``    -- 50-digit mpmath evaluation for tiny inputs.
* ``metrics.py``  -- the error measures used to compare another encoder with this one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NO_POWER = 1
NO_L2 = 2

def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (strict IEEE double, no contraction, OpenMP over frames)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
            "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OracleLib:
    """ctypes view of one build of the C oracle (the default build, or a test's own copy)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        i64, i32, u32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint, ctypes.c_double
        p = ctypes.c_void_p
        lib.fvo_posteriors.argtypes = [i64, i32, i32, p, p, p, p, p]
        lib.fvo_encode_tau.argtypes = [i64, i32, i32, p, p, p, p, u32, f64, p]
        lib.fvo_encode_tau_f64.argtypes = [i64, i32, i32, p, p, p, p, u32, f64, p]
        lib.fvo_encode_tau_f64.restype = ctypes.c_int
        lib.fvo_encode.argtypes = [i64, i32, i32, p, p, p, p, u32, p]
        lib.fvo_encode_batch.argtypes = [i32, p, i32, i32, p, p, p, p, u32, i32, p]
        lib.fvo_max_threads.argtypes = []
        for f in (lib.fvo_posteriors, lib.fvo_encode_tau, lib.fvo_encode, lib.fvo_encode_batch,
                  lib.fvo_max_threads):
            f.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def posteriors(self, X, weights, means, variances) -> np.ndarray:
        """gamma [N x K] in float64 (steps 1-4)."""
        w, mu, var, K, D = _model(weights, means, variances)
        X = _f32(X).reshape(-1, D)
        out = np.empty((X.shape[0], K), dtype=np.float64)
        rc = self.lib.fvo_posteriors(X.shape[0], K, D, _ptr(X), _ptr(w), _ptr(mu), _ptr(var),
                                     _ptr(out))
        if rc:
            raise RuntimeError("oracle posteriors failed")
        return out

    def encode(self, X, weights, means, variances, flags: int = 0,
               tau: float | None = None) -> np.ndarray:
        """Fisher vector [2KD] in float64: [u (K x D) ; v (K x D)], signed-sqrt and L2 unless
        flagged off."""
        w, mu, var, K, D = _model(weights, means, variances)
        X = _f32(X).reshape(-1, D)
        out = np.empty(2 * K * D, dtype=np.float64)
        t = -1.0 if tau is None else float(tau)
        rc = self.lib.fvo_encode_tau(X.shape[0], K, D, _ptr(X), _ptr(w), _ptr(mu), _ptr(var),
                                     int(flags), t, _ptr(out))
        if rc:
            raise RuntimeError("oracle encode failed")
        return out

    def encode_f64(self, X, weights, means, variances, flags: int = 0,
                   tau: float | None = None) -> np.ndarray:
        """As encode, for float64 descriptors (used as given, no rounding to float32)."""
        w, mu, var, K, D = _model(weights, means, variances)
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, D)
        out = np.empty(2 * K * D, dtype=np.float64)
        t = -1.0 if tau is None else float(tau)
        rc = self.lib.fvo_encode_tau_f64(X.shape[0], K, D, _ptr(X), _ptr(w), _ptr(mu), _ptr(var),
                                         int(flags), t, _ptr(out))
        if rc:
            raise RuntimeError("oracle encode failed")
        return out

    def encode_batch(self, X, offsets, weights, means, variances, flags: int = 0,
                     nthreads: int = 1) -> np.ndarray:
        """[B x 2KD]; frame b is rows offsets[b]:offsets[b+1].  nthreads spreads whole frames."""
        w, mu, var, K, D = _model(weights, means, variances)
        X = _f32(X).reshape(-1, D)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        B = off.shape[0] - 1
        out = np.empty((B, 2 * K * D), dtype=np.float64)
        rc = self.lib.fvo_encode_batch(B, _ptr(off), K, D, _ptr(X), _ptr(w), _ptr(mu), _ptr(var),
                                       int(flags), int(nthreads), _ptr(out))
        if rc:
            raise RuntimeError("oracle encode_batch failed")
        return out

    def max_threads(self) -> int:
        return int(self.lib.fvo_max_threads())


_default = None


def _load() -> OracleLib:
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _default = OracleLib(_LIB)
    return _default


def compile_variant(src_text: str, out_path: str) -> OracleLib:
    """Compile a (test-modified) copy of the oracle source and load it.  Used by the tests that
    plant mistakes in the oracle to show that the pins catch them."""
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                           "-shared", c_path, "-o", out_path, "-lm"])
    return OracleLib(out_path)


def source() -> str:
    with open(_SRC) as f:
        return f.read()


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _model(weights, means, variances):
    w, mu, var = _f32(weights), _f32(means), _f32(variances)
    K, D = mu.shape
    assert w.shape == (K,) and var.shape == (K, D)
    return w, mu, var, K, D


def posteriors(X, weights, means, variances) -> np.ndarray:
    return _load().posteriors(X, weights, means, variances)


def encode(X, weights, means, variances, flags: int = 0, tau: float | None = None) -> np.ndarray:
    return _load().encode(X, weights, means, variances, flags, tau)


def encode_batch(X, offsets, weights, means, variances, flags: int = 0,
                 nthreads: int = 1) -> np.ndarray:
    return _load().encode_batch(X, offsets, weights, means, variances, flags, nthreads)


def max_threads() -> int:
    return _load().max_threads()


def encode_gmm(X, g, flags: int = 0, tau: float | None = None) -> np.ndarray:
    return encode(X, g.weights, g.means, g.variances, flags, tau)


def project(X, A, mean) -> np.ndarray:
    """The projection prologue y = A (x - m) in float64 (Sec. 3.1: PCA of the SIFT values plus
    the appended coordinates, written as one affine map): X [N, Din], A [D, Din], mean [Din],
    all promoted exactly from float32; one library matrix product."""
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    A64 = np.asarray(A, dtype=np.float32).astype(np.float64)
    m64 = np.asarray(mean, dtype=np.float32).astype(np.float64)
    return (X64 - m64) @ A64.T


def encode_projected(X, A, mean, g, flags: int = 0, tau: float | None = None) -> np.ndarray:
    """Fisher vector of the projected descriptors, the projection kept in float64."""
    return _load().encode_f64(project(X, A, mean), g.weights, g.means, g.variances, flags, tau)


def em_step(X, weights, means, variances, var_floor: float = 1e-6, lib: OracleLib | None = None):
    """One EM iteration in float64 (the training the paper does beforehand, Sec. 3.1), by
    definition: gamma from the oracle's posteriors (steps 1-4); n_k = sum_t gamma_tk;
    w_k = n_k / N; mu_k = sum_t gamma_tk x_t / n_k; var_kd = max(sum_t gamma_tk (x_td -
    mu_kd)^2 / n_k, floor) (a component with n_k = 0: w = 0, mu = 0, var = floor); and the
    log-likelihood sum_t ln sum_k w_k N(x_t; mu_k, var_k) of the input model, with the
    log-sum-exp taken by scipy.  Returns (w, mu, var, loglik) in float64."""
    from scipy.special import logsumexp
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    w0 = np.asarray(weights, dtype=np.float32).astype(np.float64)
    mu0 = np.asarray(means, dtype=np.float32).astype(np.float64)
    var0 = np.asarray(variances, dtype=np.float32).astype(np.float64)
    N, D = X64.shape
    gam = (lib or _load()).posteriors(X, weights, means, variances)
    nk = gam.sum(axis=0)
    K = nk.shape[0]
    w = nk / N
    mu = np.zeros((K, D))
    var = np.full((K, D), float(var_floor))
    for k in range(K):
        if nk[k] > 0:
            mu[k] = gam[:, k] @ X64 / nk[k]
            var[k] = np.maximum(gam[:, k] @ (X64 - mu[k]) ** 2 / nk[k], var_floor)
    logj = np.empty((N, K))
    for k in range(K):
        logj[:, k] = (np.log(w0[k]) - 0.5 * np.log(2 * np.pi * var0[k]).sum()
                      - 0.5 * (((X64 - mu0[k]) ** 2) / var0[k]).sum(axis=1))
    return w, mu, var, float(logsumexp(logj, axis=1).sum())
