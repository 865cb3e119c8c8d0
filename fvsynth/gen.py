"""Seeded generators (numpy PCG64).  Recipes:

* gmm(K, D, seed): rng = default_rng(seed); weights ~ Dirichlet(1_K), means ~ N(0,1)^{KxD},
  variances ~ U[0.5, 2]^{KxD}, drawn in that order.  All three are cast to float32 and the
  float32 arrays *are* the model.  The float64 weights are kept only for sampling labels.
* frame(g, N, seed, outlier_frac): rng = default_rng(seed); labels ~ Cat(weights64);
  x = mean[label] + sqrt(var[label]) * z, z ~ N(0, I); then round(outlier_frac*N) rows,
  chosen without replacement, are replaced by U[-4, 4]^D.  Cast to float32.  With
  clustered=True the rows are then stably reordered by label (a frame whose neighbouring
  descriptors come from the same component, as neighbouring patches of one region do).
* batch_sizes(B, seed=1, lo=2000, hi=20000): default_rng(seed).integers(lo, hi+1, B).
* pca(D, seed, n_sift=128): a stand-in for a trained PCA of 128-D SIFT descriptors reduced to
  m = D - 2 dimensions plus two appended coordinates.  rng = default_rng(seed);
  Q = orthonormal [n_sift x m] (QR of N(0,1)^{n_sift x m}, signs fixed so diag(R) > 0);
  sift_mean ~ U[0, 0.2]^{n_sift}.  A = [[Q^T, 0], [0, I_2]] ([D x (n_sift + 2)]) and
  mean = [sift_mean, 0, 0], cast to float32.
* raw_frame(g, p, N, seed, outlier_frac, noise=0.05): y = frame(g, N, seed, outlier_frac) in
  D dimensions; n ~ N(0, noise^2)^{N x n_sift} from default_rng(seed + 1_000_003);
  sift = sift_mean + y[:, :m] Q^T + n (I - Q Q^T); raw = [sift, y[:, m:]], cast to float32.
  So A (raw - mean) = y up to the float32 rounding of raw.
* image(H, W, seed): a grayscale video-frame stand-in in [0, 1]: rng = default_rng(seed);
  a smooth field sum_{q<6} a_q sin(2 pi (f_q . (x, y)) + p_q) with a_q ~ U[0.05, 0.2],
  |f_q| ~ U[1/64, 1/8] cycles per pixel at a uniform angle, p_q ~ U[0, 2 pi); plus 12
  axis-aligned rectangles (corners uniform in the frame) adding U[-0.3, 0.3] each; plus
  N(0, 0.03^2) pixel noise; then mapped affinely onto [0, 1] (no clipping), cast to float32.
* serving_plan(...): 16 streams, Poisson arrivals at a rate per stream, resolutions
  assigned round-robin from 320x240 .. 640x480, N = 8000 * area / (320*240).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Gmm:
    weights: np.ndarray    # [K] float32
    means: np.ndarray      # [K, D] float32
    variances: np.ndarray  # [K, D] float32
    weights64: np.ndarray  # [K] float64 (sampling only)

    @property
    def K(self) -> int:
        return int(self.means.shape[0])

    @property
    def D(self) -> int:
        return int(self.means.shape[1])


def gmm(K: int, D: int, seed: int = 0) -> Gmm:
    rng = np.random.default_rng(seed)
    w64 = rng.dirichlet(np.ones(K))
    mu = rng.standard_normal((K, D))
    var = rng.uniform(0.5, 2.0, (K, D))
    return Gmm(weights=w64.astype(np.float32), means=mu.astype(np.float32),
               variances=var.astype(np.float32), weights64=w64)


def frame(g: Gmm, N: int, seed: int, outlier_frac: float = 0.0,
          clustered: bool = False) -> np.ndarray:
    rng = np.random.default_rng(seed)
    K, D = g.K, g.D
    labels = rng.choice(K, size=N, p=g.weights64 / g.weights64.sum())
    z = rng.standard_normal((N, D))
    mu = g.means.astype(np.float64)
    sd = np.sqrt(g.variances.astype(np.float64))
    x = mu[labels] + sd[labels] * z
    n_out = int(round(outlier_frac * N))
    if n_out > 0:
        rows = rng.choice(N, size=n_out, replace=False)
        x[rows] = rng.uniform(-4.0, 4.0, (n_out, D))
    if clustered:
        x = x[np.argsort(labels, kind="stable")]
    return np.ascontiguousarray(x.astype(np.float32))


@dataclass(frozen=True)
class Pca:
    A: np.ndarray      # [D, Din] float32
    mean: np.ndarray   # [Din] float32
    Q: np.ndarray      # [n_sift, m] float64 (generation only)

    @property
    def Din(self) -> int:
        return int(self.A.shape[1])

    @property
    def D(self) -> int:
        return int(self.A.shape[0])


def pca(D: int, seed: int = 0, n_sift: int = 128) -> Pca:
    m = D - 2
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n_sift, m)))
    q = q * np.sign(np.diag(r))[None, :]
    sift_mean = rng.uniform(0.0, 0.2, n_sift)
    A = np.zeros((D, n_sift + 2))
    A[:m, :n_sift] = q.T
    A[m, n_sift] = 1.0
    A[m + 1, n_sift + 1] = 1.0
    mean = np.concatenate([sift_mean, [0.0, 0.0]])
    return Pca(A=A.astype(np.float32), mean=mean.astype(np.float32), Q=q)


def raw_frame(g: Gmm, p: Pca, N: int, seed: int, outlier_frac: float = 0.0,
              noise: float = 0.05) -> np.ndarray:
    y = frame(g, N, seed, outlier_frac).astype(np.float64)
    q = p.Q
    m = q.shape[1]
    n = np.random.default_rng(seed + 1_000_003).standard_normal((N, q.shape[0])) * noise
    perp = n - (n @ q) @ q.T
    sift = p.mean[:q.shape[0]].astype(np.float64) + y[:, :m] @ q.T + perp
    return np.ascontiguousarray(np.concatenate([sift, y[:, m:]], axis=1).astype(np.float32))


def raw_batch(g: Gmm, p: Pca, sizes, seed0: int = 200, outlier_frac: float = 0.05):
    frames = [raw_frame(g, p, int(n), seed0 + f, outlier_frac) for f, n in enumerate(sizes)]
    offsets = np.zeros(len(frames) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([f.shape[0] for f in frames])
    X = np.concatenate(frames, axis=0) if frames else np.zeros((0, p.Din), np.float32)
    return np.ascontiguousarray(X), offsets


def batch_sizes(B: int, seed: int = 1, lo: int = 2000, hi: int = 20000) -> np.ndarray:
    return np.random.default_rng(seed).integers(lo, hi + 1, B).astype(np.int64)


def batch_frames(g: Gmm, sizes, seed0: int = 200, outlier_frac: float = 0.05):
    """Frames of the given sizes, frame f drawn with seed seed0 + f.  Returns (X, offsets)."""
    frames = [frame(g, int(n), seed0 + f, outlier_frac) for f, n in enumerate(sizes)]
    offsets = np.zeros(len(frames) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([f.shape[0] for f in frames])
    X = np.concatenate(frames, axis=0) if frames else np.zeros((0, g.D), np.float32)
    return np.ascontiguousarray(X), offsets


def image(H: int, W: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    f = np.zeros((H, W))
    for _ in range(6):
        a = rng.uniform(0.05, 0.2)
        fr = rng.uniform(1.0 / 64, 1.0 / 8)
        ang = rng.uniform(0.0, 2 * np.pi)
        ph = rng.uniform(0.0, 2 * np.pi)
        f += a * np.sin(2 * np.pi * fr * (np.cos(ang) * xx + np.sin(ang) * yy) + ph)
    for _ in range(12):
        x0, x1 = np.sort(rng.integers(0, W + 1, 2))
        y0, y1 = np.sort(rng.integers(0, H + 1, 2))
        f[y0:y1, x0:x1] += rng.uniform(-0.3, 0.3)
    f += rng.standard_normal((H, W)) * 0.03
    lo, hi = f.min(), f.max()
    f = (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)
    return np.ascontiguousarray(f.astype(np.float32))


def images(n: int, H: int, W: int, seed0: int = 0) -> np.ndarray:
    """n frames, frame i drawn by image(H, W, seed0 + i): [n, H, W] float32."""
    return np.ascontiguousarray(np.stack([image(H, W, seed0 + i) for i in range(n)]))


RESOLUTIONS = ((320, 240), (400, 300), (480, 360), (560, 420), (640, 480))


def serving_plan(n_streams: int = 16, rate_hz: float = 30.0, duration_s: float = 22.0,
                 pool: int = 8, base_n: int = 8000):
    """Open-loop arrival schedule: list of (t_arrival_s, stream, pool_index), sorted by time,
    plus the descriptor count of each stream.  Stream s uses default_rng(10000 + s) for its
    exponential inter-arrival gaps; its pool frame p is drawn with seed 100000 + 100*s + p."""
    sizes = []
    events = []
    for s in range(n_streams):
        w, h = RESOLUTIONS[s % len(RESOLUTIONS)]
        sizes.append(int(round(base_n * (w * h) / (320 * 240))))
        rng = np.random.default_rng(10000 + s)
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= duration_s:
                break
            events.append((t, s, k % pool))
            k += 1
    events.sort()
    return events, sizes


# Named workloads (K, D, N or batch recipe).  Descriptions only; data is drawn on demand.
WORKLOADS = {
    "c1_oracle_k64_d64_n2000": dict(K=64, D=64, gmm_seed=0, N=2000, frame_seed=0, outliers=0.0),
    "c2_frame_k256_d64_n8000": dict(K=256, D=64, gmm_seed=0, N=8000, frame_seed=100, outliers=0.05),
    "c4_batch64_k256_d64": dict(K=256, D=64, gmm_seed=0, B=64, sizes_seed=1, frame_seed0=200,
                                outliers=0.05),
    "c5_serving_k512_d80": dict(K=512, D=80, gmm_seed=0, streams=16, rate_hz=30.0),
}


def workload(name: str):
    """Return (gmm, X, offsets) for a single-frame or batch workload."""
    w = WORKLOADS[name]
    g = gmm(w["K"], w["D"], w["gmm_seed"])
    if "N" in w:
        X = frame(g, w["N"], w["frame_seed"], w["outliers"])
        return g, X, np.array([0, X.shape[0]], dtype=np.int64)
    if "B" in w:
        sizes = batch_sizes(w["B"], w["sizes_seed"])
        X, off = batch_frames(g, sizes, w["frame_seed0"], w["outliers"])
        return g, X, off
    raise ValueError(f"workload {name} is not a frame or batch workload")


def array_sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
