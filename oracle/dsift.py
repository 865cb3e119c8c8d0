"""Flat-window dense SIFT in float64 -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The plain definition of the descriptor front end that feeds the Fisher-vector encoder
(Sec. 3.1 of the GPU-FV paper: per scale, every pixel's gradient falls into 8 orientation
bins, a triangular (flat-window) convolution follows, and each descriptor takes the 8
orientation values of 4 x 4 spatial bins, 128 values, sampled at a stride of S pixels;
Sec. 3.2: the triangular convolution is applied once along each image dimension; Sec. 4: a
stride of 4 and 9 scales from 2 down to 1/8 by factors of sqrt(2), 8 scales without the
largest one).  Written from the definitions, with no blocking, pruning or reordering: every
output value is its formula evaluated on the whole image.

Readings where the paper is silent (each one is a parameter or a documented choice here):
  resize       bilinear sampling at pixel centres, u = (x + 1/2) / s - 1/2, clamped to the
               image; output size round(s * W) x round(s * H)
  gradient     central differences (I[x+1] - I[x-1]) / 2 inside the image, one-sided
               differences at its first and last column / row
  orientation  t = 8 * atan2(gy, gx) / (2 pi) taken in [0, 8); the magnitude is shared by the
               two nearest bins, floor(t) with weight 1 - frac(t) and floor(t) + 1 (mod 8) with
               weight frac(t)
  flat window  tri(d) = (B - |d|) / B^2 for |d| < B, zero outside the image, along y then x
               (the convolution of two width-B windowed sums, normalised to sum 1)
  sampling     spatial bin (i, j) of a descriptor whose first bin centre is (x0, y0) reads the
               filtered maps at (x0 + i B, y0 + j B); descriptors start at x0 = y0 = 0 and step
               by S while x0 + 3B <= W - 1 and y0 + 3B <= H - 1; value index (4 j + i) * 8 + o
  normalise    SIFT's: L2 normalise, clamp entries at 0.2, L2 normalise again (a zero vector
               stays zero)
  coordinates  the descriptor centre (x0 + 1.5 B, y0 + 1.5 B), taken at its pixel's centre
               (+ 1/2), divided by the scaled image's width and height, minus 1/2, so that they
               lie in (-1/2, 1/2) and mirror exactly with the image; appended as two more
               values (Sec. 3.1's "normalized X and Y"), so a row has 130 values
"""
from __future__ import annotations

import math

import numpy as np

NBO = 8   # orientation bins (Sec. 3.1)
NBP = 4   # spatial bins per dimension (Sec. 3.1: 4 on X and 4 on Y)
CLAMP = 0.2


def paper_scales(n: int = 8):
    """Sec. 4: scales 2, 2/sqrt(2), ..., 1/8 (nine); the 8-scale setting drops the largest."""
    all9 = [2.0 ** (1.0 - 0.5 * k) for k in range(9)]
    return all9[9 - n:] if n <= 9 else all9


def resize(img, s: float):
    """Bilinear resize by factor s (reading above); s == 1 returns the image unchanged."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    if s == 1.0:
        return img.copy()
    Hs, Ws = int(round(s * H)), int(round(s * W))
    v = np.clip((np.arange(Hs) + 0.5) / s - 0.5, 0.0, H - 1.0)
    u = np.clip((np.arange(Ws) + 0.5) / s - 0.5, 0.0, W - 1.0)
    y0 = np.floor(v).astype(np.int64)
    x0 = np.floor(u).astype(np.int64)
    y1 = np.minimum(y0 + 1, H - 1)
    x1 = np.minimum(x0 + 1, W - 1)
    fy = (v - y0)[:, None]
    fx = (u - x0)[None, :]
    top = img[y0][:, x0] * (1.0 - fx) + img[y0][:, x1] * fx
    bot = img[y1][:, x0] * (1.0 - fx) + img[y1][:, x1] * fx
    return top * (1.0 - fy) + bot * fy


def gradient(img):
    """(gx, gy): central differences inside, one-sided at the borders (reading above)."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    gx = np.zeros((H, W))
    gy = np.zeros((H, W))
    if W > 1:
        gx[:, 1:W - 1] = 0.5 * (img[:, 2:] - img[:, :W - 2])
        gx[:, 0] = img[:, 1] - img[:, 0]
        gx[:, W - 1] = img[:, W - 1] - img[:, W - 2]
    if H > 1:
        gy[1:H - 1, :] = 0.5 * (img[2:, :] - img[:H - 2, :])
        gy[0, :] = img[1, :] - img[0, :]
        gy[H - 1, :] = img[H - 1, :] - img[H - 2, :]
    return gx, gy


def orientation_maps(img):
    """G [8, H, W]: each pixel's gradient magnitude shared by its two nearest orientation bins
    (Sec. 3.1: the gradients fall into 8 orientation bins)."""
    gx, gy = gradient(img)
    H, W = gx.shape
    m = np.hypot(gx, gy)
    th = np.arctan2(gy, gx)
    th = np.where(th < 0.0, th + 2.0 * math.pi, th)
    t = NBO * th / (2.0 * math.pi)
    t = np.where(t >= NBO, t - NBO, t)
    b = np.floor(t).astype(np.int64)
    f = t - b
    G = np.zeros((NBO, H, W))
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    np.add.at(G, (b % NBO, yy, xx), (1.0 - f) * m)
    np.add.at(G, ((b + 1) % NBO, yy, xx), f * m)
    return G


def tri_weight(d: int, B: int) -> float:
    return (B - abs(d)) / float(B * B) if abs(d) < B else 0.0


def tri_conv(a, B: int, axis: int):
    """Direct triangular convolution along `axis` with zero padding: out[t] = sum over |d| < B
    of tri(d) a[t + d] (Sec. 3.2's flat window, one dimension)."""
    a = np.asarray(a, dtype=np.float64)
    a = np.moveaxis(a, axis, -1)
    n = a.shape[-1]
    out = np.zeros_like(a)
    for t in range(n):
        acc = np.zeros(a.shape[:-1])
        for d in range(-(B - 1), B):
            if 0 <= t + d < n:
                acc = acc + tri_weight(d, B) * a[..., t + d]
        out[..., t] = acc
    return np.moveaxis(out, -1, axis)


def grid(H: int, W: int, B: int, S: int):
    """First-bin centres (x0, y0) of the descriptors of an H x W image, row-major in y0 then
    x0 (every bin centre inside the image)."""
    xs = list(range(0, W - 1 - 3 * B + 1, S)) if W - 1 - 3 * B >= 0 else []
    ys = list(range(0, H - 1 - 3 * B + 1, S)) if H - 1 - 3 * B >= 0 else []
    return [(x0, y0) for y0 in ys for x0 in xs]


def normalise(v):
    """SIFT normalisation: L2, clamp at 0.2, L2 (a zero vector stays zero)."""
    v = np.asarray(v, dtype=np.float64).copy()
    n = math.sqrt(float(np.sum(v * v)))
    if n == 0.0:
        return v
    v = v / n
    v = np.minimum(v, CLAMP)
    n = math.sqrt(float(np.sum(v * v)))
    return v / n if n > 0.0 else v


def descriptors(img, B: int = 4, S: int = 4):
    """Rows [N, 130] of one scale: 128 normalised SIFT values (index (4 j + i) * 8 + o) and the
    two normalised centre coordinates."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    G = orientation_maps(img)
    F = tri_conv(tri_conv(G, B, axis=1), B, axis=2)
    pts = grid(H, W, B, S)
    rows = np.zeros((len(pts), NBP * NBP * NBO + 2))
    for n, (x0, y0) in enumerate(pts):
        # v[(4 j + i) * 8 + o] = F[o, y0 + j B, x0 + i B]
        v = F[:, y0:y0 + NBP * B:B, x0:x0 + NBP * B:B].transpose(1, 2, 0).reshape(-1)
        rows[n, :128] = normalise(v)
        rows[n, 128] = (x0 + 1.5 * B + 0.5) / W - 0.5
        rows[n, 129] = (y0 + 1.5 * B + 0.5) / H - 0.5
    return rows


def extract(img, scales=None, B: int = 4, S: int = 4):
    """All scales' rows, concatenated in scale order (Sec. 3.1: descriptors are extracted for
    all the scales of the image)."""
    scales = paper_scales(8) if scales is None else scales
    img = np.asarray(img, dtype=np.float32).astype(np.float64)
    return np.concatenate([descriptors(resize(img, s), B, S) for s in scales], axis=0)


def count(H: int, W: int, scales=None, B: int = 4, S: int = 4) -> int:
    scales = paper_scales(8) if scales is None else scales
    n = 0
    for s in scales:
        Hs, Ws = (H, W) if s == 1.0 else (int(round(s * H)), int(round(s * W)))
        n += len(grid(Hs, Ws, B, S))
    return n
