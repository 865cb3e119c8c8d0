"""Pins of the float64 dense-SIFT oracle (oracle/dsift.py) to facts outside it: library routines,
closed forms and exact symmetries of the definition.  Each pin takes the oracle module (or a
planted-mistake copy of it) and raises AssertionError when the module disagrees.

  gradient      numpy.gradient (central differences inside, one-sided first differences at
                the edges) on a random image
  binning       per pixel, the 8 orientation values sum to the gradient magnitude, and a
                gradient pointing exactly at a bin centre lands in that bin alone
  tri_conv      the direct convolution equals numpy.convolve with the triangle kernel, and the
                paper's two windowed sums (a width-B box sum, then another, Sec. 3.2)
  ramp          a linear ramp I = a x + b y: every interior descriptor is the closed form of 16
                equal spatial bins holding (1 - f) m and f m in orientation bins floor(t), +1
  edge          a vertical step edge with bin size 5 and stride 3: closed form of which spatial
                bins see the edge (pins the bin spacing and the value layout)
  constant      a constant image gives zero SIFT values at every descriptor
  transpose     the transposed image's descriptors are the original ones with x and y
                exchanged, spatial bins (i, j) -> (j, i) and orientation o -> (2 - o) mod 8,
                and the two centre coordinates swapped
  flip          the mirrored image's descriptors are the original ones mirrored, i -> 3 - i and
                o -> (4 - o) mod 8, and the x coordinate negated
  shift         moving the image by the stride moves interior descriptors by one grid step
                (to rounding)
  normalise     SIFT normalisation of a vector with one dominant entry (closed form)
  resize        factor 1/2 is the 2 x 2 box mean; a ramp stays a ramp (bilinear is exact on
                linear functions)
  count         the descriptor count of a 320 x 240 frame over the 8 scales, by hand
"""
from __future__ import annotations

import math

import numpy as np


def rand_img(H, W, seed):
    rng = np.random.default_rng(seed)
    # a smooth field plus noise, in [0, 1]
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    f = 0.5 + 0.25 * np.sin(xx / 7.0 + seed) * np.cos(yy / 5.0) + 0.1 * rng.standard_normal((H, W))
    return np.clip(f, 0.0, 1.0).astype(np.float32)


def pin_gradient(ds):
    img = rand_img(23, 31, 1).astype(np.float64)
    gx, gy = ds.gradient(img)
    ry, rx = np.gradient(img)
    assert np.allclose(gx, rx, rtol=0, atol=1e-15) and np.allclose(gy, ry, rtol=0, atol=1e-15)


def pin_binning(ds):
    img = rand_img(19, 17, 2).astype(np.float64)
    G = ds.orientation_maps(img)
    gx, gy = np.gradient(img)[1], np.gradient(img)[0]
    assert G.shape[0] == 8
    assert np.allclose(G.sum(axis=0), np.hypot(gx, gy), rtol=1e-13, atol=1e-15)
    assert np.all(G >= -1e-15)
    # a ramp whose gradient points at bin centre 3 (135 degrees): all mass in bin 3
    yy, xx = np.meshgrid(np.arange(9), np.arange(9), indexing="ij")
    ramp = -1.0 * xx + 1.0 * yy
    G = ds.orientation_maps(ramp)
    assert np.allclose(G[3], math.sqrt(2.0), rtol=1e-12)
    assert np.allclose(np.delete(G, 3, axis=0), 0.0, atol=1e-12)


def pin_tri_conv(ds):
    rng = np.random.default_rng(3)
    for B in (1, 2, 4, 5):
        x = rng.standard_normal(37)
        got = ds.tri_conv(x[None, :], B, axis=1)[0]
        k = np.array([(B - abs(d)) / (B * B) for d in range(-(B - 1), B)])
        assert np.allclose(got, np.convolve(x, k, mode="same"), rtol=0, atol=1e-13), B
        # the paper's form: a backward windowed sum of width B, then a forward one
        c = np.concatenate([[0.0], np.cumsum(np.concatenate([x, np.zeros(B)]))])
        s1 = np.array([c[t + 1] - c[max(0, t - B + 1)] for t in range(len(x) + B - 1)])
        c2 = np.concatenate([[0.0], np.cumsum(s1)])
        two = np.array([c2[min(len(s1), t + B)] - c2[t] for t in range(len(x))]) / (B * B)
        assert np.allclose(got, two, rtol=0, atol=1e-12), B


def pin_ramp(ds):
    B, S = 4, 4
    H, W = 40, 44
    a, b = 0.37, -0.21
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    rows = ds.descriptors(a * xx + b * yy, B, S)
    m = math.hypot(a, b)
    th = math.atan2(b, a) % (2 * math.pi)
    t = 8 * th / (2 * math.pi)
    o0 = int(math.floor(t))
    f = t - o0
    v = np.zeros(128)
    for sp in range(16):
        v[sp * 8 + o0 % 8] += (1 - f) * m
        v[sp * 8 + (o0 + 1) % 8] += f * m
    v = v / np.linalg.norm(v)
    v = np.minimum(v, 0.2)
    v = v / np.linalg.norm(v)
    n_in = 0
    for n, (x0, y0) in enumerate(ds.grid(H, W, B, S)):
        if x0 >= B and y0 >= B and x0 + 3 * B <= W - 1 - B and y0 + 3 * B <= H - 1 - B:
            assert np.allclose(rows[n, :128], v, rtol=0, atol=1e-12), (x0, y0)
            n_in += 1
    assert n_in >= 4


def pin_edge(ds):
    """A vertical step edge with bin size 5 and stride 3: only orientation 0 is nonzero, and the
    spatial bins that see the edge are those whose centre x0 + 5 i lies within 4 columns of
    the edge's two gradient columns (central differences 1/2 at c - 1 and c)."""
    B, S, c = 5, 3, 23
    H, W = 36, 47
    img = np.zeros((H, W))
    img[:, c:] = 1.0
    rows = ds.descriptors(img, B, S)

    def tri(d):
        return (B - abs(d)) / (B * B) if abs(d) < B else 0.0
    n_chk = 0
    for n, (x0, y0) in enumerate(ds.grid(H, W, B, S)):
        if y0 < B or y0 + 3 * B > H - 1 - B:
            continue  # rows whose vertical filter reaches the border
        v = np.zeros(128)
        for j in range(4):
            for i in range(4):
                x = x0 + i * B
                v[(4 * j + i) * 8] = 0.5 * (tri(c - 1 - x) + tri(c - x))
        if np.any(v):
            v = v / np.linalg.norm(v)
            v = np.minimum(v, 0.2)
            v = v / np.linalg.norm(v)
        assert np.allclose(rows[n, :128], v, rtol=0, atol=1e-12), (x0, y0)
        n_chk += 1
    assert n_chk >= 20


def pin_constant(ds):
    rows = ds.descriptors(np.full((30, 37), 0.6), 4, 4)
    assert rows.shape[0] > 0 and np.all(rows[:, :128] == 0.0)


def _perm_transpose():
    p = np.zeros(128, np.int64)
    for j in range(4):
        for i in range(4):
            for o in range(8):
                p[(4 * i + j) * 8 + (2 - o) % 8] = (4 * j + i) * 8 + o
    return p


def pin_transpose(ds):
    B, S = 4, 4
    img = rand_img(37, 37, 4).astype(np.float64)
    r = ds.descriptors(img, B, S)
    rt = ds.descriptors(img.T.copy(), B, S)
    pts = ds.grid(37, 37, B, S)
    idx = {p: n for n, p in enumerate(pts)}
    p = _perm_transpose()
    for n, (x0, y0) in enumerate(pts):
        nt = idx[(y0, x0)]
        assert np.allclose(rt[nt, p], r[n, :128], rtol=0, atol=1e-12), (x0, y0)
        assert rt[nt, 128] == r[n, 129] and rt[nt, 129] == r[n, 128]


def pin_flip(ds):
    B, S = 4, 4
    W = 3 * B + 1 + 6 * S  # the descriptor grid maps onto itself under mirroring
    img = rand_img(29, W, 5).astype(np.float64)
    r = ds.descriptors(img, B, S)
    rf = ds.descriptors(img[:, ::-1].copy(), B, S)
    pts = ds.grid(29, W, B, S)
    idx = {pt: n for n, pt in enumerate(pts)}
    p = np.zeros(128, np.int64)
    for j in range(4):
        for i in range(4):
            for o in range(8):
                p[(4 * j + (3 - i)) * 8 + (4 - o) % 8] = (4 * j + i) * 8 + o
    for n, (x0, y0) in enumerate(pts):
        nf = idx[(W - 1 - 3 * B - x0, y0)]
        assert np.allclose(rf[nf, p], r[n, :128], rtol=0, atol=1e-12), (x0, y0)
        # the centre mirrors: x -> -x, y unchanged
        assert abs(rf[nf, 128] + r[n, 128]) <= 1e-15 and rf[nf, 129] == r[n, 129]


def pin_shift(ds):
    B, S = 4, 4
    img = rand_img(33, 60, 6).astype(np.float64)
    sh = img[:, S:].copy()
    r = ds.descriptors(img, B, S)
    rs = ds.descriptors(sh, B, S)
    pa = {p: n for n, p in enumerate(ds.grid(33, 60, B, S))}
    ps = ds.grid(33, 60 - S, B, S)
    n_chk = 0
    for n, (x0, y0) in enumerate(ps):
        # support of a descriptor: bin centres +- (B - 1), gradients +- 1
        if x0 - B >= 0 and x0 + 3 * B + B <= 60 - S - 1:
            assert np.allclose(rs[n, :128], r[pa[(x0 + S, y0)], :128], rtol=0,
                               atol=1e-14), (x0, y0)
            n_chk += 1
    assert n_chk >= 4


def pin_normalise(ds):
    v = np.array([10.0] + [1.0] * 15)
    g = ds.normalise(v)
    # after the first L2 step the first entry exceeds 0.2 and is clamped; the others are
    # 1 / sqrt(115) < 0.2
    c = 1.0 / math.sqrt(115.0)
    ref = np.array([0.2] + [c] * 15)
    ref = ref / math.sqrt(0.04 + 15 * c * c)
    assert np.allclose(g, ref, rtol=0, atol=1e-15)
    assert np.all(ds.normalise(np.zeros(5)) == 0.0)


def pin_resize(ds):
    img = rand_img(20, 26, 7).astype(np.float64)
    half = ds.resize(img, 0.5)
    box = 0.25 * (img[0::2, 0::2] + img[1::2, 0::2] + img[0::2, 1::2] + img[1::2, 1::2])
    assert half.shape == (10, 13) and np.allclose(half, box, rtol=0, atol=1e-15)
    assert np.array_equal(ds.resize(img, 1.0), img)
    yy, xx = np.meshgrid(np.arange(30), np.arange(40), indexing="ij")
    ramp = 0.3 * xx - 0.7 * yy
    s = 1.0 / math.sqrt(2.0)
    r = ds.resize(ramp, s)
    ys = (np.arange(r.shape[0]) + 0.5) / s - 0.5
    xs = (np.arange(r.shape[1]) + 0.5) / s - 0.5
    inside = (ys[:, None] >= 0) & (ys[:, None] <= 29) & (xs[None, :] >= 0) & (xs[None, :] <= 39)
    ref = 0.3 * xs[None, :] - 0.7 * ys[:, None]
    assert np.allclose(r[inside], np.broadcast_to(ref, r.shape)[inside], rtol=0, atol=1e-12)


def pin_count(ds):
    # 8 scales sqrt(2) ... 1/8 of 320 x 240 (sizes round(s W) x round(s H)); B = S = 4:
    # per dimension floor((n - 13) / 4) + 1 descriptors
    sizes = [(453, 339), (320, 240), (226, 170), (160, 120), (113, 85), (80, 60), (57, 42),
             (40, 30)]
    n = sum(((w - 13) // 4 + 1) * ((h - 13) // 4 + 1) for w, h in sizes)
    assert ds.count(240, 320) == n
    img = rand_img(48, 64, 8)
    assert ds.extract(img, scales=[1.0, 0.5]).shape == (ds.count(48, 64, scales=[1.0, 0.5]), 130)


PINS = [pin_gradient, pin_binning, pin_tri_conv, pin_ramp, pin_edge, pin_constant, pin_transpose, pin_flip,
        pin_shift, pin_normalise, pin_resize, pin_count]
