"""Dense-SIFT front end (fv_dsift / fv_encode_images): the HIP path against the float64 oracle
(oracle/dsift.py, pinned in test_dsift_oracle.py) on seeded synthetic frames.

Gate for the descriptors (derived from the arithmetic): every value is a float32 evaluation of
the resampling (values in [0, 1]), central differences, the magnitude and angle, the two
window sums and SIFT's normalisation, about 30 roundings deep, each of relative size
u = 2^-24.  Before normalisation the error of a descriptor's vector v is then at most about
30 u * (sum of the magnitudes it holds) <= 30 u * sqrt(128) ||v|| (the entries are
non-negative), so after dividing by ||v|| (and the clamp and second division, which do not
enlarge it by more than a factor of 1 / ||clamped||, below 2.3 for these frames) every entry
is within ~ 30 * 11.3 * 2.3 u ~ 5e-5 in the worst case and a few u typically.  The gate is
    max |g - o| <= 2e-5 per value, and the per-descriptor L2 error <= 2e-5,
with the coordinates (one division each) within 2 u.  The FV of identical rows meets the
encoder's own gates (E_inf, E_2 <= 1e-5 FP32); the end-to-end FV from the image is gated at
1e-4 (the descriptors' float32 rounding propagates through the posteriors).
"""
import sys

import numpy as np
import pytest

import fvsynth
import oracle
from oracle import dsift as odsift
from oracle.metrics import errors

pytestmark = pytest.mark.gpu

DIM = 130
TOL_VAL = 2e-5
U = 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_03498_amd as fvmod
    fvmod.load()
    return fvmod


def compare_rows(name, got, ref):
    got = np.asarray(got, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    d = np.abs(got - ref)
    dv = d[:, :128]
    dc = d[:, 128:]
    per = np.sqrt(np.sum(dv * dv, axis=1)) if len(dv) else np.zeros(0)
    say(f"  {name}: rows={ref.shape[0]} max|d|={dv.max() if dv.size else 0:.3e} "
        f"max per-row L2={per.max() if per.size else 0:.3e} coords {dc.max() if dc.size else 0:.2e}")
    assert np.all(np.isfinite(got))
    if dv.size:
        assert dv.max() <= TOL_VAL and per.max() <= TOL_VAL
        assert np.all(dc <= 2 * U * np.maximum(np.abs(ref[:, 128:]), 0.5))


GEOMS = [
    # (name, H, W, scales (None: the paper's 8), bin, step)
    ("320x240_8scales", 240, 320, None, 4, 4),
    ("ragged_upsample", 97, 131, [2.0, 1.0, 0.7], 4, 4),
    ("bin6_step3", 150, 170, [1.0, 0.5], 6, 3),
    ("bin16_two_tiles", 60, 300, [1.0], 16, 7),
    ("bin1_step1_thin", 5, 600, [1.0, 1.3], 1, 1),
    ("bin3_step5_9scales", 200, 260, "nine", 3, 5),
]


@pytest.mark.parametrize("geom", GEOMS, ids=[g[0] for g in GEOMS])
def test_dsift_matches_oracle(fv, geom):
    import torch
    name, H, W, scales, B, S = geom
    img = fvsynth.image(H, W, 11 + H)
    if scales == "nine":
        sc, ns = None, 9
        osc = odsift.paper_scales(9)
    else:
        sc, ns = scales, (8 if scales is None else len(scales))
        osc = odsift.paper_scales(8) if scales is None else scales
    say(f"[gpu] dsift {name}: {H}x{W} bin={B} step={S}")
    ref = odsift.extract(img, osc, B, S)
    assert fv.dsift_rows(H, W, sc, ns, B, S) == ref.shape[0]
    got = fv.dsift(torch.from_numpy(img).cuda(), sc, ns, B, S).cpu().numpy()
    assert got.shape == (1, ref.shape[0], DIM)
    compare_rows(name, got[0], ref)


def test_dsift_640x480_paper_scales(fv):
    """The largest serving resolution, 8 scales (73,125 descriptors)."""
    import torch
    img = fvsynth.image(480, 640, 5)
    say("[gpu] dsift 640x480, 8 scales")
    ref = odsift.extract(img)
    got = fv.dsift(torch.from_numpy(img).cuda()).cpu().numpy()[0]
    compare_rows("640x480", got, ref)


def test_dsift_batch_equals_single_and_host(fv):
    """Several images in one call give each image's single-call rows bitwise; host input and
    output give the same bits as device input and output."""
    import torch
    imgs = fvsynth.images(3, 120, 160, 40)
    say("[gpu] dsift batch of 3 (120x160)")
    allr = fv.dsift(torch.from_numpy(imgs).cuda()).cpu().numpy()
    for i in range(3):
        one = fv.dsift(torch.from_numpy(imgs[i]).cuda()).cpu().numpy()[0]
        assert np.array_equal(allr[i], one)
    host = fv.dsift(imgs)
    assert isinstance(host, np.ndarray) and np.array_equal(host, allr)
    ref = odsift.extract(imgs[1])
    compare_rows("batch image 1", allr[1], ref)


def test_dsift_constant_and_empty(fv):
    """A constant image has no gradient: every SIFT value is exactly zero (coordinates as
    usual).  An image too small for one descriptor yields no rows and no launch; zero images
    is a no-op."""
    import torch
    img = np.full((64, 80), 0.37, np.float32)
    got = fv.dsift(torch.from_numpy(img).cuda(), [1.0, 0.5]).cpu().numpy()[0]
    ref = odsift.extract(img, [1.0, 0.5])
    assert got.shape == ref.shape
    assert np.all(got[:, :128] == 0.0)
    compare_rows("constant", got, ref)
    assert fv.dsift_rows(10, 10, [1.0], 1, 4, 4) == 0
    out = fv.dsift(torch.zeros(10, 10, device="cuda"), [1.0], 1, 4, 4)
    assert tuple(out.shape) == (1, 0, DIM)
    out = fv.dsift(torch.zeros(0, 40, 40, device="cuda"), [1.0], 1, 4, 4)
    assert tuple(out.shape) == (0, fv.dsift_rows(40, 40, [1.0], 1, 4, 4), DIM)


def test_dsift_rejects_bad_arguments(fv):
    for args in [(0, 10, [1.0], 1, 4, 4), (10, 10, [0.0], 1, 4, 4), (10, 10, [1.0], 1, 0, 4),
                 (10, 10, [1.0], 1, 4, 0), (10, 10, [float("nan")], 1, 4, 4),
                 (10, 10, None, 10, 4, 4)]:
        with pytest.raises(fv.FvError) as ei:
            fv.dsift_rows(*args)
        assert ei.value.code == fv.E_INVAL
    with pytest.raises(fv.FvError) as ei:
        fv.dsift_rows(10, 10, [1.0], 1, 17, 4)
    assert ei.value.code == fv.E_UNSUPPORTED


def image_gmm(y, K, seed):
    """A GMM placed on the projected rows (test data, not the method): means at K random rows,
    every variance a quarter of the rows' per-dimension variance, equal weights."""
    rng = np.random.default_rng(seed)
    mu = y[rng.choice(y.shape[0], K, replace=False)]
    var = np.tile(np.maximum(y.var(axis=0) * 0.25, 1e-4), (K, 1))
    w = np.full(K, 1.0 / K)
    return fvsynth.Gmm(weights=w.astype(np.float32), means=mu.astype(np.float32),
                       variances=var.astype(np.float32), weights64=w)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16_split"])
def test_encode_images_chain(fv, prec):
    """fv_encode_images = fv_dsift -> projection -> encode: for two 320 x 240 frames (too few
    chunks to fill the GPU as one batch) each image goes through fv_encode, bitwise the same as
    the separate calls; the FV of the GPU's own rows meets the encoder gates against the
    oracle's float64 projection and encode; end to end from the images, within 1e-4."""
    import torch
    tol = {0: 1e-5, 1: 1e-3}[prec]
    imgs = fvsynth.images(2, 240, 320, 70)
    p = fvsynth.pca(64, 9)
    ph = fv.pca_load(p.A, p.mean)
    y0 = oracle.project(odsift.extract(imgs[0]), p.A, p.mean)
    g = image_gmm(y0, 256, 3)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    say(f"[gpu] encode_images 2 x 320x240, K=256 D=64 prec={prec}")
    imd = torch.from_numpy(imgs).cuda()
    got = fv.encode_images(h, ph, imd, precision=prec).cpu().numpy()
    rows = fv.dsift(imd)
    sep = np.stack([fv.encode_projected(h, ph, rows[i].contiguous(), precision=prec).cpu().numpy()
                    for i in range(2)])
    assert np.array_equal(got, sep)
    rows_h = rows.cpu().numpy()
    for i in range(2):
        ref_rows = oracle.encode_projected(rows_h[i], p.A, p.mean, g)
        e = errors(got[i], ref_rows)
        say(f"  image {i} vs oracle on the GPU rows: e_inf={e['e_inf']:.2e} e_2={e['e_2']:.2e}")
        assert e["e_inf"] <= tol and e["e_2"] <= tol
        ref_all = oracle.encode_projected(odsift.extract(imgs[i]), p.A, p.mean, g)
        e2 = errors(got[i], ref_all)
        say(f"  image {i} end to end vs oracle: e_inf={e2['e_inf']:.2e} e_2={e2['e_2']:.2e}")
        assert e2["e_inf"] <= max(tol, 1e-4) and e2["e_2"] <= max(tol, 1e-4)
    host = fv.encode_images(h, ph, imgs, precision=prec)
    assert np.array_equal(host, got)
    h.free()
    ph.free()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16_split"])
def test_encode_images_batch(fv, prec):
    """Seventy 120 x 160 frames fill the GPU as one batch: fv_encode_images equals the dense
    SIFT rows encoded by fv_encode_batch_projected (one frame per image) bitwise, and two of its
    vectors meet the gates against the oracle's chain from those images."""
    import torch
    imgs = fvsynth.images(70, 120, 160, 500)
    p = fvsynth.pca(64, 4)
    ph = fv.pca_load(p.A, p.mean)
    y0 = oracle.project(odsift.extract(imgs[0]), p.A, p.mean)
    g = image_gmm(y0, 256, 5)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    say(f"[gpu] encode_images 70 x 160x120 prec={prec}")
    imd = torch.from_numpy(imgs).cuda()
    got = fv.encode_images(h, ph, imd, precision=prec).cpu().numpy()
    rows = fv.dsift(imd)
    n = rows.shape[1]
    off = np.arange(71, dtype=np.int64) * n
    sep = fv.encode_batch_projected(h, ph, rows.reshape(-1, DIM), off, precision=prec).cpu().numpy()
    assert np.array_equal(got, sep)
    tol = {0: 1e-4, 1: 1e-3}[prec]
    for i in (0, 69):
        ref = oracle.encode_projected(odsift.extract(imgs[i]), p.A, p.mean, g)
        e = errors(got[i], ref)
        say(f"  image {i}: e_inf={e['e_inf']:.2e} e_2={e['e_2']:.2e}")
        assert e["e_inf"] <= tol and e["e_2"] <= tol
    h.free()
    ph.free()
