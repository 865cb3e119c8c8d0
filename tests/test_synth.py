"""Seeded generators: reproducible bytes, shapes and the outlier recipe."""
import json
import os

import numpy as np

import fvsynth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_manifest_matches():
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "golden", "make_synth_manifest.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    with open(os.path.join(HERE, "golden", "synth_manifest.json")) as f:
        stored = json.load(f)
    assert mk.manifest() == stored


def test_frame_recipe():
    g = fvsynth.gmm(256, 64, 0)
    assert g.weights.dtype == np.float32 and g.means.shape == (256, 64)
    assert g.variances.min() >= 0.5 and g.variances.max() <= 2.0
    X = fvsynth.frame(g, 8000, 100, 0.05)
    assert X.shape == (8000, 64) and X.dtype == np.float32
    # exactly round(0.05 N) rows are uniform outliers in [-4, 4]; they are bounded
    assert np.abs(X).max() < 20
    # the clustered frame holds the same rows, reordered so that labels do not decrease
    Xc = fvsynth.frame(g, 8000, 100, 0.05, clustered=True)
    assert np.array_equal(np.sort(Xc.view(np.uint32), axis=None), np.sort(X.view(np.uint32), axis=None))
    assert not np.array_equal(Xc, X)
    sizes = fvsynth.batch_sizes(64, 1)
    assert sizes.min() >= 2000 and sizes.max() <= 20000 and len(sizes) == 64


def test_pca_recipe():
    g = fvsynth.gmm(32, 64, 0)
    p = fvsynth.pca(64, 0)
    assert p.A.shape == (64, 130) and p.mean.shape == (130,) and p.A.dtype == np.float32
    Q = p.A[:62, :128].astype(np.float64)
    assert np.allclose(Q @ Q.T, np.eye(62), atol=1e-6)           # orthonormal rows
    assert np.array_equal(p.A[62:, 128:], np.eye(2, dtype=np.float32))  # coordinates pass
    assert np.all(p.A[62:, :128] == 0) and np.all(p.A[:62, 128:] == 0) and np.all(p.mean[128:] == 0)
    X = fvsynth.raw_frame(g, p, 500, 3, 0.05)
    assert X.shape == (500, 130) and X.dtype == np.float32
    # the coordinates are the last two dimensions of the GMM sample, unchanged
    y = fvsynth.frame(g, 500, 3, 0.05)
    assert np.array_equal(X[:, 128:], y[:, 62:])


def test_serving_plan():
    ev, sizes = fvsynth.serving_plan(duration_s=2.0)
    assert sizes[:5] == [8000, 12500, 18000, 24500, 32000]
    assert all(ev[i][0] <= ev[i + 1][0] for i in range(len(ev) - 1))
    assert 16 * 30 * 2 * 0.7 < len(ev) < 16 * 30 * 2 * 1.3
