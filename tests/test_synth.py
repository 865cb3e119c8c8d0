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


def test_serving_plan():
    ev, sizes = fvsynth.serving_plan(duration_s=2.0)
    assert sizes[:5] == [8000, 12500, 18000, 24500, 32000]
    assert all(ev[i][0] <= ev[i + 1][0] for i in range(len(ev) - 1))
    assert 16 * 30 * 2 * 0.7 < len(ev) < 16 * 30 * 2 * 1.3
