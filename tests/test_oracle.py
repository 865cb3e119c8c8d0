"""The FP64 oracle against facts fixed by the mathematics (not by its own formulas)."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from oracle import brute
import oracle_pins as P
from oracle.metrics import errors


@pytest.fixture(scope="module")
def o():
    return oracle._load()


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(o, pin):
    pin(o)


def test_mpmath_brute_force(o):
    rng = np.random.default_rng(7)
    for N, K, D in ((5, 3, 2), (6, 2, 2), (4, 1, 2), (3, 3, 1)):
        w = rng.dirichlet(np.ones(K)).astype(np.float32)
        mu = rng.standard_normal((K, D)).astype(np.float32)
        var = rng.uniform(0.5, 2.0, (K, D)).astype(np.float32)
        X = (rng.standard_normal((N, D)) * 1.5).astype(np.float32)
        for flags in (0, 1, 2, 3):
            ref = np.array(brute.encode(X, w, mu, var, power=not (flags & 1), l2=not (flags & 2)))
            got = o.encode(X, w, mu, var, flags=flags)
            assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_batch_equals_frames_bitwise(o):
    import fvsynth
    g = fvsynth.gmm(16, 8, 5)
    sizes = [0, 37, 1, 200, 64]
    X, off = fvsynth.batch_frames(g, sizes, seed0=40)
    for nt in (1, 4):
        got = o.encode_batch(X, off, g.weights, g.means, g.variances, nthreads=nt)
        for b in range(len(sizes)):
            ref = o.encode(X[off[b]:off[b + 1]], g.weights, g.means, g.variances)
            assert np.array_equal(got[b], ref)


def test_threshold_mode(o):
    import fvsynth
    g = fvsynth.gmm(8, 4, 1)
    X = fvsynth.frame(g, 300, 2, 0.05)
    base = o.encode(X, g.weights, g.means, g.variances)
    assert np.array_equal(o.encode(X, g.weights, g.means, g.variances, tau=0.0), base)
    assert np.all(o.encode(X, g.weights, g.means, g.variances, tau=2.0) == 0)
    # a threshold only removes terms with gamma <= tau: the change is bounded by them
    thr = o.encode(X, g.weights, g.means, g.variances, flags=3, tau=1e-6)
    raw = o.encode(X, g.weights, g.means, g.variances, flags=3)
    assert 0 < np.max(np.abs(thr - raw)) < 1e-4 * np.max(np.abs(raw))


def test_invalid_sizes(o):
    w = np.ones(1, np.float32)
    with pytest.raises(Exception):
        o.encode(np.zeros((1, 0), np.float32), w, np.zeros((1, 0), np.float32),
                 np.ones((1, 0), np.float32))


# Plant plausible mistakes in a copy of the oracle: each must be caught by at least one pin.
MUTANTS = {
    "drop_minus_one_in_V": ("(z * z - 1.0) * g", "(z * z) * g"),
    "sign_in_U": ("U[(size_t)k * D + d] += z * g;", "U[(size_t)k * D + d] -= z * g;"),
    "variance_as_std": ("s[(size_t)k * D + d] = 1.0 / sqrt(v);", "s[(size_t)k * D + d] = 1.0 / v;"),
    "drop_logdet": ("double l = log((double)w[k]) - logdet_half[k] - 0.5 * delta;",
                    "double l = log((double)w[k]) - 0.5 * delta;"),
    "drop_log_weight": ("double l = log((double)w[k]) - logdet_half[k] - 0.5 * delta;",
                        "double l = -logdet_half[k] - 0.5 * delta;"),
    "no_sqrt2_in_v": ("sqrt(2.0 * (double)w[k])", "sqrt((double)w[k])"),
    "weight_not_sqrt": ("double cu = 1.0 / ((double)N * sqrt((double)w[k]));",
                        "double cu = 1.0 / ((double)N * (double)w[k]);"),
    "transposed_mean": ("((double)x[d] - (double)mu[(size_t)k * D + d]) * s[(size_t)k * D + d];\n        U",
                        "((double)x[d] - (double)mu[(size_t)d * K % (K * D) + k % D]) * s[(size_t)k * D + d];\n        U"),
    "max_not_reset": ("double m = -INFINITY;\n    for (int k = 0; k < K; ++k) {\n      double delta",
                      "static double m = -INFINITY;\n    for (int k = 0; k < K; ++k) {\n      double delta"),
    "missing_half": ("- 0.5 * delta;", "- delta;"),
    "no_division_by_N": ("double cu = 1.0 / ((double)N * sqrt",
                         "double cu = 1.0 / ((double)1 * sqrt"),
    "l1_instead_of_l2": ("ss += out[i] * out[i];", "ss += fabs(out[i]);"),
    "threshold_inverted": ("if (tau >= 0.0 && !(g > tau)) continue;",
                           "if (tau >= 0.0 && (g > tau)) continue;"),
    "threshold_ignored": ("if (tau >= 0.0 && !(g > tau)) continue;",
                          "if (tau > 1e300 && !(g > tau)) continue;"),
    "unsigned_sqrt": ("out[i] = (p > 0.0) ? sqrt(p) : ((p < 0.0) ? -sqrt(-p) : 0.0);",
                      "out[i] = sqrt(fabs(p));"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    src = oracle.source()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as td:
        lib = oracle.compile_variant(mutated, os.path.join(td, f"mut_{name}.so"))
        caught = []
        for pin in P.ALL_PINS:
            try:
                pin(lib)
            except AssertionError:
                caught.append(pin.__name__)
            except Exception:
                caught.append(pin.__name__ + "(error)")
        assert caught, f"no pin catches mutant {name}"


def test_projection_brute_force_and_recovery():
    """oracle.project against a pure-Python loop on a tiny input (brute force), and on a
    synthetic raw frame it returns the GMM sample the frame was built from."""
    import fvsynth
    rng = np.random.default_rng(7)
    A = rng.standard_normal((3, 5)).astype(np.float32)
    m = rng.standard_normal(5).astype(np.float32)
    X = rng.standard_normal((4, 5)).astype(np.float32)
    got = oracle.project(X, A, m)
    for t in range(4):
        for c in range(3):
            ref = 0.0
            for k in range(5):
                ref += float(A[c, k]) * (float(X[t, k]) - float(m[k]))
            assert abs(got[t, c] - ref) <= 1e-14 * (1 + abs(ref))
    g = fvsynth.gmm(16, 64, 1)
    p = fvsynth.pca(64, 2)
    Xr = fvsynth.raw_frame(g, p, 300, 5, 0.05)
    y = fvsynth.frame(g, 300, 5, 0.05)
    assert np.max(np.abs(oracle.project(Xr, p.A, p.mean) - y)) < 2e-6
    # and the FV of the float64 projection agrees with the FV of the float32 sample it came from
    e = errors(oracle.encode_projected(Xr, p.A, p.mean, g), oracle.encode_gmm(y, g))
    assert e["e_2"] < 1e-4
