"""The error measures of oracle.metrics on constructed vectors (CPU)."""
import numpy as np

from oracle.metrics import errors, per_block, raw_errors


def _unit(phi):
    """The improved-FV normalisation of a raw vector: signed square root, then unit L2."""
    p = np.sign(phi) * np.sqrt(np.abs(phi))
    return p / np.linalg.norm(p)


def test_identical_and_zero_vectors():
    rng = np.random.default_rng(0)
    o = _unit(rng.standard_normal(64))
    assert errors(o, o) == {"e_inf": 0.0, "e_2": 0.0, "e_1": 0.0}
    z = np.zeros(16)
    e = errors(z, z)
    assert e["e_inf"] == 0.0 and e["e_2"] == 0.0 and e["e_1"] == 0.0
    # a nonzero candidate against a zero reference: absolute differences
    e = errors(np.full(16, 0.5), z)
    assert e["e_inf"] == 0.25 and np.isclose(e["e_2"], 2.0)


def test_s_domain_undoes_the_square_root():
    """For o = unit(phi), s(o) = o|o| equals phi / ||phi||_1 exactly (up to rounding)."""
    rng = np.random.default_rng(1)
    phi = rng.standard_normal(200) * np.exp(rng.uniform(-8, 0, 200))
    o = _unit(phi)
    assert np.allclose(o * np.abs(o), phi / np.abs(phi).sum(), rtol=1e-12, atol=1e-18)


def test_sign_flip_and_single_entry():
    rng = np.random.default_rng(2)
    o = _unit(rng.standard_normal(50))
    e = errors(-o, o)
    assert np.isclose(e["e_inf"], 2.0) and np.isclose(e["e_2"], 2.0)
    g = o.copy()
    i = int(np.argmax(np.abs(o)))
    g[i] *= 1.0 + 1e-6
    s = lambda y: y * np.abs(y)
    expect = abs(s(g[i]) - s(o[i])) / np.max(np.abs(s(o)))
    e = errors(g, o)
    assert np.isclose(e["e_inf"], expect, rtol=1e-9)
    assert np.isclose(e["e_2"], abs(g[i] - o[i]), rtol=1e-9)


def test_normalise_and_raw():
    rng = np.random.default_rng(3)
    o = rng.standard_normal(40)
    assert errors(3.0 * o, o, normalise=True)["e_inf"] < 1e-15
    r = raw_errors(o * (1 + 1e-7), o)
    assert np.isclose(r["rel_inf"], 1e-7 * np.max(np.abs(o)) / np.max(np.abs(o)), rtol=1e-6)
    assert np.isclose(r["rel_2"], 1e-7, rtol=1e-6)


def test_per_block_locates_the_error():
    K, D = 8, 5
    rng = np.random.default_rng(4)
    o = _unit(rng.standard_normal(2 * K * D))
    g = o.copy()
    g[K * D + 3 * D + 2] += 1e-4  # v block of component 3
    pb = per_block(g, o, K, D, worst=3)
    assert pb["worst"][0][:2] == ("v", 3)
    assert sum(pb["log10_hist"].values()) == 2 * K
    assert np.isclose(pb["max"], errors(g, o)["e_inf"])
