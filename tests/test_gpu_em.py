"""EM training step (fv_em_step) on the device against the oracle's float64 EM step.

Tolerances, from the arithmetic: the step's inputs are the encoder's posteriors, whose relative
error is set by the logit error -- about 1e-5 in FP32 and 1e-3 for the split forms on ordinary
rows, up to ~1e-2 (split) on the uniform outlier rows, whose logits reach ~10^3 in magnitude.
A relative error delta in the gammas of a component moves mu_k by about delta E|x - mu_k| (a
few sigma) and var_k by delta E|z^2 - 1|; the sums' FP32 rounding, amplified by the
S2/S0 - mu^2 cancellation (1 + mu^2/var), adds ~1e-5.  A component with only a few
descriptors' worth of mass, fed mostly by soft outlier rows, carries those rows' error, so the
gates are two-fold:
  worst component, n_k >= 10   |d mu| / sigma, |d var| / var, |d w| / w
                               <= 1e-4 (FP32), 3e-3 (split)
  mass-weighted, n_k >= 1      sum_k n_k (|d mu|/sigma + |d var|/var) / N
                               <= 1e-5 (FP32), 1e-3 (split)
and |d w| <= tol w + 1e-7 for every component, the log-likelihood to 1e-6 relative (FP32),
1e-4 (split).
"""
import sys

import numpy as np
import pytest

import fvsynth
import oracle

pytestmark = pytest.mark.gpu


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


def _tol(prec):
    # (worst component, mass-weighted, log-likelihood)
    return (1e-4, 1e-5, 1e-6) if prec == 0 else (3e-3, 1e-3, 1e-4)


def check_step(name, got, ref, N, prec):
    w, mu, var, ll = got
    rw, rmu, rvar, rll = ref
    tol, tol_m, tol_ll = _tol(prec)
    nk = rw * N
    ok = nk >= 1.0
    big = nk >= 10.0
    sd = np.sqrt(rvar)
    d_mu = np.max(np.abs(mu - rmu) / sd, axis=1)
    d_var = np.max(np.abs(var - rvar) / rvar, axis=1)
    e_mu, e_var = d_mu[big].max(), d_var[big].max()
    e_w = np.max((np.abs(w - rw) / rw)[big])
    e_m = float(np.sum((nk * (d_mu + d_var))[ok]) / N)
    e_ll = abs(ll - rll) / abs(rll)
    say(f"  {name}: n_k>=10 worst mu {e_mu:.2e} var {e_var:.2e} w {e_w:.2e} (n_k>=1: mu "
        f"{d_mu[ok].max():.2e} var {d_var[ok].max():.2e}); mass-weighted {e_m:.2e}; loglik "
        f"{e_ll:.2e} ({big.sum()} / {ok.sum()} / {ok.size} components)")
    assert np.all(np.isfinite(mu)) and np.all(np.isfinite(var)) and np.all(var > 0)
    assert np.all(np.abs(w - rw) <= tol * rw + 1e-7)
    assert e_mu <= tol and e_var <= tol and e_w <= tol and e_m <= tol_m and e_ll <= tol_ll


CASES = [
    # (name, K, D, N, gmm_seed, frame_seed)
    ("k256_d64_n8000", 256, 64, 8000, 0, 100),
    ("k33_d17_n1000", 33, 17, 1000, 2, 3),
    ("k512_d80_n6000", 512, 80, 6000, 0, 12),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16_split"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_em_step_matches_oracle(fv, case, prec):
    import torch
    name, K, D, N, gs, fs = case
    say(f"[gpu] em step {name} prec={prec}")
    g = fvsynth.gmm(K, D, gs)
    X = fvsynth.frame(g, N, fs, 0.05)
    # start from a perturbed model so that the step moves the parameters
    rng = np.random.default_rng(gs + 1)
    mu0 = (g.means + 0.3 * rng.standard_normal(g.means.shape)).astype(np.float32)
    var0 = (g.variances * rng.uniform(0.8, 1.25, g.variances.shape)).astype(np.float32)
    h = fv.gmm_load(g.weights, mu0, var0)
    got = fv.em_step(h, torch.from_numpy(X).cuda(), precision=prec, var_floor=1e-3)
    ref = oracle.em_step(X, g.weights, mu0, var0, var_floor=1e-3)
    check_step(name, got, ref, N, prec)
    # host input gives the same bits
    goth = fv.em_step(h, X, precision=prec, var_floor=1e-3)
    for a, b in zip(got[:3], goth[:3]):
        assert np.array_equal(a, b)
    assert got[3] == goth[3]


def test_em_fit_increases_likelihood(fv):
    """Five FP32 iterations from a perturbed start: the log-likelihood never decreases (EM's
    monotonicity, up to the FP32 rounding of the likelihood) and every iteration agrees with
    the oracle's iteration from the same input model."""
    say("[gpu] em fit")
    K, D, N = 64, 32, 6000
    g = fvsynth.gmm(K, D, 5)
    X = fvsynth.frame(g, N, 50, 0.0)
    rng = np.random.default_rng(9)
    w = np.full(K, 1.0 / K, np.float32)
    mu = (g.means + 0.5 * rng.standard_normal(g.means.shape)).astype(np.float32)
    var = np.ones((K, D), np.float32)
    lls = []
    for it in range(5):
        h = fv.gmm_load(w, mu, var)
        got = fv.em_step(h, X, var_floor=1e-3)
        h.free()
        ref = oracle.em_step(X, w, mu, var, var_floor=1e-3)
        check_step(f"iter{it}", got, ref, N, 0)
        w, mu, var, ll = got
        lls.append(ll)
    say(f"  loglik: {[round(v, 3) for v in lls]}")
    for a, b in zip(lls, lls[1:]):
        assert b >= a - 1e-7 * abs(a)
    assert lls[-1] > lls[0]


def test_em_step_errors(fv):
    g = fvsynth.gmm(8, 4, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    with pytest.raises(fv.FvError):
        fv.em_step(h, np.zeros((0, 4), np.float32))
    with pytest.raises(fv.FvError):
        fv.em_step(h, np.zeros((5, 4), np.float32), var_floor=-1.0)


def test_em_single_component_closed_form(fv):
    """K = 1: every posterior is exactly 1, so the step returns w = 1, the sample mean and the
    biased sample variance (numpy, float64), and the log-likelihood of a single Gaussian."""
    say("[gpu] em K=1 closed form")
    rng = np.random.default_rng(4)
    D, N = 24, 5000
    X = (rng.standard_normal((N, D)) * rng.uniform(0.5, 2.0, D) + rng.uniform(-1, 1, D)).astype(np.float32)
    X64 = X.astype(np.float64)
    mu0 = np.zeros((1, D), np.float32)
    var0 = np.ones((1, D), np.float32)
    h = fv.gmm_load(np.ones(1, np.float32), mu0, var0)
    w, mu, var, ll = fv.em_step(h, X, var_floor=1e-6)
    assert w[0] == 1.0
    assert np.max(np.abs(mu[0] - X64.mean(axis=0)) / X64.std(axis=0)) < 1e-5
    assert np.max(np.abs(var[0] / X64.var(axis=0) - 1.0)) < 1e-5
    ll_ref = float(np.sum(-0.5 * (X64 ** 2).sum(axis=1) - 0.5 * D * np.log(2 * np.pi)))
    assert abs(ll - ll_ref) < 1e-6 * abs(ll_ref)
    # the variance floor binds for a constant feature
    Xc = X.copy()
    Xc[:, 3] = 0.25
    _, _, varc, _ = fv.em_step(h, Xc, var_floor=1e-3)
    assert varc[0, 3] == np.float32(1e-3)
