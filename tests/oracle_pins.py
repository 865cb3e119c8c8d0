"""Checks that pin the FP64 oracle to facts other than its own formulas.

Each function takes an ``OracleLib`` (the real build, or a copy with a planted mistake) and
raises AssertionError when the oracle disagrees with the fact it checks.  The facts:

* posteriors == sklearn GaussianMixture(covariance_type='diag').predict_proba  (library)
* posteriors of two equal-variance 1-D components == logistic in x             (closed form)
* U_kd == sigma_kd * sum_t d log p(x_t) / d mu_kd and
  V_kd == sigma_kd * sum_t d log p(x_t) / d sigma_kd, with log p from
  torch.distributions (MixtureSameFamily), differentiated by autograd           (library)
* K = 1: u, v from the sample mean and biased variance (numpy)                  (closed form)
* descriptors placed on well-separated means: u == 0, v_k == -n_k/(N sqrt(2 w_k))
* x drawn from the model: sqrt(N) u and sqrt(N) v have mean 0, variance 1      (statistics)
  -- this pins the 1/sqrt(w_k) and 1/sqrt(2 w_k) normalisations, which the paper does
  not print
* translation, scaling, negation, component / descriptor permutation, duplication
* ||phi||_2 == 1 after L2; N = 0 and phi == 0 give zeros                         (definition)
* EM step: n_k, means and variances == sklearn's diagonal M-step
  (_estimate_gaussian_parameters, reg_covar 0) on the sklearn posteriors, log-likelihood ==
  sum of GaussianMixture.score_samples                                          (library)
* with the posterior threshold tau (Algorithm 1's test), U and V == the autograd
  per-descriptor gradients summed over the (t, k) whose torch posterior exceeds tau
                                                                                 (library)
"""
from __future__ import annotations

import numpy as np

RAW = 3  # NO_POWER | NO_L2


def _dyadic_model(rng, K, D, scale=16.0):
    w = rng.dirichlet(np.ones(K)).astype(np.float32)
    mu = (np.round(rng.standard_normal((K, D)) * scale) / scale).astype(np.float32)
    var = (1.0 + rng.integers(0, 16, (K, D)) / 16.0).astype(np.float32) * 0.5
    return w, mu, var


def _dyadic_X(rng, N, D, scale=16.0):
    return (np.round(rng.standard_normal((N, D)) * 1.3 * scale) / scale).astype(np.float32)


def pin_posteriors_sklearn(o, seed=0):
    from sklearn.mixture import GaussianMixture
    rng = np.random.default_rng(seed)
    for K, D, N in ((5, 3, 200), (16, 8, 300)):
        w = rng.dirichlet(np.ones(K)).astype(np.float32)
        mu = (rng.standard_normal((K, D)) * 0.7).astype(np.float32)
        var = rng.uniform(0.5, 2.0, (K, D)).astype(np.float32)
        X = (rng.standard_normal((N, D)) * 1.2).astype(np.float32)
        # rows on the means first, then descriptors far from every component: the posteriors
        # must stay finite and normalised (the shift by the row maximum is per descriptor)
        far = np.full((3, D), 60.0, np.float32) * np.array([[1], [-1], [0.5]], np.float32)
        X = np.concatenate([mu, X, far]).astype(np.float32)
        gm = GaussianMixture(n_components=K, covariance_type="diag")
        gm.weights_ = w.astype(np.float64)
        gm.means_ = mu.astype(np.float64)
        gm.covariances_ = var.astype(np.float64)
        gm.precisions_cholesky_ = 1.0 / np.sqrt(var.astype(np.float64))
        ref = gm.predict_proba(X.astype(np.float64))
        got = o.posteriors(X, w, mu, var)
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) < 1e-12, np.max(np.abs(got - ref))
        assert np.max(np.abs(got.sum(1) - 1.0)) < 1e-14
        assert got.min() >= 0.0 and got.max() <= 1.0


def pin_posteriors_logistic(o):
    # two 1-D components with a common variance: log(g1/g2) = a + b x (linear discriminant)
    w = np.array([0.375, 0.625], np.float32)
    mu = np.array([[-0.5], [1.25]], np.float32)
    var = np.array([[0.75], [0.75]], np.float32)
    x = np.linspace(-3, 3, 97).astype(np.float32)[:, None]
    w64, m64, v64 = w.astype(np.float64), mu[:, 0].astype(np.float64), float(var[0, 0])
    a = np.log(w64[0] / w64[1]) - (m64[0] ** 2 - m64[1] ** 2) / (2 * v64)
    b = (m64[0] - m64[1]) / v64
    g1 = 1.0 / (1.0 + np.exp(-(a + b * x[:, 0].astype(np.float64))))
    got = o.posteriors(x, w, mu, var)
    assert np.max(np.abs(got[:, 0] - g1)) < 1e-13
    assert np.max(np.abs(got[:, 1] - (1 - g1))) < 1e-13


def pin_gradient_autograd(o, seed=1):
    import torch
    from torch.distributions import Categorical, Independent, MixtureSameFamily, Normal
    rng = np.random.default_rng(seed)
    for K, D, N in ((4, 3, 150), (12, 6, 400)):
        w = rng.dirichlet(np.ones(K)).astype(np.float32)
        mu = (rng.standard_normal((K, D)) * 0.8).astype(np.float32)
        var = rng.uniform(0.5, 2.0, (K, D)).astype(np.float32)
        X = (rng.standard_normal((N, D)) * 1.3).astype(np.float32)
        mu_t = torch.tensor(mu.astype(np.float64), requires_grad=True)
        sd_t = torch.tensor(np.sqrt(var.astype(np.float64)), requires_grad=True)
        mix = MixtureSameFamily(Categorical(probs=torch.tensor(w.astype(np.float64))),
                                Independent(Normal(mu_t, sd_t), 1))
        mix.log_prob(torch.tensor(X.astype(np.float64))).sum().backward()
        sd = sd_t.detach().numpy()
        U_ref = sd * mu_t.grad.numpy()
        V_ref = sd * sd_t.grad.numpy()
        phi = o.encode(X, w, mu, var, flags=RAW)
        w64 = w.astype(np.float64)[:, None]
        U = phi[:K * D].reshape(K, D) * N * np.sqrt(w64)
        V = phi[K * D:].reshape(K, D) * N * np.sqrt(2 * w64)
        for got, ref in ((U, U_ref), (V, V_ref)):
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            assert err < 1e-11, err


def pin_threshold_autograd(o, seed=5, tau=1e-6):
    """Threshold mode against per-descriptor gradients: the (t, k) term of U (V) is the
    gradient of log p(x_t) with respect to mu_k (sigma_k) times sigma_k; the term enters only
    when the posterior of k given x_t, from torch's log densities, exceeds tau."""
    import torch
    from torch.distributions import Categorical, Independent, MixtureSameFamily, Normal
    rng = np.random.default_rng(seed)
    K, D, N = 6, 4, 120
    w = rng.dirichlet(np.ones(K) * 2).astype(np.float32)
    mu = (rng.standard_normal((K, D)) * 2.5).astype(np.float32)
    var = rng.uniform(0.4, 1.2, (K, D)).astype(np.float32)
    X = (mu[rng.integers(0, K, N)] + rng.standard_normal((N, D)) * 0.8).astype(np.float32)
    X64 = torch.tensor(X.astype(np.float64))
    w_t = torch.tensor(w.astype(np.float64))
    mu0 = torch.tensor(mu.astype(np.float64))
    sd0 = torch.tensor(np.sqrt(var.astype(np.float64)))

    def per_desc(m, s):
        return MixtureSameFamily(Categorical(probs=w_t), Independent(Normal(m, s), 1)).log_prob(X64)

    Jm, Js = torch.autograd.functional.jacobian(per_desc, (mu0, sd0))  # [N, K, D] each
    comp = Independent(Normal(mu0, sd0), 1).log_prob(X64[:, None, :]) + torch.log(w_t)
    post = torch.softmax(comp, dim=1).numpy()
    # every decision is far from the boundary, and the threshold removes some terms
    assert np.min(np.abs(np.log(post) - np.log(tau))) > 1e-3
    keep = post > tau
    assert 0 < np.count_nonzero(~keep) < keep.size // 2
    sd = sd0.numpy()
    U_ref = sd * np.einsum("tk,tkd->kd", keep, Jm.numpy())
    V_ref = sd * np.einsum("tk,tkd->kd", keep, Js.numpy())
    phi = o.encode(X, w, mu, var, flags=RAW, tau=tau)
    w64 = w.astype(np.float64)[:, None]
    U = phi[:K * D].reshape(K, D) * N * np.sqrt(w64)
    V = phi[K * D:].reshape(K, D) * N * np.sqrt(2 * w64)
    for got, ref in ((U, U_ref), (V, V_ref)):
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err < 1e-11, err
    # and the dropped terms are not negligible at this precision
    full = o.encode(X, w, mu, var, flags=RAW)
    assert np.max(np.abs(full - phi)) > 1e-9 * np.max(np.abs(full))


def pin_em_step_sklearn(o, seed=6):
    """The oracle's EM step against sklearn's diagonal M-step on sklearn's posteriors and
    against the summed sklearn log-likelihood of the input model."""
    import oracle
    from sklearn.mixture import GaussianMixture
    from sklearn.mixture._gaussian_mixture import _estimate_gaussian_parameters
    rng = np.random.default_rng(seed)
    for K, D, N in ((4, 3, 300), (12, 8, 500)):
        w = rng.dirichlet(np.ones(K) * 2).astype(np.float32)
        mu = (rng.standard_normal((K, D)) * 1.5).astype(np.float32)
        var = rng.uniform(0.5, 2.0, (K, D)).astype(np.float32)
        X = (mu[rng.integers(0, K, N)] + rng.standard_normal((N, D))).astype(np.float32)
        X64 = X.astype(np.float64)
        gm = GaussianMixture(n_components=K, covariance_type="diag")
        gm.weights_ = w.astype(np.float64)
        gm.means_ = mu.astype(np.float64)
        gm.covariances_ = var.astype(np.float64)
        gm.precisions_cholesky_ = 1.0 / np.sqrt(var.astype(np.float64))
        nk, m_ref, v_ref = _estimate_gaussian_parameters(X64, gm.predict_proba(X64), 0.0, "diag")
        w1, m1, v1, ll = oracle.em_step(X, w, mu, var, var_floor=0.0, lib=o)
        assert np.max(np.abs(w1 - nk / N)) < 1e-12
        assert np.max(np.abs(m1 - m_ref)) < 1e-10 * np.max(np.abs(m_ref))
        assert np.max(np.abs(v1 - v_ref) / v_ref) < 1e-9
        ll_ref = gm.score_samples(X64).sum()
        assert abs(ll - ll_ref) < 1e-10 * abs(ll_ref), (ll, ll_ref)


def pin_single_component(o, seed=2):
    rng = np.random.default_rng(seed)
    for D, N, wk in ((5, 300, 1.0), (7, 64, 0.37)):
        w = np.array([wk], np.float32)
        mu = rng.standard_normal((1, D)).astype(np.float32)
        var = rng.uniform(0.5, 2.0, (1, D)).astype(np.float32)
        X = (rng.standard_normal((N, D)) * 1.5 + 0.3).astype(np.float32)
        g = o.posteriors(X, w, mu, var)
        assert np.all(g == 1.0)
        X64 = X.astype(np.float64)
        m, s2 = X64.mean(0), X64.var(0)
        mu64, var64, w64 = mu[0].astype(np.float64), var[0].astype(np.float64), float(w[0])
        u_ref = (m - mu64) / np.sqrt(var64) / np.sqrt(w64)
        v_ref = ((s2 + (m - mu64) ** 2) / var64 - 1.0) / np.sqrt(2 * w64)
        phi = o.encode(X, w, mu, var, flags=RAW)
        assert np.max(np.abs(phi[:D] - u_ref)) < 1e-12
        assert np.max(np.abs(phi[D:] - v_ref)) < 1e-12


def pin_on_means(o):
    K, D = 4, 3
    w = np.array([0.125, 0.25, 0.5, 0.125], np.float32)
    mu = np.array([[0, 0, 0], [400, 0, 0], [0, 400, 0], [0, 0, 400]], np.float32)
    var = np.array([[1, 2, 0.5], [1.5, 1, 1], [0.75, 0.75, 2], [1, 1, 1]], np.float32)
    counts = np.array([3, 1, 5, 2])
    X = np.repeat(mu, counts, axis=0)
    N = X.shape[0]
    phi = o.encode(X, w, mu, var, flags=RAW)
    u = phi[:K * D].reshape(K, D)
    v = phi[K * D:].reshape(K, D)
    assert np.all(u == 0.0)
    v_ref = -counts[:, None] / (N * np.sqrt(2 * w.astype(np.float64)[:, None]))
    assert np.max(np.abs(v - v_ref)) < 1e-15


def pin_unit_variance(o, seeds=24):
    # components far apart => hard assignments; then sqrt(N) u_kd and sqrt(N) v_kd are sums of
    # independent standardised terms with mean 0 and variance exactly 1.
    K, D, N = 8, 16, 3000
    rng = np.random.default_rng(123)
    w = rng.dirichlet(np.ones(K) * 4).astype(np.float32)
    mu = (np.arange(K)[:, None] * 60.0 + rng.standard_normal((K, D))).astype(np.float32)
    var = rng.uniform(0.5, 2.0, (K, D)).astype(np.float32)
    us, vs = [], []
    for s in range(seeds):
        r = np.random.default_rng(1000 + s)
        lab = r.choice(K, N, p=w.astype(np.float64) / w.astype(np.float64).sum())
        X = (mu[lab].astype(np.float64) + np.sqrt(var[lab].astype(np.float64)) *
             r.standard_normal((N, D))).astype(np.float32)
        phi = o.encode(X, w, mu, var, flags=RAW)
        us.append(phi[:K * D] * np.sqrt(N))
        vs.append(phi[K * D:] * np.sqrt(N))
    us, vs = np.concatenate(us), np.concatenate(vs)
    n = us.size
    for a in (us, vs):
        assert abs(a.mean()) < 5.0 / np.sqrt(n), a.mean()
        assert abs(a.var() - 1.0) < 6.0 * np.sqrt(2.0 / n) + 0.02, a.var()


def pin_invariances(o, seed=3):
    rng = np.random.default_rng(seed)
    K, D, N = 6, 5, 120
    w, mu, var = _dyadic_model(rng, K, D)
    X = _dyadic_X(rng, N, D)
    base = o.encode(X, w, mu, var)
    raw = o.encode(X, w, mu, var, flags=RAW)
    tol = 1e-12
    # translation of descriptors and means (exact in float32 for these dyadic values)
    b = np.float32(3.0)
    assert np.max(np.abs(o.encode(X + b, w, mu + b, var) - base)) < tol
    # scaling x, mu by c and var by c^2
    assert np.max(np.abs(o.encode(X * 2, w, mu * 2, var * 4) - base)) < tol
    # negation: u flips sign, v unchanged
    neg = o.encode(-X, w, -mu, var, flags=RAW)
    assert np.max(np.abs(neg[:K * D] + raw[:K * D])) < tol * np.max(np.abs(raw))
    assert np.max(np.abs(neg[K * D:] - raw[K * D:])) < tol * np.max(np.abs(raw))
    # permuting components permutes the blocks
    p = rng.permutation(K)
    per = o.encode(X, w[p], mu[p], var[p])
    assert np.max(np.abs(per[:K * D].reshape(K, D) - base[:K * D].reshape(K, D)[p])) < tol
    assert np.max(np.abs(per[K * D:].reshape(K, D) - base[K * D:].reshape(K, D)[p])) < tol
    # permuting or duplicating descriptors changes nothing (normalised by N)
    q = rng.permutation(N)
    assert np.max(np.abs(o.encode(X[q], w, mu, var) - base)) < tol
    assert np.max(np.abs(o.encode(np.concatenate([X, X]), w, mu, var, flags=RAW) - raw)) < \
        tol * np.max(np.abs(raw))
    # mirrored pairs about a single mean give u == 0
    m1 = np.array([[0.5, -1.0]], np.float32)
    v1 = np.array([[0.25, 2.0]], np.float32)
    d = _dyadic_X(rng, 20, 2)
    Xm = np.concatenate([m1 + d, m1 - d]).astype(np.float32)
    assert np.max(np.abs(o.encode(Xm, np.array([1.0], np.float32), m1, v1, flags=RAW)[:2])) < 1e-14


def pin_normalisation(o, seed=4):
    rng = np.random.default_rng(seed)
    K, D, N = 6, 5, 80
    w, mu, var = _dyadic_model(rng, K, D)
    X = _dyadic_X(rng, N, D)
    phi = o.encode(X, w, mu, var)
    assert abs(np.linalg.norm(phi) - 1.0) < 1e-14
    assert abs(np.sum(np.abs(phi * np.abs(phi))) - 1.0) < 1e-13   # sum |s(phi)| = 1
    raw = o.encode(X, w, mu, var, flags=RAW)
    pw = o.encode(X, w, mu, var, flags=2)                           # power only
    l2 = o.encode(X, w, mu, var, flags=1)                           # L2 only
    assert np.allclose(pw * np.abs(pw), raw, rtol=1e-13, atol=1e-300)
    assert np.all(np.sign(pw) == np.sign(raw))
    assert abs(np.linalg.norm(l2) - 1.0) < 1e-14
    assert np.allclose(l2 * np.linalg.norm(raw), raw, rtol=1e-12, atol=1e-300)
    # N = 0 -> zeros; a frame whose statistics vanish exactly -> zeros (no division by 0)
    z = o.encode(np.zeros((0, D), np.float32), w, mu, var)
    assert z.shape == (2 * K * D,) and np.all(z == 0)
    one = o.encode(np.array([[0.0], [1.0]], np.float32), np.array([1.0], np.float32),
                   np.array([[0.5]], np.float32), np.array([[0.25]], np.float32))
    assert np.all(one == 0)


ALL_PINS = (pin_posteriors_sklearn, pin_posteriors_logistic, pin_gradient_autograd,
            pin_single_component, pin_on_means, pin_unit_variance, pin_invariances,
            pin_normalisation, pin_threshold_autograd, pin_em_step_sklearn)
