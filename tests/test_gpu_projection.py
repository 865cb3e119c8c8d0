"""Projection prologue (fv_pca_load / fv_project / fv_encode_projected): the HIP path against
the oracle's float64 projection y = A (x - m) and the oracle's FV of that float64 projection.

The projection alone is checked entrywise against a rigorous float32 dot-product bound: with
u = 2^-24 and n = Din + 2 roundings per output (Din products accumulated onto the rounded
bias -A m),
    |y_gpu - y| <= n u (|A m| + sum_k |A_ck| |x_tk|) / (1 - n u) + u |A m|.
The split-bf16 projection of the 16-bit forms (fv_project with PROJ_SPLIT16) forms every
product a x as ah xh + al xh + ah xl with ah = rne(a), al = rne(a - ah) (and likewise for x): the
dropped al xl and the two lo roundings leave at most 3 * 2^-18 (1 + 2^-8) |a| |x| per product,
which adds 2^-16 sum_k |A_ck| |x_tk| to the float32 bound above (taken with n = 3 Din + 2).
The encodings use the usual gates: E_inf, E_2 <= 1e-5 (FP32), 1e-3 (split forms).
Inputs: a stand-in PCA (orthonormal 128 -> 62 block plus two pass-through coordinates, Din =
130, D = 64) and raw descriptors built so that their projection is a GMM sample.
"""
import sys

import numpy as np
import pytest

import fvsynth
import oracle
from oracle.metrics import errors

pytestmark = pytest.mark.gpu

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


def projection_bound(X, A, m, split16=False):
    A64 = A.astype(np.float64)
    am = np.abs(A64 @ m.astype(np.float64))
    n = (3 if split16 else 1) * X.shape[1] + 2
    ax = np.abs(X.astype(np.float64)) @ np.abs(A64).T
    s = ax + am[None, :]
    b = n * U * s / (1 - n * U) + U * am[None, :]
    return b + (2.0 ** -16) * ax if split16 else b


@pytest.mark.parametrize("Din,D,N", [(130, 64, 5000), (128, 64, 777), (130, 82, 3001),
                                     (7, 5, 33), (256, 96, 1000)])
def test_project_matches_float64(fv, Din, D, N):
    import torch
    say(f"[gpu] project Din={Din} D={D} N={N}")
    rng = np.random.default_rng(Din * 1000 + D)
    A = (rng.standard_normal((D, Din)) / np.sqrt(Din)).astype(np.float32)
    m = rng.uniform(0.0, 0.2, Din).astype(np.float32)
    X = (m + rng.standard_normal((N, Din)) * 0.5).astype(np.float32)
    p = fv.pca_load(A, m)
    ref = oracle.project(X, A, m)
    bound = projection_bound(X, A, m)
    got = fv.project(p, torch.from_numpy(X).cuda()).cpu().numpy()
    err = np.abs(got.astype(np.float64) - ref)
    say(f"  max|err|={err.max():.3e}  max err/bound={np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    # host pointers give the same bits; an unaligned device row start (Din odd) is accepted
    assert np.array_equal(fv.project(p, X), got)
    # the split-bf16 contraction of the 16-bit forms, against its own bound
    got16 = fv.project(p, torch.from_numpy(X).cuda(), split16=True).cpu().numpy()
    err16 = np.abs(got16.astype(np.float64) - ref)
    bound16 = projection_bound(X, A, m, split16=True)
    say(f"  split16: max|err|={err16.max():.3e}  max err/bound={np.max(err16 / bound16):.3f}")
    assert np.all(err16 <= bound16)
    assert np.array_equal(fv.project(p, X, split16=True), got16)


CASES = [
    # (name, K, D, N, gmm_seed, pca_seed, frame_seed)
    ("k256_d64_n8000", 256, 64, 8000, 0, 0, 100),
    ("k64_d64_n2000", 64, 64, 2000, 0, 1, 0),
    ("k512_d82_n3001", 512, 82, 3001, 2, 3, 7),
]


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp32", "bf16_split", "fp16_split"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_encode_projected_matches_oracle(fv, case, prec):
    import torch
    name, K, D, N, gs, ps, fs = case
    say(f"[gpu] encode_projected {name} prec={prec}")
    g = fvsynth.gmm(K, D, gs)
    p = fvsynth.pca(D, ps)
    X = fvsynth.raw_frame(g, p, N, fs, 0.05)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    hp = fv.pca_load(p.A, p.mean)
    ref = oracle.encode_projected(X, p.A, p.mean, g)
    got = fv.encode_projected(h, hp, torch.from_numpy(X).cuda(), precision=prec).cpu().numpy()
    e = errors(got, ref)
    tol = 1e-5 if prec == 0 else 1e-3
    say(f"  e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e} e_1={e['e_1']:.3e}")
    assert np.all(np.isfinite(got))
    assert e["e_inf"] <= tol and e["e_2"] <= tol, e
    # host input gives the same bits; the projection + encode equals encode of fv_project's
    # output (the same kernels in the same order; the 16-bit forms project with the split)
    assert np.array_equal(fv.encode_projected(h, hp, X, precision=prec), got)
    Y = fv.project(hp, torch.from_numpy(X).cuda(), split16=prec != 0)
    assert np.array_equal(fv.encode(h, Y, precision=prec).cpu().numpy(), got)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16_split"])
def test_encode_batch_projected(fv, prec):
    import torch
    say(f"[gpu] encode_batch_projected prec={prec}")
    g = fvsynth.gmm(256, 64, 0)
    p = fvsynth.pca(64, 0)
    sizes = [2500, 0, 1, 1100, 33, 4096]
    X, off = fvsynth.raw_batch(g, p, sizes, seed0=300)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    hp = fv.pca_load(p.A, p.mean)
    got = fv.encode_batch_projected(h, hp, torch.from_numpy(X).cuda(), off,
                                    precision=prec).cpu().numpy()
    tol = 1e-5 if prec == 0 else 1e-3
    for b, n in enumerate(sizes):
        if n == 0:
            assert np.all(got[b] == 0)
            continue
        e = errors(got[b], oracle.encode_projected(X[off[b]:off[b + 1]], p.A, p.mean, g))
        say(f"  frame{b}(N={n}) e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e}")
        assert e["e_inf"] <= tol and e["e_2"] <= tol, (b, e)
    assert np.array_equal(fv.encode_batch_projected(h, hp, X, off, precision=prec), got)


def test_projected_graph_replays_and_mismatch(fv, monkeypatch):
    """Captured sequences include the projection: replays with new input contents equal the
    direct encode bitwise; a projection of another output width is refused."""
    import torch
    say("[gpu] projected graph replays")
    g = fvsynth.gmm(256, 64, 0)
    p = fvsynth.pca(64, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    hp = fv.pca_load(p.A, p.mean)
    frames = [fvsynth.raw_frame(g, p, 8000, 100 + i, 0.05) for i in range(3)]
    stream = torch.cuda.Stream()
    Xd = torch.empty(8000, 130, device="cuda")
    out = torch.empty(2 * 256 * 64, device="cuda")
    monkeypatch.setenv("FV_GRAPH", "0")
    direct = []
    for X in frames:
        Xd.copy_(torch.from_numpy(X))
        direct.append(fv.encode_projected(h, hp, Xd, out=out.clone(), stream=stream).cpu().numpy())
    monkeypatch.setenv("FV_GRAPH", "1")
    for rep in range(3):
        for i, X in enumerate(frames):
            Xd.copy_(torch.from_numpy(X))
            torch.cuda.synchronize()
            fv.encode_projected(h, hp, Xd, out=out, flags=fv.ASYNC, stream=stream)
            stream.synchronize()
            got = out.cpu().numpy()
            _ = torch.ones(1000, device="cuda").sum().item()
            assert np.array_equal(got, direct[i]), (rep, i)
    other = fv.pca_load(np.eye(32, 130, dtype=np.float32), np.zeros(130, np.float32))
    with pytest.raises(fv.FvError):
        fv.encode_projected(h, other, frames[0][:10])


def test_projected_threshold_mode(fv):
    """The projection prologue composes with the posterior threshold: against the oracle's
    tau mode on the float64 projection."""
    import torch
    say("[gpu] projected + threshold")
    g = fvsynth.gmm(256, 64, 0)
    p = fvsynth.pca(64, 0)
    X = fvsynth.raw_frame(g, p, 4000, 17, 0.05)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    hp = fv.pca_load(p.A, p.mean)
    for prec, tol in ((0, 1e-5), (1, 1e-3)):
        ref = oracle.encode_projected(X, p.A, p.mean, g, tau=fv.THRESHOLD_TAU)
        got = fv.encode_projected(h, hp, torch.from_numpy(X).cuda(), precision=prec,
                                  flags=fv.THRESHOLD).cpu().numpy()
        e = errors(got, ref)
        say(f"  prec={prec} e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e}")
        assert e["e_inf"] <= tol and e["e_2"] <= tol, e
