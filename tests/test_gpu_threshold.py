"""Posterior threshold mode (FV_THRESHOLD) of the HIP path against the oracle's tau mode.

A term (t, k) enters the statistics only if gamma_tk > 1e-6 (Algorithm 1's test, with the
clustered skip of Sec. 3.3 in the kernels).  Each side takes that decision in its own
precision (the oracle in FP64, the kernels in FP32), so a term whose posterior lies within
rounding of the threshold may be kept by one side and dropped by the other.  The
un-normalised checks allow exactly that: elementwise,
    |got - ref| <= tol * max|ref| + (summed magnitude of every term whose FP64 posterior lies
                                      within a factor exp(+-0.05) of tau).
The normalised checks use the usual gates (E_inf, E_2 <= 1e-5 for FP32, 1e-3 for the split
forms); there a flipped boundary term moves an entry by far less than the gate.
Clustered frames (rows grouped by component) make most MFMA steps skippable in every form.
"""
import sys

import numpy as np
import pytest

import fvsynth
import oracle
from oracle.metrics import errors

pytestmark = pytest.mark.gpu

TAU = 1e-6
BAND = 0.05  # |ln gamma - ln tau| below this: either decision is correct


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_03498_amd as fvmod
    fvmod.load()
    assert fvmod.THRESHOLD_TAU == TAU
    return fvmod


def _tol(prec):
    return 1e-5 if prec == 0 else 1e-3


def boundary_bound(X, g):
    """Per entry of the un-normalised vector, the summed |contribution| of the terms whose
    FP64 posterior is within the band around tau; and how many such terms there are."""
    P = oracle.posteriors(X, g.weights, g.means, g.variances)
    amb = np.abs(np.log(np.maximum(P, 1e-300)) - np.log(TAU)) < BAND
    K, D = g.K, g.D
    N = X.shape[0]
    bu = np.zeros((K, D))
    bv = np.zeros((K, D))
    sd = np.sqrt(g.variances.astype(np.float64))
    for t, k in zip(*np.nonzero(amb)):
        z = (X[t].astype(np.float64) - g.means[k].astype(np.float64)) / sd[k]
        bu[k] += P[t, k] * np.abs(z)
        bv[k] += P[t, k] * np.abs(z * z - 1.0)
    w = g.weights.astype(np.float64)[:, None]
    bound = np.concatenate([(bu / (N * np.sqrt(w))).ravel(), (bv / (N * np.sqrt(2 * w))).ravel()])
    return bound, int(amb.sum())


def check_raw(name, got, ref, bound, tol):
    got = np.asarray(got, np.float64)
    lim = tol * np.max(np.abs(ref)) + bound
    worst = np.max(np.abs(got - ref) - lim)
    say(f"  {name} raw: max|d|={np.max(np.abs(got - ref)):.3e} max|ref|={np.max(np.abs(ref)):.3e}")
    assert np.all(np.isfinite(got)) and worst <= 0, (name, worst)


def check_norm(name, got, ref, tol):
    e = errors(got, ref)
    say(f"  {name}: e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e}")
    assert np.all(np.isfinite(got)), name
    assert e["e_inf"] <= tol and e["e_2"] <= tol, (name, e)


CASES = [
    # (name, K, D, N, gmm_seed, frame_seed, outliers, clustered)
    ("k256_d64_n8000", 256, 64, 8000, 0, 100, 0.05, False),
    ("k256_d64_n8000_clustered", 256, 64, 8000, 0, 100, 0.05, True),
    ("k64_d32_n2000", 64, 32, 2000, 9, 7, 0.05, False),
    ("k33_d17_n1000_ragged_clustered", 33, 17, 1000, 2, 3, 0.05, True),
    ("k512_d80_n6000_clustered", 512, 80, 6000, 0, 12, 0.05, True),
]


@pytest.fixture(params=["fused", "split"])
def path(request, monkeypatch):
    monkeypatch.setenv("FV_PATH", request.param)
    return request.param


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp32", "bf16_split", "fp16_split"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_threshold_single_frame(fv, case, prec, path):
    import torch
    name, K, D, N, gs, fs, out_frac, clus = case
    say(f"[gpu] threshold {name} prec={prec} path={path}")
    g = fvsynth.gmm(K, D, gs)
    X = fvsynth.frame(g, N, fs, out_frac, clustered=clus)
    h = fv.gmm_load(g.weights, g.means, g.variances, device=0)
    Xd = torch.from_numpy(X).cuda()
    tol = _tol(prec)
    ref = oracle.encode_gmm(X, g, tau=TAU)
    got = fv.encode(h, Xd, precision=prec, flags=fv.THRESHOLD).cpu().numpy()
    check_norm(name, got, ref, tol)
    bound, n_amb = boundary_bound(X, g)
    say(f"  terms within the band around tau: {n_amb}")
    raw_ref = oracle.encode_gmm(X, g, flags=3, tau=TAU)
    raw = fv.encode(h, Xd, precision=prec,
                    flags=fv.THRESHOLD | fv.NO_POWER_NORM | fv.NO_L2_NORM).cpu().numpy()
    check_raw(name, raw, raw_ref, bound, tol)
    # the threshold changes the result (terms below tau were there to drop) ...
    full = fv.encode(h, Xd, precision=prec, flags=fv.NO_POWER_NORM | fv.NO_L2_NORM).cpu().numpy()
    assert not np.array_equal(full, raw)
    # ... and host pointers give the same bits as device pointers
    assert np.array_equal(fv.encode(h, X, precision=prec, flags=fv.THRESHOLD), got)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16_split"])
def test_threshold_batch(fv, prec, path):
    import torch
    say(f"[gpu] threshold batch prec={prec} path={path}")
    g = fvsynth.gmm(256, 64, 0)
    sizes = [2500, 0, 1, 1100, 33, 4096]
    frames = [fvsynth.frame(g, n, 300 + f, 0.05, clustered=(f % 2 == 0)) for f, n in enumerate(sizes)]
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    X = np.ascontiguousarray(np.concatenate(frames, axis=0))
    h = fv.gmm_load(g.weights, g.means, g.variances, device=0)
    got = fv.encode_batch(h, torch.from_numpy(X).cuda(), off, precision=prec,
                          flags=fv.THRESHOLD).cpu().numpy()
    for b, n in enumerate(sizes):
        if n == 0:
            assert np.all(got[b] == 0)
            continue
        ref = oracle.encode_gmm(frames[b], g, tau=TAU)
        check_norm(f"frame{b}(N={n})", got[b], ref, _tol(prec))
    raw = fv.encode_batch(h, torch.from_numpy(X).cuda(), off, precision=prec,
                          flags=fv.THRESHOLD | fv.NO_POWER_NORM | fv.NO_L2_NORM).cpu().numpy()
    for b, n in enumerate(sizes):
        if n == 0:
            continue
        bound, _ = boundary_bound(frames[b], g)
        check_raw(f"frame{b}", raw[b], oracle.encode_gmm(frames[b], g, flags=3, tau=TAU), bound,
                  _tol(prec))


def test_threshold_graph_replays_keep_the_mode(fv, monkeypatch):
    """Captured sequences are cached per flag set: alternating threshold on and off on one
    stream and buffer replays the matching graph each time."""
    import torch
    say("[gpu] threshold graph replays")
    g = fvsynth.gmm(256, 64, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    X = fvsynth.frame(g, 8000, 100, 0.05, clustered=True)
    stream = torch.cuda.Stream()
    Xd = torch.from_numpy(X).cuda()
    out = torch.empty(2 * 256 * 64, device="cuda")
    monkeypatch.setenv("FV_GRAPH", "0")
    direct = {f: fv.encode(h, Xd, out=out.clone(), flags=f, stream=stream).cpu().numpy()
              for f in (0, fv.THRESHOLD)}
    assert not np.array_equal(direct[0], direct[fv.THRESHOLD])
    monkeypatch.setenv("FV_GRAPH", "1")
    for rep in range(3):
        for f in (0, fv.THRESHOLD):
            torch.cuda.synchronize()
            fv.encode(h, Xd, out=out, flags=f | fv.ASYNC, stream=stream)
            stream.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()
            assert np.array_equal(out.cpu().numpy(), direct[f]), (rep, f)


def test_threshold_server(fv):
    """The serving front end passes the threshold flag through to its batches."""
    import time
    say("[gpu] threshold server")
    g = fvsynth.gmm(256, 64, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    cfg = fv.server_config(precision=fv.PREC_FP32, n_streams=2, flags=fv.THRESHOLD)
    frames = [fvsynth.frame(g, n, 50 + i, 0.05) for i, n in enumerate((3000, 800, 5000))]
    with fv.Server(h, cfg) as srv:
        tickets = [srv.submit(X) for X in frames]
        outs = {}
        t_end = time.time() + 60.0
        while len(outs) < len(tickets):
            assert time.time() < t_end, "server did not finish"
            t = srv.next_done(1000.0)
            if t is not None:
                rc, out, _ = srv.poll(t)
                assert rc == fv.OK, rc
                outs[t] = out
    for X, t in zip(frames, tickets):
        check_norm("server", outs[t], oracle.encode_gmm(X, g, tau=TAU), 1e-5)


def test_threshold_single_component_and_tiny_frames(fv):
    """K = 1 (every posterior is 1: the threshold removes nothing, so the result equals the
    exact encode bitwise) and frames of 1 and 2 descriptors."""
    import torch
    say("[gpu] threshold K=1 and tiny frames")
    g = fvsynth.gmm(1, 8, 5)
    X = fvsynth.frame(g, 100, 6)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    for prec in (0, 1):
        a = fv.encode(h, X, precision=prec)
        b = fv.encode(h, X, precision=prec, flags=fv.THRESHOLD)
        assert np.array_equal(a, b)
    g = fvsynth.gmm(64, 32, 1)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    for n in (1, 2):
        X = fvsynth.frame(g, n, 40 + n, 0.0)
        ref = oracle.encode_gmm(X, g, tau=TAU)
        got = fv.encode(h, torch.from_numpy(X).cuda(), flags=fv.THRESHOLD).cpu().numpy()
        check_norm(f"n={n}", got, ref, 1e-5)
