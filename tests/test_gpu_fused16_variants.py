"""The three fused 16-bit statistics kernels at 256 components (fused16_variant 1: two barriers
per tile; 2: single-role waves; 3: pipelined, one barrier per tile, statistics operand read
transposed from the row-major tile) against the FP64 oracle and against each other.

Variants 1 and 3 form every value with the same operations in the same order (the same split
operands, the same MFMA sequence per accumulator, the same softmax normaliser and S0 order), so
their vectors must be bitwise equal; variant 2 differs in rounding only and meets the gates.
Cases: a ragged batch (empty, one-row, partial-tile and multi-chunk frames) through the dynamic
persistent launch, the same with the grid capped at three workgroups (every workgroup runs
several items), threshold mode, a single large frame, and D = 64, 48, 20 (DP = 64, 48, 32).
Gates: E_inf, E_2 <= 1e-3 for the split forms; the plain-bf16 control form is checked for
finite values and for the equality of variants 1 and 3 only.
"""
import os
import sys

import numpy as np
import pytest

import fvsynth
import oracle
from oracle.metrics import errors

pytestmark = pytest.mark.gpu

SIZES = [2500, 0, 1, 1100, 33, 4096, 31, 2049]
TOL = {1: 1e-3, 2: 1e-3}
PNAME = {1: "bf16_split", 2: "fp16_split", 3: "bf16"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nthreads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def fv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_03498_amd as fvmod
    fvmod.load()
    return fvmod


def encode_variants(fv, h, Xd, off, prec, flags=0, single=False):
    outs = {}
    for v in (1, 2, 3):
        fv.set_tuning(h, fused16_variant=v)
        if single:
            outs[v] = fv.encode(h, Xd, precision=prec, flags=flags).cpu().numpy()
        else:
            outs[v] = fv.encode_batch(h, Xd, off, precision=prec, flags=flags).cpu().numpy()
    fv.set_tuning(h)
    return outs


@pytest.mark.parametrize("D", [64, 48, 20])
@pytest.mark.parametrize("prec", [1, 2, 3], ids=["bf16_split", "fp16_split", "bf16"])
def test_batch_variants(fv, prec, D, monkeypatch):
    import torch
    for k in ("FV_PATH", "FV_MAX_GRID", "FV_BATCH_CHUNK", "FV_FUSED16"):
        monkeypatch.delenv(k, raising=False)
    monkeypatch.setenv("FV_PATH", "fused")
    g = fvsynth.gmm(256, D, 7)
    h = fv.gmm_load(g.weights, g.means, g.variances, device=0)
    X, off = fvsynth.batch_frames(g, SIZES, seed0=900 + D)
    ref = oracle.encode_batch(X, off, g.weights, g.means, g.variances, nthreads=nthreads())
    Xd = torch.from_numpy(X).cuda()
    say(f"[gpu] fused16 variants {PNAME[prec]} D={D} sizes={SIZES}")
    outs = encode_variants(fv, h, Xd, off, prec)
    d = np.abs(outs[1].astype(np.float64) - outs[3])
    half = d.shape[1] // 2
    say(f"  variants 1 vs 3: {int((d > 0).sum())} values differ, max |d| = {d.max():.3e} "
        f"(first-order part {d[:, :half].max():.3e}, second-order part {d[:, half:].max():.3e})")
    for v in (1, 2, 3):
        e = errors(outs[v][0], ref[0])
        say(f"  variant {v} frame 0: e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e}")
    assert np.array_equal(outs[1], outs[3]), "variants 1 and 3 differ"
    for v in (2, 3):
        for b, n in enumerate(SIZES):
            if n == 0:
                assert np.all(outs[v][b] == 0)
                continue
            assert np.all(np.isfinite(outs[v][b]))
            if prec in TOL:
                e = errors(outs[v][b], ref[b])
                assert e["e_inf"] <= TOL[prec] and e["e_2"] <= TOL[prec], (v, b, e)
    # the persistent loop: three workgroups run all items
    monkeypatch.setenv("FV_MAX_GRID", "3")
    capped = encode_variants(fv, h, Xd, off, prec)
    for v in (1, 2, 3):
        assert np.array_equal(capped[v], outs[v]), v
    h.free()


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16_split", "fp16_split"])
def test_threshold_and_single_frame_variants(fv, prec, monkeypatch):
    import torch
    for k in ("FV_PATH", "FV_MAX_GRID", "FV_BATCH_CHUNK", "FV_FUSED16"):
        monkeypatch.delenv(k, raising=False)
    g = fvsynth.gmm(256, 64, 3)
    h = fv.gmm_load(g.weights, g.means, g.variances, device=0)
    X, off = fvsynth.batch_frames(g, SIZES, seed0=950)
    Xd = torch.from_numpy(X).cuda()
    monkeypatch.setenv("FV_PATH", "fused")
    say(f"[gpu] fused16 variants threshold mode {PNAME[prec]}")
    th = encode_variants(fv, h, Xd, off, prec, flags=fv.THRESHOLD)
    assert np.array_equal(th[1], th[3])
    for b, n in enumerate(SIZES):
        if n:
            ref_t = oracle.encode_gmm(X[off[b]:off[b + 1]], g, tau=fv.THRESHOLD_TAU)
            e = errors(th[3][b], ref_t)
            assert e["e_inf"] <= TOL[prec] and e["e_2"] <= TOL[prec], (b, e)
    Xf = fvsynth.frame(g, 20000, 77, 0.05)
    reff = oracle.encode_gmm(Xf, g)
    say(f"[gpu] fused16 variants single frame N=20000 {PNAME[prec]}")
    single = encode_variants(fv, h, torch.from_numpy(Xf).cuda(), None, prec, single=True)
    assert np.array_equal(single[1], single[3])
    e = errors(single[3], reff)
    assert e["e_inf"] <= TOL[prec] and e["e_2"] <= TOL[prec], e
    h.free()
