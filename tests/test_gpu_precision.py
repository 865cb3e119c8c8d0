"""Split-precision forms (bf16 / fp16 hi-lo operands, three products, FP32 accumulation) and
the plain-bf16 control, through the C ABI, against the FP64 oracle.

Gate: E_inf <= 1e-3 and E_2 <= 1e-3 for BF16_SPLIT and FP16_SPLIT; the plain-bf16 form is a
control that must stay finite and be clearly less accurate than the split form."""
import dataclasses
import sys

import numpy as np
import pytest

import fvsynth
import oracle
from oracle.metrics import errors, per_block

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-3


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


@pytest.fixture(scope="module")
def c2():
    g = fvsynth.gmm(256, 64, 0)
    X = fvsynth.frame(g, 8000, 100, 0.05)
    return g, X, oracle.encode_gmm(X, g)


FORMS = [("bf16_split", 1), ("fp16_split", 2)]


@pytest.mark.parametrize("path", ["fused", "split"])
@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
def test_split_forms_c2_frame(fv, c2, form, path, monkeypatch):
    import torch
    name, prec = form
    monkeypatch.setenv("FV_PATH", path)
    g, X, ref = c2
    say(f"[gpu] {name} path={path} K=256 D=64 N=8000")
    h = fv.gmm_load(g.weights, g.means, g.variances)
    got = fv.encode(h, torch.from_numpy(X).cuda(), precision=prec).cpu().numpy()
    e = errors(got, ref)
    pb = per_block(got, ref, 256, 64, worst=3)
    say(f"  e_inf={e['e_inf']:.3e} e_2={e['e_2']:.3e} e_1={e['e_1']:.3e} worst blocks={pb['worst']}")
    assert np.all(np.isfinite(got))
    assert e["e_inf"] <= TOL_SPLIT and e["e_2"] <= TOL_SPLIT, e


def test_plain_bf16_control_is_worse(fv, c2):
    import torch
    g, X, ref = c2
    say("[gpu] plain bf16 control")
    h = fv.gmm_load(g.weights, g.means, g.variances)
    Xd = torch.from_numpy(X).cuda()
    plain = fv.encode(h, Xd, precision=3).cpu().numpy()
    split = fv.encode(h, Xd, precision=1).cpu().numpy()
    ep, es = errors(plain, ref), errors(split, ref)
    say(f"  plain bf16: {ep}\n  bf16 split: {es}")
    assert np.all(np.isfinite(plain))
    assert ep["e_2"] < 0.2
    assert ep["e_2"] > 5 * es["e_2"]


@pytest.mark.parametrize("form", FORMS, ids=[f[0] for f in FORMS])
def test_split_forms_ragged_and_batch(fv, form):
    import torch
    name, prec = form
    g = fvsynth.gmm(33, 17, 2)
    sizes = [1000, 1, 0, 77]
    X, off = fvsynth.batch_frames(g, sizes, seed0=60)
    say(f"[gpu] {name} ragged batch K=33 D=17")
    ref = oracle.encode_batch(X, off, g.weights, g.means, g.variances)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    got = fv.encode_batch(h, torch.from_numpy(X).cuda(), off, precision=prec).cpu().numpy()
    for b, n in enumerate(sizes):
        if n == 0:
            assert np.all(got[b] == 0)
            continue
        e = errors(got[b], ref[b])
        say(f"  frame {b} N={n}: {e}")
        assert e["e_inf"] <= TOL_SPLIT and e["e_2"] <= TOL_SPLIT
    one = fv.encode(h, torch.from_numpy(X[:1000]).cuda(), precision=prec).cpu().numpy()
    e = errors(one, ref[0])
    assert e["e_inf"] <= TOL_SPLIT and e["e_2"] <= TOL_SPLIT


def test_bf16_split_large_k(fv):
    import torch
    g = fvsynth.gmm(512, 80, 0)
    X = fvsynth.frame(g, 8000, 100000, 0.05)
    say("[gpu] bf16_split K=512 D=80 N=8000")
    ref = oracle.encode_gmm(X, g)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    got = fv.encode(h, torch.from_numpy(X).cuda(), precision=1).cpu().numpy()
    e = errors(got, ref)
    say(f"  {e}")
    assert e["e_inf"] <= TOL_SPLIT and e["e_2"] <= TOL_SPLIT


def test_fp16_split_refuses_models_beyond_fp16_range(fv):
    """A variance of 1e-6 puts 1/(2 sigma^2) log2 e = 7.2e5 into the E-step operand, beyond
    fp16's largest finite value: the fp16 split is refused (FV_E_UNSUPPORTED) by the encoder,
    the batch, the EM step and the server, and a model inside the range is not."""
    import torch
    say("[gpu] fp16 split range check")
    g = fvsynth.gmm(64, 16, 3)
    var = g.variances.copy()
    var[5, 3] = 1e-6
    g = dataclasses.replace(g, variances=var)
    X = fvsynth.frame(g, 3000, 4, 0.0)
    h = fv.gmm_load(g.weights, g.means, var)
    Xd = torch.from_numpy(X).cuda()
    for call in (lambda: fv.encode(h, Xd, precision=2),
                 lambda: fv.encode_batch(h, Xd, np.array([0, 1000, 3000], np.int64), precision=2),
                 lambda: fv.em_step(h, X, precision=2)):
        with pytest.raises(fv.FvError) as ei:
            call()
        assert ei.value.code == fv.E_UNSUPPORTED
    with pytest.raises(fv.FvError) as ei:
        fv.Server(h, fv.server_config(precision=2))
    assert ei.value.code == fv.E_UNSUPPORTED
    # FP32 and the bf16 split keep the FP32 exponent range: finite, unit-norm vectors (their
    # accuracy on so stiff a model -- sigma = 1e-3 in one coordinate -- is not gated here)
    for prec in (0, 1):
        got = fv.encode(h, Xd, precision=prec).cpu().numpy().astype(np.float64)
        say(f"  precision {prec}: E_inf vs oracle {errors(got, oracle.encode_gmm(X, g))['e_inf']:.2e}")
        assert np.all(np.isfinite(got)) and abs(np.linalg.norm(got) - 1.0) < 1e-5
    # a model inside the range still takes the fp16 split
    h2 = fv.gmm_load(g.weights, g.means, np.maximum(var, 0.5).astype(np.float32))
    assert np.all(np.isfinite(fv.encode(h2, Xd, precision=2).cpu().numpy()))
