"""fv_encode_noalloc: the allocation-free single-frame encode, on the library's fixed per-GPU
scratch, called through the C ABI and checked against fv_encode (the same kernels and plan, so
the bits agree) and against the FP64 oracle's gates, on two calls in a row with the second
input smaller; the device's free memory does not move across the calls; frames whose
intermediates exceed the scratch and host pointers are refused."""
import ctypes
import sys

import numpy as np
import pytest

import fvsynth
import oracle
from oracle.metrics import errors

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-3, 2: 1e-3}


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


def call_noalloc(fv, h, Xd, out, prec, stream, flags=0):
    """fv_encode_noalloc through ctypes (device X and out)."""
    lib = fv.load()
    f = fv.X_DEVICE | fv.OUT_DEVICE | flags
    return lib.fv_encode_noalloc(ctypes.c_void_p(h.handle), ctypes.c_void_p(Xd.data_ptr()),
                                 int(Xd.shape[0]), ctypes.c_void_p(out.data_ptr()), int(prec), f,
                                 ctypes.c_void_p(stream.cuda_stream))


CASES = [
    # (name, K, D, first N, second N, precisions)
    ("k256_d64", 256, 64, 8000, 1500, (0, 1, 2)),
    ("k512_d80", 512, 80, 32000, 8000, (1, 0)),
    ("k64_d64", 64, 64, 2000, 1, (0,)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_encode(fv, case):
    import torch
    name, K, D, n1, n2, precs = case
    g = fvsynth.gmm(K, D, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    stream = torch.cuda.Stream()
    X1 = fvsynth.frame(g, n1, 100, 0.05)
    X2 = fvsynth.frame(g, n2, 101, 0.05)
    ref1, ref2 = oracle.encode_gmm(X1, g), oracle.encode_gmm(X2, g)
    X1d, X2d = torch.from_numpy(X1).cuda(), torch.from_numpy(X2).cuda()
    for prec in precs:
        say(f"[gpu] noalloc {name} prec={prec}: N={n1} then N={n2}")
        out1 = torch.full((2 * K * D,), float("nan"), device="cuda")
        out2 = torch.full((2 * K * D,), float("nan"), device="cuda")
        # warm-up on both entry points (code objects loaded, library workspace allocated)
        assert call_noalloc(fv, h, X2d, out2, prec, stream) == 0
        e1 = fv.encode(h, X1d, precision=prec, stream=stream)
        e2 = fv.encode(h, X2d, precision=prec, stream=stream)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        assert call_noalloc(fv, h, X1d, out1, prec, stream) == 0
        assert call_noalloc(fv, h, X2d, out2, prec, stream) == 0
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (free0, free1)
        g1, g2 = out1.cpu().numpy(), out2.cpu().numpy()
        assert np.array_equal(g1, e1.cpu().numpy())
        assert np.array_equal(g2, e2.cpu().numpy())
        for tag, got, ref in (("first", g1, ref1), ("second", g2, ref2)):
            e = errors(got, ref)
            say(f"  {tag}: e_inf={e['e_inf']:.2e} e_2={e['e_2']:.2e}")
            assert e["e_inf"] <= TOL[prec] and e["e_2"] <= TOL[prec]
        # FV_ASYNC calls on one stream are ordered: the first result is not disturbed
        o3 = torch.empty_like(out1)
        o4 = torch.empty_like(out2)
        assert call_noalloc(fv, h, X1d, o3, prec, stream, fv.ASYNC) == 0
        assert call_noalloc(fv, h, X2d, o4, prec, stream, fv.ASYNC) == 0
        stream.synchronize()
        assert np.array_equal(o3.cpu().numpy(), g1) and np.array_equal(o4.cpu().numpy(), g2)
    fv.stream_release(stream)
    h.free()


def test_noalloc_refuses(fv):
    """Intermediates beyond the fixed scratch: FV_E_UNSUPPORTED with nothing launched (the
    output keeps its contents); host pointers: FV_E_INVAL."""
    import torch
    g = fvsynth.gmm(512, 80, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    stream = torch.cuda.Stream()
    n = 3_000_000  # two-pass normalisers alone: 16 bytes per row = 48 MB, plus 21 MB partials
    say(f"[gpu] noalloc refusal: K=512 D=80 N={n}")
    Xd = torch.zeros(n, 80, device="cuda")
    out = torch.full((2 * 512 * 80,), 7.0, device="cuda")
    assert call_noalloc(fv, h, Xd, out, 1, stream) == fv.E_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
    del Xd
    X = np.zeros((10, 80), np.float32)
    o = np.zeros(2 * 512 * 80, np.float32)
    lib = fv.load()
    rc = lib.fv_encode_noalloc(ctypes.c_void_p(h.handle), ctypes.c_void_p(X.ctypes.data), 10,
                               ctypes.c_void_p(o.ctypes.data), 0, 0, ctypes.c_void_p(0))
    assert rc == fv.E_INVAL
    fv.stream_release(stream)
    h.free()
