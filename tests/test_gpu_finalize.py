"""The finalize step's two workgroup shapes (4 dimensions x 256 components for launches with
many tiles, 1 dimension x 64 components otherwise) sum the same slots in the same order and
form the norm from the same per-(dimension, 64-component block) partial sums, so a frame
encoded alone (narrow shape) equals the same frame inside a large batch (wide shape) bitwise.
The batch also puts its frames in the finalize's longest-first order, which must not move any
frame's output row."""
import sys

import numpy as np
import pytest

import fvsynth

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


@pytest.mark.parametrize("K,D,prec", [(256, 64, 0), (256, 64, 1), (512, 80, 1), (100, 22, 0),
                                      (1024, 93, 1), (32, 16, 0)],
                         ids=["k256_fp32", "k256_bf16s", "k512_d80_bf16s", "k100_d22_fp32",
                              "k1024_d93_bf16s", "k32_d16_fp32"])
def test_wide_and_narrow_finalize_agree(fv, K, D, prec):
    import torch
    g = fvsynth.gmm(K, D, 5)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    # enough frames that the batch launch takes the wide shape: B * ceil(D / 4) * ceil(Kp / 256)
    # >= 512 tiles; sizes from one slot to three chunk groups of 1024-row chunks, unsorted
    kp = 256 * ((K + 255) // 256)
    B = -(-512 // ((D + 3) // 4 * (kp // 256))) + 3
    rng = np.random.default_rng(11)
    sizes = [int(x) for x in rng.integers(1, 40000 if B < 100 else 8000, size=B)]
    sizes[0], sizes[1], sizes[2] = 0, 1, 33 * 1024 + 5   # empty, one row, three groups
    say(f"[gpu] finalize shapes K={K} D={D} prec={prec} B={B} rows={sum(sizes)}")
    X, off = fvsynth.batch_frames(g, sizes, seed0=900)
    Xd = torch.from_numpy(X).cuda()
    stream = torch.cuda.Stream()
    out = torch.empty(B, 2 * K * D, device="cuda")
    fv.encode_batch(h, Xd, off, out=out, precision=prec, stream=stream)
    stream.synchronize()
    got = out.cpu().numpy()
    one = torch.empty(1, 2 * K * D, device="cuda")
    for b in range(B):
        fv.encode_batch(h, Xd[off[b]:off[b + 1]], np.array([0, off[b + 1] - off[b]], np.int64),
                        out=one, precision=prec, stream=stream)
        stream.synchronize()
        alone = one.cpu().numpy()[0]
        assert np.array_equal(got[b], alone), (b, sizes[b])
    assert np.all(got[0] == 0.0)
    h.free()
