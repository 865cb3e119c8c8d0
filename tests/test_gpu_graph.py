"""Graph capture and replay of the launch sequences (device-resident X and out on a stream):
every replay, with eager work and synchronisation in between, must equal the direct
(uncaptured) encode bitwise, including when the input data or the batch table change."""
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


@pytest.mark.parametrize("prec", [0, 1])
def test_single_frame_replays(fv, prec, monkeypatch):
    import torch
    say(f"[gpu] graph single frame precision={prec}")
    g = fvsynth.gmm(256, 64, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    frames = [fvsynth.frame(g, 8000, 100 + i, 0.05) for i in range(3)]
    stream = torch.cuda.Stream()
    Xd = torch.empty(8000, 64, device="cuda")
    out = torch.empty(2 * 256 * 64, device="cuda")
    monkeypatch.setenv("FV_GRAPH", "0")
    direct = []
    for X in frames:
        Xd.copy_(torch.from_numpy(X))
        direct.append(fv.encode(h, Xd, out=out.clone(), precision=prec, stream=stream).cpu().numpy())
    monkeypatch.setenv("FV_GRAPH", "1")
    for rep in range(3):
        for i, X in enumerate(frames):
            Xd.copy_(torch.from_numpy(X))          # same pointer, new contents
            torch.cuda.synchronize()
            fv.encode(h, Xd, out=out, precision=prec, flags=fv.ASYNC, stream=stream)
            stream.synchronize()
            got = out.cpu().numpy()
            _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
            assert np.array_equal(got, direct[i]), (rep, i)


def test_batch_replays_with_new_table(fv, monkeypatch):
    import torch
    say("[gpu] graph batch")
    g = fvsynth.gmm(256, 64, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    shapes = [[1000, 3000, 500], [2000, 2000, 500], [3000, 1000, 500]]   # same items and groups
    data = [fvsynth.batch_frames(g, s, seed0=10 * i) for i, s in enumerate(shapes)]
    stream = torch.cuda.Stream()
    Xd = torch.empty(4500, 64, device="cuda")
    out = torch.empty(3, 2 * 256 * 64, device="cuda")
    monkeypatch.setenv("FV_GRAPH", "0")
    direct = []
    for X, off in data:
        Xd.copy_(torch.from_numpy(X))
        direct.append(fv.encode_batch(h, Xd, off, out=out.clone(), stream=stream).cpu().numpy())
    monkeypatch.setenv("FV_GRAPH", "1")
    for rep in range(3):
        for i, (X, off) in enumerate(data):
            Xd.copy_(torch.from_numpy(X))
            torch.cuda.synchronize()
            fv.encode_batch(h, Xd, off, out=out, flags=fv.ASYNC, stream=stream)
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), direct[i]), (rep, i)


@pytest.mark.parametrize("K,D,prec", [(256, 64, 0), (256, 64, 1), (512, 80, 1), (512, 80, 0)],
                         ids=["fused_fp32", "fused_bf16s", "twopass_bf16s", "twopass_fp32"])
def test_batch_graph_serves_every_shape(fv, K, D, prec, monkeypatch):
    """Batches of different frame counts, sizes and chunk counts on one stream share the
    captured graphs (the kernels read the batch's sizes from the work table; the grids depend
    on the stream's capacities only; one graph per half of the double-buffered table
    staging): after the first two batches (the first sets the capacities), no batch that fits
    them captures again, and every replay equals the eager (uncaptured) encode bitwise, with
    eager work between the replays."""
    import torch
    say(f"[gpu] shape-independent batch graph K={K} D={D} prec={prec}")
    g = fvsynth.gmm(K, D, 1)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    shapes = [[9000, 7000, 4000, 3000, 1000, 2500, 777, 33],  # largest first: sets the capacities
              [1, 0, 5000], [1100], [2000, 2000, 2000, 2000, 2000], [0], [4096, 1024, 3000],
              [31, 32, 33, 1023, 1024, 1025]]
    rows_max = max(sum(s) for s in shapes)
    data = [fvsynth.batch_frames(g, s, seed0=300 + 10 * i) for i, s in enumerate(shapes)]
    stream = torch.cuda.Stream()
    Xd = torch.zeros(rows_max, D, device="cuda")
    out = torch.zeros(8, 2 * K * D, device="cuda")
    monkeypatch.setenv("FV_GRAPH", "0")
    direct = []
    for X, off in data:
        Xd[:X.shape[0]].copy_(torch.from_numpy(X))
        B = off.size - 1
        direct.append(fv.encode_batch(h, Xd[:X.shape[0]], off, out=out[:B].clone(),
                                      precision=prec, stream=stream).cpu().numpy())
    monkeypatch.setenv("FV_GRAPH", "1")
    c0 = None
    seen = 0
    captured_by = []
    for rep in range(2):
        for i, (X, off) in enumerate(data):
            B = off.size - 1
            Xd[:X.shape[0]].copy_(torch.from_numpy(X))
            torch.cuda.synchronize()
            cb = fv.graph_counters()[0]
            fv.encode_batch(h, Xd[:X.shape[0]], off, out=out[:B], precision=prec,
                            flags=fv.ASYNC, stream=stream)
            stream.synchronize()
            assert np.array_equal(out[:B].cpu().numpy(), direct[i]), (rep, i)
            _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
            seen += 1
            if seen <= 2:
                c0 = fv.graph_counters()[0]   # after the captures for both staging halves
            elif fv.graph_counters()[0] != cb:
                captured_by.append((rep, shapes[i]))
    c1, r1 = fv.graph_counters()
    say(f"  captures after the first batch: {c1 - c0} {captured_by}; replays so far {r1}")
    assert c1 == c0, captured_by
    fv.stream_release(stream)
    h.free()


def test_reloaded_models_do_not_replay_stale_graphs(fv, monkeypatch):
    """Captured sequences are keyed by the handle's load serial, not its address: a model
    loaded after another was freed (its handle may land at the freed address, its constants
    elsewhere) is encoded with its own constants.  Each reload cycle's graph result must equal
    the direct encode with that model; the same holds for projection handles."""
    import torch
    say("[gpu] graph cache across free and reload")
    stream = torch.cuda.Stream()
    X = fvsynth.frame(fvsynth.gmm(256, 64, 0), 8000, 100, 0.05)
    Xd = torch.from_numpy(X).cuda()
    out = torch.empty(2 * 256 * 64, device="cuda")
    addrs = set()
    for cycle in range(4):
        g = fvsynth.gmm(256, 64, 20 + cycle)
        h = fv.gmm_load(g.weights, g.means, g.variances)
        addrs.add(h.handle)
        monkeypatch.setenv("FV_GRAPH", "0")
        ref = fv.encode(h, Xd, out=out.clone(), stream=stream).cpu().numpy()
        monkeypatch.setenv("FV_GRAPH", "1")
        for _ in range(2):
            fv.encode(h, Xd, out=out, flags=fv.ASYNC, stream=stream)
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), cycle
        h.free()
    say(f"  distinct handle addresses over 4 loads: {len(addrs)}")
    g = fvsynth.gmm(256, 64, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    R = torch.from_numpy(fvsynth.raw_frame(g, fvsynth.pca(64, 0), 4000, 5, 0.05)).cuda()
    for cycle in range(3):
        p = fvsynth.pca(64, cycle)
        hp = fv.pca_load(p.A, p.mean)
        monkeypatch.setenv("FV_GRAPH", "0")
        ref = fv.encode_projected(h, hp, R, out=out.clone(), stream=stream).cpu().numpy()
        monkeypatch.setenv("FV_GRAPH", "1")
        for _ in range(2):
            fv.encode_projected(h, hp, R, out=out, flags=fv.ASYNC, stream=stream)
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), ("pca", cycle)
        hp.free()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16_split"])
def test_autotuner_keeps_results_within_tolerance(fv, tmp_path, monkeypatch, prec):
    """The autotuner's axes (path x chunk, then the statistics grid, then for a fused 16-bit
    batch at 256 components the kernel variant): every trial runs, the chosen settings are the
    handle's tuning, the tuned batch meets the oracle gates and is bitwise the batch encoded
    with those settings set by hand, and the cached choice is applied to a second handle."""
    import torch
    import oracle
    from oracle.metrics import errors
    from paper_1604_03498_amd import autotune
    monkeypatch.setenv("FV_TUNE_CACHE", str(tmp_path / "tune.json"))
    say(f"[gpu] autotuner prec={prec}")
    g = fvsynth.gmm(256, 64, 0)
    X, off = fvsynth.batch_frames(g, [5000, 2500, 9000], seed0=70)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    Xd = torch.from_numpy(X).cuda()
    cfg = autotune.tune_batch(h, Xd, off, prec, chunks=(512, 2048), reps=2)
    say(f"  chosen {cfg['batch_path']}/{cfg['batch_chunk']}/grid {cfg['batch_grid']}/variant "
        f"{cfg['fused16_variant']} from {[(t['batch_path'], t['batch_chunk'], t['batch_grid'], t['fused16_variant'], round(t['ms'], 3)) for t in cfg['trials']]}")
    n_var = len(autotune.VARIANTS) if (prec != 0 and any(
        t["batch_path"] == 1 and t["fused16_variant"] for t in cfg["trials"])) else 0
    assert not cfg["cached"] and len(cfg["trials"]) == 4 + len(autotune.GRIDS) + n_var
    if prec == 1:
        assert n_var == len(autotune.VARIANTS) or cfg["batch_path"] == 2
    tun = fv.get_tuning(h)
    for k in ("batch_chunk", "batch_path", "batch_grid", "fused16_variant"):
        assert tun[k] == cfg[k], k
    got = fv.encode_batch(h, Xd, off, precision=prec).cpu().numpy()
    ref = oracle.encode_batch(X, off, g.weights, g.means, g.variances)
    tol = 1e-5 if prec == 0 else 1e-3
    for b in range(3):
        e = errors(got[b], ref[b])
        assert e["e_inf"] <= tol and e["e_2"] <= tol
    h2 = fv.gmm_load(g.weights, g.means, g.variances)
    assert autotune.apply(h2, prec, int(off[-1]))
    assert fv.get_tuning(h2) == fv.get_tuning(h)
    assert np.array_equal(fv.encode_batch(h2, Xd, off, precision=prec).cpu().numpy(), got)


@pytest.mark.parametrize("graph", ["1", "0"], ids=["graph", "eager"])
def test_back_to_back_batches_keep_their_tables(fv, graph, monkeypatch):
    """Batches queued back to back on one stream without waiting (FV_ASYNC): the host builds
    each call's work table in the staging half the call before last used, so it must not
    overwrite a half whose copy has not run yet.  Every batch must equal the same batch encoded
    alone, bitwise, whatever was queued around it."""
    import torch
    say(f"[gpu] back-to-back batches, FV_GRAPH={graph}")
    monkeypatch.setenv("FV_GRAPH", graph)
    g = fvsynth.gmm(256, 64, 2)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    shapes = [[9000, 300, 4100], [1, 2, 3, 5000], [12000], [700, 700, 700, 700, 700, 700],
              [0, 3000], [2500, 2501, 2502, 1023, 1025]]
    data = [fvsynth.batch_frames(g, s, seed0=700 + 10 * i) for i, s in enumerate(shapes)]
    stream = torch.cuda.Stream()
    xs = [torch.from_numpy(X).cuda() for X, _ in data]
    outs = [torch.full((off.size - 1, 2 * 256 * 64), -1.0, device="cuda") for _, off in data]
    alone = []
    for (X, off), Xd in zip(data, xs):
        o = torch.empty(off.size - 1, 2 * 256 * 64, device="cuda")
        fv.encode_batch(h, Xd, off, out=o, precision=1, stream=stream)
        stream.synchronize()
        alone.append(o.cpu().numpy())
    torch.cuda.synchronize()
    for rep in range(3):
        for i in range(len(data)):
            fv.encode_batch(h, xs[i], data[i][1], out=outs[i], precision=1, flags=fv.ASYNC,
                            stream=stream)
        stream.synchronize()
        for i in range(len(data)):
            assert np.array_equal(outs[i].cpu().numpy(), alone[i]), (rep, shapes[i])
            outs[i].fill_(-1.0)
        torch.cuda.synchronize()
    fv.stream_release(stream)
    h.free()
