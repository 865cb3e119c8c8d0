"""Serving loop on the GPU: results against the FP64 oracle, bitwise equality of a frame
served alone and inside a mix, and budget-forced queueing."""
import sys
import time

import numpy as np
import pytest

import fvsynth
import oracle
from oracle.metrics import errors

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


def drain(s, tickets, timeout=60.0):
    res, pending, t0 = {}, set(tickets), time.time()
    while pending and time.time() - t0 < timeout:
        t = s.next_done(200.0)
        if t is None or t not in pending:
            continue
        res[t] = s.poll(t)
        pending.discard(t)
    assert not pending, f"{len(pending)} requests never finished"
    return res


def test_server_results_match_oracle_and_batch(fv):
    say("[gpu] server fp32 K=256 D=64")
    g = fvsynth.gmm(256, 64, 0)
    sizes = [3000, 17, 8000, 0, 1200, 9001]
    frames = [fvsynth.frame(g, n, 500 + i, 0.05) for i, n in enumerate(sizes)]
    h = fv.gmm_load(g.weights, g.means, g.variances)
    with fv.Server(h, fv.server_config(precision=fv.PREC_FP32, n_streams=2)) as s:
        tickets = [s.submit(X) for X in frames]
        res = drain(s, tickets)
    X, off = np.concatenate(frames), np.cumsum([0] + sizes)
    batch = fv.encode_batch(h, X, off)
    for i, t in enumerate(tickets):
        rc, out, st = res[t]
        assert rc == fv.OK, rc
        assert np.array_equal(out, batch[i]), f"frame {i} differs from the batched encode"
        if sizes[i] == 0:
            assert np.all(out == 0)
            continue
        e = errors(out, oracle.encode_gmm(frames[i], g))
        say(f"  frame {i} N={sizes[i]} frames-in-launch={st['batch_frames']} e_inf={e['e_inf']:.2e}")
        assert e["e_inf"] <= 1e-5 and e["e_2"] <= 1e-5


@pytest.mark.parametrize("K,D,prec", [(256, 64, 0), (512, 80, 1)])
def test_alone_equals_mix_bitwise(fv, K, D, prec):
    say(f"[gpu] server alone vs mix K={K} D={D} precision={prec}")
    g = fvsynth.gmm(K, D, 0)
    target = fvsynth.frame(g, 12500, 77, 0.05)
    others = [fvsynth.frame(g, n, 900 + i, 0.05) for i, n in enumerate([8000, 3000, 18000, 500, 9999])]
    h = fv.gmm_load(g.weights, g.means, g.variances)
    with fv.Server(h, fv.server_config(precision=prec, n_streams=1)) as s:
        t = s.submit(target)
        alone = drain(s, [t])[t]
    assert alone[0] == fv.OK and alone[2]["batch_frames"] == 1
    # a batching window long enough for all submissions puts the target in a shared launch
    with fv.Server(h, fv.server_config(precision=prec, n_streams=1, batch_window_us=2e5)) as s:
        ts = [s.submit(o) for o in others[:3]] + [s.submit(target)] + [s.submit(o) for o in others[3:]]
        res = drain(s, ts)
    mixed = res[ts[3]]
    assert mixed[0] == fv.OK
    say(f"  alone: 1 frame per launch; mixed: {mixed[2]['batch_frames']} frames in the launch")
    assert mixed[2]["batch_frames"] == 6
    assert np.array_equal(alone[1], mixed[1])
    e = errors(alone[1], oracle.encode_gmm(target, g))
    say(f"  vs oracle: {e}")
    tol = 1e-5 if prec == 0 else 1e-3
    assert e["e_inf"] <= tol and e["e_2"] <= tol


def test_small_budget_forces_queueing(fv):
    say("[gpu] server small budget")
    g = fvsynth.gmm(64, 32, 3)
    frames = [fvsynth.frame(g, 4000, 40 + i, 0.05) for i in range(8)]
    h = fv.gmm_load(g.weights, g.means, g.variances)
    # footprint of one 4000-row frame, measured by probing: a budget of about 1.5 frames
    with fv.Server(h, fv.server_config(n_streams=4)) as probe:
        t = probe.submit(frames[0])
        drain(probe, [t])
        per = probe.stats()["peak_admitted_bytes"]
    with fv.Server(h, fv.server_config(n_streams=4, hbm_budget_bytes=int(per * 1.5))) as s:
        tickets = [s.submit(X) for X in frames]
        res = drain(s, tickets)
        st = s.stats()
    assert st["peak_admitted_bytes"] <= int(per * 1.5)
    for i, t in enumerate(tickets):
        rc, out, _ = res[t]
        assert rc == fv.OK
        e = errors(out, oracle.encode_gmm(frames[i], g))
        assert e["e_inf"] <= 1e-5 and e["e_2"] <= 1e-5


def test_budget_bounds_device_memory(fv):
    """The budget bounds the device memory the server holds (its lanes' buffers and encoder
    workspaces, kept between launches): the drop of the device's free memory while serving a
    mix of the serving shape's frames stays within the budget plus a fixed overhead of 16 MiB
    (streams, events, executable graphs, runtime pools), and the memory comes back when the
    server is destroyed."""
    import threading
    import torch
    say("[gpu] server device memory within the budget, K=512 D=80 bf16 split")
    g = fvsynth.gmm(512, 80, 0)
    sizes = [8000, 32000, 12500, 24500, 18000, 8000, 32000, 12500]
    frames = [fvsynth.frame(g, n, 1300 + i, 0.05) for i, n in enumerate(sizes)]
    h = fv.gmm_load(g.weights, g.means, g.variances)
    budget = 64 << 20
    overhead = 16 << 20
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    low = [free0]
    stop = threading.Event()

    def sample():
        while not stop.is_set():
            low[0] = min(low[0], torch.cuda.mem_get_info()[0])
            time.sleep(0.001)

    th = threading.Thread(target=sample, daemon=True)
    th.start()
    try:
        cfg = fv.server_config(precision=fv.PREC_BF16_SPLIT, n_streams=2, hbm_budget_bytes=budget)
        with fv.Server(h, cfg) as s:
            tickets = [s.submit(X) for X in frames] + [s.submit(X) for X in frames[::-1]]
            res = drain(s, tickets)
            st = s.stats()
            low[0] = min(low[0], torch.cuda.mem_get_info()[0])
    finally:
        stop.set()
        th.join()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    drop = free0 - low[0]
    say(f"  held peak {st['peak_admitted_bytes'] / 2**20:.1f} MiB, device free-memory drop "
        f"{drop / 2**20:.1f} MiB (budget 64 MiB + 16 MiB), after destroy {(free0 - free1) / 2**20:.1f} MiB")
    assert st["peak_admitted_bytes"] <= budget
    assert drop <= budget + overhead
    assert free0 - free1 <= overhead
    for i, t in enumerate(tickets):
        assert res[t][0] == fv.OK, (i, res[t][0])
    ref = oracle.encode_gmm(frames[1], g)
    e = errors(res[tickets[1]][1], ref)
    assert e["e_inf"] <= 1e-3 and e["e_2"] <= 1e-3
    h.free()


def test_device_submission_matches_host_submission(fv):
    import torch
    say("[gpu] server device-resident frames, bf16 split K=512 D=80")
    g = fvsynth.gmm(512, 80, 0)
    sizes = [8000, 123, 12500, 0, 2048]
    frames = [fvsynth.frame(g, n, 700 + i, 0.05) for i, n in enumerate(sizes)]
    dev = [torch.from_numpy(X).cuda() for X in frames]
    h = fv.gmm_load(g.weights, g.means, g.variances)
    cfg = fv.server_config(precision=fv.PREC_BF16_SPLIT, n_streams=2)
    with fv.Server(h, cfg) as s:
        host = drain(s, [s.submit(X) for X in frames])
        host = [host[t] for t in sorted(host)]
    with fv.Server(h, cfg) as s:
        tickets = [s.submit_device(Xd) for Xd in dev]
        res = drain(s, tickets)
        assert not s._device_inputs
    for i, t in enumerate(tickets):
        rc, out, st = res[t]
        assert rc == fv.OK and host[i][0] == fv.OK
        # frame-relative chunking: bitwise equal whatever launches the frames shared
        assert np.array_equal(out, host[i][1]), f"frame {i} differs from the host submission"
        if sizes[i] == 0:
            assert np.all(out == 0)
            continue
        e = errors(out, oracle.encode_gmm(frames[i], g))
        say(f"  frame {i} N={sizes[i]} e_inf={e['e_inf']:.2e}")
        assert e["e_inf"] <= 1e-3 and e["e_2"] <= 1e-3


def test_stream_release_and_server_cycles(fv):
    """fv_stream_release frees a stream's cached scratch, staging and graphs: device memory
    comes back, and the next encode on that stream allocates and captures again with the same
    bits.  Servers release their lane streams on destroy: repeated create / encode / destroy
    cycles give the same results and do not accumulate device memory."""
    import torch
    say("[gpu] stream release and server cycles")
    g = fvsynth.gmm(512, 80, 0)
    h = fv.gmm_load(g.weights, g.means, g.variances)
    frames = [fvsynth.frame(g, n, 70 + i, 0.05) for i, n in enumerate((32000, 32000, 8000))]
    X, off = np.concatenate(frames), np.cumsum([0, 32000, 32000, 8000])
    Xd = torch.from_numpy(X).cuda()
    out = torch.empty(3, 2 * 512 * 80, device="cuda")
    st = torch.cuda.Stream()
    fv.stream_release(st)                                   # never used: nothing to do
    fv.encode_batch(h, Xd, off, out=out, precision=1, flags=fv.ASYNC, stream=st)
    st.synchronize()
    first = out.cpu().numpy()
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info()[0]
    fv.stream_release(st)
    after = torch.cuda.mem_get_info()[0]
    say(f"  released {(after - before) / 2**20:.1f} MiB")
    assert after - before >= 16 << 20                      # partial slots alone are ~21 MiB
    out.zero_()
    torch.cuda.synchronize()
    fv.encode_batch(h, Xd, off, out=out, precision=1, flags=fv.ASYNC, stream=st)
    st.synchronize()
    assert np.array_equal(out.cpu().numpy(), first)
    fv.stream_release(st)

    def cycle():
        with fv.Server(h, fv.server_config(precision=fv.PREC_BF16_SPLIT, n_streams=2,
                                           max_batch_frames=1)) as s:
            ts = [s.submit(F) for F in frames]
            res = drain(s, ts)
        return [res[t][1] for t in ts]

    ref = cycle()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for c in range(4):
        got = cycle()
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), c
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"  free device memory change over 4 server cycles: {(free1 - free0) / 2**20:.1f} MiB")
    assert free0 - free1 < 16 << 20
