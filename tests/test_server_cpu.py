"""Serving loop on the CPU with the host-only fake executor: admission, continuous batching,
budget, queue limits, deadlines, injected device errors, ticket handling."""
import threading
import time

import numpy as np
import pytest

import paper_1604_03498_amd as fv

K, D = 4, 3
OUT = 2 * K * D


def fake(**kw):
    base = dict(executor=fv.EXEC_FAKE, fake_K=K, fake_D=D, fake_us_per_krow=2000.0, n_streams=2)
    base.update(kw)
    return fv.Server(None, fv.server_config(**base))


def drain(s, tickets, timeout=10.0):
    res, t0 = {}, time.time()
    pending = set(tickets)
    while pending and time.time() - t0 < timeout:
        t = s.next_done(100.0)
        if t is None or t not in pending:
            continue
        rc, out, st = s.poll(t)
        res[t] = (rc, out, st)
        pending.discard(t)
    assert not pending, f"{len(pending)} requests never finished"
    return res


def test_lifecycle_and_timestamps():
    with fake() as s:
        t = s.submit(np.ones((300, D), np.float32))
        res = drain(s, [t])
        rc, out, st = res[t]
        assert rc == fv.OK and out.shape == (OUT,) and np.all(out == 0)
        assert st["t_submit_us"] <= st["t_admit_us"] <= st["t_start_us"] <= st["t_done_us"]
        assert st["rows"] == 300 and st["batch_frames"] == 1
        assert s.poll(t)[0] == fv.E_NOTFOUND        # consumed
        assert s.poll(12345)[0] == fv.E_NOTFOUND


def test_continuous_batching_groups_waiting_requests():
    with fake(n_streams=1, fake_us_per_krow=20000.0) as s:
        tickets = [s.submit(np.zeros((1000, D), np.float32)) for _ in range(12)]
        res = drain(s, tickets)
        frames = [res[t][2]["batch_frames"] for t in tickets]
        assert all(res[t][0] == fv.OK for t in tickets)
        assert max(frames) > 1                       # later arrivals shared a launch
        st = s.stats()
        assert st["completed"] == 12 and st["launches"] < 12
        # one stream + FIFO admission: requests finish in submission order
        done = [res[t][2]["t_done_us"] for t in tickets]
        assert done == sorted(done)


def test_budget_limits_in_flight_bytes_and_rejects_oversized():
    per = 1000 * D * 4 + OUT * 4                     # fake footprint of one 1000-row frame
    with fake(hbm_budget_bytes=2 * per, n_streams=4, fake_us_per_krow=5000.0) as s:
        tickets = [s.submit(np.zeros((1000, D), np.float32)) for _ in range(10)]
        res = drain(s, tickets)
        assert all(r[0] == fv.OK for r in res.values())
        st = s.stats()
        assert 0 < st["peak_admitted_bytes"] <= 2 * per
        rc, t = s.try_submit(np.zeros((10000, D), np.float32))
        assert rc == fv.E_BUDGET and t is None
        assert s.stats()["rejected"] == 1


def test_queue_full_returns_again():
    with fake(max_queue=3, n_streams=1, max_batch_frames=1, fake_us_per_krow=1e6) as s:
        codes = [s.try_submit(np.zeros((1000, D), np.float32))[0] for _ in range(8)]
        assert fv.E_AGAIN in codes
        assert codes.count(fv.OK) <= 4               # one running + three queued


def test_deadline_fails_waiting_requests():
    with fake(n_streams=1, max_batch_frames=1, fake_us_per_krow=100000.0, deadline_ms=30.0) as s:
        tickets = [s.submit(np.zeros((1000, D), np.float32)) for _ in range(4)]
        res = drain(s, tickets, timeout=20.0)
        codes = [res[t][0] for t in tickets]
        assert codes[0] == fv.OK                     # admitted immediately
        assert fv.E_TIMEOUT in codes[1:]
        assert s.stats()["failed"] >= 1


def test_cancel_withdraws_queued_and_finished_requests():
    """fv_server_cancel: a queued request is withdrawn (never launched, never reported); one
    already in a launch answers PENDING and completes normally; a finished, unpolled one is
    dropped with its completion notice; unknown or consumed tickets are NOT_FOUND."""
    def wait_for(pred, timeout=10.0):
        t0 = time.time()
        while not pred():
            assert time.time() - t0 < timeout, "condition never reached"
            time.sleep(0.002)

    with fake(n_streams=1, max_batch_frames=1, fake_us_per_krow=100000.0) as s:
        a = s.submit(np.zeros((1000, D), np.float32))            # 100 ms launch
        wait_for(lambda: s.stats()["in_flight"] == 1)
        b = s.submit(np.zeros((1000, D), np.float32))
        c = s.submit(np.zeros((10, D), np.float32))
        assert s.cancel(b) == fv.OK
        assert s.cancel(b) == fv.E_NOTFOUND
        assert s.cancel(a) == fv.PENDING
        assert s.cancel(987654) == fv.E_NOTFOUND
        res = drain(s, [a, c])
        assert res[a][0] == fv.OK and res[c][0] == fv.OK
        assert s.next_done(50.0) is None                          # b is never reported
        assert s.poll(b)[0] == fv.E_NOTFOUND
        e = s.submit(np.zeros((10, D), np.float32))
        wait_for(lambda: s.stats()["completed"] == 3)
        assert s.cancel(e) == fv.OK                               # finished, not polled
        assert s.poll(e)[0] == fv.E_NOTFOUND
        assert s.next_done(50.0) is None
        st = s.stats()
        assert st["cancelled"] == 2 and st["completed"] == 3 and st["queued"] == 0


def test_injected_device_error_fails_only_that_batch():
    with fake(n_streams=1, max_batch_frames=1, fake_fail_every=2, fake_us_per_krow=100.0) as s:
        tickets = [s.submit(np.zeros((100, D), np.float32)) for _ in range(6)]
        res = drain(s, tickets)
        codes = [res[t][0] for t in tickets]
        assert codes.count(fv.E_DEVICE) == 3 and codes.count(fv.OK) == 3
        assert all(res[t][1] is None for t in tickets if res[t][0] != fv.OK)


def test_threads_submit_concurrently():
    with fake(fake_us_per_krow=50.0) as s:
        out, lock = [], threading.Lock()

        def worker(n):
            for i in range(25):
                t = s.submit(np.full((50 + i, D), n, np.float32))
                with lock:
                    out.append(t)

        ths = [threading.Thread(target=worker, args=(n,)) for n in range(4)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        assert len(set(out)) == 100
        res = drain(s, out)
        assert all(r[0] == fv.OK for r in res.values())
        assert s.stats()["rows_done"] == sum(50 + i for i in range(25)) * 4


def test_empty_frame_and_invalid_arguments():
    with fake() as s:
        t = s.submit(np.zeros((0, D), np.float32))
        assert drain(s, [t])[t][0] == fv.OK
        with pytest.raises(ValueError):
            s.submit(np.zeros((3, D + 1), np.float32))
    with pytest.raises(fv.FvError):
        fv.Server(None, fv.server_config(executor=fv.EXEC_FAKE))         # no K/D without a GMM
    with pytest.raises(fv.FvError):
        fv.Server(None, fv.server_config(executor=fv.EXEC_HIP))          # HIP executor needs a GMM
    with pytest.raises(fv.FvError):
        fv.Server(None, fv.server_config(executor=fv.EXEC_FAKE, fake_K=1, fake_D=1, precision=9))


def test_oversized_frame_is_refused_without_a_budget():
    """With an unlimited budget a frame past the encoder's row limit (2^40 / D rows) is refused
    with FV_E_UNSUPPORTED before anything is read or allocated (the staging size would
    overflow)."""
    import ctypes
    lib = fv.load()
    buf = np.zeros((1, D), np.float32)
    with fake(hbm_budget_bytes=0) as s:
        tk = ctypes.c_uint64()
        for n in ((1 << 40) // D + 1, 1 << 62):
            rc = lib.fv_server_submit(ctypes.c_void_p(s.handle), buf.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.c_int64(n), ctypes.byref(tk))
            assert rc == fv.E_UNSUPPORTED
        t = s.submit(np.ones((10, D), np.float32))        # the server still works
        assert drain(s, [t])[t][0] == fv.OK


def test_destroy_with_work_outstanding():
    s = fake(n_streams=1, fake_us_per_krow=10000.0)
    for _ in range(5):
        s.submit(np.zeros((500, D), np.float32))
    s.close()                                        # drops queued requests, waits for the launch


def test_batching_window_collects_frames():
    with fake(n_streams=1, batch_window_us=1e5, fake_us_per_krow=10.0) as s:
        tickets = [s.submit(np.zeros((100, D), np.float32)) for _ in range(5)]
        res = drain(s, tickets)
        assert all(res[t][0] == fv.OK and res[t][2]["batch_frames"] == 5 for t in tickets)
        assert res[tickets[0]][2]["t_admit_us"] - res[tickets[0]][2]["t_submit_us"] >= 0.9e5


def test_device_submission_keeps_frame_until_done():
    # the fake executor never reads X; the binding must keep the frame referenced until the
    # ticket has finished, then release it
    with fake(n_streams=1) as s:
        X = np.ones((500, D), np.float32)
        t = s.submit_device(X)
        assert t in s._device_inputs
        res = drain(s, [t])
        assert res[t][0] == fv.OK and res[t][2]["rows"] == 500
        assert t not in s._device_inputs
        with pytest.raises(ValueError):
            s.submit_device(np.ones((5, D + 1), np.float32))
