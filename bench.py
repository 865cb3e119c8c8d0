#!/usr/bin/env python3
"""Benchmark of the Fisher-vector encoding hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp32,bf16_split,fp16_split]
                    [--no-frame] [--no-cpu-baseline] [--calib-copy-mb M]

One step = one full pass of the encoder (work-table copy, load + square, E-step contraction,
soft assignment, statistics contraction, chunk reduction, u/v assembly, signed square root,
L2) over one batch of synthetic input already resident in device memory: 64 frames with
N_f uniform in [2,000, 20,000] descriptors (686,155 in all), D = 64, K = 256 GMM, 5% uniform
outliers per frame, encoded by fv_encode_batch as one persistent, graph-captured launch
sequence.  `value` is FP32 descriptors/s over the K timed steps (HIP events on the launch
stream around every step; median, p10 and p90 of the per-step times are reported too); the
bf16 and fp16 hi-lo split forms are timed the same way under "forms", each with its
per-frame error against the FP64 oracle.  The single 8,000-descriptor frame (fv_encode), the
paper's threshold mode, the projection prologue, the EM step and the serving form are
reported as extras.  The GMM load (per-model constant precompute) happens once before timing
and is reported separately.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

# MI355X dense peaks: FP32 MFMA 157.3 TFLOP/s; BF16 / FP16 MFMA 2.5 PFLOP/s.
PEAK_TFLOPS = {"fp32": 157.3, "bf16_split": 2500.0, "fp16_split": 2500.0, "bf16": 2500.0}
PREC_CODE = {"fp32": 0, "bf16_split": 1, "fp16_split": 2, "bf16": 3}
PRODUCTS = {"fp32": 1, "bf16_split": 3, "fp16_split": 3, "bf16": 1}
DTYPE = {"fp32": "f32", "bf16_split": "bf16x3", "fp16_split": "f16x3", "bf16": "bf16"}
METRIC = "descriptors/sec encoded (K=256,D=64), BF16-split vs FP32; p99 frame latency"


SRC_DIR = os.path.join(HERE, "paper_1604_03498_amd", "csrc")
TRAFFIC_JSON = os.path.join(HERE, "profiles", "hbm_traffic.json")
# statistics kernels of each path at D = 64 (as named in rocprofv3 traces)
STATS_KERNELS = {
    ("fp32", "split"): ["fused_f32_kernel<64, 8, true, false, true>", "sliced_f32_kernel<64, 8, false, true>"],
    ("fp32", "fused"): ["fused_f32_kernel<64, 8, false, false, false>"],
    ("bf16_split", "split"): ["lse16_kernel<64, 8>", "sliced16r_kernel<64, false>"],
    ("bf16_split", "fused"): ["fused16p_kernel<64, false, false>"],
    ("fp16_split", "split"): ["lse16_kernel<64, 8>", "sliced16r_kernel<64, false>"],
    ("fp16_split", "fused"): ["fused16p_kernel<64, false, false>"],
}


def kernel_source_hash():
    """SHA-256 over the library's kernel and host sources: HBM counters taken on other sources
    do not describe the kernels that run now."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(SRC_DIR)):
        if name.endswith((".hip", ".inc", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(SRC_DIR, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def short_kernel(name):
    m = re.search(r"::(\w+_kernel(?:<[^>]*>)?)", name.replace("(anonymous namespace)", "anon"))
    return m.group(1) if m else name.split("(")[0][-60:]


def load_traffic(form, path, launches_per_step):
    """HBM bytes per statistics step from the committed counter summary, or None when it is
    absent, lacks these kernels, or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    names = STATS_KERNELS.get((form, path))
    per = t.get("kernels", {})
    if not names or not all(n in per for n in names):
        return None
    fetch = sum(per[n]["read_bytes"] for n in names)
    write = sum(per[n]["write_bytes"] for n in names)
    return {"bytes": (fetch + write) * launches_per_step, "read_bytes": fetch * launches_per_step,
            "write_bytes": write * launches_per_step, "kernels": names,
            "from": "profiles/hbm_traffic.json"}


def pmc_summary(fetch_dir, write_dir, calib_mb):
    """Per-kernel HBM bytes from two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, both with --calib-copy-mb): the counters of the plain calib_mb MiB device copy
    at the end of the run give the scale from counter units to bytes.  Writes
    profiles/hbm_traffic.json (with the source hash) and prints a markdown table."""
    def per_dispatch(d, counter):
        rows = []
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as f:
                rows += [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
        acc = {}
        for r in rows:
            k = (r["Dispatch_Id"], r["Kernel_Name"])
            acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        return acc
    fetch = per_dispatch(fetch_dir, "FETCH_SIZE")
    write = per_dispatch(write_dir, "WRITE_SIZE")
    expect = calib_mb * (1 << 20)

    def calib(acc):
        copies = [v for (d, n), v in acc.items() if "copyBuffer" in n or "copy" in n.lower()]
        return expect / (max(copies) * 1024.0) if copies else None
    fr, wr = calib(fetch), calib(write)
    if fr is None or wr is None:
        raise SystemExit("no calibration copy kernel found in the counter runs")

    def mean_by_kernel(acc):
        out = {}
        for (d, n), v in acc.items():
            out.setdefault(short_kernel(n), []).append(v)
        return {k: (sum(v) / len(v), len(v)) for k, v in out.items()}
    mf, mw = mean_by_kernel(fetch), mean_by_kernel(write)
    kernels = {}
    for k in sorted(set(mf) & set(mw)):
        if not k.endswith(">") and "_kernel" not in k:
            continue
        kernels[k] = {"read_bytes": mf[k][0] * 1024.0 * fr, "write_bytes": mw[k][0] * 1024.0 * wr,
                      "fetch_kib_raw": mf[k][0], "write_kib_raw": mw[k][0], "dispatches": mf[k][1]}
    # a second summary on the same sources (the other workload) adds to the first
    try:
        with open(TRAFFIC_JSON) as f:
            prev = json.load(f)
        if prev.get("source_sha256") == kernel_source_hash():
            kernels = {**prev.get("kernels", {}), **kernels}
    except (OSError, ValueError):
        pass
    out = {"source_sha256": kernel_source_hash(), "calibration_copy_mib": calib_mb,
           "read_scale": fr, "write_scale": wr, "kernels": kernels}
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(f"scales: read x{fr:.3f}, write x{wr:.3f} (counter KiB -> bytes x1024)")
    print("| kernel | dispatches | FETCH_SIZE (KiB, raw) | reads (MiB) | WRITE_SIZE (KiB, raw) | writes (MiB) |")
    print("|---|---|---|---|---|---|")
    for k, v in kernels.items():
        print(f"| `{k}` | {v['dispatches']} | {v['fetch_kib_raw']:.1f} | {v['read_bytes'] / 2**20:.2f} | "
              f"{v['write_kib_raw']:.1f} | {v['write_bytes'] / 2**20:.2f} |")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50,
                    help="timed steps (batches) of the headline workload")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frame-steps", type=int, default=300,
                    help="timed encodes of the single-frame extra")
    ap.add_argument("--frame-warmup", type=int, default=30)
    ap.add_argument("--forms", default="fp32,bf16_split,fp16_split")
    ap.add_argument("--latency-samples", type=int, default=300)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-frame", action="store_true",
                    help="skip the single-frame forms (profiling the batch alone)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch with the default tuning instead of the measuring autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-em", action="store_true", help="skip the EM-step measurement")
    ap.add_argument("--no-projection", action="store_true",
                    help="skip the projection-prologue measurements")
    ap.add_argument("--no-dsift", action="store_true",
                    help="skip the dense-SIFT front end measurement")
    ap.add_argument("--no-paper-mode", action="store_true",
                    help="skip the posterior-threshold (paper mode) measurements")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serving-seconds", type=float, default=4.0,
                    help="measured seconds of each open-loop serving run (0: skip)")
    ap.add_argument("--sweep", default="1,4,16,64",
                    help="serving saturation sweep: arrival-rate multipliers of the 30 Hz streams, "
                         "2 s each ('' to skip)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (HBM-counter scale)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this "
                         "script made with --calib-copy-mb into profiles/hbm_traffic.json; no GPU")
    return ap.parse_args()


def path_of(K, N, n_cu, fv_path_env):
    """The statistics path the library picks for one frame (mirrors its rule)."""
    if fv_path_env in ("fused", "split"):
        return fv_path_env
    if K > 256:
        return "split"
    return "split" if N < 4 * 32 * n_cu else "fused"


def time_form(fv, torch, h, Xd, off, out, form, steps, warmup, stream, lat_samples, batch,
              flags=0):
    prec = PREC_CODE[form]
    fl = fv.ASYNC | flags

    def step():
        if batch:
            fv.encode_batch(h, Xd, off, out=out, precision=prec, flags=fl, stream=stream)
        else:
            fv.encode(h, Xd, out=out, precision=prec, flags=fl, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed region: `steps` encodes (graph replays of the captured launch sequence)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # kernel durations: HIP events around every statistics / finalize launch on `stream`
    # (event timing runs the same launches uncaptured)
    fv.kernel_timing(True)
    for _ in range(max(5, min(steps, 50))):
        step()
    torch.cuda.synchronize()
    st_ms, st_n = fv.kernel_timing_read(0)
    fi_ms, fi_n = fv.kernel_timing_read(1)
    fv.kernel_timing(False)
    lat = []
    if lat_samples:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(lat_samples):
            e0.record(stream)
            step()
            e1.record(stream)
            e1.synchronize()
            lat.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    return elapsed, st_ms / max(st_n, 1), st_n, fi_ms / max(fi_n, 1), np.array(lat)


def trial_name(t):
    n = f"{'fused' if t['batch_path'] == 1 else 'split'}/{t['batch_chunk']}"
    if t.get("batch_grid"):
        n += f"/grid{t['batch_grid']}"
    if t.get("fused16_variant"):
        n += f"/v{t['fused16_variant']}"
    return n


def apply_tuned(fv, h, tuned):
    """The autotuner's choice for a form, recorded in the batch results."""
    fv.set_tuning(h, batch_path=1 if tuned["path"] == "fused" else 2, batch_chunk=tuned["chunk"],
                  batch_grid=tuned.get("grid", 0), fused16_variant=tuned.get("variant", 0))


def time_steps(torch, step, steps, warmup, stream):
    """`warmup` untimed steps, then `steps` timed ones with a HIP event recorded on `stream`
    before the first and after every step; the region is bracketed by device
    synchronisations.  Returns (GPU ms of all steps, per-step ms array, wall seconds)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return ev[0].elapsed_time(ev[steps]), per, wall


def kernel_avgs(fv, torch, step, reps):
    """Average device duration of the statistics and finalize launches over `reps` uncaptured
    steps (events bracket every launch on its own stream)."""
    fv.kernel_timing(True)
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    st_ms, st_n = fv.kernel_timing_read(0)
    fi_ms, fi_n = fv.kernel_timing_read(1)
    fv.kernel_timing(False)
    return st_ms / max(st_n, 1), st_n, fi_ms / max(fi_n, 1), fi_n


def step_stats(per):
    return {"median": float(np.median(per)), "p10": float(np.percentile(per, 10)),
            "p90": float(np.percentile(per, 90)), "min": float(per.min()),
            "max": float(per.max()), "samples": int(per.size)}


def roofline(form, K, D, ndesc, stats_avg_ms, path, launches_per_step=1):
    alg = 8.0 * K * D * ndesc                      # algorithmic flops of the two contractions
    # the two-pass path computes the E-step twice, except FP32 with one component group, whose
    # first pass hands the posterior factors to the second (up to DP = 64)
    handover = (form == "fp32" and path == "split" and K <= 256 and D <= 64
                and os.environ.get("FV_SPLIT_GAMMA", "1") != "0")
    execd = alg * PRODUCTS[form] * (1.5 if path == "split" and not handover else 1.0)
    achieved = alg / (stats_avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[form]
    tr = load_traffic(form, path, launches_per_step) if D == 64 else None
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": tr["bytes"] if tr else None,
            "traffic_detail": tr,
            "mfma_util": round(execd / (stats_avg_ms * 1e-3) / 1e12 / peak, 4),
            "kernel": ("fused statistics kernel" if path == "fused" else
                       "two-pass statistics: row log-sum-exp pass (writing the posterior factors) "
                       "+ component-sliced pass" if handover else
                       "two-pass statistics: row log-sum-exp pass + component-sliced pass"),
            "kernel_avg_us": round(stats_avg_ms * 1e3, 3)}


def run_serving(fv, seconds, warm_s, budget_bytes, form="bf16_split", pool=2, n_streams=2,
                rate_mult=1.0, device_input=False):
    """Open-loop serving run: 16 camera streams, Poisson arrivals at 30 Hz each, frames of
    8,000-32,000 descriptors (320x240 .. 640x480), D = 80, K = 512.  Latency is measured from
    each frame's scheduled arrival time to the completion of its encode (so a late submit
    counts against the server), over the frames that arrive after the warm-up."""
    import threading
    import fvsynth
    g = fvsynth.gmm(512, 80, 0)
    events, sizes = fvsynth.serving_plan(rate_hz=30.0 * rate_mult, duration_s=warm_s + seconds,
                                         pool=pool)
    frames = {(st, p): fvsynth.frame(g, sizes[st], 100000 + 100 * st + p, 0.05)
              for st in range(len(sizes)) for p in range(pool)}
    if device_input:  # frames already resident in HBM: no staging copy at submit time
        import torch
        frames = {k: torch.from_numpy(v).cuda() for k, v in frames.items()}
        torch.cuda.synchronize()
    submit = (lambda s_, X: s_.try_submit_device(X)) if device_input else (lambda s_, X: s_.try_submit(X))
    h = fv.gmm_load(g.weights, g.means, g.variances, device=0)
    cfg = fv.server_config(precision=PREC_CODE[form], n_streams=n_streams,
                           hbm_budget_bytes=int(budget_bytes))
    srv = fv.Server(h, cfg)
    for st in range(len(sizes)):          # warm every frame size once (buffers, code objects)
        t = submit(srv, frames[(st, 0)])[1]
        while srv.next_done(1000.0) != t:
            pass
        srv.poll(t, want_out=False)
    srv.stats(reset=True)
    sub = {}
    done = {}
    submitting = threading.Event()
    submitting.set()
    finished = threading.Event()

    def collect():
        while submitting.is_set() or len(done) < len(sub):
            t = srv.next_done(100.0)
            if t is None:
                continue
            rc, _, stt = srv.poll(t, want_out=False)
            done[t] = (rc, stt)
        finished.set()

    th = threading.Thread(target=collect, daemon=True)
    th.start()
    t0 = time.perf_counter()
    window = warm_s + seconds
    dropped = 0
    for (t_arr, st, p) in events:
        wait = t0 + t_arr - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        ts = time.perf_counter()
        if ts - t0 > window:         # saturated: arrivals past the window are not submitted
            dropped += 1
            continue
        while True:
            rc, tk = submit(srv, frames[(st, p)])
            if rc == fv.OK:
                break
            time.sleep(0.0005)
        sub[tk] = (t_arr, ts - t0, sizes[st])
    submitting.clear()
    finished.wait(timeout=120.0)
    wall = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    # a frame counts if it completed after the warm-up; its completion time on the submitter's
    # clock is its submit time plus the server's submit-to-done interval
    lat, rows, fails, frames_in_launch, t_last = [], 0, 0, [], warm_s
    for tk, (t_arr, t_sub, n) in sub.items():
        if tk not in done:
            continue
        rc, stt = done[tk]
        t_end = t_sub + (stt["t_done_us"] - stt["t_submit_us"]) * 1e-6
        if t_end < warm_s:
            continue
        if rc != fv.OK:
            fails += 1
            continue
        lat.append((t_end - t_arr) * 1e3)
        rows += n
        t_last = max(t_last, t_end)
        frames_in_launch.append(stt["batch_frames"])
    lat = np.array(lat)
    return {"form": form, "streams": len(sizes), "rate_hz_per_stream": 30.0 * rate_mult,
            "frame_sizes": sorted(set(sizes)), "K": 512, "D": 80,
            "measured_s": seconds, "frames": int(lat.size), "failed": fails, "not_submitted": dropped,
            "offered_desc_per_s": float(sum(sizes) * 30.0 * rate_mult),
            "throughput_desc_per_s": rows / max(t_last - warm_s, 1e-9),  # to the last completion
            "latency_ms_from_arrival": {"p50": float(np.percentile(lat, 50)) if lat.size else None,
                                        "p99": float(np.percentile(lat, 99)) if lat.size else None,
                                        "max": float(lat.max()) if lat.size else None},
            "mean_frames_per_launch": float(np.mean(frames_in_launch)) if frames_in_launch else None,
            "budget_bytes": int(budget_bytes), "peak_admitted_bytes": int(stats["peak_admitted_bytes"]),
            "gpu_busy_fraction": stats["busy_s"] / max(wall - warm_s, 1e-9), "n_streams": n_streams,
            "busy_note": "sum of launch durations over the server's streams / wall time (can exceed 1 "
                         "when launches on different streams overlap)",
            "input": ("device memory (fv_server_submit_device; device-to-device gather in the launch)"
                      if device_input else
                      "host memory (submit copies into pinned staging; H2D inside the launch)")}


def c5_capacity(fv, torch, dev, stream, forms, steps):
    """GPU throughput at the serving shape with inputs already in device memory: one frame of
    each of the 16 camera streams' sizes (8,000-32,000 descriptors, K = 512, D = 80) encoded
    as one batch (graph replays).  Set beside the serving sweep, it separates the device's
    capacity from the host-side staging of the serving runs."""
    import fvsynth
    g = fvsynth.gmm(512, 80, 0)
    _, sizes = fvsynth.serving_plan(duration_s=1.0)
    frames = [fvsynth.frame(g, n, 100000 + 100 * st, 0.05) for st, n in enumerate(sizes)]
    X = np.concatenate(frames)
    off = np.zeros(len(frames) + 1, np.int64)
    off[1:] = np.cumsum([f.shape[0] for f in frames])
    h = fv.gmm_load(g.weights, g.means, g.variances, device=0)
    Xd = torch.from_numpy(X).to(dev)
    out = {}
    for form in forms:
        o = torch.empty(len(frames), 2 * 512 * 80, dtype=torch.float32, device=dev)
        el, st_avg, _, fi_avg, _ = time_form(fv, torch, h, Xd, off, o, form, steps, 2, stream, 0, True)
        out[form] = {"value": int(off[-1]) * steps / el, "ms_per_batch": el * 1e3 / steps,
                     "statistics_us": round(st_avg * 1e3, 2), "finalize_us": round(fi_avg * 1e3, 2)}
        log(f"[bench] c5 capacity form={form}: {out[form]['value']:.3e} desc/s")
    out["config"] = {"K": 512, "D": 80, "frames": len(frames), "descriptors": int(off[-1])}
    return out


def oracle_c1():
    """The oracle on the small configuration (K = 64, D = 64, N = 2,000): seconds per frame on
    one thread, and frames/s with whole frames spread over the host threads."""
    import fvsynth
    import oracle
    g, X, _ = fvsynth.workload("c1_oracle_k64_d64_n2000")
    t0 = time.perf_counter()
    oracle.encode_batch(X, np.array([0, X.shape[0]], np.int64), g.weights, g.means, g.variances,
                        nthreads=1)
    one = time.perf_counter() - t0
    nthreads = max(1, min(16, os.cpu_count() or 1))
    Xs = np.concatenate([X] * nthreads)
    o = np.arange(nthreads + 1, dtype=np.int64) * X.shape[0]
    t0 = time.perf_counter()
    oracle.encode_batch(Xs, o, g.weights, g.means, g.variances, nthreads=nthreads)
    allc = time.perf_counter() - t0
    return {"seconds_per_frame_1_thread": one, "frames_per_s_all_threads": nthreads / allc,
            "threads": nthreads, "workload": "c1_oracle_k64_d64_n2000"}


def cpu_baseline_batch(g, X, off, seconds):
    """The FP64 oracle on the host cores over a bounded sample of the headline workload: the
    whole batch, frames spread over the threads, repeated until `seconds` elapse (at least
    once).  Returns (the baseline record, the oracle's vectors of the first pass)."""
    import oracle
    nthreads = max(1, min(16, os.cpu_count() or 1))
    ref, reps, t0 = None, 0, time.perf_counter()
    while reps == 0 or time.perf_counter() - t0 < seconds:
        r = oracle.encode_batch(X, off, g.weights, g.means, g.variances, nthreads=nthreads)
        if ref is None:
            ref = r
        reps += 1
    dt = time.perf_counter() - t0
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    done = reps * int(off[-1])
    return ({"value": done / dt, "unit": "descriptors/s", "cores": nthreads, "kind": "oracle",
             "cpu_model": model, "host_cpus": os.cpu_count(),
             "sample": f"{reps} pass(es) over the whole batch ({off.size - 1} frames, {done} "
                       f"descriptors) in {dt:.1f} s; FP64 C oracle, whole frames spread over "
                       f"{nthreads} threads"}, ref)


def main():
    a = parse()
    if a.pmc_summary:
        pmc_summary(a.pmc_summary[0], a.pmc_summary[1], a.calib_copy_mb or 256)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: run with --gpus 1 (frames would shard across "
                                   "GPUs with only the results gathered; not built)"}))
        sys.exit(2)
    import torch
    import fvsynth
    import paper_1604_03498_amd as fv

    dev = torch.device("cuda:0")
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    forms = [f for f in a.forms.split(",") if f]
    stream = torch.cuda.Stream(device=dev)

    # ---- headline: the 64-frame batch, one graph-replayed fv_encode_batch per step
    g, Xb, offb = fvsynth.workload("c4_batch64_k256_d64")
    K, D = g.K, g.D
    nb, B = int(offb[-1]), int(offb.size - 1)
    t0 = time.perf_counter()
    h = fv.gmm_load(g.weights, g.means, g.variances, device=0)
    gmm_load_ms = (time.perf_counter() - t0) * 1e3
    hb = h
    Xbd = torch.from_numpy(Xb).to(dev)
    from paper_1604_03498_amd import autotune
    batch, batch_out = {}, {}
    for form in forms:
        prec = PREC_CODE[form]
        outb = torch.empty(B, 2 * K * D, dtype=torch.float32, device=dev)
        if a.no_autotune:
            fv.set_tuning(hb)
            tuned = {"batch_path": 1 if path_of(K, nb, n_cu, None) == "fused" else 2,
                     "batch_chunk": fv.get_tuning(hb)["batch_chunk"] or 1024, "trials": []}
        else:
            tuned = autotune.tune_batch(hb, Xbd, offb, prec, stream=stream, reps=10,
                                        use_cache=False)
        bpath = {1: "fused", 2: "split"}[tuned["batch_path"]]
        log(f"[bench] batch form={form} tuned path={bpath} chunk={tuned['batch_chunk']} "
            f"grid={tuned.get('batch_grid', 0)} variant={tuned.get('fused16_variant', 0)} "
            f"warmup={a.warmup} steps={a.steps}")

        def bstep(prec=prec, outb=outb):
            fv.encode_batch(hb, Xbd, offb, out=outb, precision=prec, flags=fv.ASYNC,
                            stream=stream)
        tot_ms, per, wall = time_steps(torch, bstep, a.steps, a.warmup, stream)
        st_avg, st_n, fi_avg, _ = kernel_avgs(fv, torch, bstep, max(5, min(a.steps, 20)))
        rf = roofline(form, K, D, nb, st_avg, bpath)
        ms = tot_ms / a.steps
        rf["step_frac"] = round(8.0 * K * D * nb / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[form], 4)
        batch[form] = {"value": nb / (ms * 1e-3), "ms_per_step": ms, "step_ms": step_stats(per),
                       "wall_ms_per_step": wall * 1e3 / a.steps, "roofline": rf,
                       "finalize_avg_us": round(fi_avg * 1e3, 3), "stats_launches": st_n,
                       "tuned": {"path": bpath, "chunk": tuned["batch_chunk"],
                                 "grid": tuned.get("batch_grid", 0),
                                 "variant": tuned.get("fused16_variant", 0),
                                 "trials_ms": {trial_name(t): round(t["ms"], 4)
                                               for t in tuned["trials"]}}}
        batch_out[form] = outb.cpu().numpy()
        log(f"[bench]   {batch[form]['value']:.4e} desc/s, {ms:.4f} ms/step (median "
            f"{batch[form]['step_ms']['median']:.4f}), stats kernel {rf['kernel_avg_us']} us, "
            f"frac {rf['frac']}, mfma util {rf['mfma_util']}")
    fv.set_tuning(hb)
    batch["config"] = {"workload": "c4_batch64_k256_d64", "frames": B, "descriptors": nb}

    # ---- extra: the single 8,000-descriptor frame (fv_encode), every form
    _, X, off = fvsynth.workload("c2_frame_k256_d64_n8000")
    N = int(X.shape[0])
    Xd = torch.from_numpy(X).to(dev)
    path = path_of(K, N, n_cu, os.environ.get("FV_PATH"))
    results, outputs = {}, {}
    for form in ([] if a.no_frame else forms):
        out = torch.empty(2 * K * D, dtype=torch.float32, device=dev)
        log(f"[bench] frame form={form} path={path} warmup={a.frame_warmup} steps={a.frame_steps}")
        el, st_avg, st_n, fi_avg, lat = time_form(fv, torch, h, Xd, off, out, form, a.frame_steps,
                                                   a.frame_warmup, stream, a.latency_samples, False)
        r = {"value": N * a.frame_steps / el, "ms_per_step": el * 1e3 / a.frame_steps,
             "roofline": roofline(form, K, D, N, st_avg, path),
             "finalize_avg_us": round(fi_avg * 1e3, 3), "launches": st_n}
        if lat.size:
            r["latency_ms"] = {"p10": float(np.percentile(lat, 10)),
                               "p50": float(np.percentile(lat, 50)),
                               "p90": float(np.percentile(lat, 90)),
                               "p99": float(np.percentile(lat, 99)),
                               "max": float(lat.max()), "samples": int(lat.size)}
            r["value_from_event_p50"] = N / (r["latency_ms"]["p50"] * 1e-3)
        # end to end from host memory: X in pinned host memory, the output back in host memory
        # (the H2D and D2H copies inside each call)
        if a.latency_samples:
            Xh = torch.from_numpy(X).pin_memory()
            outh = torch.empty(2 * K * D, dtype=torch.float32).pin_memory()
            for _ in range(5):
                fv.encode(h, Xh, out=outh, precision=PREC_CODE[form], stream=stream)
            hl = []
            for _ in range(min(100, a.latency_samples)):
                t0h = time.perf_counter()
                fv.encode(h, Xh, out=outh, precision=PREC_CODE[form], stream=stream)
                hl.append((time.perf_counter() - t0h) * 1e3)
            hl = np.array(hl)
            r["host_input_end_to_end"] = {
                "value": N / (np.median(hl) * 1e-3), "p50_ms": float(np.median(hl)),
                "p90_ms": float(np.percentile(hl, 90)), "samples": int(hl.size),
                "note": "pinned host X and output; H2D, encode and D2H in each synchronous call"}
        results[form] = r
        outputs[form] = out.cpu().numpy()
        log(f"[bench]   {r['value']:.4e} desc/s, {r['ms_per_step']:.4f} ms/step, "
            f"stats {r['roofline']['kernel_avg_us']} us")

    # The paper's posterior threshold (gamma > 1e-6, skipped MFMA steps): the same frame, the
    # same frame with its rows grouped by generating component, and the batch
    paper = {}
    paper_out = {}
    if not a.no_paper_mode and not a.no_frame:
        Xc = fvsynth.frame(g, N, fvsynth.WORKLOADS["c2_frame_k256_d64_n8000"]["frame_seed"], 0.05,
                           clustered=True)
        Xcd = torch.from_numpy(Xc).to(dev)
        if batch:
            # the batch's frames, each with its rows grouped by generating component
            w4 = fvsynth.WORKLOADS["c4_batch64_k256_d64"]
            sz = fvsynth.batch_sizes(w4["B"], w4["sizes_seed"])
            Xbc = np.concatenate([fvsynth.frame(g, int(n), w4["frame_seed0"] + f, w4["outliers"],
                                                clustered=True) for f, n in enumerate(sz)])
            Xbcd = torch.from_numpy(np.ascontiguousarray(Xbc)).to(dev)
        for form in forms:
            paper[form] = {}
            for name, xin in (("frame", Xd), ("frame_clustered", Xcd)):
                out = torch.empty(2 * K * D, dtype=torch.float32, device=dev)
                el, st_avg, _, _, _ = time_form(fv, torch, h, xin, off, out, form, a.frame_steps,
                                                a.frame_warmup, stream, 0, False, fv.THRESHOLD)
                paper[form][name] = {"value": N * a.frame_steps / el,
                                     "ms_per_step": el * 1e3 / a.frame_steps,
                                     "stats_avg_us": round(st_avg * 1e3, 3)}
                paper_out[(form, name)] = out.cpu().numpy()
                log(f"[bench] paper mode {name} form={form}: {N * a.frame_steps / el:.4e} desc/s, "
                    f"stats {st_avg * 1e3:.3f} us")
            if batch and form in batch:
                outb = torch.empty(offb.size - 1, 2 * K * D, dtype=torch.float32, device=dev)
                apply_tuned(fv, hb, batch[form]["tuned"])
                for name, xin in (("batch", Xbd), ("batch_clustered", Xbcd)):
                    el, st_avg, _, _, _ = time_form(fv, torch, hb, xin, offb, outb, form,
                                                    a.batch_steps, 2, stream, 0, True,
                                                    fv.THRESHOLD)
                    nb = int(offb[-1])
                    paper[form][name] = {"value": nb * a.batch_steps / el,
                                         "ms_per_step": el * 1e3 / a.batch_steps,
                                         "stats_avg_us": round(st_avg * 1e3, 3),
                                         "path": batch[form]["tuned"]["path"]}
                    log(f"[bench] paper mode {name} form={form}: "
                        f"{nb * a.batch_steps / el:.4e} desc/s, stats {st_avg * 1e3:.1f} us")
        if batch:
            fv.set_tuning(hb)

    # Projection prologue (raw 130-value descriptors -> D = 64 by y = A (x - m), then the
    # encode), on the same frame and batch drawn through the stand-in PCA
    projected = {}
    if not a.no_projection and not a.no_frame:
        pc = fvsynth.pca(D, 0)
        hp = fv.pca_load(pc.A, pc.mean)
        w2 = fvsynth.WORKLOADS["c2_frame_k256_d64_n8000"]
        Xr = fvsynth.raw_frame(g, pc, N, w2["frame_seed"], w2["outliers"])
        Xrd = torch.from_numpy(Xr).to(dev)
        runs = [("frame", Xrd, None)]
        if batch:
            w4 = fvsynth.WORKLOADS["c4_batch64_k256_d64"]
            Xrb, offrb = fvsynth.raw_batch(g, pc, fvsynth.batch_sizes(w4["B"], w4["sizes_seed"]),
                                           w4["frame_seed0"], w4["outliers"])
            runs.append(("batch", torch.from_numpy(Xrb).to(dev), offrb))
        for form in forms:
            projected[form] = {}
            for name, xin, offr in runs:
                nrows = int(xin.shape[0])
                shape = (2 * K * D,) if offr is None else (offr.size - 1, 2 * K * D)
                out = torch.empty(shape, dtype=torch.float32, device=dev)
                prec = PREC_CODE[form]
                if offr is not None and form in batch:
                    apply_tuned(fv, hb, batch[form]["tuned"])

                def pstep():
                    if offr is None:
                        fv.encode_projected(h, hp, xin, out=out, precision=prec, flags=fv.ASYNC,
                                            stream=stream)
                    else:
                        fv.encode_batch_projected(h, hp, xin, offr, out=out, precision=prec,
                                                  flags=fv.ASYNC, stream=stream)
                steps = a.frame_steps if offr is None else a.batch_steps
                for _ in range(a.frame_warmup if offr is None else 2):
                    pstep()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    pstep()
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                fv.kernel_timing(True)
                for _ in range(max(5, min(steps, 50))):
                    pstep()
                torch.cuda.synchronize()
                pr_ms, pr_n = fv.kernel_timing_read(2)
                fv.kernel_timing(False)
                pr_avg = pr_ms / max(pr_n, 1)
                # projection algorithmic bytes: read Din, write D floats per descriptor
                pbytes = nrows * 4.0 * (Xr.shape[1] + D)
                projected[form][name] = {
                    "value": nrows * steps / el, "ms_per_step": el * 1e3 / steps,
                    "projection_avg_us": round(pr_avg * 1e3, 3),
                    "projection_gbps": round(pbytes / (pr_avg * 1e-3) / 1e9, 1) if pr_avg > 0 else None}
                log(f"[bench] projected {name} form={form}: {nrows * steps / el:.4e} desc/s, "
                    f"projection {pr_avg * 1e3:.2f} us")
        if batch:
            fv.set_tuning(hb)
        hp.free()

    # Dense-SIFT front end: synthetic 320x240 grayscale frames, the 8 scales sqrt 2 .. 1/8, bin
    # 4, stride 4 (the paper's setting); descriptors alone (HBM-bound: the image in, 520 bytes
    # per 130-value row out), and image -> Fisher vector (dense SIFT, projection 130 -> 64,
    # batched encode), for one frame and a batch of 64
    dsift = {}
    if not a.no_dsift:
        Hi, Wi, nimg = 240, 320, 64
        imgs = torch.from_numpy(fvsynth.images(nimg, Hi, Wi, 900)).to(dev)
        rows_per = fv.dsift_rows(Hi, Wi)
        rows_out = torch.empty(nimg, rows_per, fv.DSIFT_DIM, dtype=torch.float32, device=dev)
        pcd = fvsynth.pca(D, 0)
        hpd = fv.pca_load(pcd.A, pcd.mean)
        dsift = {"config": {"H": Hi, "W": Wi, "scales": 8, "bin": 4, "step": 4,
                            "rows_per_image": rows_per, "K": K, "D": D}, "runs": {}}
        for name, n in (("frame", 1), ("batch", nimg)):
            im, ro = imgs[:n], rows_out[:n]

            def dstep(im=im, ro=ro):
                fv.dsift(im, out=ro, flags=fv.ASYNC, stream=stream)
            steps = 200 if n == 1 else 20
            _, per, _ = time_steps(torch, dstep, steps, 5, stream)
            ms = float(np.median(per))
            gbytes = n * (4.0 * Hi * Wi + 4.0 * fv.DSIFT_DIM * rows_per)
            run = {"images": n, "dsift_ms": ms, "dsift_ms_per_image": ms / n,
                   "dsift_rows_per_s": n * rows_per / (ms * 1e-3),
                   "dsift_gbps": round(gbytes / (ms * 1e-3) / 1e9, 1), "encode_images": {}}
            for form in forms:
                outi = torch.empty(n, 2 * K * D, dtype=torch.float32, device=dev)

                def estep(im=im, outi=outi, prec=PREC_CODE[form]):
                    fv.encode_images(h, hpd, im, out=outi, precision=prec, flags=fv.ASYNC,
                                     stream=stream)
                _, per, _ = time_steps(torch, estep, steps, 5, stream)
                ems = float(np.median(per))
                run["encode_images"][form] = {"ms": ems, "ms_per_image": ems / n,
                                              "images_per_s": n / (ems * 1e-3)}
            dsift["runs"][name] = run
            log(f"[bench] dense SIFT {name} ({n} x {Wi}x{Hi}): {ms / n:.4f} ms/image, "
                f"{run['dsift_gbps']} GB/s; image->FV " +
                ", ".join(f"{f} {v['ms_per_image']:.4f} ms/image"
                          for f, v in run["encode_images"].items()))
        hpd.free()

    # EM training step on the batch's descriptors as one training set (the encoder's first
    # pass and statistics pass, then the M-step and log-likelihood reductions)
    em = {}
    if not a.no_em and batch:
        for form in forms:
            Xbd_ = Xbd
            for _ in range(2):
                fv.em_step(hb, Xbd_, precision=PREC_CODE[form], var_floor=1e-3, stream=stream)
            steps = max(3, a.batch_steps // 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fv.em_step(hb, Xbd_, precision=PREC_CODE[form], var_floor=1e-3, stream=stream)
            el = time.perf_counter() - t0
            nb = int(Xbd_.shape[0])
            em[form] = {"value": nb * steps / el, "ms_per_step": el * 1e3 / steps,
                        "descriptors": nb}
            log(f"[bench] em step form={form}: {nb * steps / el:.4e} desc/s, "
                f"{el * 1e3 / steps:.3f} ms/step")

    serving = []
    if a.serving_seconds > 0:
        for budget in (2 << 30, 64 << 20):
            log(f"[bench] serving budget={budget >> 20} MiB for {a.serving_seconds} s")
            r = run_serving(fv, a.serving_seconds, 1.0, budget)
            log(f"[bench]   p50 {r['latency_ms_from_arrival']['p50']:.3f} ms, p99 "
                f"{r['latency_ms_from_arrival']['p99']:.3f} ms, {r['throughput_desc_per_s']:.3e} desc/s")
            serving.append(r)
    sweep = []
    mults = [float(x) for x in a.sweep.split(",") if x] if a.serving_seconds > 0 else []
    for dev_in, mult in [(d, m) for d in (False, True) for m in mults]:
        log(f"[bench] serving sweep x{mult:g} ({'device' if dev_in else 'host'} input, "
            f"budget 2048 MiB, 2 s)")
        r = run_serving(fv, 2.0, 0.5, 2 << 30, rate_mult=mult, device_input=dev_in)
        sweep.append({k: r[k] for k in ("rate_hz_per_stream", "offered_desc_per_s",
                                         "throughput_desc_per_s", "latency_ms_from_arrival",
                                         "mean_frames_per_launch", "gpu_busy_fraction",
                                         "frames", "failed", "not_submitted", "input")})
        p99 = r["latency_ms_from_arrival"]["p99"]
        log(f"[bench]   offered {r['offered_desc_per_s']:.3e}, served {r['throughput_desc_per_s']:.3e} "
            f"desc/s, p99 {p99 if p99 is None else round(p99, 2)} ms, "
            f"frames/launch {r['mean_frames_per_launch']}, not submitted {r['not_submitted']}")

    c5 = {}
    if not a.no_frame:
        c5 = c5_capacity(fv, torch, dev, stream, forms, a.batch_steps)

    if a.calib_copy_mb > 0:
        n = a.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {a.calib_copy_mb} MiB done")

    prim = forms[0]
    res = batch[prim]
    result = {
        "metric": METRIC, "value": res["value"], "unit": "descriptors/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prim],
        "data": "synthetic (seeded GMM-sampled descriptors, 5% uniform outliers per frame)",
        "config": {"workload": "c4_batch64_k256_d64", "K": K, "D": D, "frames": B,
                   "descriptors": nb, "precision": prim, "path": res["tuned"]["path"],
                   "chunk": res["tuned"]["chunk"]},
        "roofline": res["roofline"], "step_ms": res["step_ms"],
        "gmm_load_ms": round(gmm_load_ms, 3),
        "forms": {f: r for f, r in batch.items() if f != "config"},
        "timing": "HIP events on the launch stream before the first and after every step "
                  "(graph replays of fv_encode_batch); value = descriptors x steps / event time; "
                  "roofline from the statistics kernel's event-timed launches",
    }
    if results:
        result["frame"] = {"config": {"workload": "c2_frame_k256_d64_n8000", "frames": 1,
                                      "descriptors": N, "path": path},
                           "forms": results}
    if serving:
        result["serving"] = serving
    if sweep:
        result["serving_sweep"] = sweep
    if c5:
        result["c5_capacity_device_input"] = c5
    if em:
        result["em_step"] = {
            "forms": em,
            "note": "one EM iteration (host-returned model and log-likelihood) over all rows of "
                    "the 64-frame batch as one training set, K = 256, D = 64"}
    if dsift:
        dsift["note"] = ("synthetic frames (fvsynth.images); dsift_gbps = (image bytes + 520 "
                         "bytes per descriptor row) / median time; encode_images = dense SIFT, "
                         "projection 130 -> 64 and the batched encode of each image's rows, one "
                         "vector per image (the paper: 34 ms per 320x240 frame for dense SIFT + "
                         "FV at K = 256, D = 82 on a K40)")
        result["dense_sift"] = dsift
    if projected:
        result["projected_din130"] = {
            "forms": projected,
            "note": "raw 130-value descriptors (128 stand-in SIFT + 2 coordinates) projected to "
                    "D = 64 by y = A (x - m) on the GPU, then encoded; the same GMM and frames"}
    if paper:
        result["paper_threshold_mode"] = {
            "tau": fv.THRESHOLD_TAU, "forms": paper,
            "note": "terms with posterior <= tau left out; MFMA steps with no term above tau "
                    "skipped; *_clustered = the same descriptors, each frame's rows grouped by "
                    "generating component"}
    if not a.no_cpu_baseline:
        import oracle
        from oracle.metrics import errors, per_block
        # the oracle on the whole batch, all host threads: the reference for every frame of the
        # timed outputs, and the first sample of the CPU baseline
        cb, refb = cpu_baseline_batch(g, Xb, offb, a.cpu_seconds)
        result["cpu_baseline"] = cb
        for f in forms:
            per = [errors(batch_out[f][b], refb[b]) for b in range(B)]
            worst = int(np.argmax([e["e_inf"] for e in per]))
            result["forms"][f]["error_vs_oracle"] = {
                "e_inf_max": max(e["e_inf"] for e in per), "e_2_max": max(e["e_2"] for e in per),
                "e_1_max": max(e["e_1"] for e in per),
                "e_inf_median": float(np.median([e["e_inf"] for e in per])),
                "frames": B, "worst_frame": worst,
                "per_frame_e_inf": [float(f"{e['e_inf']:.3e}") for e in per]}
            result["forms"][f]["error_per_block_worst_frame"] = per_block(
                batch_out[f][worst], refb[worst], K, D, worst=10)
        result["oracle_c1"] = oracle_c1()
        if results:
            ref = oracle.encode_gmm(X, g)
            for f in forms:
                results[f]["error_vs_oracle"] = errors(outputs[f], ref)
                results[f]["error_per_block"] = per_block(outputs[f], ref, K, D, worst=10)
        if paper:
            ref_t = oracle.encode_gmm(X, g, tau=fv.THRESHOLD_TAU)
            ref_tc = oracle.encode_gmm(Xc, g, tau=fv.THRESHOLD_TAU)
            for f in forms:
                paper[f]["frame"]["error_vs_oracle"] = errors(paper_out[(f, "frame")], ref_t)
                paper[f]["frame_clustered"]["error_vs_oracle"] = errors(
                    paper_out[(f, "frame_clustered")], ref_tc)
    print(json.dumps(result), flush=True)


def reap_children():
    """Nothing this run started may outlive it: name any child process still running (on
    stderr), then end it by its pid."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    for k in kids:
        try:
            log(f"child process still running at exit: pid {k.pid} {' '.join(k.cmdline())[:120]}")
            k.terminate()
        except psutil.Error:
            pass
    psutil.wait_procs(kids, timeout=5)


if __name__ == "__main__":
    try:
        main()
    finally:
        reap_children()
