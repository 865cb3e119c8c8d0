"""bench.py on the CPU: the multi-GPU refusal, and the committed HBM counter summary covering
every statistics kernel the roofline looks up (a renamed kernel would otherwise turn
`roofline.traffic` into null without any error)."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_summary_covers_every_stats_kernel():
    b = _bench()
    with open(b.TRAFFIC_JSON) as f:
        t = json.load(f)
    if t.get("source_sha256") != b.kernel_source_hash():
        pytest.skip("counter summary taken on other kernel sources (bench reports traffic null)")
    missing = sorted({n for names in b.STATS_KERNELS.values() for n in names} - set(t["kernels"]))
    assert not missing, f"kernels without HBM counters: {missing}"
    for (form, path) in b.STATS_KERNELS:
        tr = b.load_traffic(form, path, 1)
        assert tr is not None and tr["bytes"] > 0, (form, path)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
