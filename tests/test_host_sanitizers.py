"""Host code of the library under the sanitizers, on the CPU (no GPU needed).

tests/native/host_checks.cpp drives the C ABI's argument validation and the serving loop with
its host executor from several threads (submit, cancel, poll, wait, statistics, destroy with
work outstanding).  The two host-side translation units that hold that logic (fv_api.cpp,
fv_server.cpp) are compiled host-only with the sanitizer on their host code (the flags go to
the host compiler only, after -Xarch_host), and the checks link them ahead of libfv.so, which
supplies the kernel launchers (never called here).  Variants: AddressSanitizer +
UndefinedBehaviorSanitizer + LeakSanitizer, and ThreadSanitizer.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

import paper_1604_03498_amd as fv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_03498_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "native", "host_checks.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

VARIANTS = {
    "address_undefined": (["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"],
                          {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
    "thread": (["-Xarch_host", "-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
}


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in r.stderr.splitlines()
            if "packed-fp32-ops" not in ln and "unknown target feature" not in ln]
    assert r.returncode == 0, " ".join(cmd) + "\n" + "\n".join(msgs[-40:])


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_host_code_under_sanitizer(variant, tmp_path):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    lib = fv.lib_path()
    assert os.path.exists(lib), "build the library first (python -m paper_1604_03498_amd.build)"
    san, env_extra = VARIANTS[variant]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-Xarch_host", "-fno-omit-frame-pointer",
              "-I", INCLUDE, "-I", CSRC] + san
    jobs = []
    objs = []
    for src in ("fv_api.cpp", "fv_server.cpp"):
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        jobs.append([HIPCC, "-x", "hip", "--offload-host-only", "--offload-arch=gfx950",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + common +
                    ["-c", os.path.join(CSRC, src), "-o", obj])
    main_obj = str(tmp_path / "host_checks.o")
    jobs.append([HIPCC, "-x", "c++"] + common + ["-c", DRIVER, "-o", main_obj])
    with ThreadPoolExecutor(3) as ex:
        list(ex.map(_run, jobs))
    exe = str(tmp_path / "host_checks")
    _run([HIPCC] + san + [main_obj] + objs +
         [lib, "-Wl,-rpath," + os.path.dirname(lib), "-o", exe])
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "host checks passed" in r.stdout, (r.stdout + r.stderr)[-6000:]
