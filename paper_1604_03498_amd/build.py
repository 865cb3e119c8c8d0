"""Build libfv.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_1604_03498_amd.build

Every HIP source is compiled with packed-FP32 instruction selection disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops), for gfx950 only.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfv.so")

SOURCES = ["fv_api.cpp", "fv_server.cpp", "fv_kernels.hip", "fv_split.hip", "fv_finalize.hip",
           "fv_dsift.hip", "fv_dsift_host.cpp", "fv_noalloc.hip",
           "fv_form_bf16s.hip", "fv_form_f16s.hip", "fv_form_bf16.hip", "fv_project.hip",
           "fv_em.hip"]
# Statistics kernels built without NaN-preserving max semantics: every fmaxf of an MFMA or
# lane-exchange result otherwise gets a canonicalising v_max per input (about 60 extra VALU per
# 32-row wave-tile in the row maxima).  A NaN descriptor still makes its frame's statistics
# NaN (it reaches every sum through exp2); the finalize, whose signed square root maps NaN to 0
# by comparisons, keeps IEEE semantics.
NO_NAN_SOURCES = {"fv_kernels.hip", "fv_split.hip", "fv_form_bf16s.hip", "fv_form_f16s.hip",
                  "fv_form_bf16.hip"}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def hipcc_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-command-line-argument",
            "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False, out: str = LIB) -> str:
    with tempfile.TemporaryDirectory(prefix="fvbuild_") as td:
        objs = [os.path.join(td, src + ".o") for src in SOURCES]
        cmds = [[HIPCC] + hipcc_flags() + (["-fno-honor-nans"] if src in NO_NAN_SOURCES else []) +
                ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
                for src, obj in zip(SOURCES, objs)]
        procs = []
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        for src, p in zip(SOURCES, procs):
            _, err = p.communicate()
            msgs = [ln for ln in (err or "").splitlines()
                    if "packed-fp32-ops" not in ln and "unknown target feature" not in ln]
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + "\n".join(msgs))
            if verbose and msgs:
                print("\n".join(msgs))
        tmp_lib = os.path.join(td, "libfv.so")
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp_lib]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stderr)
        shutil.copyfile(tmp_lib, out + ".tmp")
        os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    # python -m paper_1604_03498_amd.build [-v] [--out PATH]  (default: in-tree libfv.so)
    args = sys.argv[1:]
    dest = args[args.index("--out") + 1] if "--out" in args else LIB
    print(build(verbose="-v" in args, out=dest))
