"""Writes synth_manifest.json: SHA-256 of the float32 bytes of each named synthetic input.
Run from the repository root: python tests/golden/make_synth_manifest.py
Only the seeded generators are called (no encoder is involved)."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import fvsynth  # noqa: E402


def manifest():
    out = {}
    for name in ("c1_oracle_k64_d64_n2000", "c2_frame_k256_d64_n8000"):
        g, X, off = fvsynth.workload(name)
        out[name] = {"weights": fvsynth.array_sha256(g.weights), "means": fvsynth.array_sha256(g.means),
                     "variances": fvsynth.array_sha256(g.variances), "X": fvsynth.array_sha256(X),
                     "shape": list(X.shape)}
    sizes = fvsynth.batch_sizes(64, 1)
    out["c4_batch64_sizes"] = {"sizes": [int(v) for v in sizes], "total": int(sizes.sum())}
    g5 = fvsynth.gmm(512, 80, 0)
    out["c5_gmm_k512_d80"] = {"means": fvsynth.array_sha256(g5.means)}
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_manifest.json")
    with open(path, "w") as f:
        json.dump(manifest(), f, indent=1, sort_keys=True)
    print("wrote", path)
