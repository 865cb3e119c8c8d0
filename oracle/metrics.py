"""Error measures between a candidate Fisher vector g and the FP64 oracle o (test infra).

With s(y) = y*|y|, a unit-L2 vector o satisfies s(o) = phi/||phi||_1 exactly, so comparing
in the s-domain undoes the infinite slope of the signed square root at zero.

* e_inf  = max_i |s(g_i) - s(o_i)| / max_j |s(o_j)|      (per entry, relative to the largest)
* e_2    = ||g - o||_2                                     (normwise on the final vector)
* e_1    = max_i |s(g_i) - s(o_i)| / max(|s(o_i)|, 1/L)   (strict per entry, floor 1/L; L=2KD)
For vectors produced without the L2 step the caller passes normalise=True to compare
directions (both scaled to unit norm first).
"""
from __future__ import annotations

import numpy as np


def _s(y):
    return y * np.abs(y)


def errors(g, o, normalise: bool = False) -> dict:
    g = np.asarray(g, dtype=np.float64).ravel()
    o = np.asarray(o, dtype=np.float64).ravel()
    if g.shape != o.shape:
        raise ValueError("shape mismatch")
    if normalise:
        ng, no = np.linalg.norm(g), np.linalg.norm(o)
        g = g / ng if ng > 0 else g
        o = o / no if no > 0 else o
    L = o.size
    so, sg = _s(o), _s(g)
    diff = np.abs(sg - so)
    top = np.max(np.abs(so)) if L else 0.0
    e_inf = float(np.max(diff) / top) if top > 0 else float(np.max(diff) if L else 0.0)
    e_2 = float(np.linalg.norm(g - o))
    floor = np.maximum(np.abs(so), 1.0 / max(L, 1))
    e_1 = float(np.max(diff / floor)) if L else 0.0
    return {"e_inf": e_inf, "e_2": e_2, "e_1": e_1}


def raw_errors(g, o) -> dict:
    """Plain relative measures for un-normalised vectors: max|g-o|/max|o| and ||g-o||/||o||."""
    g = np.asarray(g, dtype=np.float64).ravel()
    o = np.asarray(o, dtype=np.float64).ravel()
    top = np.max(np.abs(o)) if o.size else 0.0
    no = np.linalg.norm(o)
    return {"rel_inf": float(np.max(np.abs(g - o)) / top) if top > 0 else float(np.max(np.abs(g - o), initial=0.0)),
            "rel_2": float(np.linalg.norm(g - o) / no) if no > 0 else float(np.linalg.norm(g - o))}


def per_block(g, o, K: int, D: int, worst: int = 10) -> dict:
    """Max s-domain error per (component, order) block, relative to the largest |s(o)|."""
    g = np.asarray(g, dtype=np.float64).reshape(2, K, D)
    o = np.asarray(o, dtype=np.float64).reshape(2, K, D)
    so, sg = _s(o), _s(g)
    top = np.max(np.abs(so))
    blk = np.max(np.abs(sg - so), axis=2) / (top if top > 0 else 1.0)   # [2, K]
    order = np.argsort(blk.ravel())[::-1][:worst]
    hist, edges = np.histogram(np.log10(np.maximum(blk.ravel(), 1e-30)), bins=np.arange(-30, 1))
    return {"max": float(blk.max()),
            "worst": [("u" if i // K == 0 else "v", int(i % K), float(blk.ravel()[i])) for i in order],
            "log10_hist": {int(e): int(c) for e, c in zip(edges[:-1], hist) if c}}
