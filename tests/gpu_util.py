"""Helpers shared by the GPU tests: problem set-up, the oracle side, metrics."""
import json
import os
import time

import numpy as np

import tseit_synth as ts
from oracle import fit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
METRICS = os.environ.get("D2IP_METRICS", os.path.join(ROOT, "gpurun_out", "parity_metrics.jsonl"))


def record(name, **kw):
    """Append measured numbers of a GPU test to the metrics file (if its folder exists)."""
    kw["test"] = name
    kw["time"] = time.time()
    d = os.path.dirname(METRICS)
    if os.path.isdir(d):
        with open(METRICS, "a") as f:
            f.write(json.dumps(kw, default=float) + "\n")
    print("[metrics]", json.dumps(kw, default=float), flush=True)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(n, rings, levels, C, seed, frames=1, breathing=False):
    return ts.make_problem(n, rings, levels, C, seed, frames=frames, breathing=breathing)


def oracle_problem(p):
    return fit.Problem(p["J"], p["mask"], p["Z"], p["n"], p["levels"], p["base_ch"])


def make_ctx(lib, probs, precision="fp32", graph=False, shared_geometry=False):
    """One context over a list of problem dicts (one instance each)."""
    geos, insts = [], []
    for i, p in enumerate(probs):
        if shared_geometry and i > 0:
            insts.append((0, p["levels"], p["base_ch"]))
            continue
        geos.append((p["n"], p["J"].shape[0]))
        insts.append((len(geos) - 1, p["levels"], p["base_ch"]))
    ctx = lib.Context(geos, insts, precision=precision, graph=graph)
    done = set()
    for i, p in enumerate(probs):
        g = insts[i][0]
        ctx.load_problem(i, p, set_geometry=g not in done)
        done.add(g)
    return ctx


def per_tensor_rel(g_gpu, g_ref, levels, C):
    out = {}
    off = 0
    for name, shape, _ in ts.param_specs(levels, C):
        k = int(np.prod(shape))
        out[name] = rel(g_gpu[off:off + k], g_ref[off:off + k])
        off += k
    return out


def elementwise(a, ref, tol):
    """max over elements of |a - ref| / (tol * (max|ref| + |ref|)): at most 1
    when every element lies within tol of the array's scale and of its own
    magnitude (so an error confined to a few voxels, taps or channels shows
    even when the relative L2 over the whole array stays small)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = tol * (np.max(np.abs(ref)) + np.abs(ref))
    return float(np.max(np.abs(a - ref) / np.maximum(scale, 1e-300)))


def per_tensor_elementwise(g_gpu, g_ref, levels, C, tol):
    out = {}
    off = 0
    for name, shape, _ in ts.param_specs(levels, C):
        k = int(np.prod(shape))
        out[name] = elementwise(g_gpu[off:off + k], g_ref[off:off + k], tol)
        off += k
    return out
