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


def oracle_gradient_floor(p):
    """The oracle's one-iteration gradient from theta_0 moved by one FP32 ulp
    per entry (random direction): how far FP32 rounding of theta_0 alone moves
    the gradient being compared (its sensitivity floor)."""
    from tests.golden.make_golden import ulp_perturb
    pr = oracle_problem(p)
    _, g, _ = pr.loss_and_grad(ulp_perturb(p["theta0"]).astype(np.float64),
                               p["dv"][0].astype(np.float64))
    return g


def oracle_kink_variants(p, rel_tau=1e-6, max_kinks=3, theta=None, dv=None):
    """Oracle one-iteration gradients with the ReLU decisions whose
    pre-activation lies within rel_tau of its tensor's median magnitude taken
    the other way, every non-empty combination of them (none if there are more
    than max_kinks).  Such a decision rests on the last bits of the
    pre-activation, which FP32 arithmetic can put on either side of the kink;
    the derivative there is 0 or 1 and the two gradients differ by whole
    terms.  A flipped decision moves the forward value by at most rel_tau of
    the scale."""
    from oracle import net
    pr = oracle_problem(p)
    th = np.asarray(p["theta0"] if theta is None else theta, dtype=np.float64)
    dv = np.asarray(p["dv"][0] if dv is None else dv, dtype=np.float64)
    orig = net.relu
    calls = []

    def spy(x):
        a = np.abs(x).ravel()
        calls.append(np.flatnonzero(a < rel_tau * np.median(a)))
        return orig(x)
    try:
        net.relu = spy
        pr.loss_and_grad(th, dv)
        kinks = [(ci, int(j)) for ci, idx in enumerate(calls) for j in idx]
        if not kinks or len(kinks) > max_kinks:
            return []
        out = []
        for sel in range(1, 2 ** len(kinks)):
            flips = [kinks[b] for b in range(len(kinks)) if (sel >> b) & 1]
            count = [0]

            def flipped(x, flips=flips, count=count):
                ci = count[0]
                count[0] += 1
                y = orig(x).copy()
                yf, xf = y.reshape(-1), x.reshape(-1)
                for c, j in flips:
                    if c == ci:  # taken inactive, or active with a value below any scale
                        yf[j] = 0.0 if xf[j] > 0 else 1e-300
                return y
            net.relu = flipped
            out.append(pr.loss_and_grad(th, dv)[1])
        return out
    finally:
        net.relu = orig


def _grad_bounds(g, gref, levels, C, tol, tol_tensor, tol_elem):
    per = per_tensor_rel(g, gref, levels, C)
    pel = per_tensor_elementwise(g, gref, levels, C, tol_elem)
    out = dict(grad_rel=rel(g, gref), worst_tensor=max(per.items(), key=lambda kv: kv[1]),
               worst_elementwise=max(pel.items(), key=lambda kv: kv[1]))
    ok = (out["grad_rel"] < tol and out["worst_tensor"][1] < tol_tensor and
          out["worst_elementwise"][1] <= 1.0)
    return ok, out, per, pel


def check_gradient(g, gref, levels, C, tol, tol_tensor, tol_elem, floor_fn=None, kink_fn=None):
    """Relative L2 of the whole gradient within `tol`, of every tensor within
    `tol_tensor`, and every value within `tol_elem` of its tensor's scale.
    Where that fails: the same bounds against any oracle gradient with the
    ReLU decisions taken within FP32 resolution of the kink the other way
    (`kink_fn`), or, where `floor_fn` gives the oracle's gradient from a 1-ulp
    perturbed theta_0, within 3x that floor (the gradient is no better
    conditioned than that).  Returns the numbers, with "ok"."""
    ok, out, per, pel = _grad_bounds(g, gref, levels, C, tol, tol_tensor, tol_elem)
    out["floor"] = None
    out["kink_alternative"] = None
    if ok:
        out["ok"] = True
        return out
    if kink_fn is not None:
        alts = kink_fn()
        out["kink_alternatives"] = len(alts)
        for k, ga in enumerate(alts):
            ok_k, out_k, _, _ = _grad_bounds(g, ga, levels, C, tol, tol_tensor, tol_elem)
            if ok_k:
                out["kink_alternative"] = dict(index=k, **out_k)
                out["ok"] = True
                return out
    if floor_fn is None:
        out["ok"] = False
        return out
    gf = floor_fn()
    fper = per_tensor_rel(gf, gref, levels, C)
    fpel = per_tensor_elementwise(gf, gref, levels, C, tol_elem)
    out["floor"] = rel(gf, gref)
    out["floor_worst_tensor"] = max(fper.items(), key=lambda kv: kv[1])
    ok = out["grad_rel"] < max(tol, 3 * out["floor"])
    ok = ok and all(per[k] < max(tol_tensor, 3 * fper[k]) for k in per)
    ok = ok and all(pel[k] <= max(1.0, 3 * fpel[k]) for k in pel)
    out["ok"] = ok
    return out


def shadow_sequence(lib, p, iters, lr, tol=1e-5):
    """Run one sequence (frames of iters[f] iterations, TPP, Adam restarted per
    frame) on the GPU one iteration at a time beside the FP64 oracle, whose
    Adam step at each iteration takes the oracle gradient or, where the GPU's
    gradient matches it better, the oracle gradient with the ReLU decisions
    within FP32 resolution of a kink taken the other way.

    Returns dict(gpu=[image per frame], ref=[shadowed oracle image per frame],
    flips=[iterations at which a flipped decision was taken],
    departure=first iteration whose GPU gradient is farther than `tol` from
    every such oracle gradient (None if none), entry=[relative distance of the
    GPU's image from the oracle's at the start of each iteration],
    grad=[relative gradient distance per iteration]).  From the departure on
    the two trajectories are no longer the same one: the network is piecewise
    linear, its gradient jumps where a pre-activation crosses zero, and Adam
    turns such a difference into whole +-lr steps."""
    from oracle import fit
    pr = oracle_problem(p)
    ctx = make_ctx(lib, [p])
    ctx.set_adam(lr=lr)
    st = fit.State(p["theta0"])
    out = dict(gpu=[], ref=[], flips=[], departure=None, entry=[], grad=[])
    it = 0
    try:
        for f, k in enumerate(iters):
            dv = np.asarray(p["dv"][f], dtype=np.float64)
            if f > 0:
                ctx.set_frame(0, p["dv"][f])
                ctx.reset_optimizer(0)
                st.reset_optimizer()
            for _ in range(k):
                it += 1
                out["entry"].append(rel(ctx.read_image(0), pr.image(st.theta)))
                ctx.run(1)
                gg = ctx.get_grad(0)
                _, g, _ = pr.loss_and_grad(st.theta, dv)
                if rel(gg, g) > tol:
                    alts = oracle_kink_variants(p, theta=st.theta, dv=dv)
                    if alts:
                        best = min(alts, key=lambda a: rel(gg, a))
                        if rel(gg, best) < rel(gg, g):
                            g = best
                            out["flips"].append(it)
                out["grad"].append(rel(gg, g))
                if out["grad"][-1] > tol and out["departure"] is None:
                    out["departure"] = it
                st.theta, st.m, st.v, st.t = fit.adam_step(st.theta, g, st.m, st.v, st.t, lr)
            out["gpu"].append(ctx.read_image(0))
            out["ref"].append(pr.image(st.theta))
    finally:
        ctx.close()
    return out
