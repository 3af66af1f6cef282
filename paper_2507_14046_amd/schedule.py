"""The D2IP frame schedule on a fitting context (Sec. III-B, III-C, Eqs. (6)-(9)).

UPWS (Eqs. (6)-(7)): starting from the Kaiming parameters, the network is
fitted to one arbitrary single-frame task for N0 iterations; the resulting
parameters start the sequence.  TPP (Eqs. (8)-(9)): every later frame starts
from the previous frame's final parameters.  Between frames only the
measurement changes; Adam's moments and step count restart.  With the 4D-TV
term on, each finished frame's image joins the temporal history.

The paper's tsEIT schedule (Sec. IV-C): UPWS 1800 iterations, first frame 450,
later frames 250, learning rate 5e-4.  Its ablation (Sec. V, Fig. 8) compares
the runtime of D2IP without UPWS and/or TPP; `ablation` measures the same
comparison as iterations (and seconds) each variant needs to bring every
frame's loss down to the loss the full schedule reaches on that frame.

Host orchestration only: every iteration runs in the library's kernels.  The
functions drive instance `inst` of a context holding that one instance
(`Context.run` advances every instance of a context).
"""
import time

import numpy as np

PAPER_SCHEDULE = dict(upws=1800, first=450, later=250, lr=5e-4)


def _single(ctx):
    if len(ctx.instances) != 1:
        raise ValueError("the schedule drives a context holding one instance")


def warm_start(ctx, theta0, dv, iters, inst=0):
    """UPWS: theta0 fitted to the measurement dv for `iters` iterations.
    Returns the fitted parameters (host array)."""
    _single(ctx)
    ctx.set_params(inst, theta0)
    ctx.set_frame(inst, dv)
    ctx.reset_optimizer(inst)
    if iters > 0:
        ctx.run(iters)
    return ctx.get_params(inst)


def run_sequence(ctx, dvs, first_iters, later_iters, theta_start=None, tpp=True, tv=False,
                 inst=0):
    """Fit the frames `dvs` in order (first frame `first_iters` iterations,
    later frames `later_iters`).  With tpp every frame starts from the
    previous frame's parameters, else from the sequence's starting parameters
    (`theta_start`, or the instance's parameters at the call).  With tv every
    finished frame's image joins the 4D-TV history (cleared at the start).
    Returns (images [F, n^3], last reported loss per frame, seconds)."""
    _single(ctx)
    if theta_start is not None:
        ctx.set_params(inst, theta_start)
    start = ctx.get_params(inst)
    if tv:
        ctx.clear_history(inst)
    images, losses = [], []
    t0 = time.perf_counter()
    for f, dv in enumerate(dvs):
        if f > 0 and not tpp:
            ctx.set_params(inst, start)
        ctx.set_frame(inst, dv)
        ctx.reset_optimizer(inst)
        losses.append(float(ctx.run(first_iters if f == 0 else later_iters)[inst]))
        images.append(ctx.read_image(inst))
        if tv:
            ctx.commit_frame(inst)
    return np.stack(images), np.array(losses), time.perf_counter() - t0


def iterations_to_target(ctx, target, cap, chunk=10, inst=0):
    """Run the current frame until the reported loss (the loss at the
    parameters before the chunk's last update) is <= target, checking every
    `chunk` iterations, at most `cap` iterations.  Returns (iterations,
    last loss, reached)."""
    k, loss = 0, float("inf")
    while k < cap:
        n = min(chunk, cap - k)
        loss = float(ctx.run(n)[inst])
        k += n
        if loss <= target:
            return k, loss, True
    return k, loss, False


VARIANTS = (
    # name, starts from the UPWS parameters, propagates parameters across frames
    ("full", True, True),
    ("no_tpp", True, False),
    ("no_upws", False, True),
    ("no_upws_no_tpp", False, False),
)


def ablation(ctx, theta0, dvs, dv_warm, sched=PAPER_SCHEDULE, target_factor=1.05, cap_factor=8,
             chunk=10, inst=0):
    """Iterations and seconds that D2IP and its variants without UPWS and/or
    TPP need per frame to reach the target loss: `target_factor` x the loss
    the full schedule (UPWS, then first/later iterations with TPP) reports at
    the end of that frame.  A frame stops at `cap_factor` x its scheduled
    iterations if the target is not reached (reported as not reached).  The
    UPWS phase (fitting `dv_warm` from theta0) runs once; its iterations and
    seconds are reported apart, as the paper's warm start can be reused
    across tasks."""
    _single(ctx)
    ctx.set_adam(lr=sched["lr"])
    t0 = time.perf_counter()
    theta_w = warm_start(ctx, theta0, dv_warm, sched["upws"], inst)
    t_upws = time.perf_counter() - t0
    _, final, t_sched = run_sequence(ctx, dvs, sched["first"], sched["later"], theta_w, True,
                                     inst=inst)
    targets = target_factor * final
    out = dict(schedule=dict(sched), frames=len(dvs), target_factor=target_factor,
               cap_factor=cap_factor, chunk=chunk,
               upws=dict(iterations=sched["upws"], seconds=t_upws),
               scheduled_full=dict(iterations=sched["first"] + (len(dvs) - 1) * sched["later"],
                                   seconds=t_sched, final_losses=final.tolist()),
               variants={})
    for name, upws, tpp in VARIANTS:
        start = theta_w if upws else theta0
        ctx.set_params(inst, start)
        iters, reached = [], []
        t0 = time.perf_counter()
        for f, dv in enumerate(dvs):
            if f > 0 and not tpp:
                ctx.set_params(inst, start)
            ctx.set_frame(inst, dv)
            ctx.reset_optimizer(inst)
            cap = cap_factor * (sched["first"] if f == 0 else sched["later"])
            k, _, ok = iterations_to_target(ctx, targets[f], cap, chunk, inst)
            iters.append(k)
            reached.append(ok)
        secs = time.perf_counter() - t0
        out["variants"][name] = dict(uses_upws=upws, uses_tpp=tpp, iterations=iters,
                                     total_iterations=int(sum(iters)), seconds=secs,
                                     all_reached=bool(all(reached)),
                                     frames_reached=int(sum(reached)))
    base = out["variants"]["full"]
    for v in out["variants"].values():
        v["iterations_vs_full"] = v["total_iterations"] / max(1, base["total_iterations"])
        v["seconds_vs_full"] = v["seconds"] / base["seconds"]
    return out


def main():
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch  # noqa: F401  (HIP runtime before the library)
    import tseit_synth as ts
    from . import Context
    from . import autotune as at
    ap = argparse.ArgumentParser(description="D2IP schedule ablation on a synthetic sequence")
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--frames", type=int, default=20)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--seed", type=int, default=1)
    a = ap.parse_args()
    path = at.default_table_path()
    if os.path.exists(path):
        at.set_tuning(at.load_table(path))
    c = ts.CONFIGS["c1"]
    p = ts.make_problem(a.n, c["rings"], c["levels"], c["base_ch"], a.seed, frames=a.frames,
                        breathing=True)
    warm = ts.make_problem(a.n, c["rings"], c["levels"], c["base_ch"], a.seed + 1000)
    ctx = Context([(a.n, p["J"].shape[0])], [(0, c["levels"], c["base_ch"])],
                  precision=a.precision, graph=False)
    ctx.load_problem(0, p)
    res = ablation(ctx, p["theta0"], p["dv"], warm["dv"][0])
    ctx.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
