"""Write oracle trajectories used as stored expected values by the GPU tests.

Calls only the FP64 oracle and the seeded input generator.  For a problem it
stores the recorded losses, the image at checkpoint iterations, and the
SHA-256 of the FP32 inputs so a test can detect a generator drift on another
machine.  With --floor it also runs the oracle from theta_0 moved by one FP32
ulp per entry (random direction) and stores those images: the distance
between the two trajectories is the sensitivity floor that FP32 rounding
alone can cause.

    python tests/golden/make_golden.py c1 --iters 500 --floor
    python tests/golden/make_golden.py c2 --iters 50 --floor --grad
    python tests/golden/make_golden.py c3 --floor

c3 writes the eight breathing sequences of the 32^3 time-sequence workload
on a shortened TPP schedule (4 iterations for frame 0, then 3 per frame for
frames 1 and 2, Adam restarted per frame): each frame's image, FP32-rounded;
with --floor also the run from theta_0 moved by one FP32 ulp.

With --grad it also stores the loss and the theta-gradient of the first
iteration (at theta_0), the gradient rounded once to FP32 to keep the file
small (a relative change of at most 2^-24 per entry).  --shrink PATH rewrites
a stored file with its images rounded once to FP32 and without the stored
gradient (for files that would otherwise be tens of MB; a test can compute
the first gradient itself).
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tseit_synth as ts  # noqa: E402
from oracle import fit  # noqa: E402


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def ulp_perturb(theta, seed=12345):
    r = np.random.default_rng(seed)
    to = np.where(r.random(theta.size) < 0.5, np.inf, -np.inf).astype(np.float32)
    return np.nextafter(theta.astype(np.float32), to).astype(np.float32)


def trajectory(pr, theta0, dv, iters, lr, checkpoints, log=None):
    st = fit.State(theta0)
    losses, images = [], {}
    done = 0
    t0 = time.time()
    for c in sorted(checkpoints):
        losses += fit.run(pr, st, dv, c - done, lr)
        done = c
        images[c] = pr.image(st.theta)
        if log:
            log("iter %d loss %.6e  (%.0f s)" % (c, losses[-1], time.time() - t0))
    return np.array(losses), images


C3_ITERS = [4, 3, 3]


def sequences_c3(log, floor=False, out=None):
    """The eight sequences from theta_0, or (floor) from theta_0 moved by one
    FP32 ulp per entry, added to `out` as floor_images."""
    cfg = ts.CONFIGS["c3"]
    if out is None:
        out = dict(config="c3", iters=np.array(C3_ITERS), lr=cfg["lr"],
                   seeds=np.array(cfg["seeds"]))
    imgs, losses = [], []
    for seed in cfg["seeds"]:
        p = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], seed,
                            frames=len(C3_ITERS), breathing=True)
        pr = fit.Problem(p["J"], p["mask"], p["Z"], cfg["n"], cfg["levels"], cfg["base_ch"])
        th0 = ulp_perturb(p["theta0"]) if floor else p["theta0"]
        im, ls, _ = fit.fit_sequence(pr, th0, p["dv"], C3_ITERS, cfg["lr"])
        imgs.append(im.astype(np.float32))
        losses.append(np.concatenate([np.asarray(l) for l in ls]))
        out["sha_theta0_%d" % seed] = sha(p["theta0"])
        log("sequence %d%s: final loss %.6e" % (seed, " (floor)" if floor else "", losses[-1][-1]))
    key = "floor_" if floor else ""
    out[key + "images"] = np.stack(imgs)      # [sequence][frame][voxel]
    out[key + "losses"] = np.stack(losses)    # [sequence][iteration]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["c0", "c1", "c2", "c3"], nargs="?", default="c1")
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--floor", action="store_true")
    ap.add_argument("--grad", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--shrink", default=None)
    a = ap.parse_args()

    def log(m):
        print(m, flush=True)

    if a.shrink:
        z = dict(np.load(a.shrink))
        z.pop("grad1", None)
        for k in ("images", "floor_images"):
            if k in z:
                z[k] = z[k].astype(np.float32)
        np.savez_compressed(a.shrink, **z)
        log("shrunk " + a.shrink)
        return

    if a.config == "c3":
        path = a.out or os.path.join(HERE, "oracle_c3_tpp.npz")
        if a.floor and os.path.exists(path):  # add the floor run to the stored file
            out = sequences_c3(log, floor=True, out=dict(np.load(path)))
        else:
            out = sequences_c3(log)
            if a.floor:
                sequences_c3(log, floor=True, out=out)
        np.savez_compressed(path, **out)
        log("wrote " + path)
        return
    cfg = ts.CONFIGS[a.config]
    iters = a.iters or cfg["iters"]
    cps = sorted({c for c in (1, 5, 10, 20, 50, 100, 200, 300, 500, 1000) if c <= iters} | {iters})
    p = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], cfg["seed"])
    pr = fit.Problem(p["J"], p["mask"], p["Z"], cfg["n"], cfg["levels"], cfg["base_ch"])

    out = dict(config=a.config, iters=iters, lr=cfg["lr"], checkpoints=np.array(cps),
               sha_J=sha(p["J"]), sha_Z=sha(p["Z"]), sha_theta0=sha(p["theta0"]),
               sha_dv=sha(p["dv"]))
    if a.grad:
        L1, g1, _ = pr.loss_and_grad(np.asarray(p["theta0"], dtype=np.float64),
                                     np.asarray(p["dv"][0], dtype=np.float64))
        out["loss1"] = L1
        out["grad1"] = g1.astype(np.float32)
        log("iteration 1 gradient stored (loss %.6e)" % L1)
    losses, imgs = trajectory(pr, p["theta0"], p["dv"][0], iters, cfg["lr"], cps, log)
    out["losses"] = losses
    out["images"] = np.stack([imgs[c] for c in cps])
    if a.floor:
        fl, fimgs = trajectory(pr, ulp_perturb(p["theta0"]), p["dv"][0], iters, cfg["lr"], cps, log)
        out["floor_losses"] = fl
        out["floor_images"] = np.stack([fimgs[c] for c in cps])
    path = a.out or os.path.join(HERE, "oracle_%s_%d.npz" % (a.config, iters))
    np.savez_compressed(path, **out)
    log("wrote " + path)


if __name__ == "__main__":
    main()
