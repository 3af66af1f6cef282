"""Autotuner of the convolution launch shapes.

Each pass (forward, input gradient, weight gradient) of each convolution of a
workload is timed in isolation on the GPU (``d2ip_time_conv``) for every valid
launch shape: voxel tile, output-channel tile, staged channel chunk and split
(split-K for passes 0/1, voxel splits for the weight gradient).  The fastest
shape per pass becomes an entry of the process-wide tuning table that later
plans use (``d2ip_set_tuning``).  Tables are plain JSON lists of entries.

    python -m paper_2507_14046_amd.autotune --workload c1 --out table.json
"""
import argparse
import ctypes
import json
import os
import sys

from . import _lib as L
from .context import _descs, _prec

FIELDS = ("n", "cin", "cout", "taps", "pass", "prologue", "precision")
SHAPE = ("tile", "bn", "ck", "split")


def _to_c(entries):
    arr = (L.TuningEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i] = L.TuningEntry(e["n"], e["cin"], e["cout"], e["taps"], e["pass"], e["prologue"],
                               e["precision"], L.ConvShape(*[e["shape"][k] for k in SHAPE]))
    return arr


def _from_c(t):
    return {"n": t.n, "cin": t.cin, "cout": t.cout, "taps": t.taps, "pass": t.pass_,
            "prologue": t.prologue, "precision": t.precision,
            "shape": {k: getattr(t.shape, k) for k in SHAPE}}


def set_tuning(entries):
    """Install `entries` (list of dicts) as the process-wide tuning table."""
    lib = L.load()
    L.check(lib.d2ip_set_tuning(_to_c(entries), len(entries)))


def plan_convs(geometries, instances, precision="fp32", graph=False, inst=0):
    """Conv passes of instance `inst` with the shapes the current plan picks."""
    lib = L.load()
    G, I = _descs(geometries, instances)
    cnt = ctypes.c_int()
    args = (G, len(geometries), I, len(instances), _prec(precision), L.FLAG_GRAPH if graph else 0,
            inst)
    L.check(lib.d2ip_plan_convs(*args, None, 0, ctypes.byref(cnt)))
    arr = (L.TuningEntry * max(1, cnt.value))()
    L.check(lib.d2ip_plan_convs(*args, arr, cnt.value, ctypes.byref(cnt)))
    return [_from_c(arr[i]) for i in range(cnt.value)]


def _key(e):
    return tuple(e[k] for k in FIELDS)


def candidates(e):
    """Every launch shape of the pass `e` the library accepts (host check)."""
    lib = L.load()
    out = []
    kin = e["cin"] if e["pass"] != 1 else e["cout"]
    for tile in (0, 1, 2):
        for ck in (8, 16, 32):
            if kin % ck:
                continue
            if e["pass"] == 2:
                for split in (1, 2, 4, 8, 16, 24, 32, 48, 64):
                    out.append(dict(tile=tile, bn=0, ck=ck, split=split))
            else:
                nch = kin // ck
                for bn in (16, 32, 64):
                    for split in range(1, nch + 1):
                        if nch % split == 0 and split <= 8:
                            out.append(dict(tile=tile, bn=bn, ck=ck, split=split))
    good = []
    for sh in out:
        t = _to_c([dict(e, shape=sh)])
        nb = ctypes.c_size_t()
        if lib.d2ip_time_conv_bytes(t, ctypes.byref(nb)) == L.OK:
            good.append(sh)
    return good


def time_pass(e, shape, reps=20, device=0):
    """Mean ms per launch of pass `e` with `shape` (standalone, zero operands)."""
    import torch
    lib = L.load()
    t = _to_c([dict(e, shape=shape)])
    nb = ctypes.c_size_t()
    L.check(lib.d2ip_time_conv_bytes(t, ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=torch.device("cuda", device))
    stream = torch.cuda.current_stream(ws.device)
    ms = ctypes.c_double()
    L.check(lib.d2ip_time_conv(t, ctypes.c_void_p(ws.data_ptr()), nb.value,
                               ctypes.c_void_p(stream.cuda_stream), reps, ctypes.byref(ms)))
    return ms.value


def tune(geometries, instances, precision="fp32", reps=20, log=None):
    """Tuning entries for every distinct conv pass of the workload."""
    seen = {}
    set_tuning([])  # time the heuristic's choice as the baseline
    for i in range(len(instances)):
        for e in plan_convs(geometries, instances, precision, inst=i):
            seen.setdefault(_key(e), e)
    table = []
    for key, e in seen.items():
        base = time_pass(e, e["shape"], reps)
        best, best_ms = e["shape"], base
        for sh in candidates(e):
            ms = time_pass(e, sh, reps)
            if ms < best_ms:
                best, best_ms = sh, ms
        if log:
            log("n=%-3d %3d->%-3d taps %2d pass %d pro %d: %.4f ms -> %.4f ms %s"
                % (e["n"], e["cin"], e["cout"], e["taps"], e["pass"], e["prologue"], base,
                   best_ms, best))
        table.append(dict(e, shape=best, ms=best_ms, heuristic_ms=base))
    return table


def save(table, path):
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def load_table(path):
    with open(path) as f:
        return [{k: v for k, v in e.items() if k in FIELDS or k == "shape"} for e in json.load(f)]


def workload(name):
    """(geometries, instances) of a named synthetic workload."""
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import tseit_synth as ts
    c = ts.CONFIGS[name]
    M = {1: 208, 2: 928}
    if "instances" in c:
        geos, insts = [], []
        for it in c["instances"]:
            g = (it["n"], M[it["rings"]])
            if g not in geos:
                geos.append(g)
            insts.append((geos.index(g), c["levels"], it["base_ch"]))
        return geos, insts
    return [(c["n"], M[c["rings"]])], [(0, c["levels"], c["base_ch"])]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    geos, insts = workload(a.workload)
    table = tune(geos, insts, a.precision, a.reps,
                 log=lambda m: print(m, file=sys.stderr, flush=True))
    save(table, a.out)


if __name__ == "__main__":
    main()
