"""Autotuner of the convolution launch shapes.

Each pass (forward, input gradient, weight gradient) of each convolution of a
workload is timed in isolation on the GPU (``d2ip_time_conv``) for every valid
launch shape: voxel tile, output-channel tile, staged channel chunk and split
(split-K for passes 0/1, voxel splits for the weight gradient).  A weight
gradient's cost also counts the reading of its per-split partials by the
batched reduction that follows (``reduce_ms``).  The cheapest shape per pass
becomes an entry of the process-wide tuning table that later plans use
(``d2ip_set_tuning``).  Tables are plain JSON lists of entries.

    python -m paper_2507_14046_amd.autotune --out paper_2507_14046_amd/tuned_mi355x.json
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
                for split in (1, 2, 4, 8, 16, 24, 32, 48, 64, 96, 128, 192, 256):
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


# rate at which partial bytes are charged to a weight gradient (bytes per ms).
# The batched reduction reads them at about 3.9 TB/s on MI355X (83 MB in
# 21.5 us), but it runs on the critical path after both streams join, while the
# weight gradients overlap the input-gradient chain; charging 2.5 TB/s weights
# the exposed reduction above the overlapped launch.
REDUCE_BYTES_PER_MS = 2.5e9


def reduce_ms(e, shape):
    """Time the batched reduction spends on the partials of pass `e` (0 for
    passes 0/1): splits x (weights + bias) FP32 partials per output tile."""
    if e["pass"] != 2:
        return 0.0
    cout16 = (e["cout"] + 15) // 16 * 16
    return shape["split"] * cout16 * (e["taps"] * e["cin"] + 1) * 4 / REDUCE_BYTES_PER_MS


def tune(geometries, instances, precision="fp32", reps=10, log=None, margin=0.97, passes=(0, 1, 2)):
    """Tuning entries for every distinct conv pass (of the listed `passes`)
    of the workload.

    Every valid shape is timed with `reps` launches; the three cheapest and
    the heuristic's shape are timed again with 3 * reps launches, and a shape
    replaces the heuristic's only if its cost (launch time plus `reduce_ms`)
    is lower by more than 1 - margin.  `ms` in an entry is the launch time."""
    seen = {}
    set_tuning([])  # the heuristic's choice is the baseline
    for i in range(len(instances)):
        for e in plan_convs(geometries, instances, precision, inst=i):
            if e["pass"] in passes:
                seen.setdefault(_key(e), e)
    table = []
    cost = lambda e, sh, ms: ms + reduce_ms(e, sh)
    for key, e in seen.items():
        first = sorted(((cost(e, sh, time_pass(e, sh, reps)), i, sh)
                        for i, sh in enumerate(candidates(e))), key=lambda t: (t[0], t[1]))
        finals = [sh for _, _, sh in first[:3]]
        base = time_pass(e, e["shape"], 3 * reps)
        best, best_ms = e["shape"], base
        for sh in finals:
            ms = time_pass(e, sh, 3 * reps)
            if cost(e, sh, ms) < margin * cost(e, e["shape"], base) and \
                    cost(e, sh, ms) < cost(e, best, best_ms):
                best, best_ms = sh, ms
        if log:
            log("n=%-3d %3d->%-3d taps %2d pass %d pro %d: %.4f ms -> %.4f ms %s"
                % (e["n"], e["cin"], e["cout"], e["taps"], e["pass"], e["prologue"], base,
                   best_ms, best))
        table.append(dict(e, shape=best, ms=best_ms, heuristic_ms=base))
    return table


def merge(*tables):
    """One table from several (the first entry of a key wins)."""
    out, keys = [], set()
    for t in tables:
        for e in t:
            if _key(e) not in keys:
                keys.add(_key(e))
                out.append(e)
    return out


def update(base, new):
    """`base` in its order with the entries of `new` in place of those with the
    same key, then the entries of `new` that `base` lacks."""
    by_key = {_key(e): e for e in new}
    out = [by_key.pop(_key(e), e) for e in base]
    return out + [e for e in new if _key(e) in by_key]


def save(table, path):
    with open(path, "w") as f:
        json.dump(table, f, indent=0)


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


WORKLOADS = ("c0", "c1", "c2", "c3", "c4")
PRECISIONS = ("fp32", "bf16x3", "bf16")


def tune_all(workloads=WORKLOADS, precisions=PRECISIONS, reps=10, log=None, passes=(0, 1, 2)):
    """One table for every conv pass (of the listed `passes`) of the named
    workloads and precisions."""
    tables = []
    for w in workloads:
        geos, insts = workload(w)
        for prec in precisions:
            for k in sorted({tuple(i) for i in insts}):
                tables.append(tune([geos[k[0]]], [(0, k[1], k[2])], prec, reps, log,
                                   passes=passes))
    return merge(*tables)


def default_table_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="all", help="c0..c4 or all")
    ap.add_argument("--precision", default="all")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--passes", default="0,1,2", help="conv passes to tune (0 forward, "
                    "1 input gradient, 2 weight gradient)")
    ap.add_argument("--base", default=None, help="table whose other entries are kept")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    ws = WORKLOADS if a.workload == "all" else (a.workload,)
    ps = PRECISIONS if a.precision == "all" else (a.precision,)
    passes = tuple(int(x) for x in a.passes.split(","))
    table = tune_all(ws, ps, a.reps, log, passes)
    if a.base:
        with open(a.base) as f:
            table = update(json.load(f), table)
    save(table, a.out)


if __name__ == "__main__":
    main()
