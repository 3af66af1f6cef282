"""Benchmark of the D2IP fitting iteration on one MI355X.

A step is one DIP iteration of the whole hot path (network forward, J sigma,
loss, J^T, network backward, Adam) over the 32^3 / 928-measurement / 3-level /
16-channel workload, inputs resident in HBM.

The default run is one process:
  * each precision form (fp32, bf16x3, bf16), with the stored tuning table,
    launched as one captured hipGraph per iteration and as eager launches on
    the context's two streams: an untimed 500-iteration fit whose images are
    compared with the stored FP64 oracle images at every stored checkpoint
    (the form's image error, whatever --steps and --warmup are), then --warmup
    untimed and --steps timed iterations (HIP events on the context stream);
    the faster launch mode is the form's rate;
  * plain FP32 (heuristic launch shapes, eager launches) the same way;
  * tsEIT frames/s: one breathing sequence fitted frame after frame with TPP
    (500 iterations for the first frame, 50 per later frame), chosen form and
    plain FP32;
  * the kernel table of the chosen form (each kernel timed with HIP events on
    the context stream) and the roofline entry of its dominant kernel;
  * the FP64 oracle on the host's cores (cpu_baseline).
`value` is the it/s of the fastest form whose image error after 500
iterations is within its bound (FP32 1e-5, BF16 forms 2e-3, or 3x the
oracle's own 1-ulp sensitivity at that iteration when larger).

The other workloads (--configs: 16^3, 64^3, eight 32^3 sequences, sixteen
uneven instances; --ops: the depthwise-separable and SE operators and the
module variants of the network; --ablation: the UPWS/TPP schedule ablation)
each run in a child process of their own and are reported under "sections".

    python bench.py [--steps 480] [--warmup 20] [--gpus 1] [--configs] [--ops] [--ablation]

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import glob
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DIP iterations/s and tsEIT frames/s at 32^3 vs plain FP32, at stated image error"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
ERR_BOUND = {"fp32": 1e-5, "bf16x3": 2e-3, "bf16": 2e-3}
DTYPE = {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3"}
M_OF_RINGS = {1: 208, 2: 928}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def golden_image(cfg_name, iters, floor=False):
    """Stored FP64 oracle image after `iters` iterations (or, with floor, the
    relative distance to the oracle's own run from a 1-ulp perturbed theta_0)."""
    for path in sorted(glob.glob(os.path.join(ROOT, "tests", "golden",
                                              "oracle_%s_*.npz" % cfg_name))):
        z = np.load(path)
        cps = list(z["checkpoints"])
        if iters not in cps:
            continue
        img = z["images"][cps.index(iters)]
        if not floor:
            return img
        if "floor_images" not in z:
            return None
        return rel_err(z["floor_images"][cps.index(iters)], img)
    return None


def rel_err(img, ref):
    if ref is None:
        return None
    return float(np.linalg.norm(img - ref) / np.linalg.norm(ref))


def conv_flops(n, cin, cout, taps):
    return 2.0 * n ** 3 * cin * cout * taps


def network_fwd_flops(levels, C, n):
    """Forward FLOPs of the network: stem 1->C, every ResBlock's two 3x3x3
    convs and its 1x1x1 projection when channels change, the 1x1x1 head."""
    f = conv_flops(n, 1, C, 27) + conv_flops(n, C, 1, 1)
    for (m, cin, cout) in block_convs(levels, C, n):
        f += conv_flops(m, cin, cout, 27) + conv_flops(m, cout, cout, 27)
        if cin != cout:
            f += conv_flops(m, cin, cout, 1)
    return f


def iteration_roofline(cfg, prec, M, qa, P, measured_ms):
    """Per-iteration lower bound from the serial phases: convs (forward, input
    gradient and weight gradient = 3 x forward FLOPs) at the MFMA peak of the
    form's operands, two streams of the compact J and Adam (28 B/param) at the
    HBM peak; `frac` = bound sum / measured time."""
    conv_us = 3 * network_fwd_flops(cfg["levels"], cfg["base_ch"], cfg["n"]) / (
        PEAK_TFLOPS[prec] * 1e12) * 1e6
    j_us = 2 * 4.0 * M * qa / (HBM_PEAK_GBS * 1e9) * 1e6
    adam_us = 28.0 * P / (HBM_PEAK_GBS * 1e9) * 1e6
    s = conv_us + j_us + adam_us
    return dict(conv_us=conv_us, j_us=j_us, adam_us=adam_us, sum_us=s,
                max_us=max(conv_us, j_us, adam_us), measured_us=measured_ms * 1e3,
                frac=s / (measured_ms * 1e3))


def block_convs(levels, C, n):
    """(level grid n, cin, cout) of conv1 of every ResBlock in flat order."""
    out = []
    for l in range(levels):
        out.append((n >> l, C if l == 0 else C << (l - 1), C << l))
    for l in range(levels - 2, -1, -1):
        out.append((n >> l, (C << (l + 1)) + (C << l), C << l))
    return out


def tuned(d2ip, at, geos, insts, prec, cache):
    """Tuning entries for this workload and precision: from the stored table
    of this chip if it covers every pass, else tuned now (once per run)."""
    key = (tuple(geos), tuple(insts), prec)
    if key not in cache:
        stored = cache.get("stored")
        if stored is None:
            path = at.default_table_path()
            stored = cache["stored"] = at.load_table(path) if os.path.exists(path) else []
        keys = {at._key(e): e for e in stored}
        at.set_tuning([])
        need = []
        for i in range(len(insts)):
            need += at.plan_convs(geos, insts, prec, inst=i)
        if need and all(at._key(e) in keys for e in need):
            cache[key] = [keys[at._key(e)] for e in need]
        else:
            t0 = time.time()
            cache[key] = at.tune(geos, insts, prec)
            cache.setdefault("fresh", []).extend(cache[key])
            log("  tuned %d conv passes for %s in %.1f s" % (len(cache[key]), prec,
                                                             time.time() - t0))
    return cache[key]


def traffic_record(at, kernel, form, table):
    """HBM bytes per launch of `kernel` from a stored counter record, if its
    sources and tuned launch shape are unchanged since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*traffic*.md"))):
        for line in open(path):
            if not line.startswith("traffic-record: "):
                continue
            rec = json.loads(line[len("traffic-record: "):])
            if rec["kernel"] != kernel or rec["form"] != form:
                continue
            h = hashlib.sha256()
            for src in rec["sources"]:
                h.update(open(os.path.join(ROOT, src), "rb").read())
            if h.hexdigest() != rec["sources_sha256"]:
                continue
            shape = next((e["shape"] for e in table
                          if all(e[k] == v for k, v in rec["pass"].items())), None)
            if shape is None or any(shape[k] != rec["shape"][k] for k in ("tile", "ck", "split")):
                continue
            return rec["bytes_per_launch"]
    return None


def timed_run(ctx, steps, torch):
    """ms of `steps` iterations of every instance (HIP events on the context stream)."""
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    ctx.run(steps, sync=False)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def single_form(d2ip, at, p, cfg, prec, steps, warmup, torch, graph=True, tune=True, cache=None,
                tv=False):
    geos = [(cfg["n"], p["J"].shape[0])]
    insts = [(0, cfg["levels"], cfg["base_ch"])]
    at.set_tuning(tuned(d2ip, at, geos, insts, prec, cache) if tune else [])
    ctx = d2ip.Context(geos, insts, precision=prec, graph=graph)
    ctx.load_problem(0, p)
    ctx.set_adam(lr=cfg["lr"])
    if tv:
        ctx.set_tv()  # Sec. III-E coefficients; a first frame has no temporal history
    ctx.run(warmup)
    ms = timed_run(ctx, steps, torch)
    loss = float(ctx.run(0)[0])
    return ctx, ms, loss, ctx.read_image(0)


def kernel_table(d2ip, ctx, p, cfg, prec):
    """Per-kernel mean launch time (HIP events) and algorithmic work."""
    L = d2ip._lib
    M = p["J"].shape[0]
    qa = int(p["mask"].sum())
    P = ctx.n_params[0]
    rows = []
    jbytes = 4.0 * M * qa
    for name, kid, work in (("jvec", L.KERNEL_JVEC, jbytes), ("jtvec", L.KERNEL_JTVEC, jbytes)):
        ms = ctx.time_kernel(0, kid, 0, 50)
        rows.append(dict(kernel=name, ms=ms, bound="hbm", work=work, unit="GB/s",
                         achieved=work / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS))
    for k, (n, cin, cout) in enumerate(block_convs(cfg["levels"], cfg["base_ch"], cfg["n"])):
        fl = conv_flops(n, cin, cout, 27)
        for name, kid in (("conv_fwd", L.KERNEL_CONV_FWD), ("conv_dgrad", L.KERNEL_CONV_DGRAD),
                          ("conv_wgrad", L.KERNEL_CONV_WGRAD)):
            ms = ctx.time_kernel(0, kid, k, 20)
            rows.append(dict(kernel="%s[block%d %d^3 %d->%d]" % (name, k, n, cin, cout), ms=ms,
                             bound="mfma", work=fl, unit="TFLOP/s",
                             achieved=fl / (ms * 1e-3) / 1e12, peak=PEAK_TFLOPS[prec]))
    ms = ctx.time_kernel(0, L.KERNEL_ADAM, 0, 50)
    rows.append(dict(kernel="adam", ms=ms, bound="hbm", work=28.0 * P, unit="GB/s",
                     achieved=28.0 * P / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS))
    for r in rows:
        r["frac"] = r["achieved"] / r["peak"]
    return rows


def dwsep_ops(d2ip, torch, shapes=((64, 64, 64), (32, 16, 16))):
    """The depthwise-separable convolution's operators (depthwise 3x3x3:
    forward, input gradient, weight gradient; pointwise 1x1x1 forward) through
    the op-level C-ABI on synthetic channels-last FP32 tensors, each launch
    timed with HIP events on the stream it is enqueued on.  Algorithmic bytes
    of a pass: its two voxel tensors (read + write, or the two reads of a
    weight gradient), 4 bytes per value; the pointwise passes, GEMMs of
    2 n^3 C Cout flops, are priced both ways (HBM bytes and FP32 flops)."""
    import ctypes
    L = d2ip._lib
    lib = L.load()
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    g = torch.Generator(device="cuda").manual_seed(2507)
    out = {}
    for n, C, Co in shapes:
        V = n ** 3
        x = torch.randn(V, C, device="cuda", generator=g)
        w = 0.2 * torch.randn(C, 27, device="cuda", generator=g)
        b = torch.randn(C, device="cuda", generator=g)
        gy = torch.randn(V, C, device="cuda", generator=g)
        y, gx = torch.empty_like(x), torch.empty_like(x)
        gw, gb = torch.empty_like(w), torch.empty_like(b)
        wp = 0.2 * torch.randn(Co, C, 1, 1, 1, device="cuda", generator=g)
        bp = torch.randn(Co, device="cuda", generator=g)
        yp = torch.empty(V, Co, device="cuda")
        nb = ctypes.c_size_t()
        L.check(lib.d2ip_op_dwconv3d_bytes(n, C, ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        gyp = torch.randn(V, Co, device="cuda", generator=g)
        gwp, gbp = torch.empty(Co, C, device="cuda"), torch.empty(Co, device="cuda")
        pb = ctypes.c_size_t()
        L.check(lib.d2ip_op_pwconv3d_bytes(n, C, Co, ctypes.byref(pb)))
        pws = torch.empty(pb.value, dtype=torch.uint8, device="cuda")
        calls = {
            "dw_forward": lambda: lib.d2ip_op_dwconv3d_forward(P(x), P(w), P(b), P(y), n, C, sp),
            "dw_input_grad": lambda: lib.d2ip_op_dwconv3d_backward(
                None, P(w), P(gy), P(gx), None, None, n, C, None, 0, sp),
            "dw_weight_grad": lambda: lib.d2ip_op_dwconv3d_backward(
                P(x), None, P(gy), None, P(gw), P(gb), n, C, P(ws), nb.value, sp),
            "pw_forward": lambda: lib.d2ip_op_pwconv3d_forward(P(y), P(wp), P(bp), P(yp), n, C,
                                                               Co, sp),
            "pw_input_grad": lambda: lib.d2ip_op_pwconv3d_backward(
                None, P(wp), P(gyp), P(gx), None, None, n, C, Co, None, 0, sp),
            "pw_weight_grad": lambda: lib.d2ip_op_pwconv3d_backward(
                P(y), None, P(gyp), None, P(gwp), P(gbp), n, C, Co, P(pws), pb.value, sp),
        }
        rows = {}
        for name, f in calls.items():
            for _ in range(5):
                L.check(f())
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(50):
                f()
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 50
            byts = 4.0 * V * (C + (Co if name.startswith("pw") else C))
            r = dict(ms=ms, bound="hbm", achieved=byts / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                     unit="GB/s")
            r["frac"] = r["achieved"] / r["peak"]
            if name.startswith("pw"):
                fl = 2.0 * V * C * Co
                r["tflops"] = fl / (ms * 1e-3) / 1e12
                r["tflops_frac_fp32"] = r["tflops"] / PEAK_TFLOPS["fp32"]
            rows[name] = r
            log("  %d^3 C=%d %-15s %8.4f ms  %7.0f GB/s (%.1f%% of HBM peak)%s"
                % (n, C, name, ms, r["achieved"], 100 * r["frac"],
                   "  %.1f TFLOP/s" % r["tflops"] if "tflops" in r else ""))
        out["%d^3 x %d -> %d" % (n, C, Co)] = rows
    return out


def se_ops(d2ip, torch, shapes=((64, 64, 16), (32, 16, 4))):
    """The Squeeze-and-Excitation unit through the op-level C-ABI (FP32,
    channels-last, HIP events per call).  Algorithmic bytes: the forward
    streams three voxel tensors (x for the channel means, x again and y for
    the scaling); the backward five (x for the recomputed means, gy and x for
    the gate gradient, gy and gx for the input gradient)."""
    import ctypes
    L = d2ip._lib
    lib = L.load()
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    g = torch.Generator(device="cuda").manual_seed(2508)
    out = {}
    for n, C, H in shapes:
        V = n ** 3
        x = 1.0 + torch.randn(V, C, device="cuda", generator=g)
        gy = torch.randn(V, C, device="cuda", generator=g)
        w1 = torch.randn(H, C, device="cuda", generator=g) / C ** 0.5
        b1 = torch.zeros(H, device="cuda")
        w2 = torch.randn(C, H, device="cuda", generator=g) / H ** 0.5
        b2 = torch.zeros(C, device="cuda")
        y, gx = torch.empty_like(x), torch.empty_like(x)
        gw1, gb1, gw2, gb2 = (torch.empty_like(t) for t in (w1, b1, w2, b2))
        nb = ctypes.c_size_t()
        L.check(lib.d2ip_op_se_bytes(n, C, H, ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        calls = {
            "se_forward": (3, lambda: lib.d2ip_op_se_forward(
                P(x), P(w1), P(b1), P(w2), P(b2), P(y), n, C, H, P(ws), nb.value, sp)),
            "se_backward": (5, lambda: lib.d2ip_op_se_backward(
                P(x), P(w1), P(b1), P(w2), P(b2), P(gy), P(gx), P(gw1), P(gb1), P(gw2), P(gb2),
                n, C, H, P(ws), nb.value, sp)),
        }
        rows = {}
        for name, (passes, f) in calls.items():
            for _ in range(5):
                L.check(f())
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(50):
                f()
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 50
            byts = passes * 4.0 * V * C
            rows[name] = dict(ms=ms, bound="hbm", achieved=byts / (ms * 1e-3) / 1e9,
                              peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
            log("  %d^3 C=%d H=%d %-12s %8.4f ms  %7.0f GB/s (%.1f%% of HBM peak)"
                % (n, C, H, name, ms, rows[name]["achieved"], 100 * rows[name]["frac"]))
        out["%d^3 x %d, H %d" % (n, C, H)] = rows
    return out


def module_ops(d2ip, torch, att_shapes=((64, 16, 32), (32, 32, 64), (64, 64, 128), (16, 128, 256)),
               head_shapes=((64, 16), (32, 16))):
    """The attention unit, the output head (sigmoid tail), pooling and
    up-sampling + concatenation through the op-level C-ABI (FP32,
    channels-last, HIP events per call).  Algorithmic bytes (4 per value):
    attention forward reads x [n^3][c] and g [(n/2)^3][cu] and writes y;
    backward reads x, g, gy and writes gx, gg; head forward reads x [n^3][C]
    and the mask and writes the image, backward reads x, the mask and gout and
    writes gx; pooling reads n^3 C and writes n^3 C / 8; up + concat reads the
    coarse d and the skip and writes the concatenation."""
    import ctypes
    L = d2ip._lib
    lib = L.load()
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    st = torch.cuda.current_stream()
    sp = ctypes.c_void_p(st.cuda_stream)
    g0 = torch.Generator(device="cuda").manual_seed(2509)
    rnd = lambda *sh: torch.randn(*sh, device="cuda", generator=g0)

    def timed(f, byts, label):
        for _ in range(5):
            L.check(f())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(50):
            f()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 50
        r = dict(ms=ms, bound="hbm", achieved=byts / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                 unit="GB/s", bytes=byts)
        r["frac"] = r["achieved"] / r["peak"]
        log("  %-34s %8.4f ms  %7.0f GB/s (%.1f%% of HBM peak)"
            % (label, ms, r["achieved"], 100 * r["frac"]))
        return r

    out = {}
    for n, c, cu in att_shapes:
        V, m3 = n ** 3, (n // 2) ** 3
        x, g, gy = rnd(V, c), rnd(m3, cu), rnd(V, c)
        wx, wg = rnd(c, c) / c ** 0.5, rnd(c, cu) / cu ** 0.5
        b, psi, bpsi = 0.1 * rnd(c), rnd(c) / c ** 0.5, 0.1 * rnd(1)
        y, gx, gg = torch.empty_like(x), torch.empty_like(x), torch.empty_like(g)
        gwx, gwg, gb, gpsi, gbpsi = (torch.empty_like(t) for t in (wx, wg, b, psi, bpsi))
        nb = ctypes.c_size_t()
        L.check(lib.d2ip_op_attention_bytes(n, c, cu, ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        key = "attention %d^3 c=%d cu=%d" % (n, c, cu)
        out[key] = dict(
            forward=timed(lambda: lib.d2ip_op_attention_forward(
                P(x), P(g), P(wx), P(wg), P(b), P(psi), P(bpsi), P(y), None, n, c, cu, P(ws),
                nb.value, sp),
                4.0 * (2 * V * c + m3 * cu), key + " fwd"),
            backward=timed(lambda: lib.d2ip_op_attention_backward(
                P(x), P(g), P(wx), P(wg), P(b), P(psi), P(bpsi), P(gy), P(gx), P(gg), P(gwx),
                P(gwg), P(gb), P(gpsi), P(gbpsi), n, c, cu, P(ws), nb.value, sp),
                4.0 * (3 * V * c + 2 * m3 * cu), key + " bwd"))
    for n, C in head_shapes:
        V = n ** 3
        x, w, b = rnd(V, C), rnd(C) / C ** 0.5, rnd(1)
        mask = (rnd(V) > -1.0).float()
        o, go, gx = torch.empty(V, device="cuda"), rnd(V), torch.empty_like(x)
        gw, gb = torch.empty_like(w), torch.empty_like(b)
        nb = ctypes.c_size_t()
        L.check(lib.d2ip_op_head_bytes(n, C, ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        key = "head (sigmoid) %d^3 C=%d" % (n, C)
        out[key] = dict(
            forward=timed(lambda: lib.d2ip_op_head_forward(P(x), P(w), P(b), P(mask), P(o), n, C,
                                                           1, sp),
                          4.0 * V * (C + 2), key + " fwd"),
            backward=timed(lambda: lib.d2ip_op_head_backward(
                P(x), P(w), P(b), P(mask), P(go), P(gx), P(gw), P(gb), n, C, 1, P(ws), nb.value,
                sp), 4.0 * V * (2 * C + 2), key + " bwd"))
    n, C = 64, 32
    V = n ** 3
    x, d = rnd(V, C), rnd(V // 8, 2 * C)
    y, cat = torch.empty(V // 8, C, device="cuda"), torch.empty(V, 3 * C, device="cuda")
    out["pool2 64^3 C=32"] = timed(lambda: lib.d2ip_op_pool2_forward(P(x), P(y), n, C, sp),
                                   4.0 * V * C * 9 / 8, "pool2 64^3 C=32")
    out["up2+concat 64^3 32+32"] = timed(
        lambda: lib.d2ip_op_up2_concat_forward(P(d), 2 * C, P(x), C, n, P(cat), sp),
        4.0 * (V // 8 * 2 * C + V * C + V * 3 * C), "up2+concat 64^3 (2C from 32^3) + C")
    return out


def module_fit(d2ip, torch, ts, reps=20):
    """The 3D-FastResUNet fitting iteration in one library call per k
    iterations (d2ip_mnet_run) at the 32^3 / 928-measurement / 3-level /
    16-channel workload: the plain network and each module mix, ms per
    iteration after 3 warm-up iterations (HIP events on the context stream)."""
    from paper_2507_14046_amd.context import ModuleFit
    cfg = ts.CONFIGS["c1"]
    p = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], cfg["seed"])
    mixes = {"plain": {}, "dwsep": dict(sep=True), "se": dict(se_ratio=4),
             "attention+sigmoid": dict(att=True, tail="sigmoid"), "aspp": dict(aspp=True),
             "all modules": dict(sep=True, se_ratio=4, att=True, tail="sigmoid", aspp=True)}
    out = {}
    for name, kw in mixes.items():
        row = {}
        for graph in (False, True):
            f = ModuleFit(cfg["n"], p["J"].shape[0], cfg["levels"], cfg["base_ch"], graph=graph,
                          **kw)
            rng = np.random.default_rng(7)
            th = (0.1 * rng.standard_normal(f.n_params)).astype(np.float32)
            f.set_problem(p["J"], p["mask"], p["Z"])
            f.set_params(th)
            f.set_frame(p["dv"][0])
            f.set_adam(lr=cfg["lr"])
            f.run(3)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(f.stream)
            f.run(reps, sync=False)
            e1.record(f.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            row["graph" if graph else "eager"] = dict(ms_per_it=ms, it_per_s=1e3 / ms)
            row["params"] = f.n_params
            f.close()
        out[name] = row
        log("  module fit %-18s eager %7.3f ms/it, graph %7.3f ms/it  (%d parameters)"
            % (name, row["eager"]["ms_per_it"], row["graph"]["ms_per_it"], row["params"]))
    return out


def dwsep_network(d2ip, torch, ts, names=("c1", "c2"), reps=10):
    """One loss + theta-gradient evaluation of the autograd network
    (`ops.DIPNet`, every operator on the library's kernels) with dense and
    with depthwise-separable ResBlock convolutions, and with the
    3D-FastResUNet modules (depthwise-separable convs, SE units, ASPP,
    attention units, sigmoid tail), FP32, on a config's problem: ms per
    evaluation (HIP events, mean of `reps` after three warm-up calls) and
    parameter counts."""
    from paper_2507_14046_amd import ops
    out = {}
    for name in names:
        c = ts.CONFIGS[name]
        p = ts.make_problem(c["n"], c["rings"], c["levels"], c["base_ch"], c["seed"])
        dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
        Z, mask, J, dv = dev(p["Z"]), dev(p["mask"].astype(np.float32)), dev(p["J"]), \
            dev(p["dv"][0])
        row = {}
        variants = {"dense": {}, "dwsep": dict(conv="dwsep"),
                    "fastres_modules": dict(conv="dwsep", se_ratio=4, att=True, tail="sigmoid",
                                            aspp=True)}
        for conv, kw in variants.items():
            model = ops.DIPNet(c["n"], c["levels"], c["base_ch"], **kw)
            g = torch.Generator(device="cuda").manual_seed(11)
            th = (0.1 * torch.randn(model.size, device="cuda", generator=g)).requires_grad_(True)

            def once():
                th.grad = None
                model.loss(th, Z, mask, J, dv).backward()
            for _ in range(3):  # first calls load kernels and size the allocator
                once()
            torch.cuda.synchronize()
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                once()
            e1.record(st)
            torch.cuda.synchronize()
            row[conv] = dict(ms_per_loss_and_grad=e0.elapsed_time(e1) / reps, params=model.size)
        row["speedup"] = row["dense"]["ms_per_loss_and_grad"] / row["dwsep"]["ms_per_loss_and_grad"]
        out[name] = row
        log("network %s: dense %.2f ms (%d params), dwsep %.2f ms (%d params), %.2fx"
            % (name, row["dense"]["ms_per_loss_and_grad"], row["dense"]["params"],
               row["dwsep"]["ms_per_loss_and_grad"], row["dwsep"]["params"], row["speedup"]))
        if "fastres_modules" in row:
            log("network %s: dwsep + SE + ASPP + attention + sigmoid tail %.2f ms (%d params)"
                % (name, row["fastres_modules"]["ms_per_loss_and_grad"],
                   row["fastres_modules"]["params"]))
    return out


def config0(d2ip, at, ts, prec, torch, cache, graph=True):
    cfg = ts.CONFIGS["c0"]
    p = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], cfg["seed"])
    ctx, ms, loss, img = single_form(d2ip, at, p, cfg, prec, cfg["iters"], 0, torch, graph=graph,
                                     cache=cache)
    ctx.close()
    return dict(workload=cfg["desc"], form=prec, launch="graph" if graph else "eager",
                it_per_s=cfg["iters"] / (ms * 1e-3),
                image_rel_err=rel_err(img, golden_image("c0", cfg["iters"])))


def config2(d2ip, at, ts, prec, torch, cache, steps=40, graph=True):
    cfg = ts.CONFIGS["c2"]
    p = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], cfg["seed"])
    ctx, ms, loss, img = single_form(d2ip, at, p, cfg, prec, steps, 3, torch, graph=graph,
                                     cache=cache)
    M, qa, P = p["J"].shape[0], int(p["mask"].sum()), ctx.n_params[0]
    kernels = None
    if not graph:
        # at 64^3 the compact J (767 MB) exceeds the MALL: the J products are
        # HBM streams; the largest conv (decoder level 0, 96 -> 32 channels)
        L = d2ip._lib
        kernels = {}
        jbytes = 4.0 * M * qa
        for name, kid in (("jvec", L.KERNEL_JVEC), ("jtvec", L.KERNEL_JTVEC)):
            kms = ctx.time_kernel(0, kid, 0, 20)
            kernels[name] = dict(ms=kms, achieved=jbytes / (kms * 1e-3) / 1e9, unit="GB/s",
                                 frac=jbytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        blocks = block_convs(cfg["levels"], cfg["base_ch"], cfg["n"])
        k = len(blocks) - 1
        n, cin, cout = blocks[k]
        fl = conv_flops(n, cin, cout, 27)
        for name, kid in (("conv_fwd", L.KERNEL_CONV_FWD), ("conv_dgrad", L.KERNEL_CONV_DGRAD),
                          ("conv_wgrad", L.KERNEL_CONV_WGRAD)):
            kms = ctx.time_kernel(0, kid, k, 5)
            kernels["%s[block%d %d^3 %d->%d]" % (name, k, n, cin, cout)] = dict(
                ms=kms, achieved=fl / (kms * 1e-3) / 1e12, unit="TFLOP/s",
                frac=fl / (kms * 1e-3) / 1e12 / PEAK_TFLOPS[prec])
    ctx.close()
    return dict(workload=cfg["desc"], form=prec, launch="graph" if graph else "eager",
                roofline=iteration_roofline(cfg, prec, M, qa, P, ms / steps), kernels=kernels,
                it_per_s=steps / (ms * 1e-3), timed_iters=steps,
                final_loss=loss, image_rel_err=None,
                note="no stored FP64 oracle trajectory at this size")


def _launch(graph):
    return ("one captured hipGraph per iteration, instances in sequence" if graph else
            "eager launches, instances concurrently on up to 4 stream lanes")


def config3(d2ip, at, ts, prec, torch, cache, frames=3, graph=True):
    """Eight sequences fitted together, frame after frame (TPP): steady-state
    frames/s over `frames` frames of 50 iterations after a 500-iteration first
    frame, and the full 100-frame schedule's rate derived from it."""
    cfg = ts.CONFIGS["c3"]
    seqs = [ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], s,
                            frames=frames + 1, breathing=True) for s in cfg["seeds"]]
    M = seqs[0]["J"].shape[0]
    geos = [(cfg["n"], M)]
    insts = [(0, cfg["levels"], cfg["base_ch"])] * len(seqs)
    at.set_tuning(tuned(d2ip, at, geos, [insts[0]], prec, cache))
    ctx = d2ip.Context(geos, insts, precision=prec, graph=graph)
    ctx.set_geometry(0, seqs[0]["J"], seqs[0]["mask"])
    for i, p in enumerate(seqs):
        ctx.load_problem(i, p, set_geometry=False)
    ctx.set_adam(lr=cfg["lr"])
    t_first = timed_run(ctx, cfg["iters"], torch)
    t_later = 0.0
    for f in range(1, frames + 1):
        for i, p in enumerate(seqs):
            ctx.set_frame(i, p["dv"][f])
            ctx.reset_optimizer(i)
        t_later += timed_run(ctx, cfg["later_iters"], torch)
    ctx.close()
    S = len(seqs)
    per_frame_ms = t_later / frames
    total_ms = t_first + (cfg["frames"] - 1) * per_frame_ms
    return dict(workload=cfg["desc"], form=prec, sequences=S, launch=_launch(graph),
                frames_per_s_steady=S / (per_frame_ms * 1e-3),
                frames_per_s_schedule=S * cfg["frames"] / (total_ms * 1e-3),
                first_frame_ms=t_first, later_frame_ms=per_frame_ms,
                sample="first frame (500 its) + %d frames of 50 its, 8 sequences; the full "
                       "100-frame rate extrapolates the measured per-frame time" % frames)


def config4(d2ip, at, ts, prec, torch, cache, iters=20, graph=True):
    cfg = ts.CONFIGS["c4"]
    geos, insts, probs = [], [], []
    for it in cfg["instances"]:
        p = ts.make_problem(it["n"], it["rings"], cfg["levels"], it["base_ch"], it["seed"])
        g = (it["n"], M_OF_RINGS[it["rings"]])
        if g not in geos:
            geos.append(g)
        insts.append((geos.index(g), cfg["levels"], it["base_ch"]))
        probs.append(p)
    table = {}
    for k in {tuple(i) for i in insts}:
        for e in tuned(d2ip, at, [geos[k[0]]], [(0, k[1], k[2])], prec, cache):
            table[tuple(e[f] for f in at.FIELDS)] = e
    at.set_tuning(list(table.values()))
    ctx = d2ip.Context(geos, insts, precision=prec, graph=graph)
    done = set()
    for i, p in enumerate(probs):
        ctx.load_problem(i, p, set_geometry=insts[i][0] not in done)
        done.add(insts[i][0])
    ctx.set_adam(lr=cfg["lr"])
    ctx.run(2)
    ms = timed_run(ctx, iters, torch)
    ctx.close()
    return dict(workload=cfg["desc"], form=prec, instances=len(insts), launch=_launch(graph),
                batched_it_per_s=iters / (ms * 1e-3),
                instance_it_per_s=len(insts) * iters / (ms * 1e-3),
                schedule_s=cfg["iters"] * ms / iters * 1e-3,
                sample="%d batched iterations timed after 2 warm-up iterations" % iters)



def golden(cfg_name, upto):
    """Stored FP64 oracle images of a workload at its checkpoints <= upto, and
    the relative distance of the oracle's own run from a 1-ulp perturbed
    theta_0 at each (the sensitivity floor)."""
    for path in sorted(glob.glob(os.path.join(ROOT, "tests", "golden",
                                              "oracle_%s_*.npz" % cfg_name))):
        z = np.load(path)
        cps = [int(c) for c in z["checkpoints"]]
        out = {}
        for i, c in enumerate(cps):
            if c <= upto:
                fl = rel_err(z["floor_images"][i], z["images"][i]) if "floor_images" in z else None
                out[c] = (z["images"][i], fl)
        if out:
            return out
    return {}


def fit_and_time(d2ip, at, p, cfg, prec, steps, warmup, torch, gold, graph, tune=True,
                 cache=None):
    """Untimed fit through the stored checkpoints (image error at each), then
    `warmup` untimed and `steps` timed iterations in the same context."""
    geos = [(cfg["n"], p["J"].shape[0])]
    insts = [(0, cfg["levels"], cfg["base_ch"])]
    at.set_tuning(tuned(d2ip, at, geos, insts, prec, cache) if tune else [])
    ctx = d2ip.Context(geos, insts, precision=prec, graph=graph)
    try:
        ctx.load_problem(0, p)
        ctx.set_adam(lr=cfg["lr"])
        errs, done = {}, 0
        last_img = None
        for k in sorted(gold):
            ctx.run(k - done)
            done = k
            last_img = ctx.read_image(0)
            errs[k] = rel_err(last_img, gold[k][0])
        loss = float(ctx.run(0)[0])
        kmax = max(gold) if gold else None
        max_abs = float(np.max(np.abs(last_img - gold[kmax][0]))) if kmax else None
        ctx.run(warmup)
        ms = timed_run(ctx, steps, torch)
        ctx.run(0)  # synchronising read: raises on a non-finite loss or parameter
    finally:
        ctx.close()
    return dict(ms=ms, errs=errs, loss_at_fit_end=loss, fit_iters=done, max_abs=max_abs)


def tpp_frames(d2ip, at, cfg, prec, torch, graph, tune=True, cache=None, frames=5):
    """tsEIT frames/s of one breathing sequence (Sec. III-C): a 500-iteration
    first frame, then `frames` frames of 50 iterations, each started from the
    previous frame's parameters (Eq. (9)) with the optimiser restarted."""
    import tseit_synth as ts
    c3 = ts.CONFIGS["c3"]
    seq = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], c3["seeds"][0],
                          frames=frames + 1, breathing=True)
    geos = [(cfg["n"], seq["J"].shape[0])]
    insts = [(0, cfg["levels"], cfg["base_ch"])]
    at.set_tuning(tuned(d2ip, at, geos, insts, prec, cache) if tune else [])
    ctx = d2ip.Context(geos, insts, precision=prec, graph=graph)
    try:
        ctx.load_problem(0, seq)
        ctx.set_adam(lr=c3["lr"])
        first_ms = timed_run(ctx, c3["iters"], torch)
        # frame transitions included: dv upload (host array) and optimiser reset
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for f in range(1, frames + 1):
            ctx.set_frame(0, seq["dv"][f])
            ctx.reset_optimizer(0)
            ctx.run(c3["later_iters"], sync=False)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        ctx.run(0)
    finally:
        ctx.close()
    return dict(frames_per_s=frames / (wall), later_frame_ms=wall * 1e3 / frames,
                later_frame_ms_gpu_events=ms / frames, first_frame_ms=first_ms,
                sample="1 sequence: first frame 500 iterations, then %d frames of 50 iterations "
                       "(dv upload + optimiser reset per frame, host wall clock)" % frames)


def cpu_baseline(p, cfg, iters=3):
    """The FP64 oracle as it stands on this host's cores: one warm-up
    iteration, then the median of `iters` timed iterations."""
    from oracle import fit
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    pr = fit.Problem(p["J"], p["mask"], p["Z"], cfg["n"], cfg["levels"], cfg["base_ch"])
    st = fit.State(p["theta0"])
    fit.run(pr, st, p["dv"][0], 1, cfg["lr"])
    ts_ = []
    for _ in range(iters):
        t0 = time.perf_counter()
        fit.run(pr, st, p["dv"][0], 1, cfg["lr"])
        ts_.append(time.perf_counter() - t0)
    med = float(np.median(ts_))
    return dict(value=1.0 / med, unit="it/s", cores=int(cores), kind="oracle",
                sample="median of %d FP64 oracle iterations of the 32^3 workload after 1 "
                       "warm-up iteration (%s s each)" % (iters, ", ".join("%.1f" % t for t in ts_)))


SECTIONS = ("c0", "c2", "c3", "c4", "ops", "network", "ablation", "kernels64")


def kernels64(d2ip, at, ts, prec, torch, cache, reps=20):
    """The 64^3 workload's kernels in one form, each timed in isolation with
    HIP events on the context stream (after two eager iterations): J sigma and
    J^T g (HBM streams of the 767 MB compact J), Adam over its 5.97 M
    parameters, and the three passes of the largest conv (decoder level 0,
    96 -> 32 channels, 43.5 GFLOP per pass)."""
    cfg = ts.CONFIGS["c2"]
    p = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], cfg["seed"])
    geos, insts = [(cfg["n"], p["J"].shape[0])], [(0, cfg["levels"], cfg["base_ch"])]
    at.set_tuning(tuned(d2ip, at, geos, insts, prec, cache))
    ctx = d2ip.Context(geos, insts, precision=prec, graph=False)
    L = d2ip._lib
    out = {}
    try:
        ctx.load_problem(0, p)
        ctx.set_adam(lr=cfg["lr"])
        ctx.run(2)
        M, qa, P = p["J"].shape[0], int(p["mask"].sum()), ctx.n_params[0]
        jb = 4.0 * M * qa
        for name, kid, work in (("jvec", L.KERNEL_JVEC, jb), ("jtvec", L.KERNEL_JTVEC, jb),
                                ("adam", L.KERNEL_ADAM, 28.0 * P)):
            ms = ctx.time_kernel(0, kid, 0, reps)
            out[name] = dict(ms=ms, bytes=work, achieved=work / (ms * 1e-3) / 1e9, unit="GB/s",
                             frac=work / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        blocks = block_convs(cfg["levels"], cfg["base_ch"], cfg["n"])
        k = len(blocks) - 1
        n, cin, cout = blocks[k]
        fl = conv_flops(n, cin, cout, 27)
        for name, kid in (("conv_fwd", L.KERNEL_CONV_FWD), ("conv_dgrad", L.KERNEL_CONV_DGRAD),
                          ("conv_wgrad", L.KERNEL_CONV_WGRAD)):
            ms = ctx.time_kernel(0, kid, k, reps)
            out["%s[block%d %d^3 %d->%d]" % (name, k, n, cin, cout)] = dict(
                ms=ms, flop=fl, achieved=fl / (ms * 1e-3) / 1e12, unit="TFLOP/s",
                frac=fl / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec])
    finally:
        ctx.close()
        at.set_tuning([])
    for name, r in out.items():
        log("  64^3 %s %-36s %9.4f ms  %9.2f %s (%.1f%% of peak)"
            % (prec, name, r["ms"], r["achieved"], r["unit"], 100 * r["frac"]))
    return dict(form=prec, kernels=out)


def run_section(name, a):
    """One optional workload in this process (the child side of --configs,
    --ops and --ablation); returns a JSON-able result."""
    import torch
    import paper_2507_14046_amd as d2ip
    from paper_2507_14046_amd import autotune as at
    import tseit_synth as ts
    cache = {}
    out = {}
    if name in ("c0", "c2", "c3", "c4"):
        fn = {"c0": config0, "c2": config2, "c3": config3, "c4": config4}[name]
        for prec in ("fp32", "bf16"):
            for graph in (True, False):
                key = prec + ("" if graph else "_eager")
                t0 = time.time()
                out[key] = fn(d2ip, at, ts, prec, torch, cache, graph=graph)
                log("%s %-10s %s (%.0f s)" % (name, key, json.dumps(out[key]), time.time() - t0))
        at.set_tuning([])
    elif name == "ops":
        out = dict(dwsep=dwsep_ops(d2ip, torch), se=se_ops(d2ip, torch),
                   modules=module_ops(d2ip, torch))
    elif name == "network":
        out = dict(autograd=dwsep_network(d2ip, torch, ts), module_fit=module_fit(d2ip, torch, ts))
    elif name == "kernels64":
        out = {prec: kernels64(d2ip, at, ts, prec, torch, cache) for prec in a.forms.split(",")}
    elif name == "ablation":
        from paper_2507_14046_amd import schedule
        cfg = ts.CONFIGS["c1"]
        seq = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], cfg["seed"],
                              frames=20, breathing=True)
        warm = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"],
                               cfg["seed"] + 1000)
        geos = [(cfg["n"], seq["J"].shape[0])]
        insts = [(0, cfg["levels"], cfg["base_ch"])]
        at.set_tuning(tuned(d2ip, at, geos, insts, a.ablation_form, cache))
        actx = d2ip.Context(geos, insts, precision=a.ablation_form, graph=False)
        actx.load_problem(0, seq)
        out = schedule.ablation(actx, seq["theta0"], seq["dv"], warm["dv"][0])
        actx.close()
        out["form"] = a.ablation_form
    if cache.get("fresh"):
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        at.save(at.merge(cache["fresh"]),
                os.path.join(ROOT, "gpurun_out", "tuned_fresh_%s.json" % name))
    return out


def spawn_section(name, a, timeout_s):
    """Run one optional workload in a child process; its result, or its exit
    status when it failed."""
    cmd = [sys.executable, os.path.abspath(__file__), "--section", name,
           "--ablation-form", a.ablation_form, "--forms", "fp32,bf16"]
    log("section %s: starting a child process" % name)
    t0 = time.time()
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, timeout=timeout_s, text=True)
    except subprocess.TimeoutExpired:
        return dict(status="timeout", seconds=time.time() - t0)
    lines = [l for l in r.stdout.splitlines() if l.startswith("SECTION_JSON: ")]
    if r.returncode != 0 or not lines:
        return dict(status="failed", returncode=r.returncode, seconds=time.time() - t0)
    res = json.loads(lines[-1][len("SECTION_JSON: "):])
    res["seconds"] = time.time() - t0
    return res


def traffic_probe(mib):
    """Plain device copies of known size: the scale of the HBM byte counters."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("traffic probe: 3 copies of %d MiB" % mib)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=480)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--forms", default="fp32,bf16x3,bf16")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--no-frames", action="store_true")
    ap.add_argument("--no-tv", action="store_true")
    ap.add_argument("--configs", action="store_true",
                    help="also the 16^3, 64^3, eight-sequence and sixteen-instance workloads")
    ap.add_argument("--ops", action="store_true",
                    help="also the depthwise-separable / SE operators and the module variants "
                         "of the network")
    ap.add_argument("--ablation", action="store_true",
                    help="also the D2IP schedule ablation (UPWS / TPP), 20 frames at 32^3")
    ap.add_argument("--ablation-form", default="fp32")
    ap.add_argument("--section", choices=SECTIONS,
                    help="run one optional workload alone in this process (kernels64: the "
                         "64^3 kernels of each --forms form) and print its result")
    ap.add_argument("--traffic-probe", type=int, default=0,
                    help="MiB copied 3 times after the kernel table (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the fitting of one instance runs on one device); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.section:
        res = run_section(a.section, a)
        if a.traffic_probe > 0:
            traffic_probe(a.traffic_probe)
        print("SECTION_JSON: " + json.dumps(res), flush=True)
        return

    import torch
    import paper_2507_14046_amd as d2ip
    from paper_2507_14046_amd import autotune as at
    from paper_2507_14046_amd.context import runtime_versions
    import tseit_synth as ts

    hip_compiled, hip_runtime = runtime_versions()
    log("HIP headers %d, runtime %d" % (hip_compiled, hip_runtime))
    cfg = ts.CONFIGS["c1"]
    p = ts.make_problem(cfg["n"], cfg["rings"], cfg["levels"], cfg["base_ch"], cfg["seed"])
    gold = golden("c1", cfg["iters"])
    kref = max(gold) if gold else None
    cache = {}
    forms = {}
    for prec in a.forms.split(","):
        runs = {}
        for graph in (True, False):
            runs[graph] = fit_and_time(d2ip, at, p, cfg, prec, a.steps, a.warmup, torch, gold,
                                       graph, cache=cache)
        graph = min(runs, key=lambda g: runs[g]["ms"])
        r = runs[graph]
        err = r["errs"].get(kref)
        floor = gold[kref][1] if kref else None
        bound = max(ERR_BOUND[prec], 3 * floor) if floor is not None else ERR_BOUND[prec]
        bounds = {k: max(ERR_BOUND[prec], 3 * gold[k][1]) if gold[k][1] is not None
                  else ERR_BOUND[prec] for k in gold}
        forms[prec] = dict(it_per_s=a.steps / (r["ms"] * 1e-3), ms_per_step=r["ms"] / a.steps,
                           launch="graph" if graph else "eager",
                           graph_it_per_s=a.steps / (runs[True]["ms"] * 1e-3),
                           eager_it_per_s=a.steps / (runs[False]["ms"] * 1e-3),
                           image_rel_err_vs_fp64_oracle=err, image_err_iteration=kref,
                           image_max_abs_err=r["max_abs"],
                           image_rel_err_by_iteration={str(k): v for k, v in r["errs"].items()},
                           image_rel_err_other_launch=runs[not graph]["errs"].get(kref),
                           error_bound_stated=ERR_BOUND[prec], oracle_floor=floor,
                           error_bound=bound,
                           checkpoints_within_bound=[k for k in sorted(r["errs"])
                                                     if r["errs"][k] <= bounds[k]],
                           loss_at_iteration_500=r["loss_at_fit_end"],
                           within_bound=(err is not None and err <= bound))
        log("form %-7s %9.1f it/s  %.4f ms/it  image err at %s: %s (bound %.2g)  (graph %.1f, "
            "eager %.1f)" % (prec, forms[prec]["it_per_s"], r["ms"] / a.steps, kref, err, bound,
                             forms[prec]["graph_it_per_s"], forms[prec]["eager_it_per_s"]))
    r = fit_and_time(d2ip, at, p, cfg, "fp32", a.steps, a.warmup, torch, gold, False, tune=False,
                     cache=cache)
    plain = dict(it_per_s=a.steps / (r["ms"] * 1e-3), ms_per_step=r["ms"] / a.steps,
                 image_rel_err_vs_fp64_oracle=r["errs"].get(kref),
                 note="FP32, heuristic launch shapes, eager launches (no graph)")
    log("plain fp32     %9.1f it/s  image err %s" % (plain["it_per_s"], plain["image_rel_err_vs_fp64_oracle"]))
    ok = [f for f in forms if forms[f]["within_bound"]]
    chosen = max(ok, key=lambda f: forms[f]["it_per_s"]) if ok else (
        "fp32" if "fp32" in forms else list(forms)[0])
    res = forms[chosen]
    chosen_graph = res["launch"] == "graph"

    frames = None
    if not a.no_frames:
        fc = tpp_frames(d2ip, at, cfg, chosen, torch, chosen_graph, cache=cache)
        fp = tpp_frames(d2ip, at, cfg, "fp32", torch, False, tune=False, cache=cache)
        frames = dict(chosen=dict(form=chosen, launch=res["launch"], **fc), plain_fp32=fp,
                      speedup=fc["frames_per_s"] / fp["frames_per_s"])
        log("tsEIT frames/s (50 it/frame, TPP): %s %.2f, plain fp32 %.2f"
            % (chosen, fc["frames_per_s"], fp["frames_per_s"]))
    with_tv = None
    if not a.no_tv:
        geos = [(cfg["n"], p["J"].shape[0])]
        insts = [(0, cfg["levels"], cfg["base_ch"])]
        at.set_tuning(tuned(d2ip, at, geos, insts, "fp32", cache))
        ctx = d2ip.Context(geos, insts, precision="fp32", graph=False)
        try:
            ctx.load_problem(0, p)
            ctx.set_adam(lr=cfg["lr"])
            ctx.set_tv()  # Sec. III-E coefficients; a first frame has no temporal history
            ctx.run(a.warmup)
            ms = timed_run(ctx, a.steps, torch)
            loss = float(ctx.run(0)[0])
        finally:
            ctx.close()
        with_tv = dict(it_per_s=a.steps / (ms * 1e-3), ms_per_step=ms / a.steps, final_loss=loss,
                       note="FP32, tuned, eager launches, loss with the 4D-TV term (lambda 0.002, "
                            "1, 0.1; first frame: spatial term only)")
        log("fp32 + 4D-TV   %9.1f it/s" % with_tv["it_per_s"])

    roof = None
    if not a.no_kernels:
        at.set_tuning(tuned(d2ip, at, [(cfg["n"], p["J"].shape[0])],
                            [(0, cfg["levels"], cfg["base_ch"])], chosen, cache))
        kctx = d2ip.Context([(cfg["n"], p["J"].shape[0])], [(0, cfg["levels"], cfg["base_ch"])],
                            precision=chosen, graph=False)
        try:
            kctx.load_problem(0, p)
            kctx.set_adam(lr=cfg["lr"])
            kctx.run(a.warmup + 1)
            rows = kernel_table(d2ip, kctx, p, cfg, chosen)
        finally:
            kctx.close()
        for r_ in rows:
            log("  %-40s %8.4f ms  %9.2f %s  (%.1f%% of %s peak)" %
                (r_["kernel"], r_["ms"], r_["achieved"], r_["unit"], 100 * r_["frac"], r_["bound"]))
        dom = max(rows, key=lambda r_: r_["ms"])
        table = tuned(d2ip, at, [(cfg["n"], p["J"].shape[0])],
                      [(0, cfg["levels"], cfg["base_ch"])], chosen, cache)
        roof = dict(kernel=dom["kernel"], bound=dom["bound"], achieved=dom["achieved"],
                    peak=dom["peak"], unit=dom["unit"], frac=dom["frac"],
                    traffic=traffic_record(at, dom["kernel"], chosen, table),
                    ms_per_launch=dom["ms"], work_per_launch=dom["work"],
                    kernels={r_["kernel"]: dict(ms=r_["ms"], achieved=r_["achieved"],
                                                unit=r_["unit"], frac=r_["frac"]) for r_ in rows})
        at.set_tuning([])
    if a.traffic_probe > 0:
        traffic_probe(a.traffic_probe)
    if cache.get("fresh"):
        # shapes tuned in this run (no stored table covered them)
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        at.save(at.merge(cache["fresh"]), os.path.join(ROOT, "gpurun_out", "tuned_fresh.json"))

    sections = {}
    wanted = ([s for s in ("c0", "c2", "c3", "c4", "kernels64") if a.configs] +
              (["ops", "network"] if a.ops else []) + (["ablation"] if a.ablation else []))
    for name in wanted:
        sections[name] = spawn_section(name, a, timeout_s=900)
        log("section %s: %s" % (name, sections[name].get("status", "ok")))
    cpu = None if a.no_cpu else cpu_baseline(p, cfg)
    if cpu:
        log("cpu baseline: %.4f it/s on %d cores (%s)" % (cpu["value"], cpu["cores"], cpu["sample"]))
    total = a.warmup + a.steps
    out = {
        "metric": METRIC,
        "value": res["it_per_s"],
        "unit": "it/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[chosen],
        "data": "synthetic",
        "config": {"workload": "32^3 voxels, 928 measurements (2 rings x 16 electrodes), "
                               "3-level residual U-Net with 16 base channels, 1 frame, "
                               "Adam lr 1e-3; image error after a 500-iteration fit, then "
                               "%d + %d iterations timed after it" % (a.warmup, a.steps),
                   "form": chosen, "launch": res["launch"], "autotuned": True, "instances": 1},
        "image_rel_err": res["image_rel_err_vs_fp64_oracle"],
        "image_err_iteration": kref,
        "image_error_bound": res["error_bound"],
        "speedup_vs_plain_fp32": res["it_per_s"] / plain["it_per_s"],
        "iteration_roofline": iteration_roofline(cfg, chosen, p["J"].shape[0],
                                                 int(p["mask"].sum()),
                                                 d2ip.param_count(cfg["levels"], cfg["base_ch"]),
                                                 res["ms_per_step"]),
        "tseit_frames_per_s": frames,
        "forms": forms,
        "plain_fp32": plain,
        "fp32_with_4d_tv": with_tv,
        "sections": sections,
        "hip_version": {"compiled": hip_compiled, "runtime": hip_runtime},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
