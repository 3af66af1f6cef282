"""Parity of the HIP fitting iteration with the FP64 oracle, through the C-ABI.

Tolerances.  The stated image bounds are 1e-5 (FP32) and 2e-3 (the BF16 forms)
relative L2 against the FP64 oracle; one-iteration gradients are held to the
same relative bound for the BF16 forms and to 5e-6 overall / 1e-4 per tensor
for FP32 (about ten times the measured 2-8e-7 / 3.6e-5), and FP32 images and
gradient tensors are also checked element by element (every value within a
fixed fraction of its array's scale).  The pure BF16 form (operands rounded
once to bfloat16, 2^-9 relative per operand) misses the 2e-3 bound already on
one forward pass (3-5e-3) and its gradients by 2-10e-2; the BF16x3 form (hi +
lo operands, product error near 2^-16) meets it for one iteration but not along
Adam trajectories, which amplify any per-iteration difference (the oracle's own
1-ulp run grows 1400-fold by iteration 500).  Those cases are strict expected
failures carrying the measured numbers, and
tests/test_gpu_bf16_rounding.py shows the BF16 kernels exact against the
oracle fed the same rounded operands.
"""
import numpy as np
import pytest

import tseit_synth as ts
from oracle import fit
from tests.gpu_util import (check_gradient, elementwise, make_ctx, oracle_gradient_floor,
                            oracle_problem, per_tensor_rel, problem, record, rel)

pytestmark = pytest.mark.gpu

CASES = {
    # name: (n, rings, levels, C, seed)
    "n16_L2_C8": (16, 1, 2, 8, 0),       # the 16^3 single-frame configuration
    "n24_L3_C8": (24, 1, 3, 8, 7),       # ragged tiles, 6^3 coarsest level
    "n16_L3_C16_M928": (16, 2, 3, 16, 3),
}

# stated bounds (relative L2 vs the FP64 oracle)
TOL_IMG = {"fp32": 1e-5, "bf16x3": 2e-3, "bf16": 2e-3}
TOL_GRAD = {"fp32": 5e-6, "bf16x3": 2e-3, "bf16": 2e-3}
# per gradient tensor; small tensors whose gradients cancel (biases and gains
# in front of a LayerNorm) carry larger relative errors than the whole vector
TOL_TENSOR = {"fp32": 1e-4, "bf16x3": 5e-3, "bf16": 5e-3}
TOL_TRAJ = {"fp32": 1e-5, "bf16x3": 2e-3, "bf16": 2e-3}
# element-wise (FP32): every value within this fraction of max|ref| + |ref|
ELEM_IMG, ELEM_GRAD = 1e-5, 3e-4
PRECS = ["fp32", "bf16x3", "bf16"]


def precs(**xfail):
    """PRECS with the named forms marked as strict expected failures."""
    return [pytest.param(p, marks=pytest.mark.xfail(strict=True, reason=xfail[p]))
            if p in xfail else p for p in PRECS]


BF16_FWD = "pure BF16 operands move the first image by 3.0-5.1e-3 (> 2e-3)"
BF16_GRAD = ("pure BF16 operands: one-iteration gradient 2-10e-2 from the FP64 oracle "
             "(exact against the oracle fed the same rounded operands)")


@pytest.fixture(scope="module")
def probs():
    return {k: problem(*v) for k, v in CASES.items()}


@pytest.mark.parametrize("prec", precs(bf16=BF16_FWD))
@pytest.mark.parametrize("case", list(CASES))
def test_forward_image(lib, probs, case, prec):
    p = probs[case]
    ctx = make_ctx(lib, [p], prec)
    img = ctx.read_image(0)
    ref = oracle_problem(p).image(p["theta0"].astype(np.float64))
    e = rel(img, ref)
    el = elementwise(img, ref, ELEM_IMG)
    record("forward_image", case=case, prec=prec, rel=e, elementwise=el)
    assert np.all(img[p["mask"] == 0] == 0.0)
    assert e < TOL_IMG[prec]
    if prec == "fp32":
        assert el <= 1.0, el


def _check_gradient(g, gref, levels, C, prec, tag, floor_fn=None, p=None, **kw):
    """Stated gradient bounds (FP32 also element-wise, against the oracle or
    the oracle with ReLU decisions within FP32 resolution of the kink taken
    the other way, or 3x the oracle's own 1-ulp floor where that is larger;
    the BF16 forms the stated bounds only)."""
    fp = prec == "fp32"
    r = check_gradient(g, gref, levels, C, TOL_GRAD[prec], TOL_TENSOR[prec],
                       ELEM_GRAD if fp else 1e30, floor_fn if fp else None,
                       (lambda: oracle_kink_variants(p)) if fp and p is not None else None)
    record(tag, prec=prec, **r, **kw)
    assert r["ok"], r


@pytest.mark.parametrize("prec", precs(bf16=BF16_GRAD))
@pytest.mark.parametrize("case", list(CASES))
def test_one_iteration_loss_and_gradient(lib, probs, case, prec):
    p = probs[case]
    ctx = make_ctx(lib, [p], prec)
    loss = ctx.run(1)[0]
    g = ctx.get_grad(0)
    pr = oracle_problem(p)
    L0, gref, _ = pr.loss_and_grad(p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64))
    assert abs(loss - L0) / L0 < TOL_IMG[prec], abs(loss - L0) / L0
    _check_gradient(g, gref, p["levels"], p["base_ch"], prec, "one_iteration",
                    floor_fn=lambda: oracle_gradient_floor(p), p=p, case=case,
                    loss_rel=abs(loss - L0) / L0)


@pytest.mark.parametrize("prec", precs(
    bf16x3="BF16x3: 50 Adam iterations at 16^3 end 2.4e-3 from the oracle (> 2e-3)",
    bf16="pure BF16: 50 Adam iterations at 16^3 end 0.15 from the oracle"))
def test_trajectory_50_iterations_16cubed(lib, probs, prec):
    p = probs["n16_L2_C8"]
    ctx = make_ctx(lib, [p], prec)
    losses = [ctx.run(1)[0] for _ in range(50)]
    img = ctx.read_image(0)
    pr = oracle_problem(p)
    st = fit.State(p["theta0"])
    lref = fit.run(pr, st, p["dv"][0], 50, 1e-3)
    ref = pr.image(st.theta)
    e = rel(img, ref)
    lrel = float(np.max(np.abs(np.array(losses) - lref) / np.array(lref)))
    el = elementwise(img, ref, ELEM_IMG * 10)
    record("trajectory50_n16", prec=prec, image_rel=e, loss_max_rel=lrel, elementwise=el)
    assert e < TOL_TRAJ[prec]
    if prec == "fp32":
        assert el <= 1.0, el


def test_tpp_two_frames_matches_oracle(lib):
    p = problem(16, 1, 2, 8, 11, frames=2, breathing=True)
    ctx = make_ctx(lib, [p])
    ctx.run(6)
    img0 = ctx.read_image(0)
    ctx.set_frame(0, p["dv"][1])          # theta carried over (TPP)
    ctx.reset_optimizer(0)
    ctx.run(4)
    img1 = ctx.read_image(0)
    pr = oracle_problem(p)
    imgs, _, _ = fit.fit_sequence(pr, p["theta0"], p["dv"], [6, 4], 1e-3)
    e0, e1 = rel(img0, imgs[0]), rel(img1, imgs[1])
    record("tpp_two_frames", rel_frame0=e0, rel_frame1=e1)
    assert e0 < 1e-5 and e1 < 1e-5


@pytest.mark.parametrize("prec", PRECS)
def test_graph_replay_matches_eager(lib, probs, prec):
    p = probs["n24_L3_C8"]
    a = make_ctx(lib, [p], prec, graph=False)
    b = make_ctx(lib, [p], prec, graph=True)
    la = [a.run(1)[0] for _ in range(3)]
    lb = [b.run(1)[0] for _ in range(3)]
    # replays with eager work and synchronisation in between
    assert la == lb
    np.testing.assert_array_equal(a.get_params(0), b.get_params(0))
    np.testing.assert_array_equal(a.read_image(0), b.read_image(0))


def test_runs_are_deterministic(lib, probs):
    p = probs["n16_L3_C16_M928"]
    a = make_ctx(lib, [p])
    b = make_ctx(lib, [p])
    a.run(3)
    b.run(3)
    np.testing.assert_array_equal(a.get_params(0), b.get_params(0))
    np.testing.assert_array_equal(a.get_grad(0), b.get_grad(0))


def test_state_save_restore_resumes_exactly(lib, probs):
    p = probs["n16_L2_C8"]
    a = make_ctx(lib, [p])
    a.run(5)
    b = make_ctx(lib, [p])
    b.run(3)
    st, t = b.get_state(0)
    assert t == 3
    c = make_ctx(lib, [p])
    c.set_state(0, st, t)
    c.run(2)
    np.testing.assert_array_equal(a.get_params(0), c.get_params(0))


def test_instances_in_one_context_match_separate(lib, probs):
    p1, p2 = probs["n16_L2_C8"], probs["n24_L3_C8"]
    both = make_ctx(lib, [p1, p2])
    l_both = both.run(3)
    s1 = make_ctx(lib, [p1])
    s2 = make_ctx(lib, [p2])
    assert l_both[0] == s1.run(3)[0]
    assert l_both[1] == s2.run(3)[0]
    np.testing.assert_array_equal(both.get_params(1), s2.get_params(0))


def test_device_inputs_match_host_inputs(lib, probs):
    import torch
    p = probs["n16_L2_C8"]
    a = make_ctx(lib, [p])
    b = lib.Context([(16, p["J"].shape[0])], [(0, 2, 8)])
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    b.set_geometry(0, dev(p["J"]), dev(p["mask"]))
    b.set_params(0, dev(p["theta0"]))
    b.set_noise_input(0, dev(p["Z"]))
    b.set_frame(0, dev(p["dv"][0]))
    assert a.run(2)[0] == b.run(2)[0]
    out = torch.empty(16 ** 3, dtype=torch.float32, device="cuda")
    b.read_image(0, out=out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), a.read_image(0))


def test_error_paths(lib, probs):
    from paper_2507_14046_amd import _lib as L
    p = probs["n16_L2_C8"]
    ctx = lib.Context([(16, 208)], [(0, 2, 8)])
    with pytest.raises(lib.D2ipError) as e:
        ctx.run(1)
    assert e.value.status == L.ESTATE
    ctx.set_geometry(0, p["J"], p["mask"])
    ctx.set_noise_input(0, p["Z"])
    with pytest.raises(lib.D2ipError) as e:
        ctx.run(1)                       # no frame yet
    assert e.value.status == L.ESTATE
    bad = p["dv"][0].copy()
    bad[3] = np.nan
    with pytest.raises(lib.D2ipError) as e:
        ctx.set_frame(0, bad)
    assert e.value.status == L.ENONFINITE
    with pytest.raises(lib.D2ipError) as e:
        ctx.set_adam(lr=-1.0)
    assert e.value.status == L.EINVAL
    ctx.set_frame(0, p["dv"][0])
    ctx.set_params(0, p["theta0"])
    assert np.isfinite(ctx.run(1)[0])


@pytest.fixture(scope="module")
def c1_reference():
    c = ts.CONFIGS["c1"]
    p = problem(c["n"], c["rings"], c["levels"], c["base_ch"], c["seed"])
    pr = oracle_problem(p)
    L0, gref, _ = pr.loss_and_grad(p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64))
    return p, L0, gref


@pytest.mark.parametrize("prec", precs(bf16="pure BF16 operands: 32^3 one-iteration gradient "
                                            "1.9e-2 from the FP64 oracle, worst tensor 0.63"))
def test_full_size_32cubed_one_iteration(lib, c1_reference, prec):
    """The 32^3 / 928-measurement / L=3 / C=16 workload, in both launch
    configurations the benchmark times (captured graph, eager launches on two
    streams): loss and every gradient tensor vs the oracle after one
    iteration, element by element for FP32."""
    p, L0, gref = c1_reference
    c = ts.CONFIGS["c1"]
    for graph in (True, False):
        ctx = make_ctx(lib, [p], prec, graph=graph)
        loss = ctx.run(1)[0]
        g = ctx.get_grad(0)
        ctx.close()
        assert abs(loss - L0) / L0 < TOL_IMG[prec]
        _check_gradient(g, gref, c["levels"], c["base_ch"], prec, "full32_one_iteration",
                        floor_fn=lambda: oracle_gradient_floor(p), p=p,
                        graph=graph, loss_rel=abs(loss - L0) / L0)


@pytest.mark.skip(reason="instance groups (batched launches) are switched off: their first GPU run crashed the host process (SIGSEGV in d2ip_run) and the cause is not yet shown")
def test_group_of_instances_matches_each_alone(lib):
    """Instances sharing geometry, levels and channels run as one group
    (batched launches, J read once for all members); each member must match
    the same instance run alone, bit for bit, across a frame switch."""
    probs = [problem(16, 2, 3, 8, s, frames=2, breathing=True) for s in (21, 22, 23)]
    grp = lib.Context([(16, 928)], [(0, 3, 8)] * 3, graph=True)
    grp.set_geometry(0, probs[0]["J"], probs[0]["mask"])
    for i, p in enumerate(probs):
        grp.load_problem(i, p, set_geometry=False)
    l_grp = grp.run(4)
    for i, p in enumerate(probs):
        grp.set_frame(i, p["dv"][1])
        grp.reset_optimizer(i)
    l_grp2 = grp.run(3)
    for i, p in enumerate(probs):
        one = make_ctx(lib, [p], graph=True)
        assert one.run(4)[0] == l_grp[i]
        one.set_frame(0, p["dv"][1])
        one.reset_optimizer(0)
        assert one.run(3)[0] == l_grp2[i]
        np.testing.assert_array_equal(one.get_params(0), grp.get_params(i))
        np.testing.assert_array_equal(one.read_image(0), grp.read_image(i))


@pytest.mark.skip(reason="instance groups (batched launches) are switched off: their first GPU run crashed the host process (SIGSEGV in d2ip_run) and the cause is not yet shown")
def test_mixed_groups_and_shared_geometry(lib):
    """Two groups on one geometry (different channel counts) plus a group on
    another geometry, as in the uneven batch; compared with the oracle."""
    pa = problem(16, 1, 2, 8, 31)
    pb = problem(16, 1, 2, 16, 32)
    pc = problem(24, 1, 3, 8, 33)
    ctx = lib.Context([(16, 208), (24, 208)], [(0, 2, 8), (0, 2, 16), (1, 3, 8), (0, 2, 8)])
    ctx.set_geometry(0, pa["J"], pa["mask"])
    ctx.set_geometry(1, pc["J"], pc["mask"])
    pd = problem(16, 1, 2, 8, 34)
    for i, p in enumerate([pa, pb, pc, pd]):
        ctx.load_problem(i, p, set_geometry=False)
    ctx.run(3)
    for i, p in enumerate([pa, pb, pc, pd]):
        pr = oracle_problem(p)
        st = fit.State(p["theta0"])
        fit.run(pr, st, p["dv"][0], 3, 1e-3)
        e = rel(ctx.read_image(i), pr.image(st.theta))
        record("mixed_groups", instance=i, image_rel=e)
        assert e < 1e-5


@pytest.mark.parametrize("case", ["n16_L2_C8", "n24_L3_C8"])
def test_every_launch_shape_family_matches_oracle(lib, probs, case):
    """Tuned launch shapes (tiles, channel tiles, chunks, split-K, voxel
    splits) other than the heuristic's give the same gradient: three tables,
    each choosing for every conv pass a different valid shape."""
    from paper_2507_14046_amd import autotune as at
    p = probs[case]
    geos, insts = [(p["n"], p["J"].shape[0])], [(0, p["levels"], p["base_ch"])]
    pr = oracle_problem(p)
    _, gref, _ = pr.loss_and_grad(p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64))
    passes = at.plan_convs(geos, insts)
    try:
        for k in range(3):
            table, seen = [], set()
            for j, e in enumerate(passes):
                cands = [c for c in at.candidates(e) if c != e["shape"]]
                key = (e["n"], e["cin"], e["cout"], e["taps"], e["pass"], e["prologue"])
                if cands and key not in seen:
                    seen.add(key)
                    table.append(dict(e, shape=cands[(7 * k + 3 * j) % len(cands)]))
            at.set_tuning(table)
            lib.check_launches(geos, insts)
            ctx = make_ctx(lib, [p])
            ctx.run(1)
            g = ctx.get_grad(0)
            record("tuned_shapes", case=case, table=k, grad_rel=rel(g, gref))
            assert rel(g, gref) < TOL_GRAD["fp32"], (k, rel(g, gref))
            ctx.close()
    finally:
        at.set_tuning([])


@pytest.mark.parametrize("case", ["n24_L3_C8", "n16_L3_C16_M928"])
def test_largest_split_k_matches_oracle(lib, probs, case):
    """Every forward and input-gradient pass forced to its largest split-K
    (each split stores a partial tile; a second launch sums the splits in
    order and runs the epilogue: bias, residual add, LayerNorm statistics),
    the 3x3x3 ones on every voxel tile in turn, on a ragged and a full grid:
    one-iteration gradient against the oracle, element by element."""
    from paper_2507_14046_amd import autotune as at
    p = probs[case]
    geos, insts = [(p["n"], p["J"].shape[0])], [(0, p["levels"], p["base_ch"])]
    table, splits = [], []
    for j, e in enumerate(at.plan_convs(geos, insts)):
        if e["pass"] == 2:
            continue
        cands = [c for c in at.candidates(e) if c["split"] > 1]
        if not cands:
            continue
        top = max(c["split"] for c in cands)
        cands = [c for c in cands if c["split"] == top]
        table.append(dict(e, shape=cands[j % len(cands)]))
        splits.append(top)
    if not table:
        pytest.skip("no pass here admits split-K")
    pr = oracle_problem(p)
    _, gref, _ = pr.loss_and_grad(p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64))
    try:
        at.set_tuning(table)
        lib.check_launches(geos, insts)
        for graph in (False, True):
            ctx = make_ctx(lib, [p], graph=graph)
            ctx.run(1)
            g = ctx.get_grad(0)
            ctx.close()
            _check_gradient(g, gref, p["levels"], p["base_ch"], "fp32", "largest_split_k",
                            floor_fn=lambda: oracle_gradient_floor(p), p=p, case=case,
                            graph=graph, passes=len(table), max_split=max(splits))
    finally:
        at.set_tuning([])


@pytest.mark.parametrize("prec", precs(bf16=BF16_GRAD))
@pytest.mark.parametrize("ck", [8, 16, 32])
@pytest.mark.parametrize("case", ["n24_L3_C8", "n16_L3_C16_M928"])
def test_weight_gradient_chunks_match_oracle(lib, probs, case, ck, prec):
    """Every 3x3x3 weight gradient forced to one channel chunk (each chunk is
    a kernel of its own: it fixes the halo prefetch and the column tiles each
    wave owns), alternating the fewest and the most voxel splits, on a ragged
    and a full grid: one-iteration gradient, per tensor, against the oracle."""
    from paper_2507_14046_amd import autotune as at
    p = probs[case]
    geos, insts = [(p["n"], p["J"].shape[0])], [(0, p["levels"], p["base_ch"])]
    table = []
    for j, e in enumerate(at.plan_convs(geos, insts, prec)):
        if e["pass"] != 2 or e["taps"] != 27:
            continue
        cands = sorted((c for c in at.candidates(e) if c["ck"] == ck),
                       key=lambda c: (c["split"], c["tile"]))
        if cands:
            table.append(dict(e, shape=cands[-1] if j % 2 else cands[0]))
    if not table:
        pytest.skip("no 3x3x3 weight gradient takes %d-channel chunks here" % ck)
    pr = oracle_problem(p)
    _, gref, _ = pr.loss_and_grad(p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64))
    try:
        at.set_tuning(table)
        lib.check_launches(geos, insts, precision=prec)
        ctx = make_ctx(lib, [p], prec)
        ctx.run(1)
        g = ctx.get_grad(0)
        ctx.close()
    finally:
        at.set_tuning([])
    _check_gradient(g, gref, p["levels"], p["base_ch"], prec, "wgrad_chunks",
                    floor_fn=lambda: oracle_gradient_floor(p), p=p, case=case, ck=ck,
                    passes=len(table))


def test_one_iteration_with_many_j_column_blocks(lib):
    """40^3: the compact J has more than 32 column blocks of 1024 voxels, so
    the residual is formed once by its own kernel before J^T g (the path of
    large grids); one iteration's loss and gradient against the oracle."""
    p = problem(40, 1, 2, 8, 5)
    qa_pad = (int(p["mask"].sum()) + 63) // 64 * 64
    assert (qa_pad + 1023) // 1024 > 32
    ctx = make_ctx(lib, [p])
    loss = ctx.run(1)[0]
    g = ctx.get_grad(0)
    ctx.close()
    pr = oracle_problem(p)
    L0, gref, _ = pr.loss_and_grad(p["theta0"].astype(np.float64), p["dv"][0].astype(np.float64))
    record("many_column_blocks_40", loss_rel=abs(loss - L0) / L0, grad_rel=rel(g, gref))
    assert abs(loss - L0) / L0 < TOL_IMG["fp32"]
    assert rel(g, gref) < TOL_GRAD["fp32"]


def test_standalone_conv_timing(lib):
    from paper_2507_14046_amd import autotune as at
    passes = at.plan_convs([(16, 208)], [(0, 2, 8)])
    for e in passes[:6]:
        ms = at.time_pass(e, e["shape"], reps=3)
        assert 0.0 < ms < 50.0


@pytest.mark.parametrize("graph", [False, pytest.param(True, marks=pytest.mark.skip(
    reason="its run with concurrent instance lanes inside a captured graph crashed the host "
           "process (SIGSEGV in d2ip_run); lanes are now eager-only and the case stays off "
           "until the cause is shown"))])
def test_instances_sharing_a_geometry_match_separate(lib, graph):
    """Two instances on one geometry (each its own launch sequence) give
    bitwise the results of each run alone."""
    pa, pb = problem(16, 1, 2, 8, 41), problem(16, 1, 2, 8, 42)
    both = make_ctx(lib, [pa, pb], graph=graph, shared_geometry=True)
    l_both = both.run(3)
    for i, p in enumerate([pa, pb]):
        one = make_ctx(lib, [p], graph=graph)
        assert one.run(3)[0] == l_both[i]
        np.testing.assert_array_equal(one.get_params(0), both.get_params(i))
        one.close()
    both.close()


@pytest.mark.parametrize("prec", precs(bf16="pure BF16 operands: 32^3 one-iteration gradient "
                                            "1.9e-2 from the FP64 oracle"))
def test_stored_tuning_table_matches_oracle(lib, c1_reference, prec):
    """The chip's stored tuning table (the bench's launch shapes) on the
    full-size 32^3 workload: one-iteration gradient against the oracle."""
    import os
    from paper_2507_14046_amd import autotune as at
    path = at.default_table_path()
    if not os.path.exists(path):
        pytest.skip("no stored tuning table")
    c = ts.CONFIGS["c1"]
    p, _, gref = c1_reference
    try:
        at.set_tuning(at.load_table(path))
        for graph in (True, False):
            ctx = make_ctx(lib, [p], precision=prec, graph=graph)
            ctx.run(1)
            g = ctx.get_grad(0)
            ctx.close()
            _check_gradient(g, gref, c["levels"], c["base_ch"], prec, "stored_table_32cubed",
                            floor_fn=lambda: oracle_gradient_floor(p), p=p,
                            graph=graph)
    finally:
        at.set_tuning([])


@pytest.mark.parametrize("prec", precs(
    bf16x3="BF16x3 along the 500-iteration fit: 2.9e-4 after iteration 1, then 8.6e-3 at 5, "
           "1.3e-2 at 10, 4.8e-2 at 500 (> 2e-3 from iteration 5 on)",
    bf16="pure BF16 along the 500-iteration fit: 1.8e-2 after iteration 1, 0.19 at 500"))
def test_trajectory_500_iterations_32cubed_vs_stored_oracle(lib, prec):
    """The benchmark workload (32^3, 928 measurements, 3 levels, 16 channels,
    500 iterations, eager launches on two streams as the benchmark reports
    them, stored tuning table) against the stored FP64 oracle trajectory; the
    captured-graph run must end on the same image bit for bit.  The oracle's
    own sensitivity (a 1-ulp change of theta_0 moves its image by `floor` at
    iteration 500) bounds what any implementation can match: FP32 must stay
    within 3 x floor at iteration 500.  The BF16 forms are held to the stated
    2e-3 at every stored checkpoint whose oracle floor is at most a third of it
    (all of them here); Adam amplifies any early difference by up to the
    factor the oracle's 1-ulp run shows (about 1400 by iteration 500), which
    their operand rounding cannot survive."""
    import os
    from paper_2507_14046_amd import autotune as at
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_c1_500.npz")
    z = np.load(path)
    c = ts.CONFIGS["c1"]
    p = problem(c["n"], c["rings"], c["levels"], c["base_ch"], c["seed"])
    cps = list(z["checkpoints"])
    ref, flo = z["images"][cps.index(500)], z["floor_images"][cps.index(500)]
    floor = rel(flo, ref)
    amp = floor / rel(z["floor_images"][cps.index(1)], z["images"][cps.index(1)])
    try:
        if os.path.exists(at.default_table_path()):
            at.set_tuning(at.load_table(at.default_table_path()))
        ctx = make_ctx(lib, [p], precision=prec, graph=False)
        losses, imgs = [], {}
        done = 0
        for cp in cps:
            losses.append(ctx.run(cp - done)[0])
            done = cp
            imgs[cp] = ctx.read_image(0)
        ctx.close()
        gctx = make_ctx(lib, [p], precision=prec, graph=True)
        gctx.run(cps[-1])
        np.testing.assert_array_equal(gctx.read_image(0), imgs[cps[-1]])
        gctx.close()
    finally:
        at.set_tuning([])
    e = {int(cp): rel(imgs[cp], z["images"][i]) for i, cp in enumerate(cps)}
    lrel = [abs(l - z["losses"][cp - 1]) / z["losses"][cp - 1] for l, cp in zip(losses, cps)]
    record("trajectory500_32cubed", prec=prec, image_rel=e, floor=floor, amplification=amp,
           loss_rel=lrel)
    assert e[1] < TOL_IMG[prec], e
    if prec == "fp32":
        assert e[500] < 3 * floor, (e[500], floor)
    else:
        floors = {int(cp): rel(z["floor_images"][i], z["images"][i]) for i, cp in enumerate(cps)}
        for cp, err in e.items():
            if floors[cp] <= TOL_IMG[prec] / 3:
                assert err <= TOL_IMG[prec], (cp, err, e)
