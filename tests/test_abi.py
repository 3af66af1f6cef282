"""Host-side checks of the C-ABI library: it loads, exports every function the
header declares, and its host-only entry points validate their arguments.
No compute call is made (no GPU needed)."""
import ctypes
import os
import re

import pytest

import tseit_synth as ts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "d2ip.h")


@pytest.fixture(scope="module")
def L():
    from paper_2507_14046_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libd2ip.so not built")
    _lib.load()
    return _lib


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(d2ip_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each compute entry point
    for name in names:
        if name != "d2ip_last_error":
            assert name in L.SIGNATURES, name


@pytest.mark.parametrize("L_,C", [(2, 8), (3, 16), (4, 32), (3, 8), (2, 16), (5, 16)])
def test_param_count_matches_generator(L, L_, C):
    from paper_2507_14046_amd import param_count
    assert param_count(L_, C) == ts.param_count(L_, C)


def test_workspace_bytes_and_validation(L):
    from paper_2507_14046_amd import workspace_bytes, D2ipError
    b1 = workspace_bytes([(32, 928)], [(0, 3, 16)])
    b2 = workspace_bytes([(32, 928)], [(0, 3, 16), (0, 3, 16)])
    assert b1 > 121 * 2 ** 20          # at least the J buffer
    assert b2 > b1
    assert b1 % 256 == 0
    assert workspace_bytes([(32, 928)], [(0, 3, 16)], precision="bf16") > 0
    bad = [
        ([(32, 928)], [(0, 1, 16)]),      # levels < 2
        ([(32, 928)], [(0, 3, 12)]),      # base_ch not 8/16/32
        ([(30, 928)], [(0, 3, 16)]),      # 30 not divisible by 4
        ([(32, 928)], [(1, 3, 16)]),      # bad geometry index
        ([(32, 0)], [(0, 3, 16)]),        # M = 0
        ([(8, 10)], [(0, 3, 16)]),        # coarsest level 2^3 -> 2 ok? 8/4 = 2 -> fine
    ]
    for geos, insts in bad[:-1]:
        with pytest.raises(D2ipError) as e:
            workspace_bytes(geos, insts)
        assert e.value.status == L.EINVAL
        assert len(L.load().d2ip_last_error()) > 0
    assert workspace_bytes(*bad[-1]) > 0
    with pytest.raises(ValueError):
        workspace_bytes([(32, 928)], [(0, 3, 16)], precision="fp8")


def test_null_pointer_errors(L):
    lib = L.load()
    assert lib.d2ip_param_count(3, 16, None) == L.EINVAL
    assert lib.d2ip_run(None, 1, None) == L.EINVAL
    assert lib.d2ip_read_image(None, 0, None, 0) == L.EINVAL
    assert lib.d2ip_destroy(None) == L.OK
    out = ctypes.c_void_p()
    g = (L.GeometryDesc * 1)(L.GeometryDesc(16, 208))
    i = (L.InstanceDesc * 1)(L.InstanceDesc(0, 2, 8))
    # null workspace
    assert lib.d2ip_create(g, 1, i, 1, 0, 0, None, 0, None, ctypes.byref(out)) == L.EINVAL
    assert b"workspace" in lib.d2ip_last_error()


def _workload(name):
    """(geometries, instances) of one named workload, one geometry per distinct grid."""
    c = ts.CONFIGS[name]
    M = {1: 208, 2: 928}
    if name == "c4":
        geos, insts = [], []
        for inst in c["instances"]:
            g = (inst["n"], M[inst["rings"]])
            if g not in geos:
                geos.append(g)
            insts.append((geos.index(g), c["levels"], inst["base_ch"]))
        return geos, insts
    geos = [(c["n"], M[c["rings"]])]
    return geos, [(0, c["levels"], c["base_ch"])] * c.get("sequences", 1)


@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3", "c4"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
def test_every_launch_stays_inside_the_workspace(L, name, prec):
    """Host-only walk of one iteration's launch schedule: each kernel
    argument's extent, implied by its shapes, lies in one workspace
    allocation (all instances, eager and graph plans)."""
    import paper_2507_14046_amd as d2ip
    geos, insts = _workload(name)
    for graph in (False, True):
        d2ip.check_launches(geos, insts, prec, graph=graph)


def _shape_tables(geos, insts, k):
    """The k-th table of non-heuristic shapes (same choice as the GPU test)."""
    from paper_2507_14046_amd import autotune as at
    at.set_tuning([])
    passes = at.plan_convs(geos, insts)
    table, seen = [], set()
    for j, e in enumerate(passes):
        cands = [c for c in at.candidates(e) if c != e["shape"]]
        key = (e["n"], e["cin"], e["cout"], e["taps"], e["pass"], e["prologue"])
        if cands and key not in seen:
            seen.add(key)
            table.append(dict(e, shape=cands[(7 * k + 3 * j) % len(cands)]))
    return table


@pytest.mark.parametrize("geo,inst", [((16, 208), (0, 2, 8)), ((24, 928), (0, 3, 8)),
                                      ((32, 928), (0, 3, 16))])
def test_tuning_tables_plan_and_stay_in_bounds(L, geo, inst):
    from paper_2507_14046_amd import autotune as at
    import paper_2507_14046_amd as d2ip
    try:
        for k in range(3):
            table = _shape_tables([geo], [inst], k)
            at.set_tuning(table)
            got = {(e["n"], e["cin"], e["cout"], e["taps"], e["pass"], e["prologue"]): e["shape"]
                   for e in at.plan_convs([geo], [inst])}
            for e in table:
                key = (e["n"], e["cin"], e["cout"], e["taps"], e["pass"], e["prologue"])
                assert got[key] == e["shape"]
            for prec in ("fp32", "bf16x3", "bf16"):
                d2ip.check_launches([geo], [inst], prec, graph=True)
    finally:
        at.set_tuning([])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("geo,inst", [((24, 928), (0, 3, 8)), ((32, 928), (0, 3, 16)),
                                      ((64, 928), (0, 4, 32))])
def test_weight_gradient_chunks_and_splits_stay_in_bounds(L, geo, inst, prec):
    """Every 3x3x3 weight gradient at each channel chunk, with the fewest and
    the most voxel splits the tiles allow (up to 256): launches stay inside
    the workspace."""
    from paper_2507_14046_amd import autotune as at
    import paper_2507_14046_amd as d2ip
    passes = [e for e in at.plan_convs([geo], [inst], prec) if e["pass"] == 2 and e["taps"] == 27]
    try:
        for ck in (8, 16, 32):
            for pick in (0, -1):
                table = []
                for e in passes:
                    cands = sorted((c for c in at.candidates(e) if c["ck"] == ck),
                                   key=lambda c: (c["split"], c["tile"]))
                    if cands:
                        table.append(dict(e, shape=cands[pick]))
                if not table:
                    continue
                at.set_tuning(table)
                d2ip.check_launches([geo], [inst], prec, graph=True)
                big = [e["shape"]["split"] for e in table if e["n"] >= 32]
                if pick == -1 and big:
                    assert max(big) > 64
    finally:
        at.set_tuning([])


def test_tuning_entry_validation(L):
    from paper_2507_14046_amd import autotune as at
    e = at.plan_convs([(32, 928)], [(0, 3, 16)])[2]
    bad = [dict(tile=0, bn=64, ck=16, split=1), dict(tile=3, bn=16, ck=16, split=1),
           dict(tile=1, bn=16, ck=12, split=1), dict(tile=1, bn=16, ck=16, split=3),
           dict(tile=0, bn=32, ck=16, split=1)]  # the last is over the LDS budget
    for sh in bad:
        with pytest.raises(Exception):
            at.set_tuning([dict(e, shape=sh)])
    assert at.plan_convs([(32, 928)], [(0, 3, 16)])[2]["shape"] == e["shape"]


def test_stored_tuning_table_plans_every_workload(L):
    """The chip's stored table is valid and keeps every launch in bounds."""
    import os
    from paper_2507_14046_amd import autotune as at
    import paper_2507_14046_amd as d2ip
    path = at.default_table_path()
    if not os.path.exists(path):
        pytest.skip("no stored tuning table")
    try:
        at.set_tuning(at.load_table(path))
        for w in at.WORKLOADS:
            geos, insts = at.workload(w)
            for prec in at.PRECISIONS:
                d2ip.check_launches(geos, insts, prec, graph=True)
    finally:
        at.set_tuning([])


def test_tuning_table_update_keeps_order_and_format(tmp_path):
    """`update` puts re-tuned entries in place of the stored ones with the same
    pass key (the stored order kept), appends passes the table lacked, and
    `save` writes the stored table's one-key-per-line format, so a partial
    re-tune rewrites only the entries it changed."""
    import json
    from paper_2507_14046_amd import autotune as at
    key = dict(n=16, cin=8, cout=8, taps=27, prologue=0, precision=0)
    base = [dict(key, **{"pass": p}, shape=dict(tile=2, bn=16, ck=8, split=1), ms=0.01)
            for p in (0, 1, 2)]
    new = [dict(key, **{"pass": 1}, shape=dict(tile=1, bn=16, ck=8, split=4), ms=0.005),
           dict(key, n=8, **{"pass": 0}, shape=dict(tile=2, bn=16, ck=8, split=1), ms=0.002)]
    out = at.update(base, new)
    assert [at._key(e) for e in out] == [at._key(e) for e in base] + [at._key(new[1])]
    assert out[0] == base[0] and out[2] == base[2] and out[1] == new[0]
    path = tmp_path / "t.json"
    at.save(out, str(path))
    text = path.read_text()
    assert json.loads(text) == out
    assert text.startswith('[\n{\n"n": 16,')


@pytest.mark.parametrize("L_,C", [(2, 8), (3, 16), (4, 32)])
@pytest.mark.parametrize("sep", [False, True])
@pytest.mark.parametrize("r", [0, 4, 64])
@pytest.mark.parametrize("att,aspp", [(False, False), (True, False), (True, True)])
def test_operator_network_layout_matches_oracle(L, L_, C, sep, r, att, aspp):
    """The autograd network's flat parameter order (dense or depthwise-separable
    ResBlock convs, with or without SE units) is the oracle's, tensor by
    tensor."""
    import numpy as np
    from oracle import net
    from paper_2507_14046_amd import ops
    mine = [int(np.prod(s)) for _, s in ops.param_shapes(L_, C, sep, r, att, aspp)]
    ref = [int(np.prod(s)) for _, ps in net.module_list(L_, C, sep, r, att, aspp=aspp)
           for _, s in ps]
    assert ops.ASPP_RATES == net.ASPP_RATES
    assert mine == ref


def test_misaligned_parameter_views_are_copied_for_the_float4_kernels(L):
    """Views into a flat parameter vector can start off a 16-byte boundary;
    the autograd wrappers hand the float4 kernels aligned copies of those."""
    import torch
    from paper_2507_14046_amd import ops
    flat = torch.zeros(1001)
    for off in range(4):
        v = flat[off + 1:off + 1 + 64].view(8, 8)
        a = ops._a16(v)
        assert a.data_ptr() % 16 == 0 and torch.equal(a, v)
    assert ops._a16(None) is None


def test_module_operators_validate_their_arguments(L):
    """The depthwise, atrous, pointwise and SE entry points reject bad sizes,
    null and misaligned pointers and short workspaces before touching the
    device (every call below returns an error from host checks alone)."""
    lib = L.load()
    nb = ctypes.c_size_t()
    sz = ctypes.byref(nb)
    for args in ((8, 6), (0, 8), (257, 8), (8, 2048), (8, 0)):
        assert lib.d2ip_op_dwconv3d_bytes(*args, sz) == L.EINVAL, args
    assert lib.d2ip_op_dwconv3d_bytes(8, 16, None) == L.EINVAL
    for args in ((8, 16, 0), (8, 16, 300), (8, 6, 2)):
        assert lib.d2ip_op_dwconv3d_dilated_bytes(*args, sz) == L.EINVAL, args
    for args in ((8, 6, 8), (8, 8, 2048), (0, 8, 8), (8, 4, 2)):
        assert lib.d2ip_op_pwconv3d_bytes(*args, sz) == L.EINVAL, args
    for args in ((8, 16, 0), (8, 16, 300), (8, 6, 4), (8, 2048, 4)):
        assert lib.d2ip_op_se_bytes(*args, sz) == L.EINVAL, args
    for ok in ((8, 16), (1, 4), (256, 1024)):
        assert lib.d2ip_op_dwconv3d_bytes(*ok, sz) == L.OK and nb.value > 0
    assert lib.d2ip_op_pwconv3d_bytes(8, 4, 4, sz) == L.OK and nb.value > 0
    assert lib.d2ip_op_se_bytes(8, 1024, 256, sz) == L.OK and nb.value > 0
    P = ctypes.c_void_p
    a, odd = P(4096), P(4100)  # never dereferenced: the checks fail first
    # null and misaligned operands
    assert lib.d2ip_op_dwconv3d_forward(None, a, None, a, 8, 16, None) == L.EINVAL
    assert lib.d2ip_op_dwconv3d_forward(odd, a, None, a, 8, 16, None) == L.EINVAL
    assert b"aligned" in lib.d2ip_last_error()
    assert lib.d2ip_op_dwconv3d_dilated_forward(a, a, None, odd, 8, 16, 2, None) == L.EINVAL
    assert lib.d2ip_op_pwconv3d_forward(a, odd, None, a, 8, 16, 16, None) == L.EINVAL
    assert lib.d2ip_op_se_forward(a, a, a, a, a, None, 8, 16, 4, a, 1 << 30, None) == L.EINVAL
    # gradients that need x without x, gx without w
    assert lib.d2ip_op_dwconv3d_backward(None, a, a, None, a, None, 8, 16, a, 1 << 30,
                                         None) == L.EINVAL
    assert lib.d2ip_op_pwconv3d_backward(a, None, a, a, None, None, 8, 16, 16, None, 0,
                                         None) == L.EINVAL
    # short workspaces
    assert lib.d2ip_op_dwconv3d_backward(a, a, a, None, a, None, 8, 16, a, 1, None) == L.ENOMEM
    assert lib.d2ip_op_dwconv3d_dilated_backward(a, a, a, None, a, None, 8, 16, 2, a, 1,
                                                 None) == L.ENOMEM
    assert lib.d2ip_op_pwconv3d_backward(a, a, a, None, a, None, 8, 16, 16, a, 1,
                                         None) == L.ENOMEM
    assert lib.d2ip_op_se_backward(a, a, a, a, a, a, a, None, None, None, None, 8, 16, 4, a, 1,
                                   None) == L.ENOMEM
    assert b"workspace too small" in lib.d2ip_last_error()


def test_network_module_operators_validate_their_arguments(L):
    """Pooling, up-sampling/concatenation, channel copy, ReLU, head and
    attention entry points reject bad sizes, null, misaligned and overlapping
    pointers and short workspaces from host checks alone; empty inputs are a
    no-op."""
    lib = L.load()
    nb = ctypes.c_size_t()
    sz = ctypes.byref(nb)
    P = ctypes.c_void_p
    a, b2, odd = P(4096), P(1 << 20), P(4100)  # never dereferenced
    assert lib.d2ip_op_pool2_forward(a, b2, 7, 16, None) == L.EINVAL
    assert lib.d2ip_op_pool2_forward(a, b2, 8, 6, None) == L.EINVAL
    assert lib.d2ip_op_pool2_backward(odd, b2, 8, 16, None) == L.EINVAL
    assert lib.d2ip_op_up2_concat_forward(a, 16, None, 8, 8, b2, None) == L.EINVAL
    assert lib.d2ip_op_up2_concat_backward(a, 16, 6, 8, b2, b2, None) == L.EINVAL
    # channel copy: ranges, multiples of 4, overlap, alignment
    assert lib.d2ip_op_channel_copy(a, 16, 8, b2, 32, 0, 12, 10, None) == L.EINVAL
    assert b"exceeds" in lib.d2ip_last_error()
    assert lib.d2ip_op_channel_copy(a, 16, 2, b2, 32, 0, 8, 10, None) == L.EINVAL
    assert lib.d2ip_op_channel_copy(a, 16, 0, P(4096 + 64), 32, 0, 16, 10, None) == L.EINVAL
    assert b"overlap" in lib.d2ip_last_error()
    assert lib.d2ip_op_channel_copy(odd, 16, 0, b2, 32, 0, 16, 10, None) == L.EINVAL
    assert lib.d2ip_op_channel_copy(a, 16, 0, b2, 32, 16, 16, 0, None) == L.OK
    # ReLU
    assert lib.d2ip_op_relu_forward(a, b2, 6, None) == L.EINVAL
    assert lib.d2ip_op_relu_forward(odd, b2, 8, None) == L.EINVAL
    assert lib.d2ip_op_relu_backward(a, None, b2, 8, None) == L.EINVAL
    assert lib.d2ip_op_relu_forward(a, b2, 0, None) == L.OK
    # head
    for args in ((8, 6), (8, 512), (0, 8), (600, 8)):
        assert lib.d2ip_op_head_bytes(*args, sz) == L.EINVAL, args
    assert lib.d2ip_op_head_bytes(8, 16, sz) == L.OK and nb.value > 0
    assert lib.d2ip_op_head_forward(a, odd, a, None, b2, 8, 16, 0, None) == L.EINVAL
    assert lib.d2ip_op_head_backward(a, a, a, None, a, b2, None, None, 8, 16, 1, a, 1,
                                     None) == L.ENOMEM
    # attention
    for args in ((7, 8, 16), (8, 260, 16), (8, 8, 516), (8, 6, 16), (0, 8, 8)):
        assert lib.d2ip_op_attention_bytes(*args, sz) == L.EINVAL, args
    assert lib.d2ip_op_attention_bytes(16, 64, 128, sz) == L.OK and nb.value > 0
    assert lib.d2ip_op_attention_bytes(16, 256, 512, sz) == L.OK and nb.value > 0
    assert lib.d2ip_op_attention_forward(a, a, a, a, a, a, None, b2, None, 8, 8, 16, a, 1 << 30,
                                         None) == L.EINVAL
    assert lib.d2ip_op_attention_forward(a, a, a, a, a, a, a, b2, None, 8, 128, 16, a, 1,
                                         None) == L.ENOMEM
    assert lib.d2ip_op_attention_backward(a, a, a, a, a, a, a, a, b2, None, None, None, None,
                                          None, None, 8, 8, 16, a, 1, None) == L.ENOMEM


@pytest.mark.parametrize("L_,C", [(3, 16), (4, 32), (2, 8)])
def test_kaiming_initialiser_moments(L, L_, C):
    """d2ip_init_params_host (Sec. III-B, Kaiming): every conv weight tensor
    has mean 0 and variance 2 / fan_in (fan_in = Cin * taps) within sampling
    error, biases 0, LayerNorm gamma 1 and beta 0 -- tensors found through the
    oracle's own parameter layout."""
    import numpy as np
    from oracle import net
    from paper_2507_14046_amd.context import kaiming_params
    th = kaiming_params(L_, C, 12345).astype(np.float64)
    mods = net.unpack(th, L_, C)
    n_w = 0
    for mod, ps in mods.items():
        for name, t in ps.items():
            if name.endswith("w") and t.ndim == 5:
                fan_in = t.shape[1] * t.shape[2] * t.shape[3] * t.shape[4]
                var = 2.0 / fan_in
                N = t.size
                assert abs(t.mean()) < 6 * np.sqrt(var / N), (mod, name)
                # the sample variance of N normals has relative sd sqrt(2 / N)
                assert abs(t.var() / var - 1) < 6 * np.sqrt(2.0 / N) + 1e-12, (mod, name)
                n_w += 1
            elif name.endswith("b") and not name.endswith("beta"):
                assert np.all(t == 0), (mod, name)
            elif name.endswith(".g"):
                assert np.all(t == 1), (mod, name)
            elif name.endswith("beta"):
                assert np.all(t == 0), (mod, name)
    assert n_w == 2 + 2 * (2 * L_ - 1) + sum(1 for l in range(L_) if l > 0) + (L_ - 1)


def test_kaiming_initialiser_is_seeded(L):
    import numpy as np
    from paper_2507_14046_amd.context import kaiming_params
    from paper_2507_14046_amd import D2ipError
    a, b, c = (kaiming_params(3, 8, s) for s in (1, 1, 2))
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    # the draws are standard normal overall: a Kolmogorov-Smirnov check on the
    # largest weight tensor rescaled to unit variance
    from scipy import stats
    from oracle import net
    w = net.unpack(kaiming_params(4, 32, 7).astype(np.float64), 4, 32)["dec0"]["conv1.w"]
    z = (w / np.sqrt(2.0 / (w.shape[1] * 27))).ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-4
    out = (ctypes.c_float * 10)()
    with pytest.raises(D2ipError):
        L.check(L.load().d2ip_init_params_host(3, 8, 1, out, 10))


def test_runtime_versions_are_reported(L):
    from paper_2507_14046_amd.context import runtime_versions
    compiled, loaded = runtime_versions()
    assert compiled >= 70000000  # ROCm 7 headers
    assert loaded >= 0


MODULE_MIXES = [dict(), dict(sep=True), dict(se_ratio=4), dict(att=True), dict(aspp=True),
                dict(sep=True, se_ratio=4, att=True, aspp=True)]


@pytest.mark.parametrize("kw", MODULE_MIXES)
@pytest.mark.parametrize("L_,C", [(2, 8), (3, 16), (4, 16)])
def test_module_network_layout_matches_the_canonical_order(L, L_, C, kw):
    """d2ip_mnet_param_count equals the flat layout the autograd network and
    the oracle use, for every module mix (host only)."""
    import numpy as np
    from oracle import net
    from paper_2507_14046_amd import ops
    from paper_2507_14046_amd.context import module_param_count
    want = int(sum(np.prod(s) for _, s in ops.param_shapes(L_, C, **kw)))
    assert module_param_count(L_, C, **kw) == want
    assert net.n_params(L_, C, kw.get("sep", False), kw.get("se_ratio", 0), kw.get("att", False),
                        kw.get("aspp", False)) == want


def test_module_network_validates_its_description(L):
    """Bad descriptions and short or misaligned workspaces are rejected by
    host checks before anything touches the device."""
    lib = L.load()
    sz = ctypes.c_size_t()
    ok = L.MnetDesc(16, 208, 3, 8, 1, 4, 1, 1, 1, 1)
    assert lib.d2ip_mnet_workspace_bytes(ctypes.byref(ok), ctypes.byref(sz)) == L.OK
    assert sz.value > 208 * 16 ** 3 * 4
    for bad in (L.MnetDesc(16, 208, 1, 8, 0, 0, 0, 0, 0, 0), L.MnetDesc(16, 208, 3, 12, 0, 0, 0, 0, 0, 0),
                L.MnetDesc(6, 208, 3, 8, 0, 0, 0, 0, 0, 0), L.MnetDesc(16, 0, 3, 8, 0, 0, 0, 0, 0, 0),
                L.MnetDesc(16, 208, 3, 8, 0, -1, 0, 0, 0, 0),
                L.MnetDesc(64, 208, 5, 32, 0, 0, 1, 0, 0, 0)):  # 512 channels at the bottleneck
        assert lib.d2ip_mnet_workspace_bytes(ctypes.byref(bad), ctypes.byref(sz)) == L.EINVAL
    h = ctypes.c_void_p()
    assert lib.d2ip_mnet_create(ctypes.byref(ok), ctypes.c_void_p(4096), 1024, None,
                                ctypes.byref(h)) == L.ENOMEM
    assert lib.d2ip_mnet_create(ctypes.byref(ok), ctypes.c_void_p(4100), 1 << 40, None,
                                ctypes.byref(h)) == L.EINVAL
    assert lib.d2ip_mnet_run(None, 1, None) == L.EINVAL
    assert lib.d2ip_mnet_destroy(None) == L.OK
