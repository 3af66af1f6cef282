"""The allocation-free J^T entry point (d2ip_op_jt_noalloc) through the C-ABI.

Its output must equal d2ip_op_jt's (same kernels, same summation order: bit
for bit) on two calls in a row, the second with a smaller input, so that the
static scratch array's leftover contents from the first call cannot leak into
the second.  Sizes beyond the static scratch are rejected on the host.
"""
import ctypes

import numpy as np
import pytest


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import os
    from paper_2507_14046_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libd2ip.so not built")
    lib = L.load()
    # host-side checks: nothing is enqueued, no device is touched
    buf = ctypes.c_void_p(256)
    assert lib.d2ip_op_jt_noalloc(buf, buf, buf, 8, 64 ** 3 + 4, None) == L.EINVAL
    assert b"static scratch" in lib.d2ip_last_error()
    assert lib.d2ip_op_jt_noalloc(buf, buf, buf, 8, 6, None) == L.EINVAL
    assert lib.d2ip_op_jt_noalloc(None, buf, buf, 8, 64, None) == L.EINVAL
    assert lib.d2ip_op_jt_noalloc(ctypes.c_void_p(260), buf, buf, 8, 64, None) == L.EINVAL


@pytest.mark.gpu
def test_noalloc_jt_matches_workspace_jt_on_two_calls(lib):
    import torch
    from paper_2507_14046_amd import _lib as L
    lib = L.load()
    dev = torch.device("cuda", 0)
    st = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(st.cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    rng = np.random.default_rng(77)
    # the full 64^3 / 928-measurement size first, then a smaller, ragged one
    for M, Q in ((928, 64 ** 3), (208, 24 ** 3 + 4)):
        print("noalloc J^T: M %d, Q %d" % (M, Q), flush=True)
        J = torch.tensor(rng.standard_normal((M, Q), dtype=np.float32), device=dev)
        g = torch.tensor(rng.standard_normal(M, dtype=np.float32), device=dev)
        ref = torch.empty(Q, device=dev)
        out = torch.full((Q,), float("nan"), device=dev)
        nb = ctypes.c_size_t()
        L.check(lib.d2ip_op_jt_bytes(M, Q, ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        L.check(lib.d2ip_op_jt(P(J), P(g), P(ref), M, Q, P(ws), nb.value, sp))
        L.check(lib.d2ip_op_jt_noalloc(P(J), P(g), P(out), M, Q, sp))
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
        # and both are J^T g (FP64 host product of the same operands)
        Jh, gh = J.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
        want = Jh.T @ gh
        err = np.max(np.abs(a - want)) / np.max(np.abs(want))
        assert err < 1e-5, err
