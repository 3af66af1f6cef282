"""Python front end of libd2ip: a thin marshalling layer over the C-ABI.

Device memory (the workspace) and the stream come from PyTorch; every step of
the fitting iteration runs in the library's HIP kernels.
"""
import ctypes

import numpy as np

from . import _lib as L


def param_count(levels, base_ch):
    lib = L.load()
    out = ctypes.c_size_t()
    L.check(lib.d2ip_param_count(levels, base_ch, ctypes.byref(out)))
    return out.value


def kaiming_params(levels, base_ch, seed):
    """Kaiming-initialised theta drawn by the library (host only)."""
    lib = L.load()
    out = np.empty(param_count(levels, base_ch), dtype=np.float32)
    L.check(lib.d2ip_init_params_host(levels, base_ch, int(seed),
                                      out.ctypes.data_as(ctypes.c_void_p), out.size))
    return out


def runtime_versions():
    """(HIP_VERSION compiled against, version of the HIP runtime in this process)."""
    lib = L.load()
    c, r = ctypes.c_int(), ctypes.c_int()
    L.check(lib.d2ip_runtime_versions(ctypes.byref(c), ctypes.byref(r)))
    return c.value, r.value


def _descs(geometries, instances):
    G = (L.GeometryDesc * len(geometries))(*[L.GeometryDesc(int(n), int(M)) for n, M in geometries])
    I = (L.InstanceDesc * len(instances))(*[L.InstanceDesc(int(g), int(lv), int(c))
                                            for g, lv, c in instances])
    return G, I


def workspace_bytes(geometries, instances, precision="fp32", graph=False):
    lib = L.load()
    G, I = _descs(geometries, instances)
    out = ctypes.c_size_t()
    L.check(lib.d2ip_workspace_bytes(G, len(geometries), I, len(instances),
                                     _prec(precision), L.FLAG_GRAPH if graph else 0,
                                     ctypes.byref(out)))
    return out.value


def check_launches(geometries, instances, precision="fp32", graph=False):
    """Host-only launch-extent check of one iteration (raises D2ipError)."""
    lib = L.load()
    G, I = _descs(geometries, instances)
    L.check(lib.d2ip_check_launches(G, len(geometries), I, len(instances), _prec(precision),
                                    L.FLAG_GRAPH if graph else 0))


def _prec(p):
    if p in ("fp32", L.PLAIN_FP32):
        return L.PLAIN_FP32
    if p in ("bf16", L.BF16_CONV):
        return L.BF16_CONV
    if p in ("bf16x3", L.BF16X3_CONV):
        return L.BF16X3_CONV
    raise ValueError("precision must be 'fp32', 'bf16' or 'bf16x3'")


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _in(x, dtype):
    """(pointer, on_device, keepalive) for an input array."""
    if _is_torch(x):
        import torch
        tdt = {np.float32: torch.float32, np.uint8: torch.uint8}[dtype]
        if x.dtype != tdt:
            raise TypeError("expected %s tensor" % tdt)
        if not x.is_cuda:
            x = x.contiguous().numpy()
        else:
            x = x.contiguous()
            return ctypes.c_void_p(x.data_ptr()), 1, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), 0, a


class Context:
    """Geometries + instances fitted together; see include/d2ip.h.

    geometries: list of (n, M); instances: list of (geometry, levels, base_ch).
    """

    def __init__(self, geometries, instances, precision="fp32", graph=False, device=0,
                 stream=None):
        import torch
        self._lib = L.load()
        self.geometries = [tuple(g) for g in geometries]
        self.instances = [tuple(i) for i in instances]
        self.precision = precision
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        nbytes = workspace_bytes(geometries, instances, precision, graph)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        G, I = _descs(geometries, instances)
        ctx = ctypes.c_void_p()
        L.check(self._lib.d2ip_create(G, len(geometries), I, len(instances), _prec(precision),
                                      L.FLAG_GRAPH if graph else 0,
                                      ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx
        self.n_params = [param_count(lv, c) for _, lv, c in self.instances]

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.d2ip_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- inputs ---------------------------------------------------------------
    def set_geometry(self, geo, J, mask):
        jp, jd, _k1 = _in(J, np.float32)
        mp, md, _k2 = _in(mask, np.uint8)
        if jd != md:
            raise ValueError("J and mask must both be host arrays or both device tensors")
        L.check(self._lib.d2ip_set_geometry(self._ctx, geo, jp, mp, jd))

    def set_params(self, inst, theta):
        p, d, _k = _in(theta, np.float32)
        L.check(self._lib.d2ip_set_params(self._ctx, inst, p, self.n_params[inst], d))

    def init_params(self, inst, seed):
        """Kaiming-initialised theta from the library's generator (Sec. III-B)."""
        L.check(self._lib.d2ip_init_params(self._ctx, inst, int(seed)))

    def set_noise_input(self, inst, z):
        p, d, _k = _in(z, np.float32)
        L.check(self._lib.d2ip_set_noise_input(self._ctx, inst, p, d))

    def set_frame(self, inst, dv):
        p, d, _k = _in(dv, np.float32)
        L.check(self._lib.d2ip_set_frame(self._ctx, inst, p, d))

    def set_adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        cfg = L.AdamCfg(lr, beta1, beta2, eps)
        L.check(self._lib.d2ip_set_adam(self._ctx, ctypes.byref(cfg)))

    def set_tv(self, lambda_tv=0.002, lambda_s=1.0, lambda_t=0.1, eps=1e-8):
        """4D-TV coefficients (lambda_tv = 0 switches the term off)."""
        cfg = L.TvCfg(lambda_tv, lambda_s, lambda_t, eps)
        L.check(self._lib.d2ip_set_tv(self._ctx, ctypes.byref(cfg)))

    def commit_frame(self, inst):
        """The image at the current theta joins the temporal history."""
        L.check(self._lib.d2ip_commit_frame(self._ctx, inst))

    def clear_history(self, inst):
        L.check(self._lib.d2ip_clear_history(self._ctx, inst))

    def reset_optimizer(self, inst):
        L.check(self._lib.d2ip_reset_optimizer(self._ctx, inst))

    # -- outputs --------------------------------------------------------------
    def get_params(self, inst):
        out = np.empty(self.n_params[inst], dtype=np.float32)
        L.check(self._lib.d2ip_get_params(self._ctx, inst, out.ctypes.data_as(ctypes.c_void_p),
                                          out.size, 0))
        return out

    def get_grad(self, inst):
        out = np.empty(self.n_params[inst], dtype=np.float32)
        L.check(self._lib.d2ip_get_grad(self._ctx, inst, out.ctypes.data_as(ctypes.c_void_p),
                                        out.size, 0))
        return out

    def get_state(self, inst):
        P = self.n_params[inst]
        out = np.empty(3 * P, dtype=np.float32)
        t = ctypes.c_int64()
        L.check(self._lib.d2ip_get_state(self._ctx, inst, out.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(t), 0))
        return out, t.value

    def set_state(self, inst, theta_m_v, t):
        p, d, _k = _in(theta_m_v, np.float32)
        L.check(self._lib.d2ip_set_state(self._ctx, inst, p, int(t), d))

    def run(self, k, sync=True):
        """k iterations of every instance; returns the last losses if sync."""
        if not sync:
            L.check(self._lib.d2ip_run(self._ctx, k, None))
            return None
        out = (ctypes.c_double * len(self.instances))()
        L.check(self._lib.d2ip_run(self._ctx, k, out))
        return np.array(out[:], dtype=np.float64)

    def read_image(self, inst, out=None):
        n = self.geometries[self.instances[inst][0]][0]
        if out is not None:
            import torch
            if out.dtype != torch.float32 or not out.is_cuda or out.numel() != n ** 3 \
                    or not out.is_contiguous():
                raise TypeError("out must be a contiguous float32 device tensor of n^3 values")
            L.check(self._lib.d2ip_read_image(self._ctx, inst, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        img = np.empty(n ** 3, dtype=np.float32)
        L.check(self._lib.d2ip_read_image(self._ctx, inst, img.ctypes.data_as(ctypes.c_void_p), 0))
        return img

    def time_kernel(self, inst, which, block=0, reps=20):
        """Mean ms per launch of one kernel (see d2ip_time_kernel)."""
        ms = ctypes.c_double()
        L.check(self._lib.d2ip_time_kernel(self._ctx, inst, which, block, reps, ctypes.byref(ms)))
        return ms.value

    # -- convenience ----------------------------------------------------------
    def load_problem(self, inst, prob, frame=0, set_geometry=True):
        """Upload one tseit_synth problem dict into instance `inst`."""
        if set_geometry:
            self.set_geometry(self.instances[inst][0], prob["J"], prob["mask"])
        self.set_params(inst, prob["theta0"])
        self.set_noise_input(inst, prob["Z"])
        self.set_frame(inst, prob["dv"][frame])


def _mnet_desc(n, M, levels, base_ch, sep=False, se_ratio=0, att=False, tail="linear",
               aspp=False, graph=False):
    if tail not in ("linear", "sigmoid"):
        raise ValueError("tail must be 'linear' or 'sigmoid'")
    return L.MnetDesc(int(n), int(M), int(levels), int(base_ch), int(bool(sep)), int(se_ratio),
                      int(bool(att)), int(tail == "sigmoid"), int(bool(aspp)), int(bool(graph)))


def module_param_count(levels, base_ch, sep=False, se_ratio=0, att=False, aspp=False, n=None):
    """Parameters of the 3D-FastResUNet variant (the grid does not matter)."""
    lib = L.load()
    d = _mnet_desc(n or (4 << levels), 1, levels, base_ch, sep, se_ratio, att, "linear", aspp)
    out = ctypes.c_size_t()
    L.check(lib.d2ip_mnet_param_count(ctypes.byref(d), ctypes.byref(out)))
    return out.value


class ModuleFit:
    """The fitting iteration of one instance of the 3D-FastResUNet variants
    (any mix of depthwise-separable convs, SE units, ASPP, attention units and
    the sigmoid tail) in the library; see d2ip_mnet_* in include/d2ip.h."""

    def __init__(self, n, M, levels, base_ch, sep=False, se_ratio=0, att=False, tail="linear",
                 aspp=False, graph=False, device=0, stream=None):
        import torch
        self._lib = L.load()
        self.n, self.M = int(n), int(M)
        self.desc = _mnet_desc(n, M, levels, base_ch, sep, se_ratio, att, tail, aspp, graph)
        out = ctypes.c_size_t()
        L.check(self._lib.d2ip_mnet_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(out)))
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.workspace = torch.empty(out.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        L.check(self._lib.d2ip_mnet_create(ctypes.byref(self.desc),
                                           ctypes.c_void_p(self.workspace.data_ptr()), out.value,
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        pc = ctypes.c_size_t()
        L.check(self._lib.d2ip_mnet_param_count(ctypes.byref(self.desc), ctypes.byref(pc)))
        self.n_params = pc.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.d2ip_mnet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_problem(self, J, mask, z):
        jp, jd, _k1 = _in(J, np.float32)
        mp, md, _k2 = _in(mask, np.uint8)
        zp, zd, _k3 = _in(z, np.float32)
        if not (jd == md == zd):
            raise ValueError("J, mask and z must all be host arrays or all device tensors")
        L.check(self._lib.d2ip_mnet_set_problem(self._h, jp, mp, zp, jd))

    def set_params(self, theta):
        p, d, _k = _in(theta, np.float32)
        L.check(self._lib.d2ip_mnet_set_params(self._h, p, self.n_params, d))

    def set_frame(self, dv):
        p, d, _k = _in(dv, np.float32)
        L.check(self._lib.d2ip_mnet_set_frame(self._h, p, d))

    def set_adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        cfg = L.AdamCfg(lr, beta1, beta2, eps)
        L.check(self._lib.d2ip_mnet_set_adam(self._h, ctypes.byref(cfg)))

    def reset_optimizer(self):
        L.check(self._lib.d2ip_mnet_reset_optimizer(self._h))

    def run(self, k, sync=True):
        if not sync:
            L.check(self._lib.d2ip_mnet_run(self._h, int(k), None))
            return None
        out = ctypes.c_double()
        L.check(self._lib.d2ip_mnet_run(self._h, int(k), ctypes.byref(out)))
        return out.value

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        L.check(self._lib.d2ip_mnet_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                               out.size, 0))
        return out

    def get_grad(self):
        out = np.empty(self.n_params, dtype=np.float32)
        L.check(self._lib.d2ip_mnet_get_grad(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                             out.size, 0))
        return out

    def read_image(self):
        img = np.empty(self.n ** 3, dtype=np.float32)
        L.check(self._lib.d2ip_mnet_read_image(self._h, img.ctypes.data_as(ctypes.c_void_p), 0))
        return img
