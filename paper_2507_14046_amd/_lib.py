"""ctypes declarations of libd2ip.so (the C-ABI in include/d2ip.h).

There is no fallback: if the shared library is missing or fails to load this
module raises, so nothing can silently run elsewhere.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libd2ip.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ENONFINITE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ENONFINITE"}
PLAIN_FP32, BF16_CONV, BF16X3_CONV = 0, 1, 2
FLAG_GRAPH = 1
KERNEL_JVEC, KERNEL_JTVEC, KERNEL_ADAM, KERNEL_CONV_FWD, KERNEL_CONV_DGRAD, KERNEL_CONV_WGRAD = range(6)


class GeometryDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("M", ctypes.c_int)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [("geometry", ctypes.c_int), ("levels", ctypes.c_int), ("base_ch", ctypes.c_int)]


class MnetDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("M", ctypes.c_int), ("levels", ctypes.c_int),
                ("base_ch", ctypes.c_int), ("sep", ctypes.c_int), ("se_ratio", ctypes.c_int),
                ("att", ctypes.c_int), ("sigmoid_tail", ctypes.c_int), ("aspp", ctypes.c_int),
                ("graph", ctypes.c_int)]


class AdamCfg(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class TvCfg(ctypes.Structure):
    _fields_ = [("lambda_tv", ctypes.c_float), ("lambda_s", ctypes.c_float),
                ("lambda_t", ctypes.c_float), ("eps", ctypes.c_float)]


class ConvShape(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int), ("bn", ctypes.c_int), ("ck", ctypes.c_int),
                ("split", ctypes.c_int)]


class TuningEntry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("cin", ctypes.c_int), ("cout", ctypes.c_int),
                ("taps", ctypes.c_int), ("pass_", ctypes.c_int), ("prologue", ctypes.c_int),
                ("precision", ctypes.c_int), ("shape", ConvShape)]


class D2ipError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


_c_size_p = ctypes.POINTER(ctypes.c_size_t)
_vp = ctypes.c_void_p
_i = ctypes.c_int

# name -> argument types (all return int status, except d2ip_last_error)
SIGNATURES = {
    "d2ip_param_count": [_i, _i, _c_size_p],
    "d2ip_init_params_host": [_i, _i, ctypes.c_uint64, _vp, ctypes.c_size_t],
    "d2ip_init_params": [_vp, _i, ctypes.c_uint64],
    "d2ip_runtime_versions": [ctypes.POINTER(_i), ctypes.POINTER(_i)],
    "d2ip_workspace_bytes": [ctypes.POINTER(GeometryDesc), _i, ctypes.POINTER(InstanceDesc), _i, _i,
                             ctypes.c_uint, _c_size_p],
    "d2ip_check_launches": [ctypes.POINTER(GeometryDesc), _i, ctypes.POINTER(InstanceDesc), _i, _i,
                            ctypes.c_uint],
    "d2ip_create": [ctypes.POINTER(GeometryDesc), _i, ctypes.POINTER(InstanceDesc), _i, _i,
                    ctypes.c_uint, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)],
    "d2ip_destroy": [_vp],
    "d2ip_set_geometry": [_vp, _i, _vp, _vp, _i],
    "d2ip_set_params": [_vp, _i, _vp, ctypes.c_size_t, _i],
    "d2ip_get_params": [_vp, _i, _vp, ctypes.c_size_t, _i],
    "d2ip_get_grad": [_vp, _i, _vp, ctypes.c_size_t, _i],
    "d2ip_set_noise_input": [_vp, _i, _vp, _i],
    "d2ip_set_frame": [_vp, _i, _vp, _i],
    "d2ip_set_adam": [_vp, ctypes.POINTER(AdamCfg)],
    "d2ip_reset_optimizer": [_vp, _i],
    "d2ip_get_state": [_vp, _i, _vp, ctypes.POINTER(ctypes.c_int64), _i],
    "d2ip_set_state": [_vp, _i, _vp, ctypes.c_int64, _i],
    "d2ip_run": [_vp, _i, ctypes.POINTER(ctypes.c_double)],
    "d2ip_read_image": [_vp, _i, _vp, _i],
    "d2ip_time_kernel": [_vp, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_double)],
    "d2ip_set_tuning": [ctypes.POINTER(TuningEntry), _i],
    "d2ip_plan_convs": [ctypes.POINTER(GeometryDesc), _i, ctypes.POINTER(InstanceDesc), _i, _i,
                        ctypes.c_uint, _i, ctypes.POINTER(TuningEntry), _i,
                        ctypes.POINTER(ctypes.c_int)],
    "d2ip_time_conv_bytes": [ctypes.POINTER(TuningEntry), _c_size_p],
    "d2ip_time_conv": [ctypes.POINTER(TuningEntry), _vp, ctypes.c_size_t, _vp, _i,
                       ctypes.POINTER(ctypes.c_double)],
    "d2ip_set_tv": [_vp, ctypes.POINTER(TvCfg)],
    "d2ip_commit_frame": [_vp, _i],
    "d2ip_clear_history": [_vp, _i],
    # standalone operators
    "d2ip_op_conv3d_bytes": [_i, _i, _i, _i, _i, _c_size_p],
    "d2ip_op_conv3d_forward": [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp, ctypes.c_size_t, _vp],
    "d2ip_op_conv3d_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp,
                                ctypes.c_size_t, _vp],
    "d2ip_op_ln_relu_bytes": [_i, _i, _c_size_p],
    "d2ip_op_ln_relu_forward": [_vp, _vp, _vp, _vp, _vp, _i, _i, _vp, ctypes.c_size_t, _vp],
    "d2ip_op_ln_relu_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _vp, ctypes.c_size_t,
                                 _vp],
    "d2ip_op_dwconv3d_bytes": [_i, _i, _c_size_p],
    "d2ip_op_dwconv3d_forward": [_vp, _vp, _vp, _vp, _i, _i, _vp],
    "d2ip_op_dwconv3d_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _vp, ctypes.c_size_t,
                                  _vp],
    "d2ip_op_dwconv3d_dilated_bytes": [_i, _i, _i, _c_size_p],
    "d2ip_op_dwconv3d_dilated_forward": [_vp, _vp, _vp, _vp, _i, _i, _i, _vp],
    "d2ip_op_dwconv3d_dilated_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp,
                                          ctypes.c_size_t, _vp],
    "d2ip_op_pwconv3d_bytes": [_i, _i, _i, _c_size_p],
    "d2ip_op_pwconv3d_forward": [_vp, _vp, _vp, _vp, _i, _i, _i, _vp],
    "d2ip_op_pwconv3d_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp,
                                  ctypes.c_size_t, _vp],
    "d2ip_op_se_bytes": [_i, _i, _i, _c_size_p],
    "d2ip_op_se_forward": [_vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, ctypes.c_size_t, _vp],
    "d2ip_op_se_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i,
                            _vp, ctypes.c_size_t, _vp],
    "d2ip_op_j_forward": [_vp, _vp, _vp, _i, _i, _vp],
    "d2ip_op_mse_loss": [_vp, _vp, _vp, _vp, _i, _vp],
    "d2ip_op_pool2_forward": [_vp, _vp, _i, _i, _vp],
    "d2ip_op_pool2_backward": [_vp, _vp, _i, _i, _vp],
    "d2ip_op_up2_concat_forward": [_vp, _i, _vp, _i, _i, _vp, _vp],
    "d2ip_op_up2_concat_backward": [_vp, _i, _i, _i, _vp, _vp, _vp],
    "d2ip_op_channel_copy": [_vp, _i, _i, _vp, _i, _i, _i, ctypes.c_size_t, _vp],
    "d2ip_op_relu_forward": [_vp, _vp, ctypes.c_size_t, _vp],
    "d2ip_op_relu_backward": [_vp, _vp, _vp, ctypes.c_size_t, _vp],
    "d2ip_mnet_param_count": [ctypes.POINTER(MnetDesc), _c_size_p],
    "d2ip_mnet_workspace_bytes": [ctypes.POINTER(MnetDesc), _c_size_p],
    "d2ip_mnet_create": [ctypes.POINTER(MnetDesc), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)],
    "d2ip_mnet_destroy": [_vp],
    "d2ip_mnet_set_problem": [_vp, _vp, _vp, _vp, _i],
    "d2ip_mnet_set_params": [_vp, _vp, ctypes.c_size_t, _i],
    "d2ip_mnet_get_params": [_vp, _vp, ctypes.c_size_t, _i],
    "d2ip_mnet_get_grad": [_vp, _vp, ctypes.c_size_t, _i],
    "d2ip_mnet_set_frame": [_vp, _vp, _i],
    "d2ip_mnet_set_adam": [_vp, ctypes.POINTER(AdamCfg)],
    "d2ip_mnet_reset_optimizer": [_vp],
    "d2ip_mnet_run": [_vp, _i, ctypes.POINTER(ctypes.c_double)],
    "d2ip_mnet_read_image": [_vp, _vp, _i],
    "d2ip_op_head_bytes": [_i, _i, _c_size_p],
    "d2ip_op_head_forward": [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp],
    "d2ip_op_head_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp,
                              ctypes.c_size_t, _vp],
    "d2ip_op_attention_bytes": [_i, _i, _i, _c_size_p],
    "d2ip_op_attention_forward": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp,
                                  ctypes.c_size_t, _vp],
    "d2ip_op_attention_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp, _vp, _i, _i, _i, _vp, ctypes.c_size_t, _vp],
    "d2ip_op_jt_bytes": [_i, _i, _c_size_p],
    "d2ip_op_jt": [_vp, _vp, _vp, _i, _i, _vp, ctypes.c_size_t, _vp],
    "d2ip_op_jt_noalloc": [_vp, _vp, _vp, _i, _i, _vp],
}

_lib = None


def load():
    """Load libd2ip.so once; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libd2ip.so is not built (run `python -m paper_2507_14046_amd.build` "
                          "or __graft_entry__.build()); there is no fallback path")
    # PyTorch ships its own HIP runtime: load it first so that the library
    # binds to the same runtime instance as the tensors and streams it is given
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    lib.d2ip_last_error.restype = ctypes.c_char_p
    lib.d2ip_last_error.argtypes = []
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def check(status):
    if status != OK:
        raise D2ipError(status, load().d2ip_last_error().decode())
    return status
