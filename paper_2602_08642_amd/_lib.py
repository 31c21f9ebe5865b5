"""ctypes loader of libaps.so: argument types only, no computation."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaps.so")

(APS_OK, APS_ERR_NULL, APS_ERR_SHAPE, APS_ERR_UNSUPPORTED, APS_ERR_WORKSPACE, APS_ERR_HIP, APS_ERR_ARG,
 APS_ERR_TOO_LARGE) = range(8)
APS_F32, APS_BF16 = 0, 1
APS_HARD, APS_RELAXED, APS_STRAIGHT_THROUGH, APS_GUMBEL, APS_DASR = range(5)
APS_ROUND_STOCHASTIC, APS_ROUND_HOLDOUT, APS_ROUND_DETERMINISTIC = range(3)
APS_FEAT_SAMPLER, APS_FEAT_KERNEL = 0, 1
APS_CONV_DIRECT, APS_CONV_POOL2, APS_CONV_UP2_CAT = 0, 1, 2
APS_MAX_LEVELS = 5
APS_MAX_NET_LAYERS = 20
APS_STATUS_COUNT_OVERFLOW, APS_STATUS_NONFINITE, APS_STATUS_CAPACITY = 1, 2, 4


class ConvLayer(C.Structure):
    _fields_ = [("w", C.c_void_p), ("b", C.c_void_p), ("cin", C.c_int), ("cout", C.c_int),
                ("ksize", C.c_int), ("relu", C.c_int)]


class NetDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("dtype", C.c_int),
                ("layer", ConvLayer * APS_MAX_NET_LAYERS)]


P, I, I64, U64, U32, F, SZ = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_uint32, C.c_float, C.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "aps_version": (I, []),
    "aps_status_string": (C.c_char_p, [I]),
    "aps_conv_packed_elems": (SZ, [I, I, I]),
    "aps_conv_pack_weights": (I, [P, I, I, I, I, P, P]),
    "aps_conv2d_fwd": (I, [P, P, I, I, I, I, I, I, P, P, I, I, I, I, P, I, I, P]),
    "aps_conv2d_fwd_head": (I, [P, P, I, I, I, I, I, I, P, P, I, I, P, P, I, I, P, I, P, I, P]),
    "aps_conv2d_fwd_head_ex": (I, [P, P, I, I, I, I, I, I, P, P, I, I, P, P, I, I, P, I, P, I, P, I, P]),
    "aps_conv2d_fwd_pool": (I, [P, P, I, I, I, I, I, I, P, P, I, I, I, P, P, P]),
    "aps_normalize_workspace_size": (SZ, [I, I, I]),
    "aps_normalize_density": (I, [P, I, I, I, F, F, P, P, SZ, P, P]),
    "aps_density_predict_workspace_size": (SZ, [I, I, I, I, I]),
    "aps_density_predict": (I, [C.POINTER(NetDesc), P, I, I, I, I, F, F, P, P, P, SZ, P, P]),
    "aps_avgpool2": (I, [P, I, I, I, I, I, P, P]),
    "aps_demodulate": (I, [P, P, I, I, I, I, I, I, I, P, P]),
    "aps_remodulate": (I, [P, P, I, I, I, I, I, I, I, P, P, P]),
    "aps_demodulate_bwd": (I, [P, P, I, I, I, I, I, I, I, P, P, P, I, P]),
    "aps_remodulate_bwd": (I, [P, P, I, I, I, I, I, I, P, P, P, I, P]),
    "aps_upsample_nearest2": (I, [P, I, I, I, P, P]),
    "aps_sample_mask_workspace_size": (SZ, [I, I, I]),
    "aps_sample_mask": (I, [P, I, I, I, U64, U32, P, P, P, I64, P, P, P, SZ, P, P]),
    "aps_sample_mask_ex": (I, [P, I, I, I, U64, U32, P, I, I, P, P, P, I64, P, P, P, SZ, P, P]),
    "aps_sample_mask_noalloc": (I, [P, I, I, I, U64, U32, P, I, I, P, P, P, I64, P, P, P, P]),
    "aps_fixture_render": (I, [P, I, P, P, I, I, I, I64, P, P]),
    "aps_scatter_samples": (I, [P, P, P, P, I64, I, I, I, I, I, F, U64, U32, P, P]),
    "aps_scatter_samples_ex": (I, [P, P, P, P, I64, I, I, I, I, I, F, U64, U32, P, I, P, P]),
    "aps_assemble_features": (I, [I, P, P, P, P, P, I, I, I, I, I, P, P]),
    "aps_assemble_features_ex": (I, [I, P, P, P, P, P, P, I, I, I, I, I, P, P]),
    "aps_kernel_predict_workspace_size": (SZ, [C.POINTER(NetDesc), I, I, I]),
    "aps_kernel_predict": (I, [C.POINTER(NetDesc), P, I, I, I, I, I, P, I, P, P, SZ, P]),
    "aps_kernel_predict_ex": (I, [C.POINTER(NetDesc), P, I, I, I, I, I, P, I, P, P, I, P, SZ, P]),
    "aps_denoise_pyramid_workspace_size": (SZ, [I, I, I, I]),
    "aps_denoise_pyramid": (I, [P, P, I, P, I, I, I, I, P, P, I, I, I, P, P, SZ, P]),
    "aps_denoise_pyramid_ex": (I, [P, P, I, P, I, I, I, I, P, P, I, I, I, I, I, P, P, P, P, SZ, P]),
    "aps_reproject": (I, [P, P, P, I, I, I, I, I, I, I, I, I, P, P]),
    "aps_upsample": (I, [P, P, I, I, I, I, I, I, I, I, I, P, P]),
    # backward
    "aps_denoise_pyramid_bwd_workspace_size": (SZ, [I, I, I, I, I, I, I, I]),
    "aps_denoise_pyramid_bwd": (I, [P, P, I, P, I, I, I, I, P, P, I, I, I, P, P, I, P, P, P, P,
                                    SZ, P]),
    "aps_reproject_bwd_workspace_size": (SZ, [I, I, I, I, I, I, I]),
    "aps_reproject_bwd": (I, [P, P, P, I, I, I, I, I, I, I, I, I, P, P, I, I, P, P, SZ, P]),
    "aps_upsample_bwd_workspace_size": (SZ, [I, I, I, I, I, I, I]),
    "aps_upsample_bwd": (I, [P, P, I, I, I, I, I, I, I, I, I, P, P, I, I, P, P, SZ, P]),
    "aps_density_predict_bwd_workspace_size": (SZ, [C.POINTER(NetDesc), I, I, I]),
    "aps_density_predict_bwd": (I, [C.POINTER(NetDesc), P, P, I, I, I, I, F, F, P, P, P, P, P, SZ, P]),
    "aps_scatter_samples_bwd": (I, [P, P, P, P, I64, I, I, I, I, I, F, U64, U32, P, P, I, P]),
    "aps_scatter_samples_bwd_ex": (I, [P, P, P, P, I64, I, I, I, I, I, F, U64, U32, P, I, P, P, P, I, P]),
    "aps_normalize_bwd_workspace_size": (SZ, [I, I, I]),
    "aps_normalize_density_bwd": (I, [P, I, I, I, F, F, P, P, P, SZ, P]),
    "aps_assemble_features_bwd": (I, [I, P, P, P, I, I, I, I, I, P, P, P, P, P]),
    "aps_assemble_features_bwd_ex": (I, [I, P, P, P, I, I, I, I, I, I, P, P, P, P, P, P]),
    "aps_conv_pack_weights_dgrad": (I, [P, I, I, I, I, P, P]),
    "aps_conv2d_bwd_data": (I, [P, P, I, I, I, I, I, P, I, I, I, P, P]),
    "aps_conv_input_grad": (I, [I, P, I, I, I, I, I, I, P, I, P, I, P]),
    "aps_conv2d_bwd_weight_workspace_size": (SZ, [I, I, I, I, I, I, I]),
    "aps_conv2d_bwd_weight": (I, [P, P, I, I, I, I, I, I, P, P, I, I, I, I, P, P, P, SZ, P]),
    # training
    "aps_tmo_loss_workspace_size": (SZ, [I, I, I]),
    "aps_tmo_loss": (I, [P, P, P, P, P, P, I, I, I, P, P, P, P, SZ, P]),
    "aps_adamw_step": (I, [P, P, P, P, I64, F, F, F, F, F, I, F, P]),
    "aps_copy_channels": (I, [P, I, I, P, I, I, I64, I, P]),
    "aps_scale_by": (I, [P, I64, P, P]),
    "aps_sumsq_workspace_size": (SZ, [I64]),
    "aps_sumsq": (I, [P, I64, P, P, SZ, P]),
}

_lib = None


def load():
    """The loaded library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2602_08642_amd.build` (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class ApsError(RuntimeError):
    def __init__(self, msg: str, status: int = -1):
        super().__init__(msg)
        self.status = status


def check(status: int, what: str = ""):
    if status != 0:
        msg = load().aps_status_string(status).decode()
        raise ApsError(f"{what}: aps status {status} ({msg})", status)
