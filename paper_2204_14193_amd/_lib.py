"""ctypes declarations of the C ABI in include/fse.h."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfse.so")


class fse_block_t(C.Structure):
    _fields_ = [("frame", C.c_int32), ("y0", C.c_int32), ("x0", C.c_int32),
                ("bh", C.c_int16), ("bw", C.c_int16), ("border", C.c_int16),
                ("fft", C.c_int16), ("iters", C.c_int32)]


class fse_volume_t(C.Structure):
    _fields_ = [("frame", C.c_int32), ("y0", C.c_int32), ("x0", C.c_int32),
                ("bt", C.c_int16), ("bh", C.c_int16), ("bw", C.c_int16), ("border", C.c_int16),
                ("tborder", C.c_int16), ("fft", C.c_int16), ("fft_t", C.c_int16), ("pad", C.c_int16),
                ("iters", C.c_int32)]


class fse_plan_desc_t(C.Structure):
    _fields_ = [("rho", C.c_float), ("gamma", C.c_float), ("max_iters", C.c_int32),
                ("flags", C.c_uint32)]


class fse_trace_t(C.Structure):
    _fields_ = [("u", C.c_uint16), ("v", C.c_uint16), ("c_re", C.c_float),
                ("c_im", C.c_float), ("r2", C.c_float)]


P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
PI32 = C.POINTER(C.c_int32)

# name -> (restype, argtypes); every function declared in include/fse.h
SIGNATURES = {
    "fse_plan_create": (I32, [C.POINTER(fse_plan_desc_t), C.POINTER(P)]),
    "fse_plan_destroy": (None, [P]),
    "fse_validate_blocks": (I32, [P, P, I32, I32, I32, I32, PI32]),
    "fse_blocks_from_mask": (I32, [P, I32, I32, I32, I64, I32, I32, I32, I32, P, I32, PI32]),
    "fse_batch3d_create": (I32, [P, P, I32, I32, I32, I32, C.POINTER(P), PI32]),
    "fse_batch3d_destroy": (None, [P]),
    "fse_batch3d_workspace_size": (I32, [P, I32, C.POINTER(C.c_size_t)]),
    "fse_batch3d_create_in": (I32, [P, P, I32, I32, I32, I32, P, C.c_size_t, C.POINTER(P), PI32]),
    "fse_extrapolate3d_batch": (I32, [P, P, P, I64, P, I64, P, P, P]),
    "fse_warm3d_extrapolate_batch": (I32, [P, P, P, I64, P, I64, P, P, P, P, I32, P]),
    "fse_batch_create": (I32, [P, P, I32, I32, I32, I32, C.POINTER(P)]),
    "fse_batch_destroy": (None, [P]),
    "fse_batch_workspace_size": (I32, [P, I32, C.c_uint32, C.POINTER(C.c_size_t)]),
    "fse_batch_create_in": (I32, [P, P, I32, I32, I32, I32, P, C.c_size_t, C.c_uint32, C.POINTER(P)]),
    "fse_batch_max_iters": (I32, [P]),
    "fse_extrapolate_batch": (I32, [P, P, P, I64, P, I64, P, P, P]),
    "fse_batch_launch_info": (I32, [P, I32, PI32, PI32, PI32, PI32]),
    "fse_batch_set_variant": (I32, [P, I32, I32]),
    "fse_batch_autotune": (I32, [P, P, P, I64, P, I64, P, I32, P, C.c_char_p, C.c_size_t]),
    "fse_batch_autotune_cached": (I32, [P, P, P, I64, P, I64, P, I32, P, C.c_char_p, C.c_size_t, C.c_char_p]),
    "fse_batch_set_timing": (I32, [P, I32]),
    "fse_batch_kernel_times": (I32, [P, P, P, P, I32]),
    "fse_last_error": (C.c_char_p, []),
    "fse_measure_lds_bandwidth": (I32, [I32, P, C.POINTER(C.c_double)]),
    "fse_cnn_num_params": (I64, []),
    "fse_cnn_create": (I32, [I32, C.c_uint64, C.POINTER(P)]),
    "fse_cnn_destroy": (None, [P]),
    "fse_cnn_set_params": (I32, [P, P]),
    "fse_cnn_get_params": (I32, [P, P, P]),
    "fse_cnn_patches": (I32, [P, P, P, I64, P, P]),
    "fse_cnn_forward": (I32, [P, P, I32, P, I32, P]),
    "fse_cnn_forward_blocks": (I32, [P, P, P, P, I64, P, P]),
    "fse_cnn_backward": (I32, [P, P, P, P, I32, C.c_float, P, P]),
    "fse_cnn_adam": (I32, [P, C.c_float, C.c_float, C.c_float, C.c_float, P]),
    "fse_cnn_topk": (I32, [P, I32, I32, P, P, P]),
    "fse_warm_extrapolate_batch": (I32, [P, P, P, I64, P, I64, P, P, P, P, I32, I32, I32, P]),
    "fse_warm_trace_stride": (I32, [P, I32, I32]),
    "fse_warm_prepare": (I32, [P, I32, I32, I32]),
    "fse_initial_power": (I32, [P, P, P, I64, P, P]),
    "fse_warm_set_restricted_gamma": (I32, [P, C.c_float]),
    "fse_warm_extrapolate_batch_noalloc": (I32, [P, P, P, I64, P, I64, P, P, P, P, I32, I32, I32, P]),
    "fse_warm_noalloc_max_blocks": (C.c_size_t, [I32]),
}

_lib = None


def lib():
    """Load libfse.so (built in-tree by paper_2204_14193_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2204_14193_amd.build` (there is no CPU fallback)")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib
