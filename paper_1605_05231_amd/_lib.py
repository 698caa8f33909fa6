"""ctypes loader for libnufftct.so (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnufftct.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, 1, 2, 3, 4
KERNEL_KB, KERNEL_MINMAX_KB = 0, 1
FP32, FP64 = 0, 1
RADIAL, DERIV = 1, 2
DERIV_RADIAL = RADIAL | DERIV
DETERMINISTIC = 4
STAGE_PAD_FFT, STAGE_INTERP, STAGE_RADIAL, STAGE_RADIAL_ADJ, STAGE_SPREAD, STAGE_IFFT_CROP = range(6)
UMB_STAGE_GRID, UMB_STAGE_GATHER = 0, 1
GR_STAGE_SPECTRA, GR_STAGE_BACKPROJECT = 0, 1
STAGE_NAMES = ["pad_fft", "interp", "radial", "radial_adj", "spread", "ifft_crop", "merge"]
TIMING_MERGE = 6

# every entry point declared in include/nufftct.h: name -> (restype, argtypes)
_p = C.c_void_p
_i64 = C.c_int64
_dp = C.POINTER(C.c_double)
SIGNATURES = {
    "nufftct_plan_create": (C.c_int, [C.POINTER(_p), _i64, _i64, C.c_int, C.c_int, C.c_double,
                                      C.c_int, _dp, _i64, _i64, _p]),
    "nufftct_plan_create_radial": (C.c_int, [C.POINTER(_p), _i64, _i64, C.c_int, C.c_int,
                                             C.c_double, C.c_int, _dp, _i64, _i64, _p]),
    "nufftct_autotune_radial": (C.c_int, [_i64, _i64, C.c_int, C.c_int, C.c_double, C.c_int, _dp,
                                          _i64, _i64, C.c_int, C.POINTER(C.c_int),
                                          C.POINTER(C.c_int), C.POINTER(C.c_double), _p]),
    "nufftct_forward": (C.c_int, [_p, _p, _p, C.c_int, _p]),
    "nufftct_adjoint": (C.c_int, [_p, _p, _p, C.c_int, _p]),
    "nufftct_forward_noalloc": (C.c_int, [_p, _p, _p, C.c_int, _p]),
    "nufftct_radial_quadrature": (C.c_int, [_dp, _i64, _dp, _i64, _dp]),
    "nufftct_set_line_weights": (C.c_int, [_p, _dp, _p]),
    "nufftct_reconstruct": (C.c_int, [_p, _p, _p, _p]),
    "nufftct_umbrella_create": (C.c_int, [C.POINTER(_p), _i64, _i64, _i64, C.c_double, C.c_double,
                                          C.c_double, _i64, _i64, C.c_double, C.c_double, _i64,
                                          C.c_int, C.c_int, _p]),
    "nufftct_umbrella1_create": (C.c_int, [C.POINTER(_p), _i64, _i64, _i64, C.c_double, C.c_double,
                                           C.c_double, _i64, _i64, C.c_double, C.c_double, _i64,
                                           C.c_int, C.c_int, _p]),
    "nufftct_umbrella_grid_shape": (C.c_int, [_p, C.POINTER(_i64)]),
    "nufftct_umbrella_stage": (C.c_int, [_p, C.c_int, _p, _p, _p]),
    "nufftct_umbrella_resample": (C.c_int, [_p, _p, _p, _p]),
    "nufftct_grangeat_create": (C.c_int, [C.POINTER(_p), _i64, _i64, _i64, C.c_double, C.c_double,
                                          C.c_double, C.c_int, C.c_int, _p]),
    "nufftct_grangeat_project": (C.c_int, [_p, _p, _p, _p]),
    "nufftct_grangeat_stage": (C.c_int, [_p, C.c_int, _p, _p, _p]),
    "nufftct_grangeat_info": (C.c_int, [_p, C.POINTER(_i64)]),
    "nufftct_grangeat_destroy": (C.c_int, [_p]),
    "nufftct_umbrella_destroy": (C.c_int, [_p]),
    "nufftct_stage": (C.c_int, [_p, C.c_int, _p, _p, C.c_int, _p]),
    "nufftct_plan_destroy": (C.c_int, [_p]),
    "nufftct_plan_info": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(C.c_int),
                                    C.POINTER(_i64), C.POINTER(_i64), C.POINTER(C.c_int),
                                    C.POINTER(_i64)]),
    "nufftct_plan_tiling": (C.c_int, [_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "nufftct_set_timing": (C.c_int, [_p, C.c_int]),
    "nufftct_get_stage_times": (C.c_int, [_p, _dp, C.POINTER(_i64), C.c_int]),
    "nufftct_batch_create": (C.c_int, [C.POINTER(_p), C.c_int, C.POINTER(_i64), C.POINTER(_i64),
                                       C.c_int, C.c_int, C.c_double, C.c_int, C.POINTER(_dp),
                                       C.POINTER(_i64), C.POINTER(_i64), _p]),
    "nufftct_batch_create_tuned": (C.c_int, [C.POINTER(_p), C.c_int, C.POINTER(_i64), C.POINTER(_i64),
                                       C.c_int, C.c_int, C.c_double, C.c_int, C.POINTER(_dp),
                                       C.POINTER(_i64), C.POINTER(_i64), _p]),
    "nufftct_batch_forward": (C.c_int, [_p, C.POINTER(_p), C.POINTER(_p), C.c_int, _p]),
    "nufftct_batch_adjoint": (C.c_int, [_p, C.POINTER(_p), C.POINTER(_p), C.c_int, _p]),
    "nufftct_batch_graph_capture": (C.c_int, [_p, C.c_int, C.POINTER(_p), C.POINTER(_p),
                                              C.c_int, _p]),
    "nufftct_batch_graph_launch": (C.c_int, [_p, C.c_int, _p]),
    "nufftct_batch_destroy": (C.c_int, [_p]),
    "nufftct_last_error": (C.c_char_p, []),
    "nufftct_version": (C.c_char_p, []),
}

_lib = None


class NufftError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nufftct error {code}: {msg}")
        self.code = code


def load() -> C.CDLL:
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != OK:
        msg = load().nufftct_last_error()
        raise NufftError(rc, msg.decode() if msg else "")
