"""ctypes declarations of libssimx.so (include/ssimx.h).

Argument marshalling only: every computation runs in the HIP library.  The
library must have been built (``python paper_2101_06354_amd/build_lib.py``);
importing this module without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
# SSIMX_LIBRARY names another build of the library to load (the host-sanitised
# build of build_lib.py --sanitize-host, for instance).
LIB_PATH = os.environ.get("SSIMX_LIBRARY") or os.path.join(HERE, "libssimx.so")

# status codes
OK, EINVAL, EDTYPE, ETOOSMALL, EWORKSPACE, EHIP, ENOTSUP, ENOMEM, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8
# dtypes
U8, U16, F32, BF16 = 0, 1, 2, 3
# windows / algorithms / padding
WIN_GAUSSIAN, WIN_BOX = 0, 1
ALGO_AUTO, ALGO_SEPARABLE, ALGO_INTEGRAL_IMAGE = 0, 1, 2
PAD_VALID, PAD_ZERO, PAD_REFLECT = 0, 1, 2
MS_RENORM, MS_CS_CLAMP, MS_SUM, MS_COARSE_SEPARATE = 1, 2, 4, 8
OP_MAP, OP_POOLED, OP_MSSSIM, OP_MAP_BACKWARD, OP_POOLED_BACKWARD, OP_MSSSIM_BACKWARD = range(6)


class Params(ctypes.Structure):
    _fields_ = [("window", c_int), ("k", c_int), ("sigma", c_float), ("C1", c_double), ("C2", c_double),
                ("stride", c_int), ("padding", c_int), ("algo", c_int)]


class Image(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("dtype", c_int), ("width", c_int), ("height", c_int),
                ("pitch", c_int64), ("batch_stride", c_int64)]


class Pair(ctypes.Structure):
    _fields_ = [("ref", Image), ("dis", Image), ("p", Params), ("map_out", c_void_p), ("map_pitch", c_int64)]


class Pool(ctypes.Structure):
    _fields_ = [("kind", c_int), ("p", c_double), ("o", c_double), ("r", c_double)]


(POOL_MEAN, POOL_COV, POOL_MEAN_DEV, POOL_MINKOWSKI, POOL_DIST_WEIGHTED, POOL_FIVE_NUMBER, POOL_PERCENTILE,
 POOL_GEOMETRIC, POOL_HARMONIC, POOL_MEDIAN, POOL_WIN_AM, POOL_WIN_GM, POOL_WIN_HM, POOL_WIN_COV) = range(14)


class SSIMXError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.ssimx_strerror(status).decode() if lib else str(status)
        extra = f" (hipError {lib.ssimx_last_hip_error()})" if status == EHIP else ""
        super().__init__(f"{where}: {msg}{extra} [status {status}]")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2101_06354_amd/build_lib.py`")
    return ctypes.CDLL(LIB_PATH)


lib = _load()

_P = POINTER(Params)
_I = POINTER(Image)
_F = POINTER(c_float)

_SIGS = {
    "ssimx_map_shape": (c_int, [_P, c_int, c_int, POINTER(c_int), POINTER(c_int)]),
    "ssimx_workspace_size": (c_int, [_P, c_int, c_int, c_int, c_int, c_int, c_int, POINTER(c_size_t)]),
    "ssim_map": (c_int, [_P, _I, _I, c_int, c_void_p, c_int64, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ssim_pooled": (c_int, [_P, _I, _I, c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ssim_pooled_lw": (c_int, [_P, _I, _I, c_int, c_float, c_float, c_void_p, c_void_p, c_size_t, c_void_p]),
    "msssim": (c_int, [_P, _F, c_int, c_int, _I, _I, c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ssimx_msssim_pyramid_layout": (c_int, [_P, c_int, c_int, c_int, c_int, c_int, POINTER(c_int64),
                                            POINTER(c_int64), POINTER(c_int), POINTER(c_int)]),
    "ssim_pooled_noalloc": (c_int, [_P, _I, _I, c_int, c_void_p, c_void_p]),
    "ssimx_noalloc_scratch_bytes": (c_size_t, []),
    "ssim_map_backward": (c_int, [_P, _I, _I, c_int, c_void_p, c_int64, c_int64, c_void_p, c_int64, c_int64,
                                  c_void_p, c_size_t, c_void_p]),
    "ssim_pooled_backward": (c_int, [_P, _I, _I, c_int, c_void_p, c_void_p, c_int64, c_int64, c_void_p, c_size_t,
                                     c_void_p]),
    "msssim_backward": (c_int, [_P, _F, c_int, c_int, _I, _I, c_int, c_void_p, c_void_p, c_int64, c_int64,
                                c_void_p, c_size_t, c_void_p]),
    "msssim_backward_values": (c_int, [_P, _F, c_int, c_int, _I, _I, c_int, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_int64, c_int64, c_void_p, c_size_t, c_void_p]),
    "ssimx_box_sums": (c_int, [c_int, c_int, c_int, _I, _I, c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ssimx_integral_images": (c_int, [_I, _I, c_int, c_void_p, c_void_p]),
    "ssimx_rgb_to_luma": (c_int, [c_void_p, c_int, c_int, c_int, c_int64, c_int64, c_int64, c_int, c_void_p,
                                  c_void_p]),
    "ssimx_luma_grad_to_rgb": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_int64, c_int64, c_int64,
                                       c_void_p]),
    "ssimx_plan_create": (c_int, [POINTER(Pair), c_int, c_void_p, POINTER(c_void_p)]),
    "ssimx_plan_run": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ssimx_plan_run_unbatched": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ssimx_plan_destroy": (c_int, [c_void_p]),
    "ssimx_plan_info": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int)]),
    "ssimx_autotune": (c_int, [_P, c_int, c_int, c_int, c_int, c_void_p, POINTER(c_int)]),
    "ssimx_tune_cache_load": (c_int, [c_char_p]),
    "ssimx_tune_cache_save": (c_int, [c_char_p]),
    "ssimx_set_tile_override": (c_int, [c_int]),
    "ssimx_num_tile_configs": (c_int, []),
    "ssimx_pool_workspace_size": (c_int, [POINTER(Pool), c_int, c_int, c_int, POINTER(c_size_t)]),
    "ssimx_pool_map": (c_int, [POINTER(Pool), c_void_p, c_int, c_int, c_int64, c_int64, c_int, c_void_p, c_void_p,
                               c_size_t, c_void_p]),
    "ssimx_scaled_pooled_workspace_size": (c_int, [_P, c_int, POINTER(Pool), c_int, c_int, c_int, c_int,
                                                   POINTER(c_size_t)]),
    "ssimx_scaled_pooled_ssim": (c_int, [_P, c_int, POINTER(Pool), _I, _I, c_int, c_void_p, c_void_p, c_size_t,
                                         c_void_p]),
    "ssimx_color_workspace_size": (c_int, [_P, c_int, c_int, c_int, POINTER(c_size_t)]),
    "ssimx_color_ssim": (c_int, [_P, c_double, c_double, c_void_p, c_void_p, c_int, c_int, c_int, c_int64, c_int64,
                                 c_int64, c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ssimx_ssim3d_workspace_size": (c_int, [_P, c_int, c_int, c_int, c_int, c_int, POINTER(c_size_t)]),
    "ssimx_ssim3d": (c_int, [_P, c_int, _I, _I, c_int, c_void_p, c_int64, c_int64, c_void_p, c_void_p, c_size_t,
                             c_void_p]),
    "ssimx_msssim3d_workspace_size": (c_int, [_P, c_int, c_int, c_int, c_int, c_int, c_int, POINTER(c_size_t)]),
    "ssimx_msssim3d": (c_int, [_P, c_int, _F, c_int, c_int, _I, _I, c_int, c_void_p, c_void_p, c_void_p, c_size_t,
                               c_void_p]),
    "ssimx_msssim_loss_workspace_size": (c_int, [_P, _F, c_int, c_int, c_int, c_int, c_int, c_int,
                                                 POINTER(c_size_t)]),
    "ssimx_msssim_loss_rgb": (c_int, [_P, _F, c_int, c_int, c_void_p, c_void_p, c_int, c_int, c_int, c_int64,
                                      c_int64, c_int64, c_int, c_void_p, c_void_p, c_void_p, c_int, c_int64,
                                      c_int64, c_int64, c_void_p, c_size_t, c_void_p]),
    "ssimx_msssim_loss_rgb_deferred": (c_int, [_P, _F, c_int, c_int, c_void_p, c_void_p, c_int, c_int, c_int,
                                               c_int64, c_int64, c_int64, c_int, c_void_p, c_void_p, c_void_p,
                                               c_size_t, c_void_p]),
    "ssimx_msssim_loss_rgb_grad": (c_int, [_P, _F, c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p,
                                           c_int, c_int64, c_int64, c_int64, c_void_p, c_size_t, c_void_p]),
    "ssimx_loss_plan_create": (c_int, [_P, _F, c_int, c_int, c_int, c_int, c_int, c_int, c_int,
                                       POINTER(c_void_p)]),
    "ssimx_loss_plan_run": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p,
                                    c_void_p, c_int64, c_int64, c_int64, c_void_p]),
    "ssimx_loss_plan_destroy": (c_int, [c_void_p]),
    "ssimx_strerror": (c_char_p, [c_int]),
    "ssimx_last_hip_error": (c_int, []),
    "ssimx_version": (c_int, []),
}

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def check(status: int, where: str) -> None:
    if status != OK:
        raise SSIMXError(status, where)


__all__ = [n for n in dir() if not n.startswith("__")]
_ = (c_int32, c_uint32)
