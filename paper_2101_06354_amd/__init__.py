"""MI355X-native SSIM / MS-SSIM (arXiv 2101.06354): HIP kernels behind a
C-ABI (include/ssimx.h), with a thin torch binding.

Importing the package loads libssimx.so and fails loudly if it is missing.
"""
from . import _lib  # noqa: F401  (raises ImportError when the library is not built)
from .ops import (MS_WEIGHTS, BatchPlan, LossPlan, SSIMConfig, autotune, box_sums, color_ssim, enhanced_ssim,  # noqa: F401
                  integral_images, luma_grad_to_rgb, map_shape, ms_ssim, ms_ssim3d, ms_ssim_backward, msssim_loss_rgb,
                  num_tile_configs, pool, rgb_to_luma, scaled_pooled_ssim, set_tile_override, ssim, ssim3d,
                  ssim_backward, ssim_lw, ssim_map_backward, temporal_pool, tune_cache_load, tune_cache_save,
                  workspace_size)
from . import autograd  # noqa: F401

__version__ = "0.1.0"
