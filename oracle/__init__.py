"""FP64 CPU oracle for SSIM / MS-SSIM (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the HIP library and imports nothing from it.
"""
from .ssim_oracle import *  # noqa: F401,F403
from .ssim_oracle import mean_pool, BT601  # noqa: F401
