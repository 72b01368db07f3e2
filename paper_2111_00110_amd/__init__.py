"""FC^2T^2 on MI355X: the explicit, ray-integral and ray-root layers of Lange & Kutz
(arXiv 2111.00110) as hand-written HIP kernels for gfx950 behind a small C-ABI."""
import torch  # noqa: F401  (load torch's HIP runtime before the library)

from .fc2t2 import (Explicit, FC2T2Error, Plan, RayIntegral, RayRoot, lib,  # noqa: F401
                    multi_indices)
