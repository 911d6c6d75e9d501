"""MI355X-native hot path of level-set shape optimisation (compliance).

The computation lives in libfo.so (HIP, gfx950) behind the C ABI of
include/fo.h; `fo` is its ctypes binding.
"""
from . import fo  # noqa: F401
from .fo import (Context, DescentOpts, SolveOpts, Stats, FoError, time_steps,  # noqa: F401
                 FO_FP64, FO_FP32_IR, FO_SCATTER_TILED, FO_SCATTER_ATOMIC)
