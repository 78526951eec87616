"""MI355X-native periodic tree-gravity force evaluation (2HOT hot path).

The compute lives in ``libhot.so`` (hand-written HIP for gfx950 behind the C
ABI in ``include/hot.h``); ``hot`` is its ctypes binding.
"""
from .hot import (HOT_FP32, HOT_FP64, Gravity, HotError, checkpointed_kdk, far_table,
                  gravity_forces, lib, make_params)

__all__ = ["Gravity", "HotError", "checkpointed_kdk", "far_table", "gravity_forces", "lib",
           "make_params",
           "HOT_FP32", "HOT_FP64"]
