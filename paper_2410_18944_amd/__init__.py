"""MI355X-native guided walk on stars.

The hot path runs in the gfx950 HIP library ``libwost.so`` behind the C ABI
declared in ``include/wost.h``; this package is its thin Python binding.
"""
from .api import Accumulator, Geometry, Problem, Records, set_launch, set_walk_pool, solve  # noqa: F401
from .guide import Guide, GuideConfig, GuideLoss, tail_pass  # noqa: F401
