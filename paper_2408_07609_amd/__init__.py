"""MI355X-native hot path of the RTi nested long-wave (tsunami) time step.

The computation lives in librti.so (HIP kernels for gfx950 behind the C ABI of
include/rti.h); ``paper_2408_07609_amd.rti`` is its ctypes binding.
"""
from .rti import *  # noqa: F401,F403
from .rti import Batch, Domain, RtiError, make_desc  # noqa: F401
