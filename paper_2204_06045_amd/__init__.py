"""MI355X bucket-elimination engine for the QAOA MaxCut energy expectation
(arXiv 2204.06045): per-edge light-cone tensor networks contracted bucket by
bucket, with merged indices, in hand-written HIP kernels for gfx950.

The C ABI is ``include/qtn.h``; ``binding`` exposes it under the same names.
"""

from .binding import *  # noqa: F401,F403
from .binding import Network, QTN_C128, QTN_C64, QTN_MIXED, QtnError  # noqa: F401
