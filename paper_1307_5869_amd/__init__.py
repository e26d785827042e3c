"""MI355X (gfx950) parallel uniform random number generation after PRAND
(Barash & Shchur, Comput. Phys. Commun. 185 (2014) 1343).

The computation lives in ``libprand.so`` (hand-written HIP kernels behind the C
ABI of ``include/prand.h``); ``prand`` is its ctypes binding and
``workloads`` the seeded synthetic inputs.
"""
from . import prand  # noqa: F401
from .prand import (  # noqa: F401
    F32, F64, U32, NAMES, NUM_GENERATORS, Context, PrandError, block_log2, independence_limit, state_bytes,
)
