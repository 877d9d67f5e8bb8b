"""MI355X-native Schwarz-preconditioned Wilson-clover solver (arxiv 1502.04025, Sec. 3).

The compute path is the HIP library libsapdd.so (C ABI in include/sapdd.h); the Python
module `sapdd` only marshals arguments into it.
"""
from .sapdd import (  # noqa: F401
    Batch, Context, Field, MgParams, Multigrid, Params, SapddError, Stats, load_library,
    F16, F16_LINKS, F32, F64, OK, EINVAL, EFULL, ENOCONV, ESINGULAR, ENAN, DEVICE_PTRS, USE_X0, NO_GRAPH, LINKS12, ELASTIC,
)
