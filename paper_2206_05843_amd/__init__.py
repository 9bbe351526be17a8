"""Level-scheduled sparse triangular solves with equation rewriting on MI355X.

The computation lives in libsptrsv.so (hand-written HIP kernels for gfx950,
C ABI in include/sptrsv.h); ``sptrsv`` is its ctypes binding. Nothing here
falls back to a CPU path: a missing library raises.
"""
from .sptrsv import (  # noqa: F401
    ORIGINAL, REWRITTEN, BATCH, THIN_ROWS, THIN_COST, LOWER, UPPER, LOWER_TRANS, UPPER_TRANS, MLP_NPARAM, Handle,
    SptrsvError, lib, mlp_forward, mlp_backward, mlp_adam, mlp_mask, mlp_actions, MAX_TIERS, EXPORTS,
)
