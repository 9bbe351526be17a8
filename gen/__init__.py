"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws matrices and right-hand sides. It holds none of the
solver's arithmetic (no substitution, no level sets, no rewriting), so the CPU
oracle and the HIP path can both consume it without sharing any method code.
"""
from .matrices import (  # noqa: F401
    Csr,
    window_random,
    stencil2d_chain,
    stencil3d_tail,
    powerlaw,
    policy_training_matrix,
    lung2_like,
    torso2_like,
    batch_window,
    rhs,
    from_dense_lower,
    transpose,
    bidiagonal,
    diagonal,
    config_matrix,
)
