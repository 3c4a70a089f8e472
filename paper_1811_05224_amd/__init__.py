"""Space-time Galerkin BEM for the 2D heat equation on MI355X (arXiv:1811.05224).

Thin binding over the C ABI of libstbem.so: every step of assembly, matrix
application, preconditioning and solving runs in the HIP kernels; this layer
only passes torch device pointers and the current HIP stream.
"""
from .api import Context, SolveInfo, StbemError  # noqa: F401
from .adjoint import HeatFluxSolve  # noqa: F401
from . import _lib  # noqa: F401
