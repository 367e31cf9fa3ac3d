"""MI355X (gfx950) linearised eikonal solver: Python binding of libsweik.so.

The binding marshals arguments to the C ABI declared in include/sweik.h;
every step of the solve runs in the library's HIP kernels.  PyTorch supplies
device memory and the stream.  There is no fallback: if the library is not
built, importing the solver functions raises.

    S = solve(f, src, h, hbar, T)                 # f: cuda float32/float64
    S, info = solve(..., return_info=True)
    path, n_points, status = backtrack(S, src, start)   # Section 6 paths
    S_fd = fd_solve(f, src, h, hbar)                    # Section 6 FD system
    S = solve_tilted(f, src, h, hbar, T)                # far field (tilted convolutions)
"""
from __future__ import annotations

from ._native import (  # noqa: F401
    SweikError, Plan, Batch, solve, solve_adjoint, solve_with_checkpoint,
    EikonalFn, eikonal, batch_solve, lib_path, load_library, INFO_FLAGS, backtrack, TRACE_STATUS,
    fd_solve, solve_gradient, solve_tilted, default_tilts,
)

__all__ = ["SweikError", "Plan", "Batch", "solve", "solve_adjoint",
           "solve_with_checkpoint", "EikonalFn", "eikonal", "batch_solve",
           "lib_path", "load_library", "INFO_FLAGS", "backtrack", "TRACE_STATUS", "fd_solve", "solve_gradient",
           "solve_tilted", "default_tilts"]
