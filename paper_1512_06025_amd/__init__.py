"""MI355X-native Bernstein-Bezier DG solver for the acoustic wave equation.

The compute path is libbbdg.so (hand-written HIP kernels for gfx950 behind a
C ABI, include/bbdg.h).  This package holds its build script, the ctypes
binding and a thin torch-facing wrapper; PyTorch supplies device memory and
streams only.
"""
from ._lib import (BBDG_BC_PRESSURE_RELEASE, BBDG_BC_RIGID, BBDG_F32, BBDG_F64,
                   BBDG_RHS_FULL, BBDG_RHS_SURFACE, BBDG_RHS_VOLUME, BBDGError, load)
from .solver import (BatchedSolver, MeshData, Misfit, Solver, alpha_table, bernstein_eval, locate_points,
                     mesh_geometry, nodal_operators, np_count)


def __getattr__(name):
    # the autograd wrapper needs torch; build it on first use
    if name == "MisfitFunction":
        from .solver import _misfit_function
        return _misfit_function()
    raise AttributeError(name)


__all__ = [
    "Solver", "BatchedSolver", "Misfit", "MisfitFunction", "MeshData", "alpha_table", "mesh_geometry", "nodal_operators", "np_count",
    "locate_points", "bernstein_eval", "load", "BBDGError",
    "BBDG_F64", "BBDG_F32", "BBDG_BC_RIGID", "BBDG_BC_PRESSURE_RELEASE",
    "BBDG_RHS_FULL", "BBDG_RHS_VOLUME", "BBDG_RHS_SURFACE",
]
