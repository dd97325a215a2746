"""MI355X (gfx950) Newton-step linear solve of pressurized phase-field fracture.

The computation lives in libfracture.so (HIP, built from csrc/ by build.py) behind the C ABI
of include/fracture.h; `binding` is its ctypes wrapper.
"""
from . import binding  # noqa: F401
from .binding import (Mesh, System, Amg, solve, update, newton, functionals, params, amg_opts, solve_opts,
                      newton_opts, mesh_desc, FractureError, FR_RESIDUAL, FR_ACTIVE_SET, FR_JACOBIAN)

__all__ = ["binding", "Mesh", "System", "Amg", "solve", "update", "newton", "functionals", "params", "amg_opts",
           "solve_opts", "newton_opts", "mesh_desc", "FractureError", "FR_RESIDUAL", "FR_ACTIVE_SET", "FR_JACOBIAN"]
