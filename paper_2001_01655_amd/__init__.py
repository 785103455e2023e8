"""topomg: multigrid-preconditioned CG for SIMP elasticity on MI355X (gfx950).

The compute lives in libtopomg.so (HIP); this package is its binding.
Importing the package loads the library and fails loudly if it is not built.
"""
from ._lib import (LIB, TmError, check, default_options, make_material, make_mesh,  # noqa: F401
                   tm_export_connectivity, tm_plan_bytes)


def __getattr__(name):
    # torch-facing classes are imported lazily so that the C ABI can be
    # inspected without initialising torch
    if name in ("Hierarchy", "SolveState", "SolveResult", "tm_batch_iterate", "density_filter"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
