"""MI355X FAS multigrid solver for the 3D Monge-Ampere equation.

Implements the method of Liu, Froese, Oberman and Xiao, "A multigrid scheme
for 3D Monge-Ampere equations": the FAS V-cycle (Algorithm 1) whose smoother
is the nonlinear Gauss-Seidel sweep that takes, at every grid point, the
smallest real root of the local cubic (eqs. 2.8-2.9).  The kernels are
hand-written HIP for gfx950 behind the C ABI of include/ma.h; this package
only marshals torch tensors into that ABI.

Submodules are imported lazily so that ``problems`` (input generators) can be
used without the HIP library.
"""
import importlib

__all__ = ["Solver", "levels", "footprint_bytes", "problems", "solver", "batch", "server"]


def __getattr__(name):
    if name in ("Solver", "levels", "footprint_bytes"):
        return getattr(importlib.import_module(".solver", __name__), name)
    if name in ("problems", "solver", "solver2d", "batch", "server", "build", "autotune"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
