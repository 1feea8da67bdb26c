"""MI355X (gfx950) stand-alone multigrid for the 2D Helmholtz equation.

Method: Dwarka & Vuik, "Stand-alone multigrid for Helmholtz revisited"
(arXiv 2308.13476). The numerical work runs in hand-written HIP kernels behind
the C ABI of include/helmg.h (libhelmg.so); this package is the thin Python
binding (`Solver`), the differentiable solve (`helmholtz_solve`) and the
seeded input generators (`workloads`).
"""
from . import workloads  # noqa: F401
from ._binding import MGError, lib  # noqa: F401


def __getattr__(name):
    # torch-dependent parts load lazily so that `workloads` works without a GPU stack
    if name == "Solver":
        from .solver import Solver
        return Solver
    if name == "helmholtz_solve":
        from .autograd import helmholtz_solve
        return helmholtz_solve
    raise AttributeError(name)
