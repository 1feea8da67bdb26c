"""Plain, slow FP64 CPU oracle of the stand-alone Helmholtz multigrid method.

TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import or run anything in this package.
The GPU product path never calls it, and it shares no code with the HIP
library: it is written independently from the paper (Dwarka & Vuik,
"Stand-alone multigrid for Helmholtz revisited", arXiv 2308.13476) with
SciPy sparse matrices as its only building blocks.

Modules
  operator  -- the discretised model problems of §2 (and a Dirichlet variant)
  transfer  -- the Bézier and linear prolongation/restriction of §4
  multigrid -- Galerkin hierarchy on the complex shifted Laplacian, weighted
               Jacobi (§3) and GMRES(3) (§5.3) smoothing, V/W cycles (§5),
               FP32-in-FP64 refinement
  twogrid   -- the dense two-grid iteration matrix of §3 for tiny grids
  adjoint   -- misfit, adjoint-state gradient w.r.t. per-node k^2
  krylov    -- flexible GMRES(m) with a multigrid cycle as right preconditioner

Every function states the passage it follows; readings of silent or garbled
passages are listed with the design notes of the repository.
"""
from .operator import (  # noqa: F401
    boundary_sides,
    node_weights,
    laplacian_1d_sommerfeld,
    helmholtz_matrix,
    shifted_laplacian,
    scaled_rhs,
    dirichlet_helmholtz_matrix,
)
from .transfer import prolongation_1d, prolongation, restriction  # noqa: F401
from .multigrid import (  # noqa: F401
    CycleOptions,
    Hierarchy,
    build_hierarchy,
    build_dirichlet_hierarchy,
    jacobi_step,
    gmres_step,
    cycle,
    solve,
    solve_refined,
    SolveResult,
)
from .krylov import fgmres, mg_preconditioner, FgmresResult  # noqa: F401
