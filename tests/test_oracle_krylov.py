"""Pins of the oracle's flexible GMRES (multigrid as a right preconditioner, §1)."""
import numpy as np
import scipy.sparse.linalg as spla

import oracle as O
from paper_2308_13476_amd import workloads as W


def _mp2a(n, k, beta):
    k2 = W.constant_k2(n, k)
    H = O.build_hierarchy(k2, 1.0 / n, beta)
    fs = O.scaled_rhs(W.point_source_rhs(n, [W.center_node(n)])[0]).ravel()
    return H, fs


def test_identity_preconditioner_is_scipy_gmres():
    """With M = I, one restart cycle of m iterations is GMRES(m): the iterate
    equals SciPy's gmres after the same m iterations (library routine)."""
    H, fs = _mp2a(32, 8.0, 0.5)
    A = H.A[0]
    m = 12
    res = O.fgmres(A, fs, lambda v: v, m=m, tol=1e-30, max_iter=m)
    ref, _ = spla.gmres(A, fs, restart=m, maxiter=1, rtol=1e-30, atol=0.0)
    assert res.iterations == m
    assert np.linalg.norm(res.x - ref) / np.linalg.norm(ref) <= 1e-10


def test_exact_preconditioner_converges_in_one_iteration():
    """With M = A^{-1} (sparse LU) the first direction solves the system."""
    H, fs = _mp2a(32, 10.0, 0.5)
    lu = spla.splu(H.A[0].tocsc())
    res = O.fgmres(H.A[0], fs, lu.solve, m=5, tol=1e-10)
    assert res.iterations == 1 and res.status == "converged" and res.true_relres <= 1e-10


def test_residual_estimate_is_monotone_and_true_at_restarts():
    """GMRES minimises the residual over a growing space: the estimate never
    increases within a cycle, and at a restart it equals the true residual."""
    H, fs = _mp2a(64, 20.0, 0.05)
    pre = O.mg_preconditioner(H, O.CycleOptions(smoother="gmres"))
    res = O.fgmres(H.A[0], fs, pre, m=4, tol=1e-8, max_iter=40)
    assert res.status == "converged"
    h = res.history
    for a in range(0, len(h), 4):
        seg = h[a:a + 4]
        assert all(seg[i + 1] <= seg[i] * (1 + 1e-12) for i in range(len(seg) - 1))
    assert abs(res.true_relres - h[-1]) <= 1e-3 * h[-1]


def test_preconditioned_iterations_fewer_than_standalone_cycles():
    """MG-preconditioned FGMRES needs fewer cycles (preconditioner applications)
    than stand-alone V-cycles for the same tolerance, also where stand-alone
    Jacobi-smoothed cycles need many (config 1 shape, shift 0.7)."""
    H, fs = _mp2a(64, 20.0, 0.7)
    opts = O.CycleOptions(smoother="jacobi")
    alone = O.solve(H, fs, opts, tol=1e-6, max_cycles=400)
    res = O.fgmres(H.A[0], fs, O.mg_preconditioner(H, opts), m=30, tol=1e-6, max_iter=400)
    assert res.status == "converged" and res.true_relres <= 1e-6 * 1.001
    assert res.iterations < alone.cycles / 2, (res.iterations, alone.cycles)
