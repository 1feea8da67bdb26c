"""Pins of the oracle's cycles and stopping rule (paper §3, §5)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_2308_13476_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mp2a(n, k):
    k2 = W.constant_k2(n, k)
    fs = O.scaled_rhs(W.point_source_rhs(n, [W.center_node(n)])[0]).ravel()
    return k2, fs


def test_converged_solution_equals_sparse_direct_solve():
    n, k = 64, 20.0
    k2, fs = _mp2a(n, k)
    H = O.build_hierarchy(k2, 1.0 / n, 1.0 / k)
    res = O.solve(H, fs, O.CycleOptions(smoother="gmres"), tol=1e-12)
    assert res.status == "converged"
    exact = spla.splu(O.helmholtz_matrix(k2, 1.0 / n).tocsc()).solve(fs)
    assert np.linalg.norm(res.x - exact) / np.linalg.norm(exact) < 1e-9


def test_v_equals_w_on_two_levels():
    n, k = 16, 8.0
    k2, fs = _mp2a(n, k)
    H = O.build_hierarchy(k2, 1.0 / n, 0.3, levels=2)
    for sm in ["jacobi", "gmres"]:
        v = O.solve(H, fs, O.CycleOptions(smoother=sm, gamma=1), tol=1e-30, max_cycles=4)
        w = O.solve(H, fs, O.CycleOptions(smoother=sm, gamma=2), tol=1e-30, max_cycles=4)
        np.testing.assert_array_equal(v.x, w.x)


def test_restriction_scale_does_not_change_the_iterates():
    """R = c P^T: Galerkin coarse operators scale by c, coarse right-hand sides by c,
    so corrections are unchanged for any c (Jacobi and GMRES are scale invariant)."""
    n, k = 32, 10.0
    k2, fs = _mp2a(n, k)
    for sm in ["jacobi", "gmres"]:
        a = O.solve(O.build_hierarchy(k2, 1 / n, 0.5, r_scale=0.25), fs, O.CycleOptions(smoother=sm), 1e-30,
                    max_cycles=5)
        b = O.solve(O.build_hierarchy(k2, 1 / n, 0.5, r_scale=1.0), fs, O.CycleOptions(smoother=sm), 1e-30,
                    max_cycles=5)
        assert np.linalg.norm(a.x - b.x) <= 1e-11 * np.linalg.norm(a.x)


def test_mesh_independent_convergence_at_k0():
    """k = 0 (Dirichlet variant; the absorbing condition turns Neumann and A_s is singular):
    the number of cycles to tolerance does not depend on h."""
    counts = []
    for n in [32, 64, 128, 256]:
        H = O.build_dirichlet_hierarchy(n, 0.0)
        f = np.zeros((n - 1) ** 2, complex)
        f[((n - 1) // 2) * (n - 1) + (n - 1) // 2] = n * n
        counts.append(O.solve(H, f, O.CycleOptions(smoother="jacobi", omega=1.5), tol=1e-8).cycles)
    assert max(counts) - min(counts) <= 1, counts
    assert max(counts) < 25


def test_paper_table8_counts_within_one():
    """GMRES(3), shift 1/k, k = 50 at kh = 0.625 (n = 80, coarsest 5 x 5 intervals), tol 1e-5."""
    g = json.load(open(os.path.join(GOLDEN, "table8_gmres_counts.json")))
    n, k = 80, float(g["k"])
    k2, fs = _mp2a(n, k)
    H = O.build_hierarchy(k2, 1.0 / n, 1.0 / k, levels=5)
    for nu, v_paper, w_paper in list(zip(g["nu"], g["V"], g["W"]))[:3]:
        v = O.solve(H, fs, O.CycleOptions(smoother="gmres", nu1=nu, nu2=nu, gamma=1), tol=1e-5).cycles
        w = O.solve(H, fs, O.CycleOptions(smoother="gmres", nu1=nu, nu2=nu, gamma=2), tol=1e-5).cycles
        assert abs(v - v_paper) <= 1 and abs(w - w_paper) <= 1, (nu, v, w)


def test_gmres_beats_jacobi_and_w_helps_gmres():
    """§5.3: GMRES(3) needs far fewer cycles than Jacobi; with a small shift W < V."""
    n, k = 64, 20.0
    k2, fs = _mp2a(n, k)
    jac = O.solve(O.build_hierarchy(k2, 1 / n, 0.7), fs, O.CycleOptions(smoother="jacobi"), 1e-6).cycles
    H = O.build_hierarchy(k2, 1 / n, 1 / k)
    gv = O.solve(H, fs, O.CycleOptions(smoother="gmres"), 1e-6).cycles
    gw = O.solve(H, fs, O.CycleOptions(smoother="gmres", gamma=2), 1e-6).cycles
    assert gv * 2.5 < jac and gw < gv


def test_divergence_and_cycle_limit_are_reported():
    n, k = 64, 40.0
    k2, fs = _mp2a(n, k)
    H = O.build_hierarchy(k2, 1 / n, 0.0)  # Jacobi on the unshifted coarse operators diverges
    res = O.solve(H, fs, O.CycleOptions(smoother="jacobi"), 1e-6, max_cycles=300, divergence=1e3)
    assert res.status == "diverged"
    H = O.build_hierarchy(k2, 1 / n, 1 / k)
    res = O.solve(H, fs, O.CycleOptions(smoother="gmres"), 1e-6, max_cycles=3)
    assert res.status == "not_converged" and res.cycles == 3


def test_restart_from_saved_iterate_is_exact():
    n, k = 32, 10.0
    k2, fs = _mp2a(n, k)
    H = O.build_hierarchy(k2, 1 / n, 0.1)
    opts = O.CycleOptions(smoother="gmres")
    full = O.solve(H, fs, opts, 1e-30, max_cycles=5)
    part = O.solve(H, fs, opts, 1e-30, max_cycles=2)
    rest = O.solve(H, fs, opts, 1e-30, max_cycles=3, x0=part.x)
    np.testing.assert_array_equal(full.x, rest.x)


@pytest.mark.parametrize("smoother,beta", [("gmres", 0.05), ("jacobi", 0.7)])
def test_fp32_refinement_reaches_fp64_tolerance(smoother, beta):
    n, k = 64, 20.0
    k2, fs = _mp2a(n, k)
    H = O.build_hierarchy(k2, 1 / n, beta)
    opts = O.CycleOptions(smoother=smoother)
    a = O.solve(H, fs, opts, 1e-6)
    b = O.solve_refined(H, fs, opts, 1e-6)
    assert b.status == "converged" and abs(a.cycles - b.cycles) <= 1
    A0 = H.A[0]
    assert np.linalg.norm(fs - A0 @ b.x) / np.linalg.norm(fs) <= 1e-6
