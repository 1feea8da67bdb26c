"""Pins of the oracle's discrete operator (paper §2) against facts fixed outside it."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_2308_13476_amd import workloads as W


def test_scaled_operator_is_complex_symmetric():
    rng = np.random.default_rng(0)
    n = 12
    k2 = rng.uniform(20.0, 90.0, size=(n + 1, n + 1))
    A = O.helmholtz_matrix(k2, 1.0 / n)
    assert abs(A - A.T).max() == 0.0
    # the unscaled operator is not symmetric: the scaling is what symmetrises it
    A_raw = O.helmholtz_matrix(k2, 1.0 / n, scaled=False)
    assert abs(A_raw - A_raw.T).max() > 0.0


def test_rows_from_ghost_elimination_by_hand():
    """Rows written out by hand for n = 4, h = 1/4, k = 3 from the central-difference
    ghost elimination u_ghost = u_mirror + 2 i h k u_b of the absorbing condition."""
    n, h, k = 4, 0.25, 3.0
    A = O.helmholtz_matrix(W.constant_k2(n, k), h, scaled=False).toarray()
    p = lambda i, j: j * (n + 1) + i  # noqa: E731
    ih2 = 1.0 / h**2  # 16
    # interior node (2, 2): 5-point stencil minus k^2
    row = A[p(2, 2)]
    assert row[p(2, 2)] == pytest.approx(4 * ih2 - 9.0)
    for q in [p(1, 2), p(3, 2), p(2, 1), p(2, 3)]:
        assert row[q] == pytest.approx(-ih2)
    assert np.count_nonzero(row) == 5
    # left edge node (0, 2): the ghost at i = -1 is folded onto (1, 2)
    row = A[p(0, 2)]
    assert row[p(0, 2)] == pytest.approx(4 * ih2 - 9.0 - 2j * k / h)
    assert row[p(1, 2)] == pytest.approx(-2 * ih2)
    assert row[p(0, 1)] == pytest.approx(-ih2) and row[p(0, 3)] == pytest.approx(-ih2)
    assert np.count_nonzero(row) == 4
    # corner (4, 4): two ghosts, two doubled couplings
    row = A[p(4, 4)]
    assert row[p(4, 4)] == pytest.approx(4 * ih2 - 9.0 - 4j * k / h)
    assert row[p(3, 4)] == pytest.approx(-2 * ih2) and row[p(4, 3)] == pytest.approx(-2 * ih2)
    assert np.count_nonzero(row) == 3


def _plane_wave_problem(n, k, theta):
    """Discrete rhs for the plane wave u* = exp(i k (x cos t + y sin t)), which solves the
    homogeneous Helmholtz equation with inhomogeneous absorbing data g = du/dn - i k u.
    The ghost elimination adds (2/h) g per boundary side to the right-hand side."""
    h = 1.0 / n
    x = np.arange(n + 1) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.exp(1j * k * (X * np.cos(theta) + Y * np.sin(theta)))
    f = np.zeros_like(u)
    c, s = np.cos(theta), np.sin(theta)
    f[:, 0] += 2.0 / h * (-1j * k * (1 + c)) * u[:, 0]      # x = 0, normal -x
    f[:, -1] += 2.0 / h * (1j * k * (c - 1)) * u[:, -1]     # x = 1, normal +x
    f[0, :] += 2.0 / h * (-1j * k * (1 + s)) * u[0, :]      # y = 0, normal -y
    f[-1, :] += 2.0 / h * (1j * k * (s - 1)) * u[-1, :]     # y = 1, normal +y
    return u, f


def test_second_order_convergence_to_plane_wave():
    """O(h^2) convergence of the discrete solution to an exact solution of the PDE + BC."""
    k, theta = 10.0, 0.3
    errs = []
    for n in [32, 64, 128, 256]:
        u_exact, f = _plane_wave_problem(n, k, theta)
        A = O.helmholtz_matrix(W.constant_k2(n, k), 1.0 / n).tocsc()
        u = spla.spsolve(A, O.scaled_rhs(f).ravel()).reshape(n + 1, n + 1)
        errs.append(np.abs(u - u_exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios[1:]), (errs, ratios)


def test_direct_solve_residual():
    n, k = 64, 20.0
    A = O.helmholtz_matrix(W.constant_k2(n, k), 1.0 / n).tocsc()
    f = O.scaled_rhs(W.point_source_rhs(n, [W.center_node(n)])[0]).ravel()
    u = spla.splu(A).solve(f)
    assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) < 1e-13


def test_shifted_laplacian_differs_only_on_the_diagonal():
    n = 8
    k2 = np.random.default_rng(1).uniform(10, 50, size=(n + 1, n + 1))
    A = O.helmholtz_matrix(k2, 1.0 / n)
    C = O.shifted_laplacian(k2, 1.0 / n, 0.7)
    D = (C - A).toarray()
    assert np.allclose(D, np.diag(np.diag(D)))
    # -(1 + i b) k^2 W: the added part is -0.7 i W k^2
    assert np.allclose(np.diag(D), -0.7j * (O.node_weights(n) * k2).ravel())
