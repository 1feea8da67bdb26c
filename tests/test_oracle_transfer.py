"""Pins of the oracle's transfer operators (paper §4, Bézier prolongation)."""
import numpy as np

import oracle as O


def test_interior_column_is_cubic_bspline_mask():
    """A coarse unit spike prolongs to [1, 4, 6, 4, 1]/8 on the fine grid."""
    P = O.prolongation_1d(16).toarray()
    col = P[:, 4]  # coarse node 4 sits on fine node 8
    expect = np.zeros(17)
    expect[6:11] = np.array([1, 4, 6, 4, 1]) / 8.0
    np.testing.assert_array_equal(col, expect)
    L = O.prolongation_1d(16, "linear").toarray()[:, 4]
    expect = np.zeros(17)
    expect[7:10] = [0.5, 1.0, 0.5]
    np.testing.assert_array_equal(L, expect)


def test_truncation_at_the_boundary():
    """Coarse indices outside the grid are dropped: fine node 0 gets (6 e0 + e1)/8."""
    P = O.prolongation_1d(8).toarray()
    np.testing.assert_array_equal(P[0, :3], [6 / 8, 1 / 8, 0])
    np.testing.assert_array_equal(P[8, -3:], [0, 1 / 8, 6 / 8])
    np.testing.assert_array_equal(P[1, :3], [0.5, 0.5, 0])


def test_symbol_on_a_periodic_grid():
    """Fourier symbol of the mask is 2 cos^4(t/2) (4th-order zero at pi); linear: 2 cos^2(t/2)."""
    m = O.prolongation_1d(64).toarray()[:, 16]
    offs = np.arange(65) - 32
    for t in np.linspace(0, np.pi, 9):
        sym = np.sum(m * np.exp(-1j * offs * t))
        assert abs(sym - 2 * np.cos(t / 2) ** 4) < 1e-14
    ml = O.prolongation_1d(64, "linear").toarray()[:, 16]
    for t in np.linspace(0, np.pi, 9):
        assert abs(np.sum(ml * np.exp(-1j * offs * t)) - 2 * np.cos(t / 2) ** 2) < 1e-14


def test_exact_on_linear_functions_inside():
    n = 32
    P = O.prolongation_1d(n).toarray()
    X = np.arange(n // 2 + 1) * 2.0
    x = np.arange(n + 1) * 1.0
    out = P @ (3.0 + 0.25 * X)
    np.testing.assert_allclose(out[1:-1], 3.0 + 0.25 * x[1:-1], rtol=0, atol=1e-14)


def test_restriction_rows_sum_to_one_and_is_scaled_transpose():
    n = 16
    R = O.restriction(n).toarray()
    P = O.prolongation(n).toarray()
    np.testing.assert_array_equal(R, 0.25 * P.T)
    nc = n // 2
    for J in range(2, nc - 1):
        for I in range(2, nc - 1):
            assert abs(R[J * (nc + 1) + I].sum() - 1.0) < 1e-15
    # interior 2D row is the outer product of [1, 4, 6, 4, 1]/16
    row = R[4 * (nc + 1) + 4].reshape(n + 1, n + 1)[6:11, 6:11]
    m = np.array([1, 4, 6, 4, 1]) / 16.0
    np.testing.assert_allclose(row, np.outer(m, m), rtol=0, atol=1e-16)


def test_2d_is_tensor_product():
    n = 8
    P = O.prolongation(n).toarray()
    P1 = O.prolongation_1d(n).toarray()
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(n // 2 + 1), rng.standard_normal(n // 2 + 1)
    coarse = np.outer(b, a).ravel()  # [J, I] with x fastest
    np.testing.assert_allclose((P @ coarse).reshape(n + 1, n + 1), np.outer(P1 @ b, P1 @ a), atol=1e-14)
