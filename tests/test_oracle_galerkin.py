"""Pins of the Galerkin coarse operators on the shifted Laplacian (paper §3, §4)."""
import numpy as np
import pytest
from scipy.signal import convolve2d

import oracle as O
from paper_2308_13476_amd import workloads as W

M1 = np.array([1, 4, 6, 4, 1]) / 8.0
M2 = np.outer(M1, M1)


def _row_stencil(A, nl, I, J, r):
    """Coefficients of row (I, J) of a level matrix on offsets [-r, r]^2, indexed [dy, dx]."""
    row = A.getrow(J * (nl + 1) + I).toarray().ravel().reshape(nl + 1, nl + 1)
    return row[J - r:J + r + 1, I - r:I + r + 1]


def _galerkin_interior(stencil):
    """Interior coarse stencil of R S P for a translation-invariant fine stencil S:
    (1/4) (M2 * S * M2) sampled at even offsets (convolution of the masks)."""
    full = 0.25 * convolve2d(convolve2d(M2, stencil), M2)
    c = full.shape[0] // 2
    r = c // 2
    return full[c - 2 * r:c + 2 * r + 1:2, c - 2 * r:c + 2 * r + 1:2]


def test_interior_stencils_match_mask_convolution():
    n, k, beta = 64, 20.0, 0.7
    h = 1.0 / n
    H = O.build_hierarchy(W.constant_k2(n, k), h, beta)
    fine = np.array([[0, -1, 0], [-1, 4, -1], [0, -1, 0]], dtype=complex) / h**2
    fine[1, 1] -= (1 + 1j * beta) * k * k
    s1 = _galerkin_interior(fine)  # 5 x 5: radius 2
    assert s1.shape == (5, 5)
    np.testing.assert_allclose(_row_stencil(H.A[1], 32, 16, 16, 2), s1, rtol=1e-13, atol=1e-9)
    s2 = _galerkin_interior(s1)  # 7 x 7: radius 3
    assert s2.shape == (7, 7)
    np.testing.assert_allclose(_row_stencil(H.A[2], 16, 8, 8, 3), s2, rtol=1e-12, atol=1e-8)


def _radius(A, nl):
    A = A.tocoo()
    I1, J1 = A.row % (nl + 1), A.row // (nl + 1)
    I2, J2 = A.col % (nl + 1), A.col // (nl + 1)
    return max(np.abs(I1 - I2).max(), np.abs(J1 - J2).max())


@pytest.mark.parametrize("transfer,radii", [("bezier", [1, 2, 3, 3, 3]), ("linear", [1, 1, 1, 1, 1])])
def test_stencil_radius_and_symmetry(transfer, radii):
    """Every level operator is complex symmetric (A = A^T, not Hermitian): A_s = W A
    and its shifted form are, and R = P^T / 4 keeps it through R C P. The stencil
    passes read the lower half of each stored stencil from the mirrored
    neighbour's upper half on the strength of this."""
    n = 64
    k2 = W.random_k2(n, 4, 10.0, 30.0)
    H = O.build_hierarchy(k2, 1.0 / n, 0.05, transfer=transfer)
    assert [_radius(A, nl) for A, nl in zip(H.A, H.n)] == radii
    for A in H.A:
        scale = abs(A).max()
        assert abs(A - A.T).max() <= 1e-14 * scale
        assert abs(A - A.conj().T).max() > 1e-3 * scale  # symmetric, not Hermitian


def test_shift_enters_only_through_the_first_coarsening():
    n = 32
    k2 = W.constant_k2(n, 12.0)
    H0 = O.build_hierarchy(k2, 1.0 / n, 0.0)
    H1 = O.build_hierarchy(k2, 1.0 / n, 0.5)
    assert abs(H0.A[0] - H1.A[0]).max() == 0.0
    # A_1(beta) - A_1(0) = -i beta R W K^2 P
    Wk = O.restriction(n) @ (O.shifted_laplacian(k2, 1 / n, 1.0) - O.helmholtz_matrix(k2, 1 / n)) @ O.prolongation(n)
    np.testing.assert_allclose((H1.A[1] - H0.A[1]).toarray(), 0.5 * Wk.toarray(), atol=1e-9)
