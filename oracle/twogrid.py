"""Dense two-grid iteration matrix on tiny grids (paper §3, Table 1 of §4).

TEST INFRASTRUCTURE ONLY (see the package header).

T_0 = (I - P A_c^{-1} R A)(I - X^{-1} A) with X = omega diag(A): one Jacobi
smoothing step followed by an exact coarse grid correction (§3). A_c is the
Galerkin product of either A itself or the shifted Laplacian C (§4, Table 1).
"""
from __future__ import annotations

import numpy as np

from .operator import helmholtz_matrix, shifted_laplacian
from .transfer import prolongation, restriction


def two_grid_matrix(k: float, n: int, beta2: float = 0.7, transfer: str = "bezier", coarse_on: str = "C",
                    omega: float = 4.5) -> np.ndarray:
    """Dense T_0 for constant k on an n-interval grid (scaled operator A_s)."""
    h = 1.0 / n
    k2 = np.full((n + 1, n + 1), float(k) ** 2)
    A = helmholtz_matrix(k2, h).toarray()
    M = shifted_laplacian(k2, h, beta2).toarray() if coarse_on == "C" else A
    P = prolongation(n, transfer).toarray()
    R = restriction(n, transfer).toarray()
    Ac = R @ M @ P
    I = np.eye(A.shape[0])
    cgc = I - P @ np.linalg.solve(Ac, R @ A)
    smoother = I - A / (omega * np.diag(A))[:, None]
    return cgc @ smoother


def spectral_norm(T: np.ndarray) -> float:
    """Largest singular value of a dense matrix."""
    return float(np.linalg.norm(T, 2))


def spectral_radius(T: np.ndarray) -> float:
    """Largest eigenvalue modulus of a dense matrix."""
    return float(np.max(np.abs(np.linalg.eigvals(T))))
