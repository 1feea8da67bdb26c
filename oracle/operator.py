"""Discrete Helmholtz operators of the model problems (paper §2).

TEST INFRASTRUCTURE ONLY (see the package header).

MP 2-A / MP 2-B (§2): -Laplace(u) - k(x,y)^2 u = f on [0,1]^2 with the
first-order absorbing (Sommerfeld) condition du/dn - i k u = 0 on the whole
boundary, discretised by second-order finite differences with h = 1/n.

Readings (the paper does not write the discrete boundary rows):
  * vertex-centred grid, n intervals, (n+1)^2 unknowns including the boundary;
  * the boundary condition is imposed with a central difference over a ghost
    node, u_ghost = u_mirror + 2 i h k u_b, which eliminates the ghost from the
    5-point row: the interior-normal neighbour gets weight 2 and the diagonal
    gains -2 i k / h per boundary side;
  * rows are scaled by W = diag(w_i w_j) with w = 1/2 on the two end nodes of a
    line and 1 elsewhere; the scaled matrix A_s = W A is complex symmetric.

Node p = (i, j) is flattened as p = j (n+1) + i (x fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def boundary_sides(n: int) -> np.ndarray:
    """s[j, i] = [i in {0, n}] + [j in {0, n}], the number of boundary sides of a node."""
    on = np.zeros(n + 1)
    on[0] = on[n] = 1.0
    return on[:, None] + on[None, :]


def node_weights(n: int) -> np.ndarray:
    """W[j, i] = w_i w_j with w = 1/2 at the two ends of a grid line, else 1."""
    w = np.ones(n + 1)
    w[0] = w[n] = 0.5
    return w[:, None] * w[None, :]


def laplacian_1d_sommerfeld(n: int) -> sp.csr_matrix:
    """1D second difference on n+1 vertex nodes (times h^2) with the ghost node of the
    absorbing boundary eliminated: rows 0 and n read (2, -2); interior rows (-1, 2, -1).

    The -2 i h k u_b part of the ghost elimination is diagonal and is added in 2D.
    """
    T = sp.diags([-np.ones(n), 2.0 * np.ones(n + 1), -np.ones(n)], [-1, 0, 1], format="lil")
    T[0, 1] = -2.0
    T[n, n - 1] = -2.0
    return T.tocsr()


def helmholtz_matrix(k2: np.ndarray, h: float, scaled: bool = True) -> sp.csr_matrix:
    """Discrete MP 2-A/2-B operator (§2).

    A = (I (x) T + T (x) I)/h^2 - diag(k^2) - (2 i / h) diag(k s), with T from
    `laplacian_1d_sommerfeld`, s the boundary side count and k = sqrt(k^2).
    Returns A_s = W A when `scaled`, else A.
    """
    n = k2.shape[0] - 1
    I = sp.identity(n + 1, format="csr")
    T = laplacian_1d_sommerfeld(n)
    lap = (sp.kron(I, T) + sp.kron(T, I)) / (h * h)
    k = np.sqrt(k2)
    s = boundary_sides(n)
    diag = -(k2 + 2j * k * s / h).ravel()
    A = (lap + sp.diags(diag)).astype(np.complex128).tocsr()
    if scaled:
        A = (sp.diags(node_weights(n).ravel()) @ A).tocsr()
    return A


def shifted_laplacian(k2: np.ndarray, h: float, beta2: float) -> sp.csr_matrix:
    """Complex shifted Laplacian used for coarsening (§4; shift beta_2 of §5).

    Reading: C = -Laplace - (1 + i beta_2) k^2 with the same absorbing boundary,
    i.e. C_s = A_s - i beta_2 W diag(k^2). The paper never writes C out; the sign
    of the shift is the one that damps together with the boundary term.
    """
    n = k2.shape[0] - 1
    A_s = helmholtz_matrix(k2, h, scaled=True)
    shift = sp.diags((node_weights(n) * k2).ravel())
    return (A_s - 1j * beta2 * shift).tocsr()


def scaled_rhs(f: np.ndarray) -> np.ndarray:
    """Right-hand side of the scaled system A_s u = W f (f given on the grid, [..., j, i])."""
    n = f.shape[-1] - 1
    return f * node_weights(n)


def dirichlet_helmholtz_matrix(n: int, h: float, k: float) -> sp.csr_matrix:
    """Interior (n-1)^2 unknowns with homogeneous Dirichlet data: -Laplace - k^2.

    Used only to check mesh-independent convergence at k = 0, where the absorbing
    condition degenerates to a Neumann one and the Sommerfeld matrix is singular.
    """
    m = n - 1
    T = sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    I = sp.identity(m)
    A = (sp.kron(I, T) + sp.kron(T, I)) / (h * h) - k * k * sp.identity(m * m)
    return A.astype(np.complex128).tocsr()
