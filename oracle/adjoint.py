"""Misfit and its adjoint-state gradient with respect to per-node k^2.

TEST INFRASTRUCTURE ONLY (see the package header).

Not in the paper. The forward model is the discretised MP 2-B operator of §2,
A_s(k^2) u = W f, solved here exactly with a sparse LU factorisation. For the
misfit J = 1/2 sum_src || S u - d ||^2 the adjoint state solves
A_s^H lambda = S^T (S u - d), and
  dJ/dk^2_p = -sum_src Re[ conj(lambda_p) (dA_s/dk^2_p)_pp u_p ],
  (dA_s/dk^2_p)_pp = -W_p (1 + i s_p / (h k_p)),
since only the diagonal of A_s depends on k^2 (the boundary term through
k = sqrt(k^2)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .operator import boundary_sides, helmholtz_matrix, node_weights, scaled_rhs


def forward(k2: np.ndarray, h: float, f: np.ndarray) -> np.ndarray:
    """Exact discrete solutions u[s] of A_s u = W f[s] for a stack of sources (S, n+1, n+1)."""
    A = helmholtz_matrix(k2, h).tocsc()
    lu = spla.splu(A)
    fs = scaled_rhs(f).reshape(f.shape[0], -1)
    return np.stack([lu.solve(fs[s]) for s in range(f.shape[0])]).reshape(f.shape)


def misfit(u: np.ndarray, rec_row: int, d: np.ndarray) -> float:
    """J = 1/2 sum over sources of || S u - d ||^2, S = restriction to receiver row `rec_row`."""
    res = u[:, rec_row, :] - d
    return 0.5 * float(np.sum(np.abs(res) ** 2))


def gradient(k2: np.ndarray, h: float, f: np.ndarray, rec_row: int, d: np.ndarray):
    """Adjoint-state gradient dJ/dk^2 (shape (n+1, n+1)) and the forward solutions."""
    n = k2.shape[0] - 1
    A = helmholtz_matrix(k2, h).tocsc()
    lu = spla.splu(A)
    AH = spla.splu(A.conj().T.tocsc())
    fs = scaled_rhs(f).reshape(f.shape[0], -1)
    Wn = node_weights(n)
    s = boundary_sides(n)
    k = np.sqrt(k2)
    dA = -Wn * (1.0 + 1j * s / (h * np.where(k > 0, k, np.inf)))
    g = np.zeros_like(k2)
    us = []
    for src in range(f.shape[0]):
        u = lu.solve(fs[src]).reshape(n + 1, n + 1)
        us.append(u)
        adj_rhs = np.zeros((n + 1, n + 1), dtype=np.complex128)
        adj_rhs[rec_row, :] = u[rec_row, :] - d[src]
        lam = AH.solve(adj_rhs.ravel()).reshape(n + 1, n + 1)
        g += -np.real(np.conj(lam) * dA * u)
    return g, np.stack(us)


def finite_difference(k2: np.ndarray, h: float, f: np.ndarray, rec_row: int, d: np.ndarray, node, rel_eps=1e-4):
    """Central difference of J in k^2 at one node (j, i), step rel_eps * k^2."""
    j, i = node
    eps = rel_eps * k2[j, i]
    kp = k2.copy()
    kp[j, i] += eps
    km = k2.copy()
    km[j, i] -= eps
    return (misfit(forward(kp, h, f), rec_row, d) - misfit(forward(km, h, f), rec_row, d)) / (2 * eps)
