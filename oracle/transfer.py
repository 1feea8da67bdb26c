"""Intergrid transfer operators (paper §4, the Bézier prolongation formula).

TEST INFRASTRUCTURE ONLY (see the package header).

The higher-order prolongation of §4 (taken from the quadratic rational Bézier
scheme) maps a coarse grid function e (spacing 2h) to the fine grid by
  fine node i even:  (e[(i-2)/2] + 6 e[i/2] + e[(i+2)/2]) / 8
  fine node i odd :  (e[(i-1)/2] + e[(i+1)/2]) / 2
The odd rule is linear interpolation (§4 notes this); the "linear" transfer of
Table 1 uses the odd rule together with injection-like e[i/2] at even nodes.

Readings: vertex grids (fine even nodes coincide with coarse nodes); coarse
indices outside the grid are dropped (truncation at the boundary); the 2D
operator is the tensor product of the 1D rule; restriction is the transpose of
prolongation (§1, §4) scaled by 1/4 so that interior rows sum to one.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def prolongation_1d(n_fine: int, kind: str = "bezier", first: int = 0, last: int | None = None) -> sp.csr_matrix:
    """1D prolongation from nodes first..n_fine/2 - (n_fine - last)/2 to nodes first..last.

    With the defaults the fine grid holds nodes 0..n_fine and the coarse grid
    0..n_fine/2 (absorbing-boundary problems). The Dirichlet variant passes
    first=1, last=n_fine-1 so that only interior nodes are unknowns.
    """
    if last is None:
        last = n_fine
    nc = n_fine // 2
    c_first = (first + 1) // 2
    c_last = last // 2
    rows, cols, vals = [], [], []

    def add(i, J, w):
        if c_first <= J <= c_last:  # coarse indices outside the grid are dropped
            rows.append(i - first)
            cols.append(J - c_first)
            vals.append(w)

    for i in range(first, last + 1):
        if i % 2 == 0:
            if kind == "bezier":
                add(i, (i - 2) // 2, 1.0 / 8.0)
                add(i, i // 2, 6.0 / 8.0)
                add(i, (i + 2) // 2, 1.0 / 8.0)
            elif kind == "linear":
                add(i, i // 2, 1.0)
            else:
                raise ValueError(kind)
        else:
            add(i, (i - 1) // 2, 0.5)
            add(i, (i + 1) // 2, 0.5)
    shape = (last - first + 1, c_last - c_first + 1)
    assert nc >= c_last
    return sp.csr_matrix((vals, (rows, cols)), shape=shape)


def prolongation(n_fine: int, kind: str = "bezier", dirichlet: bool = False) -> sp.csr_matrix:
    """2D prolongation P = P1 (x) P1 (tensor product of the 1D rule, y slow, x fast)."""
    if dirichlet:
        P1 = prolongation_1d(n_fine, kind, first=1, last=n_fine - 1)
    else:
        P1 = prolongation_1d(n_fine, kind)
    return sp.kron(P1, P1, format="csr")


def restriction(n_fine: int, kind: str = "bezier", dirichlet: bool = False, scale: float = 0.25) -> sp.csr_matrix:
    """Restriction R = scale * P^T (the paper takes R as the transpose of P)."""
    return (scale * prolongation(n_fine, kind, dirichlet).T).tocsr()
