"""Flexible GMRES with a multigrid cycle as right preconditioner.

TEST INFRASTRUCTURE ONLY (see the package header).

§1 names the deployment of multigrid on the complex shifted Laplacian as a
preconditioner for a Krylov method such as GMRES; this module writes out the
outer iteration: restarted flexible GMRES(m) in FP64 on A_s x = f_s, where
the j-th search direction is z_j = M_j(v_j), one multigrid cycle (§3, §5) on
A_s z = v_j started from z = 0 (FP64, or complex64 with FP64 coarsest solve).
Flexible (Z stored next to V) because a cycle with GMRES smoothing is a
nonlinear map of v_j.

Arnoldi uses modified Gram-Schmidt; the (j+2) x (j+1) least-squares problem
is solved with a library least-squares routine at every step, whose residual
is the iteration's residual estimate. The iterate is formed at the end of
every restart cycle, where the true relative residual is also computed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .multigrid import CycleOptions, Hierarchy, cycle


def _dot(x: np.ndarray, y: np.ndarray) -> complex:
    return complex(np.vdot(x, y))


def mg_preconditioner(hier: Hierarchy, opts: CycleOptions, fp32: bool = False):
    """z = M(v): one multigrid cycle on A_s z = v from z = 0 (complex64 cycle when fp32)."""
    def apply(v: np.ndarray) -> np.ndarray:
        dt = np.complex64 if fp32 else np.complex128
        z = cycle(hier, 0, np.zeros(v.shape, dtype=dt), v.astype(dt), opts, fp32=fp32)
        return z.astype(np.complex128)
    return apply


@dataclass
class FgmresResult:
    x: np.ndarray
    iterations: int      # preconditioner applications
    history: list        # residual estimate ||f_s - A_s x_j|| / ||f_s|| after every iteration
    status: str          # "converged" or "not_converged"
    true_relres: float   # at the returned iterate


def fgmres(A, f_s: np.ndarray, precond, m: int = 20, tol: float = 1e-6, max_iter: int = 500,
           x0: np.ndarray | None = None) -> FgmresResult:
    """Restarted right-preconditioned flexible GMRES(m) on A x = f_s (FP64).

    Per restart: r = f_s - A x, beta = ||r||, v_0 = r / beta; for j = 0..m-1:
    z_j = precond(v_j), w = A z_j, modified Gram-Schmidt against v_0..v_j into
    column j of H, v_{j+1} = w / H[j+1, j]; y_j = argmin ||beta e_1 - H y||;
    stop the cycle when ||beta e_1 - H y_j|| / ||f_s|| <= tol or j = m-1; then
    x += Z y. The solve stops when that estimate has reached tol (the true
    relative residual is returned next to it) or after max_iter applications.
    """
    f_s = np.asarray(f_s, dtype=np.complex128).ravel()
    x = np.zeros_like(f_s) if x0 is None else np.asarray(x0, dtype=np.complex128).ravel().copy()
    nf = float(np.linalg.norm(f_s))
    if nf == 0.0:
        return FgmresResult(np.zeros_like(f_s), 0, [], "converged", 0.0)
    hist: list = []
    it = 0
    while True:
        r = f_s - A @ x
        beta = float(np.linalg.norm(r))
        if beta / nf <= tol:
            return FgmresResult(x, it, hist, "converged", beta / nf)
        if it >= max_iter:
            return FgmresResult(x, it, hist, "not_converged", beta / nf)
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        y = np.zeros(0, dtype=np.complex128)
        done = False
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = A @ z
            for i in range(j + 1):
                H[i, j] = _dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            g = np.zeros(j + 2, dtype=np.complex128)
            g[0] = beta
            y = np.linalg.lstsq(H[: j + 2, : j + 1], g, rcond=None)[0]
            est = float(np.linalg.norm(g - H[: j + 2, : j + 1] @ y)) / nf
            it += 1
            hist.append(est)
            if est <= tol or it >= max_iter or H[j + 1, j] == 0.0:
                done = est <= tol
                break
            V.append(w / H[j + 1, j].real)
        for i in range(len(y)):
            x = x + y[i] * Z[i]
        if done or it >= max_iter:
            rel = float(np.linalg.norm(f_s - A @ x)) / nf
            return FgmresResult(x, it, hist, "converged" if done else "not_converged", rel)
