"""Stand-alone multigrid for the Helmholtz operator: hierarchy, smoothers, cycles.

TEST INFRASTRUCTURE ONLY (see the package header).

Follows the paper's algorithm:
  * coarse grid correction with Galerkin coarse operators (§3), built on the
    complex shifted Laplacian C instead of A (§4, Table 1; shift beta_2 of §5);
  * weighted Jacobi smoothing S = I - X^{-1} A, X = omega diag(A) (§3), so the
    damping factor is 1/omega (omega = 3/2 for Poisson, 4.5 here, §4.2 and §5);
  * alternatively GMRES(3) smoothing: each smoothing step is one restart cycle
    of three unpreconditioned GMRES iterations from the current iterate (§5.3);
  * V-cycles (gamma = 1) and W-cycles (gamma = 2) with nu pre- and nu
    post-smoothing steps (Tables 4-9), coarsening down to a small grid that is
    solved directly (§5), stopping on the relative residual (§5).

Readings: the shift enters only at the first coarsening, A_1 = R C_s P, and
deeper levels are Galerkin products of the level above, A_{l+1} = R A_l P; the
relative residual is the 2-norm of f_s - A_s u over the 2-norm of f_s.

The FP32-in-FP64 refinement (`solve_refined`) is not in the paper: the outer
residual and the correction are FP64, one cycle runs in complex64 on the
residual with a zero initial guess, and the coarsest direct solve stays FP64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .operator import dirichlet_helmholtz_matrix, helmholtz_matrix, shifted_laplacian
from .transfer import prolongation, restriction


@dataclass
class Hierarchy:
    """Level operators A[l] (A[0] = A_s), transfers P[l]: level l+1 -> l, R[l]: l -> l+1."""

    n: list
    A: list
    P: list
    R: list
    lu: tuple
    A32: list = field(default_factory=list)
    P32: list = field(default_factory=list)
    R32: list = field(default_factory=list)

    @property
    def levels(self) -> int:
        return len(self.A)


def build_hierarchy(k2: np.ndarray, h: float, beta2: float, levels: int = 0, transfer: str = "bezier",
                    coarsest_n: int = 4, r_scale: float = 0.25) -> Hierarchy:
    """Galerkin hierarchy on the shifted Laplacian (§3, §4).

    A_0 = A_s (the operator being solved), A_1 = R C_s P, A_{l+1} = R A_l P.
    `levels` = 0 coarsens until the grid has `coarsest_n` intervals per side.
    """
    n = k2.shape[0] - 1
    if levels <= 0:
        levels = 1
        m = n
        while m > coarsest_n:
            if m % 2:
                raise ValueError("grid cannot be halved down to the coarsest size")
            m //= 2
            levels += 1
    if levels < 2:
        raise ValueError("need at least two levels")
    if n % (1 << (levels - 1)):
        raise ValueError("n is not divisible by 2^(levels-1)")
    A_s = helmholtz_matrix(k2, h)
    C_s = shifted_laplacian(k2, h, beta2)
    ns, A, P, R = [n], [A_s], [], []
    for l in range(levels - 1):
        nl = ns[-1]
        Pl = prolongation(nl, transfer)
        Rl = restriction(nl, transfer, scale=r_scale)
        fine_op = C_s if l == 0 else A[-1]
        Ac = (Rl @ fine_op @ Pl).tocsr()
        Ac.sum_duplicates()
        P.append(Pl.tocsr())
        R.append(Rl.tocsr())
        A.append(Ac)
        ns.append(nl // 2)
    lu = sla.lu_factor(A[-1].toarray())
    hier = Hierarchy(n=ns, A=A, P=P, R=R, lu=lu)
    hier.A32 = [a.astype(np.complex64) for a in A]
    hier.P32 = [p.astype(np.float32) for p in P]
    hier.R32 = [r.astype(np.float32) for r in R]
    return hier


def build_dirichlet_hierarchy(n: int, k: float, coarsest_n: int = 4, transfer: str = "bezier") -> Hierarchy:
    """Galerkin hierarchy for -Laplace - k^2 with homogeneous Dirichlet data (interior unknowns).

    Only for the mesh-independence check at k = 0; the transfer rule is the §4
    formula with coarse values outside the interior taken as zero.
    """
    h = 1.0 / n
    ns, A, P, R = [n], [dirichlet_helmholtz_matrix(n, h, k)], [], []
    while ns[-1] > coarsest_n:
        nl = ns[-1]
        Pl = prolongation(nl, transfer, dirichlet=True)
        Rl = restriction(nl, transfer, dirichlet=True)
        A.append((Rl @ A[-1] @ Pl).tocsr())
        P.append(Pl.tocsr())
        R.append(Rl.tocsr())
        ns.append(nl // 2)
    lu = sla.lu_factor(A[-1].toarray())
    return Hierarchy(n=ns, A=A, P=P, R=R, lu=lu)


def jacobi_step(A: sp.csr_matrix, u: np.ndarray, f: np.ndarray, omega: float) -> np.ndarray:
    """One weighted-Jacobi step u + (omega diag(A))^{-1} (f - A u)  (§3)."""
    d = A.diagonal()
    return u + (f - A @ u) / (omega * d)


def _dot(x: np.ndarray, y: np.ndarray) -> complex:
    """Hermitian inner product sum(conj(x) y), accumulated in FP64."""
    return complex(np.vdot(x.astype(np.complex128), y.astype(np.complex128)))


def _norm(x: np.ndarray) -> float:
    return float(np.sqrt(_dot(x, x).real))


def gmres_step(A: sp.csr_matrix, u: np.ndarray, f: np.ndarray, m: int = 3, breakdown: float = 1e-14) -> np.ndarray:
    """One GMRES(m) smoothing step from the current iterate (§5.3, m = 3).

    Arnoldi with modified Gram-Schmidt on r0 = f - A u, then the (m+1) x m
    least-squares problem min || beta e1 - H y ||, then u + V_m y.
    Vectors keep the dtype of u; inner products and H are FP64.
    A subdiagonal entry below `breakdown` * beta ends the Arnoldi process early.
    """
    dt = u.dtype
    r0 = (f - A @ u).astype(dt)
    beta = _norm(r0)
    if beta == 0.0:
        return u
    V = [(r0 / beta).astype(dt)]
    H = np.zeros((m + 1, m), dtype=np.complex128)
    k = m
    for j in range(m):
        w = (A @ V[j]).astype(dt)
        for i in range(j + 1):
            H[i, j] = _dot(V[i], w)
            w = (w - dt.type(H[i, j]) * V[i]).astype(dt)
        H[j + 1, j] = _norm(w)
        if H[j + 1, j].real <= breakdown * beta:
            k = j + 1
            break
        V.append((w / H[j + 1, j].real).astype(dt))
    rhs = np.zeros(k + 1, dtype=np.complex128)
    rhs[0] = beta
    y = np.linalg.lstsq(H[: k + 1, :k], rhs, rcond=None)[0]
    for i in range(k):
        u = (u + dt.type(y[i]) * V[i]).astype(dt)
    return u


@dataclass
class CycleOptions:
    gamma: int = 1               # 1 = V-cycle, 2 = W-cycle
    smoother: str = "jacobi"     # "jacobi" or "gmres"
    nu1: int = 1
    nu2: int = 1
    omega: float = 4.5           # paper-omega: damping 1/omega


def _smooth(A, u, f, opts: CycleOptions):
    if opts.smoother == "jacobi":
        return jacobi_step(A, u, f, opts.omega)
    if opts.smoother == "gmres":
        brk = 1e-14 if u.dtype == np.complex128 else 1e-6
        return gmres_step(A, u, f, 3, brk)
    raise ValueError(opts.smoother)


def cycle(hier: Hierarchy, l: int, u: np.ndarray, f: np.ndarray, opts: CycleOptions, fp32: bool = False) -> np.ndarray:
    """Recursive multigrid cycle on level l (§3 coarse grid correction, §5 V/W cycles).

    nu1 pre-smoothing steps, residual restriction, gamma recursive cycles on the
    coarse correction starting from zero, prolongation and correction, nu2
    post-smoothing steps. The coarsest level is solved directly (FP64 LU, also
    in the FP32 cycle).
    """
    A = hier.A32 if fp32 else hier.A
    P = hier.P32 if fp32 else hier.P
    R = hier.R32 if fp32 else hier.R
    if l == hier.levels - 1:
        x = sla.lu_solve(hier.lu, f.astype(np.complex128))
        return x.astype(f.dtype)
    for _ in range(opts.nu1):
        u = _smooth(A[l], u, f, opts)
    fc = (R[l] @ (f - A[l] @ u)).astype(u.dtype)
    e = np.zeros(fc.shape, dtype=u.dtype)
    for _ in range(opts.gamma):
        e = cycle(hier, l + 1, e, fc, opts, fp32)
    u = (u + P[l] @ e).astype(u.dtype)
    for _ in range(opts.nu2):
        u = _smooth(A[l], u, f, opts)
    return u


@dataclass
class SolveResult:
    x: np.ndarray
    cycles: int
    history: list
    status: str  # "converged", "not_converged", "diverged"


def solve(hier: Hierarchy, f_s: np.ndarray, opts: CycleOptions, tol: float = 1e-6, max_cycles: int = 500,
          x0: np.ndarray | None = None, divergence: float = 1e8) -> SolveResult:
    """Stand-alone multigrid solve of A_s x = f_s in FP64 (§5).

    After every cycle the relative residual ||f_s - A_s x|| / ||f_s|| is
    compared with `tol`. Non-finite residuals, or residuals `divergence` times
    above the initial one, stop the iteration as diverged.
    """
    A0 = hier.A[0]
    f_s = np.asarray(f_s, dtype=np.complex128).ravel()
    x = np.zeros_like(f_s) if x0 is None else np.asarray(x0, dtype=np.complex128).ravel().copy()
    nf = np.linalg.norm(f_s)
    if nf == 0.0:
        return SolveResult(np.zeros_like(f_s), 0, [], "converged")
    rel0 = np.linalg.norm(f_s - A0 @ x) / nf
    if rel0 <= tol:
        return SolveResult(x, 0, [], "converged")
    hist = []
    for it in range(1, max_cycles + 1):
        x = cycle(hier, 0, x, f_s, opts)
        rel = float(np.linalg.norm(f_s - A0 @ x) / nf)
        hist.append(rel)
        if not np.isfinite(rel) or rel > divergence * rel0:
            return SolveResult(x, it, hist, "diverged")
        if rel <= tol:
            return SolveResult(x, it, hist, "converged")
    return SolveResult(x, max_cycles, hist, "not_converged")


def solve_refined(hier: Hierarchy, f_s: np.ndarray, opts: CycleOptions, tol: float = 1e-6, max_cycles: int = 500,
                  x0: np.ndarray | None = None, divergence: float = 1e8) -> SolveResult:
    """FP32 cycles inside FP64 iterative refinement (not in the paper).

    r = f_s - A_s x (FP64); e = one complex64 cycle on A e = r from e = 0 with the
    coarsest solve in FP64; x += e (FP64); stop on the FP64 relative residual.
    """
    A0 = hier.A[0]
    f_s = np.asarray(f_s, dtype=np.complex128).ravel()
    x = np.zeros_like(f_s) if x0 is None else np.asarray(x0, dtype=np.complex128).ravel().copy()
    nf = np.linalg.norm(f_s)
    if nf == 0.0:
        return SolveResult(np.zeros_like(f_s), 0, [], "converged")
    r = f_s - A0 @ x
    rel0 = np.linalg.norm(r) / nf
    if rel0 <= tol:
        return SolveResult(x, 0, [], "converged")
    hist = []
    for it in range(1, max_cycles + 1):
        r32 = r.astype(np.complex64)
        e = cycle(hier, 0, np.zeros_like(r32), r32, opts, fp32=True)
        x = x + e.astype(np.complex128)
        r = f_s - A0 @ x
        rel = float(np.linalg.norm(r) / nf)
        hist.append(rel)
        if not np.isfinite(rel) or rel > divergence * rel0:
            return SolveResult(x, it, hist, "diverged")
        if rel <= tol:
            return SolveResult(x, it, hist, "converged")
    return SolveResult(x, max_cycles, hist, "not_converged")
