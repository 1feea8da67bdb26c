"""Differentiable Helmholtz solve: forward = multigrid solve (mg_solve), backward =
the same multigrid on the adjoint system plus the gradient kernel (mg_grad).

For solutions u = A_s(k^2)^{-1} W f and a real loss L(u), PyTorch hands the
backward pass grad_u = dL/du in its convention (dL = Re <grad_u, du>); the
library returns dL/dk^2 (real, per node, summed over sources) and dL/df.
"""
from __future__ import annotations

import warnings

import torch

from . import _binding as B
from .solver import Solver


def _check_converged(info: dict, what: str, opts: dict):
    """A solve that stopped at max_cycles (MG_NOT_CONVERGED) would hand the
    optimiser a wrong solution or gradient without a signal: raise, unless the
    caller allowed it (opts["allow_unconverged"]), then warn."""
    if info["status"] != B.MG_NOT_CONVERGED:
        return
    msg = (f"{what} solve stopped at max_cycles = {opts.get('max_cycles', 500)} with relative residuals "
           f"{info['relres']} above the tolerance")
    if not opts.get("allow_unconverged", False):
        raise B.MGError(B.MG_NOT_CONVERGED, msg + " (pass allow_unconverged=True to accept it)")
    warnings.warn(msg, RuntimeWarning, stacklevel=3)


class _HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k2, f, h, shift, opts):
        solver = Solver(k2.detach(), h, shift, levels=opts.get("levels", 0), transfer=opts.get("transfer", "bezier"),
                        precision=opts.get("setup_precision", "fp64"), max_batch=f.shape[0] if f.dim() == 3 else 1,
                        coarsest_n=opts.get("coarsest_n", 4))
        u, info = solver.solve(f.detach(), tol=opts.get("tol", 1e-10), cycle=opts.get("cycle", "V"),
                               smoother=opts.get("smoother", "gmres"), nu_pre=opts.get("nu_pre", 1),
                               nu_post=opts.get("nu_post", 1), omega=opts.get("omega", 4.5),
                               max_cycles=opts.get("max_cycles", 500), precision=opts.get("precision", "fp64"))
        _check_converged(info, "forward", opts)
        if f.dim() == 2:
            u = u[0]
        ctx.solver = solver
        ctx.opts = opts
        ctx.squeeze = f.dim() == 2
        ctx.save_for_backward(u)
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        o = ctx.opts
        gk2, grhs, ginfo = ctx.solver.grad(u, grad_u.contiguous(), tol=o.get("adjoint_tol", o.get("tol", 1e-10)),
                                       cycle=o.get("cycle", "V"), smoother=o.get("smoother", "gmres"),
                                       nu_pre=o.get("nu_pre", 1), nu_post=o.get("nu_post", 1),
                                       omega=o.get("omega", 4.5), max_cycles=o.get("max_cycles", 500),
                                       precision=o.get("precision", "fp64"), want_rhs=ctx.needs_input_grad[1])
        _check_converged(ginfo, "adjoint", o)
        if grhs is not None and ctx.squeeze:
            grhs = grhs[0]
        return (gk2 if ctx.needs_input_grad[0] else None, grhs, None, None, None)


def helmholtz_solve(k2: torch.Tensor, f: torch.Tensor, h: float, shift: float = 0.0, **opts) -> torch.Tensor:
    """u = A_s(k2)^{-1} W f by stand-alone multigrid, differentiable in k2 (float64) and f (complex128).

    k2: (n+1, n+1) float64 on the GPU; f: (n+1, n+1) or (S, n+1, n+1) complex128.
    opts: tol, cycle ("V"/"W"), smoother ("gmres"/"jacobi"), nu_pre, nu_post, omega, max_cycles,
          precision ("fp64"/"fp32_refined", then setup_precision must be "fp32_refined"),
          adjoint_tol, levels, transfer, coarsest_n, allow_unconverged (default False: a forward or
          adjoint solve that reaches max_cycles above its tolerance raises MGError; True: it warns).
    """
    return _HelmholtzSolve.apply(k2, f, float(h), float(shift), opts)
