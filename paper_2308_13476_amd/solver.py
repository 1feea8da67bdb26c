"""PyTorch-facing wrapper of the C ABI: device memory and streams come from
PyTorch, every numerical step runs in libhelmg.so.

Grid functions are tensors of shape (batch, n+1, n+1) (or (n+1, n+1)),
indexed [b, j, i] with x (index i) fastest, on a ROCm device.
"""
from __future__ import annotations

import ctypes

import torch

from . import _binding as B

_TRANSFER = {"bezier": B.MG_TRANSFER_BEZIER, "linear": B.MG_TRANSFER_LINEAR}
_CYCLE = {"V": B.MG_V, "W": B.MG_W, 1: B.MG_V, 2: B.MG_W}
_SMOOTHER = {"jacobi": B.MG_JACOBI, "gmres": B.MG_GMRES3, "gmres3": B.MG_GMRES3}
_PREC = {"fp64": B.MG_FP64, "fp32_refined": B.MG_FP32_REFINED}


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(status: int, handle=None, ok=(B.MG_OK,)):
    if status not in ok:
        raise B.MGError(status, B.last_error(handle))
    return status


def _stats(cycles, rel, hist=None) -> B.SolveStats:
    """mg_solve_stats over ctypes arrays (hist may be None)."""
    return B.SolveStats(ctypes.cast(cycles, ctypes.POINTER(ctypes.c_int)),
                        ctypes.cast(rel, ctypes.POINTER(ctypes.c_double)),
                        ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)) if hist is not None else None,
                        len(hist) if hist is not None else 0, 0.0)


def _batched(t: torch.Tensor, n: int, dtype) -> torch.Tensor:
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.shape[-2:] != (n + 1, n + 1):
        raise ValueError(f"expected grid functions of shape (..., {n + 1}, {n + 1}), got {tuple(t.shape)}")
    if not t.is_cuda:
        raise ValueError("grid functions must live on the GPU")
    return t.to(dtype).contiguous()


class Solver:
    """Multigrid hierarchy for one k^2 field (mg_setup) and its solves.

    k2: float64 tensor (n+1, n+1) on the GPU; h: mesh width; shift: beta2 >= 0.
    """

    def __init__(self, k2: torch.Tensor, h: float, shift: float, levels: int = 0, transfer: str = "bezier",
                 precision: str = "fp64", max_batch: int = 1, coarsest_n: int = 4, use_graph: bool = True,
                 tune_cache: str | None = None):
        lib = B.lib()
        if k2.dim() != 2 or k2.shape[0] != k2.shape[1]:
            raise ValueError("k2 must be a square (n+1, n+1) tensor")
        self.n = k2.shape[0] - 1
        self.h = float(h)
        self.shift = float(shift)
        self.transfer = transfer
        self.max_batch = int(max_batch)
        self.setup_precision = precision
        self.handle = ctypes.c_void_p()
        self._tune_cache = tune_cache.encode() if tune_cache else None  # kept alive for the C side
        self._opts = B.SetupOpts(_PREC[precision], self.max_batch, int(coarsest_n), 1 if use_graph else -1,
                                 self._tune_cache)
        nbytes = lib.mg_workspace_bytes(self.n, int(levels), _TRANSFER[transfer], ctypes.byref(self._opts))
        if nbytes == 0:
            raise ValueError("invalid grid / level configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=k2.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.workspace.data_ptr() + off)
        self._ws_bytes = nbytes
        self.device = k2.device
        k2c = k2.to(torch.float64).contiguous()
        st = lib.mg_setup(_ptr(k2c), self.n, self.h, self.shift, int(levels), _TRANSFER[transfer],
                          ctypes.byref(self._opts), self._ws_ptr, nbytes, _stream(), ctypes.byref(self.handle))
        _check(st, None)
        lv = ctypes.c_int()
        lib.mg_level_info(self.handle, 0, None, None, ctypes.byref(lv))
        self.levels = lv.value

    # ------------------------------------------------------------------ life cycle
    def close(self):
        if self.handle:
            B.lib().mg_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_k2(self, k2: torch.Tensor):
        k2c = k2.to(torch.float64).contiguous()
        _check(B.lib().mg_update_k2(self.handle, _ptr(k2c), _stream()), self.handle)

    def level_info(self, level: int):
        n_l, r = ctypes.c_int(), ctypes.c_int()
        _check(B.lib().mg_level_info(self.handle, level, ctypes.byref(n_l), ctypes.byref(r), None), self.handle)
        return n_l.value, r.value

    # ------------------------------------------------------------------ solves
    @staticmethod
    def solve_options(nu_pre=1, nu_post=1, omega=4.5, max_cycles=500, precision="fp64", divergence=1e8):
        return B.SolveOpts(int(nu_pre), int(nu_post), float(omega), int(max_cycles), _PREC[precision],
                           float(divergence))

    def solve(self, rhs: torch.Tensor, x0: torch.Tensor | None = None, tol: float = 1e-6, cycle="V",
              smoother="gmres", nu_pre=1, nu_post=1, omega=4.5, max_cycles=500, precision="fp64",
              divergence=1e8, history=False, raise_on_error=True):
        """mg_solve: returns (x, info) with x complex128 (batch, n+1, n+1)."""
        f = _batched(rhs, self.n, torch.complex128)
        nb = f.shape[0]
        x = torch.zeros_like(f) if x0 is None else _batched(x0, self.n, torch.complex128).clone()
        opts = self.solve_options(nu_pre, nu_post, omega, max_cycles, precision, divergence)
        cycles = (ctypes.c_int * nb)()
        rel = (ctypes.c_double * nb)()
        hist = (ctypes.c_double * (nb * max_cycles))() if history else None
        stats = _stats(cycles, rel, hist)
        st = B.lib().mg_solve(self.handle, _ptr(f), _ptr(x), nb, float(tol), _CYCLE[cycle], _SMOOTHER[smoother],
                              ctypes.byref(opts), ctypes.byref(stats), _stream())
        info = {"status": st, "status_name": B.status_string(st), "cycles": list(cycles), "relres": list(rel),
                "seconds": stats.seconds}
        if hist is not None:
            h = list(hist)
            info["history"] = [[h[it * nb + b] for it in range(max(info["cycles"]))] for b in range(nb)]
        if raise_on_error and st < 0:
            raise B.MGError(st, B.last_error(self.handle))
        return x, info

    def solve_fgmres(self, rhs: torch.Tensor, x0: torch.Tensor | None = None, tol: float = 1e-6, m: int = 20,
                     cycle="V", smoother="gmres", nu_pre=1, nu_post=1, omega=4.5, max_iter=500, precision="fp64",
                     history=False, raise_on_error=True):
        """mg_solve_fgmres: FP64 flexible GMRES(m) preconditioned by one cycle per
        iteration. Returns (x, info); info["cycles"] counts iterations."""
        f = _batched(rhs, self.n, torch.complex128)
        nb = f.shape[0]
        x = torch.zeros_like(f) if x0 is None else _batched(x0, self.n, torch.complex128).clone()
        nbytes = B.lib().mg_fgmres_workspace_bytes(self.handle, int(m))
        if nbytes == 0:
            raise ValueError("restart length m must be in [1, 64]")
        kry = torch.empty(nbytes, dtype=torch.uint8, device=f.device)
        opts = self.solve_options(nu_pre, nu_post, omega, max_iter, precision)
        cycles = (ctypes.c_int * nb)()
        rel = (ctypes.c_double * nb)()
        hist = (ctypes.c_double * (nb * max_iter))() if history else None
        stats = _stats(cycles, rel, hist)
        st = B.lib().mg_solve_fgmres(self.handle, _ptr(f), _ptr(x), nb, float(tol), int(m), _CYCLE[cycle],
                                     _SMOOTHER[smoother], ctypes.byref(opts), _ptr(kry), nbytes,
                                     ctypes.byref(stats), _stream())
        info = {"status": st, "status_name": B.status_string(st), "cycles": list(cycles), "relres": list(rel),
                "seconds": stats.seconds}
        if hist is not None:
            h = list(hist)
            info["history"] = [[h[it * nb + b] for it in range(max(info["cycles"]))] for b in range(nb)]
        if raise_on_error and st < 0:
            raise B.MGError(st, B.last_error(self.handle))
        return x, info

    def tune(self, rhs: torch.Tensor, cycle="V", smoother="gmres", nu_pre=1, nu_post=1, omega=4.5,
             precision="fp64") -> dict:
        """mg_tune: times cycles of this problem under each candidate launch setting
        and keeps the fastest for later solves."""
        f = _batched(rhs, self.n, torch.complex128)
        opts = self.solve_options(nu_pre, nu_post, omega, 1, precision)
        res = B.TuneResult()
        _check(B.lib().mg_tune(self.handle, _ptr(f), f.shape[0], _CYCLE[cycle], _SMOOTHER[smoother],
                               ctypes.byref(opts), ctypes.byref(res), _stream()), self.handle)
        return {"block_cap": res.block_cap, "tail_n": res.tail_n, "level1_product": res.level1_product,
                "ms_per_cycle": res.ms_per_cycle, "candidates": res.candidates, "tall_rows": res.tall_rows,
                "small_rows": res.small_rows, "from_cache": bool(res.from_cache)}

    @staticmethod
    def solve_multi(solvers, rhs_list, x0_list=None, tol: float = 1e-6, cycle="V", smoother="gmres", nu_pre=1,
                    nu_post=1, omega=4.5, max_cycles=500, precision="fp64", divergence=1e8, raise_on_error=True):
        """mg_solve_multi: independent problems (one Solver each, any sizes) solved
        together. Returns a list of (x, info) in the order of `solvers`."""
        npb = len(solvers)
        if npb == 0 or len(rhs_list) != npb:
            raise ValueError("need one right-hand side tensor per solver")
        fs = [_batched(r, S.n, torch.complex128) for S, r in zip(solvers, rhs_list)]
        if x0_list is None:
            xs = [torch.zeros_like(f) for f in fs]
        else:
            xs = [_batched(x0, S.n, torch.complex128).clone() for S, x0 in zip(solvers, x0_list)]
        nbs = [f.shape[0] for f in fs]
        opts = Solver.solve_options(nu_pre, nu_post, omega, max_cycles, precision, divergence)
        cyc = [(ctypes.c_int * nb)() for nb in nbs]
        rel = [(ctypes.c_double * nb)() for nb in nbs]
        stats = (B.SolveStats * npb)(*[_stats(c, r) for c, r in zip(cyc, rel)])
        handles = (ctypes.c_void_p * npb)(*[S.handle for S in solvers])
        rp = (ctypes.c_void_p * npb)(*[_ptr(f) for f in fs])
        xp = (ctypes.c_void_p * npb)(*[_ptr(x) for x in xs])
        nr = (ctypes.c_int * npb)(*nbs)
        st = B.lib().mg_solve_multi(handles, npb, rp, xp, nr, float(tol), _CYCLE[cycle], _SMOOTHER[smoother],
                                    ctypes.byref(opts), stats, _stream())
        if raise_on_error and st < 0:
            failing = next((S.handle for S in solvers if B.last_error(S.handle)), None)
            raise B.MGError(st, B.last_error(failing))
        out = []
        for p in range(npb):
            info = {"status": st, "status_name": B.status_string(st), "cycles": list(cyc[p]),
                    "relres": list(rel[p]), "seconds": stats[p].seconds}
            out.append((xs[p], info))
        return out

    def grad(self, u: torch.Tensor, grad_u: torch.Tensor, tol: float = 1e-10, cycle="V", smoother="gmres",
             nu_pre=1, nu_post=1, omega=4.5, max_cycles=500, precision="fp64", want_rhs=True):
        """mg_grad: returns (grad_k2 float64 (n+1, n+1), grad_rhs complex128 or None, info)."""
        uu = _batched(u, self.n, torch.complex128)
        gu = _batched(grad_u, self.n, torch.complex128)
        nb = uu.shape[0]
        gk2 = torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=uu.device)
        grhs = torch.empty_like(uu) if want_rhs else None
        opts = self.solve_options(nu_pre, nu_post, omega, max_cycles, precision)
        cycles = (ctypes.c_int * nb)()
        rel = (ctypes.c_double * nb)()
        stats = _stats(cycles, rel)
        st = B.lib().mg_grad(self.handle, _ptr(uu), _ptr(gu), nb, float(tol), _CYCLE[cycle], _SMOOTHER[smoother],
                             ctypes.byref(opts), _ptr(gk2), _ptr(grhs) if grhs is not None else None,
                             ctypes.byref(stats), _stream())
        _check(st, self.handle, ok=(B.MG_OK, B.MG_NOT_CONVERGED))
        return gk2, grhs, {"status": st, "cycles": list(cycles), "relres": list(rel), "seconds": stats.seconds}

    # ------------------------------------------------------------------ level operations
    def _lvl_dtype(self, precision):
        return torch.complex128 if precision == "fp64" else torch.complex64

    def _lvl_vec(self, t, level, precision):
        n_l, _ = self.level_info(level)
        return _batched(t, n_l, self._lvl_dtype(precision))

    def stencil(self, level: int) -> torch.Tensor:
        n_l, r = self.level_info(level)
        out = torch.empty(((2 * r + 1) ** 2, n_l + 1, n_l + 1), dtype=torch.complex128, device=self.device)
        _check(B.lib().mg_get_stencil(self.handle, level, _ptr(out), _stream()), self.handle)
        return out

    def apply(self, level: int, x: torch.Tensor, precision="fp64") -> torch.Tensor:
        xv = self._lvl_vec(x, level, precision)
        y = torch.empty_like(xv)
        _check(B.lib().mg_apply(self.handle, level, _ptr(xv), _ptr(y), xv.shape[0], _PREC[precision], _stream()),
               self.handle)
        return y

    def residual(self, level: int, x: torch.Tensor, f: torch.Tensor, precision="fp64") -> torch.Tensor:
        xv = self._lvl_vec(x, level, precision)
        fv = self._lvl_vec(f, level, precision)
        r = torch.empty_like(xv)
        _check(B.lib().mg_residual(self.handle, level, _ptr(xv), _ptr(fv), _ptr(r), xv.shape[0], _PREC[precision],
                                   _stream()), self.handle)
        return r

    def residual_noalloc(self, level: int, x: torch.Tensor, f: torch.Tensor, r: torch.Tensor, precision="fp64"):
        """mg_residual_noalloc into the caller's r (nothing allocated, nothing
        synchronised: r is ready when the current stream reaches the kernels).
        Returns the status; raises on an error status."""
        xv = self._lvl_vec(x, level, precision)
        fv = self._lvl_vec(f, level, precision)
        if r.shape != xv.shape or r.dtype != xv.dtype or not r.is_contiguous():
            raise ValueError("r must be a contiguous tensor of x's shape and dtype")
        return _check(B.lib().mg_residual_noalloc(self.handle, level, _ptr(xv), _ptr(fv), _ptr(r), xv.shape[0],
                                                  _PREC[precision], _stream()), self.handle)

    def smooth(self, level: int, u: torch.Tensor, f: torch.Tensor, smoother="jacobi", nsteps=1, omega=4.5,
               precision="fp64") -> torch.Tensor:
        uv = self._lvl_vec(u, level, precision).clone()
        fv = self._lvl_vec(f, level, precision)
        _check(B.lib().mg_smooth(self.handle, level, _SMOOTHER[smoother], int(nsteps), float(omega), _ptr(uv),
                                 _ptr(fv), uv.shape[0], _PREC[precision], _stream()), self.handle)
        return uv

    def restrict(self, level: int, fine: torch.Tensor, precision="fp64") -> torch.Tensor:
        fv = self._lvl_vec(fine, level, precision)
        n_c, _ = self.level_info(level + 1)
        out = torch.empty((fv.shape[0], n_c + 1, n_c + 1), dtype=fv.dtype, device=fv.device)
        _check(B.lib().mg_restrict(self.handle, level, _ptr(fv), _ptr(out), fv.shape[0], _PREC[precision],
                                   _stream()), self.handle)
        return out

    def prolong_add(self, level: int, coarse: torch.Tensor, fine: torch.Tensor, precision="fp64") -> torch.Tensor:
        cv = self._lvl_vec(coarse, level + 1, precision)
        fv = self._lvl_vec(fine, level, precision).clone()
        _check(B.lib().mg_prolong_add(self.handle, level, _ptr(cv), _ptr(fv), fv.shape[0], _PREC[precision],
                                      _stream()), self.handle)
        return fv

    def coarse_solve(self, f: torch.Tensor, precision="fp64") -> torch.Tensor:
        fv = self._lvl_vec(f, self.levels - 1, precision)
        u = torch.empty_like(fv)
        _check(B.lib().mg_coarse_solve(self.handle, _ptr(fv), _ptr(u), fv.shape[0], _PREC[precision], _stream()),
               self.handle)
        return u

    def cycle(self, u: torch.Tensor, f_s: torch.Tensor, cycle="V", smoother="gmres", nu_pre=1, nu_post=1,
              omega=4.5, precision="fp64") -> torch.Tensor:
        """mg_cycle: one cycle; complex128 data, or complex64 with precision="fp32_refined"."""
        dt = torch.complex64 if precision == "fp32_refined" else torch.complex128
        uv = _batched(u, self.n, dt).clone()
        fv = _batched(f_s, self.n, dt)
        opts = self.solve_options(nu_pre, nu_post, omega, 1, precision)
        _check(B.lib().mg_cycle(self.handle, _ptr(uv), _ptr(fv), uv.shape[0], _CYCLE[cycle], _SMOOTHER[smoother],
                                ctypes.byref(opts), _stream()), self.handle)
        return uv

    # ------------------------------------------------------------------ timing hook
    def set_timing(self, kernel_class: int):
        _check(B.lib().mg_set_timing(self.handle, int(kernel_class)), self.handle)

    def get_timing(self):
        n, ms, nodes = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(B.lib().mg_get_timing(self.handle, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(nodes)),
               self.handle)
        return n.value, ms.value, nodes.value
