"""mg_residual_noalloc, the residual entry point for callers that cannot
allocate, against mg_residual through the C ABI: the same kernels on the
same inputs, so the results must agree bit for bit, on two calls in a row
(the second on a smaller level, in the other precision, with fewer vectors);
the handle's own buffers are left alone, and requests beyond the static
scratch are refused before anything is enqueued."""
import numpy as np
import pytest

import oracle as O
from paper_2308_13476_amd import workloads as W
from tests.gpu_common import node_rel, require_gpu, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _rand(n, nvec, seed, dtype=np.complex128):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nvec, n + 1, n + 1)) + 1j * rng.standard_normal((nvec, n + 1, n + 1))
    return a.astype(dtype)


def test_noalloc_residual_equals_mg_residual_on_two_calls():
    require_gpu()
    import torch
    from paper_2308_13476_amd import _binding as B
    from paper_2308_13476_amd.solver import Solver
    n = 256
    k2 = W.random_k2(n, 31, 20.0, 60.0)
    S = Solver(to_gpu(k2), 1.0 / n, 0.05, max_batch=3, precision="fp32_refined")
    H = O.build_hierarchy(k2, 1.0 / n, 0.05)
    # a solve first, so that the handle's level buffers hold data of their own
    f0 = to_gpu(W.point_source_rhs(n, [W.center_node(n)]))
    x_before, _ = S.solve(f0, tol=1e-8)
    calls = [(0, "fp64", 3, 11), (2, "fp32_refined", 2, 12)]  # second call: smaller level, fewer vectors
    for level, prec, nvec, seed in calls:
        n_l = H.n[level]
        dt = np.complex128 if prec == "fp64" else np.complex64
        x = to_gpu(_rand(n_l, nvec, seed, dt))
        f = to_gpu(_rand(n_l, nvec, seed + 100, dt))
        want = S.residual(level, x, f, precision=prec)
        r = torch.full_like(x, float("nan"))
        assert S.residual_noalloc(level, x, f, r, precision=prec) == B.MG_OK
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(r), to_np(want))
        if prec == "fp64":
            for b in range(nvec):
                ref = to_np(f)[b].ravel() - H.A[level] @ to_np(x)[b].ravel()
                assert node_rel(to_np(r)[b], ref) <= 1e-13
    # the static path never touched the handle's buffers: a repeated solve is unchanged
    x_after, _ = S.solve(f0, tol=1e-8)
    np.testing.assert_array_equal(to_np(x_after), to_np(x_before))


def test_noalloc_residual_refuses_requests_beyond_its_scratch():
    require_gpu()
    from paper_2308_13476_amd import _binding as B
    from paper_2308_13476_amd.solver import Solver, _ptr, _stream
    n = 256
    S = Solver(to_gpu(W.constant_k2(n, 30.0)), 1.0 / n, 0.05)
    x = to_gpu(_rand(n, 1, 5))
    # 3 x 20 padded complex128 planes of 257 x 257 nodes (1.36 MB each) exceed 64 MiB;
    # the check fails before any pointer is used
    st = B.lib().mg_residual_noalloc(S.handle, 0, _ptr(x), _ptr(x), _ptr(x), 20, B.MG_FP64, _stream())
    assert st == B.MG_E_ARG and "static scratch" in B.last_error(S.handle)
    st = B.lib().mg_residual_noalloc(S.handle, 0, _ptr(x), _ptr(x), _ptr(x), 0, B.MG_FP64, _stream())
    assert st == B.MG_E_ARG
    assert B.lib().mg_residual_noalloc(None, 0, _ptr(x), _ptr(x), _ptr(x), 1, B.MG_FP64, _stream()) == B.MG_E_ARG
