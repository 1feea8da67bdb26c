"""Boundary behaviour of the C ABI on the GPU: the k^2 field check of
mg_setup / mg_update_k2 (§2: k > 0 on the absorbing boundary, k^2 >= 0 and
finite everywhere), the history buffer bound, the differentiable solve's
refusal of unconverged solves, and the FP32 cycle against the oracle's own
complex64 cycle."""
import ctypes
import warnings

import numpy as np
import pytest

import oracle as O
from paper_2308_13476_amd import workloads as W
from tests.gpu_common import node_rel, rel, require_gpu, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _solver(k2, beta, **kw):
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    n = k2.shape[0] - 1
    return Solver(to_gpu(k2), 1.0 / n, beta, **kw)


@pytest.mark.parametrize("what,node,value", [("negative", (5, 7), -1.0), ("boundary zero", (0, 9), 0.0),
                                             ("corner zero", (16, 16), 0.0), ("nan", (3, 3), np.nan),
                                             ("inf", (9, 12), np.inf)])
def test_setup_rejects_an_invalid_k2_field(what, node, value):
    from paper_2308_13476_amd import _binding as B
    n = 16
    k2 = W.constant_k2(n, 6.0)
    j, i = node
    k2[j, i] = value
    with pytest.raises(B.MGError) as e:
        _solver(k2, 0.1)
    assert e.value.status == B.MG_E_ARG
    assert f"(i, j) = ({i}, {j})" in str(e.value), str(e.value)


def test_zero_inside_is_valid_and_update_keeps_the_hierarchy_on_a_bad_field():
    from paper_2308_13476_amd import _binding as B
    n = 32
    k2 = W.constant_k2(n, 8.0)
    k2[10:14, 10:14] = 0.0  # k = 0 inside the domain is allowed
    S = _solver(k2, 0.1)
    f = W.point_source_rhs(n, [W.center_node(n)])
    x0, i0 = S.solve(to_gpu(f), tol=1e-8)
    assert i0["status"] == 0
    bad = k2.copy()
    bad[n, 4] = -2.0
    with pytest.raises(B.MGError) as e:
        S.update_k2(to_gpu(bad))
    assert e.value.status == B.MG_E_ARG and "(i, j) = (4, 32)" in str(e.value)
    x1, i1 = S.solve(to_gpu(f), tol=1e-8)
    assert i1["cycles"] == i0["cycles"]
    np.testing.assert_array_equal(to_np(x1), to_np(x0))
    # the gradient at a node with k = 0 is finite and equals the oracle's
    from oracle import adjoint
    row = W.receiver_row(n)
    d = np.zeros((1, n + 1), dtype=np.complex128)
    ref, _ = adjoint.gradient(k2, 1.0 / n, f, row, d)
    u, _ = S.solve(to_gpu(f), tol=1e-13, max_cycles=400)
    import torch
    gu = torch.zeros_like(u)
    gu[:, row, :] = u[:, row, :]
    g, _, gi = S.grad(u, gu, tol=1e-13, max_cycles=400)
    g = to_np(g)
    assert gi["status"] == 0 and np.isfinite(g).all()
    assert np.abs(g - ref).max() <= 1e-8 * np.abs(ref).max()


def test_history_buffer_must_hold_max_cycles_per_rhs():
    from paper_2308_13476_amd import _binding as B
    from paper_2308_13476_amd.solver import _ptr, _stream
    n = 16
    S = _solver(W.constant_k2(n, 5.0), 0.2)
    f = to_gpu(W.point_source_rhs(n, [W.center_node(n)]))
    x = f.clone()
    opts = S.solve_options(max_cycles=20)
    cyc = (ctypes.c_int * 1)()
    relr = (ctypes.c_double * 1)()
    hist = (ctypes.c_double * 19)()
    st = B.SolveStats(ctypes.cast(cyc, ctypes.POINTER(ctypes.c_int)), ctypes.cast(relr, ctypes.POINTER(ctypes.c_double)),
                      ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), 19, 0.0)
    r = B.lib().mg_solve(S.handle, _ptr(f), _ptr(x), 1, 1e-6, B.MG_V, B.MG_GMRES3, ctypes.byref(opts),
                         ctypes.byref(st), _stream())
    assert r == B.MG_E_ARG and "history_len" in B.last_error(S.handle)
    st.history_len = 20
    r = B.lib().mg_solve(S.handle, _ptr(f), _ptr(x), 1, 1e-6, B.MG_V, B.MG_GMRES3, ctypes.byref(opts),
                         ctypes.byref(st), _stream())
    assert r == B.MG_OK and 0 < cyc[0] <= 20
    assert all(np.isfinite(hist[i]) for i in range(cyc[0]))


def test_differentiable_solve_refuses_unconverged_solves():
    import torch
    from paper_2308_13476_amd import _binding as B
    from paper_2308_13476_amd import helmholtz_solve
    require_gpu()
    n = 32
    k2 = to_gpu(W.constant_k2(n, 10.0)).requires_grad_(True)
    f = to_gpu(W.point_source_rhs(n, [W.center_node(n)]))
    with pytest.raises(B.MGError) as e:
        helmholtz_solve(k2, f, 1.0 / n, 0.1, tol=1e-12, max_cycles=2)
    assert e.value.status == B.MG_NOT_CONVERGED
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        u = helmholtz_solve(k2, f, 1.0 / n, 0.1, tol=1e-12, max_cycles=2, allow_unconverged=True)
        (torch.abs(u) ** 2).sum().backward()
    msgs = [str(x.message) for x in w]
    assert any("forward solve" in m for m in msgs) and any("adjoint solve" in m for m in msgs), msgs
    assert torch.isfinite(k2.grad).all()


@pytest.mark.parametrize("cyc", ["V", "W"])
def test_fp32_cycle_against_the_complex64_oracle_cycle(cyc):
    """The FP32 cycle of the refined solve against the oracle's cycle run in
    complex64 arithmetic (coarsest solve FP64 in both). The two differ by FP32
    rounding order only (the GPU accumulates inner products in FP64), so they
    agree to a few hundred FP32 units."""
    n = 64
    k2 = W.random_k2(n, 9, 8.0, 18.0)
    H = O.build_hierarchy(k2, 1.0 / n, 0.3)
    S = _solver(k2, 0.3, max_batch=1, precision="fp32_refined")
    rng = np.random.default_rng(77)
    f = (rng.standard_normal((1, n + 1, n + 1)) + 1j * rng.standard_normal((1, n + 1, n + 1))).astype(np.complex64)
    u = np.zeros_like(f)
    opts = O.CycleOptions(gamma=1 if cyc == "V" else 2, smoother="gmres", nu1=1, nu2=1)
    got = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle=cyc, smoother="gmres", precision="fp32_refined"))[0].ravel()
    ref32 = O.cycle(H, 0, u[0].ravel(), f[0].ravel(), opts, fp32=True)
    ref64 = O.cycle(H, 0, u[0].ravel().astype(complex), f[0].ravel().astype(complex), opts)
    d32, d64 = rel(got, ref32), rel(ref32, ref64)
    print(f"FP32 cycle ({cyc}): vs complex64 oracle {d32:.2e} (per node {node_rel(got, ref32):.2e}); "
          f"complex64 oracle vs FP64 oracle {d64:.2e}")
    assert d32 <= 2e-5 and node_rel(got, ref32) <= 2e-5, (d32, node_rel(got, ref32))
