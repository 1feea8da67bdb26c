"""Outer flexible GMRES with the multigrid cycle as preconditioner (§1) on the
GPU, against the oracle's FGMRES (oracle/krylov.py)."""
import numpy as np
import pytest

import oracle as O
from paper_2308_13476_amd import workloads as W
from tests.gpu_common import rel, require_gpu, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _setup(n, k, beta, nodes=None, precision="fp64", max_batch=1):
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    k2 = W.constant_k2(n, k)
    f = W.point_source_rhs(n, nodes or [W.center_node(n)])
    S = Solver(to_gpu(k2), 1.0 / n, beta, precision=precision, max_batch=max_batch)
    H = O.build_hierarchy(k2, 1.0 / n, beta)
    return S, H, f


@pytest.mark.parametrize("smoother,beta,m", [("gmres", 0.05, 10), ("jacobi", 0.7, 30), ("gmres", 0.05, 3)])
def test_fgmres_matches_oracle(smoother, beta, m):
    """n = 64, k = 20: iteration count within one of the oracle's, the residual
    estimates of every iteration equal, and the iterate after the GPU's
    iteration count equal to the oracle's within 1e-10 (FP64 cycles)."""
    n, k = 64, 20.0
    S, H, f = _setup(n, k, beta)
    x, info = S.solve_fgmres(to_gpu(f), tol=1e-8, m=m, smoother=smoother, history=True, max_iter=300)
    assert info["status"] == 0, info
    fs = O.scaled_rhs(f[0]).ravel()
    pre = O.mg_preconditioner(H, O.CycleOptions(smoother=smoother))
    ref = O.fgmres(H.A[0], fs, pre, m=m, tol=1e-8, max_iter=300)
    assert abs(info["cycles"][0] - ref.iterations) <= 1
    it = min(info["cycles"][0], ref.iterations)
    got = np.array(info["history"][0][:it])
    assert np.max(np.abs(got - np.array(ref.history[:it])) / np.array(ref.history[:it])) <= 1e-6
    same = O.fgmres(H.A[0], fs, pre, m=m, tol=1e-30, max_iter=info["cycles"][0])
    assert rel(to_np(x)[0], same.x) <= 1e-10
    assert info["relres"][0] <= 1e-8


def test_fgmres_fp32_preconditioner_and_batch():
    """Two sources, FP32 cycles as the preconditioner of the FP64 outer
    iteration: both reach the FP64 tolerance (true residual), in fewer
    iterations than stand-alone FP32-refined cycles need."""
    n, k = 128, 40.0
    S, H, f = _setup(n, k, 1.0 / k, nodes=[W.center_node(n), (30, 90)], precision="fp32_refined", max_batch=2)
    x, info = S.solve_fgmres(to_gpu(f), tol=1e-9, m=20, precision="fp32_refined", max_iter=300)
    assert info["status"] == 0
    _, alone = S.solve(to_gpu(f), tol=1e-9, precision="fp32_refined", max_cycles=400)
    for b in range(2):
        fs = O.scaled_rhs(f[b]).ravel()
        r = np.linalg.norm(fs - H.A[0] @ to_np(x)[b].ravel()) / np.linalg.norm(fs)
        assert r <= 1e-9 * 1.01, (b, r)
        assert info["cycles"][b] < alone["cycles"][b], (info["cycles"], alone["cycles"])


def test_fgmres_repeated_calls_reuse_dirty_memory():
    """Consecutive calls with the iteration cap 1, 2, 3, 4, 6 (each allocating a
    Krylov buffer that may hold an earlier call's data) equal the oracle's
    iterate after as many iterations (restarts every 3)."""
    n, k = 64, 20.0
    S, H, f = _setup(n, k, 0.05)
    fs = O.scaled_rhs(f[0]).ravel()
    pre = O.mg_preconditioner(H, O.CycleOptions(smoother="gmres"))
    for it in [1, 2, 3, 4, 6]:
        x, info = S.solve_fgmres(to_gpu(f), tol=1e-30, m=3, max_iter=it)
        assert info["cycles"][0] == it
        ref = O.fgmres(H.A[0], fs, pre, m=3, tol=1e-30, max_iter=it)
        assert rel(to_np(x)[0], ref.x) <= 1e-10, (it, rel(to_np(x)[0], ref.x))


def test_fgmres_batch_members_stop_at_their_own_iteration():
    """Two sources in one call, restart length 3: each member stops at its own
    iteration count and equals the oracle's iterate for that count (the
    members that finish earlier keep their final update)."""
    n, k = 64, 20.0
    nodes = [W.center_node(n), (5, 58)]
    S, H, f = _setup(n, k, 0.05, nodes=nodes, max_batch=2)
    x, info = S.solve_fgmres(to_gpu(f), tol=1e-9, m=3, max_iter=200)
    assert info["status"] == 0
    pre = O.mg_preconditioner(H, O.CycleOptions(smoother="gmres"))
    for b in range(2):
        fs = O.scaled_rhs(f[b]).ravel()
        ref = O.fgmres(H.A[0], fs, pre, m=3, tol=1e-9, max_iter=200)
        assert abs(info["cycles"][b] - ref.iterations) <= 1
        same = O.fgmres(H.A[0], fs, pre, m=3, tol=1e-30, max_iter=info["cycles"][b])
        assert rel(to_np(x)[b], same.x) <= 1e-10, (b, rel(to_np(x)[b], same.x))


@pytest.mark.parametrize("m,nb", [(20, 1), (5, 2)])
def test_fgmres_fp32_cycles_follow_the_oracle(m, nb):
    """FP32 cycles as the preconditioner (each starts from u = 0 with the
    complex64 basis vector as its first GMRES residual, written by the pass
    that forms the vector) against the oracle's FGMRES with FP64 cycles: per
    source the iteration count within one, the residual estimates of the
    common iterations within 1e-3 of each other (the preconditioners differ by
    FP32 rounding), and the true FP64 residual at the tolerance; with restarts
    (m = 5) and two sources."""
    n, k = 128, 40.0
    nodes = [W.center_node(n), (30, 90)][:nb]
    S, H, f = _setup(n, k, 1.0 / k, nodes=nodes, precision="fp32_refined", max_batch=nb)
    x, info = S.solve_fgmres(to_gpu(f), tol=1e-9, m=m, precision="fp32_refined", max_iter=300, history=True)
    assert info["status"] == 0
    pre = O.mg_preconditioner(H, O.CycleOptions(smoother="gmres"))
    for b in range(nb):
        fs = O.scaled_rhs(f[b]).ravel()
        ref = O.fgmres(H.A[0], fs, pre, m=m, tol=1e-9, max_iter=300)
        it = min(info["cycles"][b], ref.iterations)
        d = np.max(np.abs(np.array(info["history"][b][:it]) - np.array(ref.history[:it])) / np.array(ref.history[:it]))
        print(f"source {b}: {info['cycles'][b]} iterations (oracle {ref.iterations}), residual estimates "
              f"within {d:.2e}")
        assert abs(info["cycles"][b] - ref.iterations) <= 1
        assert d <= 1e-3
        r = np.linalg.norm(fs - H.A[0] @ to_np(x)[b].ravel()) / np.linalg.norm(fs)
        assert r <= 1e-9 * 1.01, (b, r)
