"""Whole-solve parity of the HIP path with the CPU oracle, batching, error paths
and the full-size benchmark configuration."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2308_13476_amd import workloads as W
from tests.gpu_common import node_rel, rel, require_gpu, to_gpu, to_np

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mp2a(n, k, nodes=None):
    k2 = W.constant_k2(n, k)
    f = W.point_source_rhs(n, nodes or [W.center_node(n)])
    return k2, f


def _solver(k2, beta, **kw):
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    n = k2.shape[0] - 1
    return Solver(to_gpu(k2), 1.0 / n, beta, **kw)


@pytest.mark.parametrize("smoother,beta,cyc,nu", [("jacobi", 0.7, "V", 1), ("gmres", 0.05, "V", 1),
                                                   ("gmres", 0.05, "W", 1), ("jacobi", 0.7, "W", 2),
                                                   ("gmres", 0.0, "V", 2)])
def test_solve_matches_oracle(smoother, beta, cyc, nu):
    """Config 1 shape (n = 64, k = 20): cycle counts within one of the oracle, and the
    iterate after the GPU's cycle count equal to the oracle's within 1e-10."""
    n, k = 64, 20.0
    k2, f = _mp2a(n, k)
    S = _solver(k2, beta)
    x, info = S.solve(to_gpu(f), tol=1e-6, cycle=cyc, smoother=smoother, nu_pre=nu, nu_post=nu, max_cycles=400)
    assert info["status"] == 0, info
    H = O.build_hierarchy(k2, 1.0 / n, beta)
    opts = O.CycleOptions(gamma=1 if cyc == "V" else 2, smoother=smoother, nu1=nu, nu2=nu)
    fs = O.scaled_rhs(f[0]).ravel()
    ref = O.solve(H, fs, opts, tol=1e-6, max_cycles=400)
    assert abs(info["cycles"][0] - ref.cycles) <= 1
    same = O.solve(H, fs, opts, tol=1e-30, max_cycles=info["cycles"][0])
    assert rel(to_np(x)[0], same.x) <= 1e-10
    assert node_rel(to_np(x)[0], same.x) <= 1e-10
    assert np.linalg.norm(fs - H.A[0] @ to_np(x)[0].ravel()) / np.linalg.norm(fs) <= 1e-6


def test_config1_jacobi_count():
    """The plain method of config 1: Jacobi V(1,1), shift 0.7, n = 64, k = 20 (oracle: 127)."""
    k2, f = _mp2a(64, 20.0)
    S = _solver(k2, 0.7)
    _, info = S.solve(to_gpu(f), tol=1e-6, cycle="V", smoother="jacobi", max_cycles=400)
    assert info["status"] == 0 and abs(info["cycles"][0] - 127) <= 1


@pytest.mark.parametrize("smoother,beta", [("gmres", 0.02), ("jacobi", 0.7)])
def test_fp32_refined_solve(smoother, beta):
    n, k = 128, 25.0
    k2, f = _mp2a(n, k)
    S = _solver(k2, beta, precision="fp32_refined")
    x, info = S.solve(to_gpu(f), tol=1e-6, smoother=smoother, precision="fp32_refined", max_cycles=500)
    assert info["status"] == 0
    H = O.build_hierarchy(k2, 1.0 / n, beta)
    fs = O.scaled_rhs(f[0]).ravel()
    r = np.linalg.norm(fs - H.A[0] @ to_np(x)[0].ravel()) / np.linalg.norm(fs)
    assert r <= 1e-6
    ref = O.solve_refined(H, fs, O.CycleOptions(smoother=smoother), tol=1e-6, max_cycles=500)
    assert abs(info["cycles"][0] - ref.cycles) <= 1
    exact = O.solve(H, fs, O.CycleOptions(smoother=smoother), tol=1e-12, max_cycles=800).x
    # error against the FP64 solution is of the order of the tolerance
    assert rel(to_np(x)[0], exact) < 1e-3


def test_batch_members_equal_solo_solves():
    n, k = 64, 15.0
    nodes = W.seeded_interior_nodes(n, 3, 4)
    k2, f = _mp2a(n, k, nodes)
    S = _solver(k2, 1.0 / k, max_batch=3, precision="fp32_refined")
    for prec in ["fp64", "fp32_refined"]:
        xb, ib = S.solve(to_gpu(f), tol=1e-6, precision=prec)
        for b in range(3):
            xs, is_ = S.solve(to_gpu(f[b:b + 1]), tol=1e-6, precision=prec)
            assert ib["cycles"][b] == is_["cycles"][0]
            np.testing.assert_array_equal(to_np(xb)[b], to_np(xs)[0])


def test_solves_are_deterministic_and_restartable():
    n, k = 64, 12.0
    k2, f = _mp2a(n, k)
    S = _solver(k2, 0.1)
    a, _ = S.solve(to_gpu(f), tol=1e-30, max_cycles=5)
    b, _ = S.solve(to_gpu(f), tol=1e-30, max_cycles=5)
    np.testing.assert_array_equal(to_np(a), to_np(b))
    p, _ = S.solve(to_gpu(f), tol=1e-30, max_cycles=2)
    q, _ = S.solve(to_gpu(f), x0=p, tol=1e-30, max_cycles=3)
    np.testing.assert_array_equal(to_np(a), to_np(q))


def test_error_paths():
    from paper_2308_13476_amd import _binding as B
    n, k = 64, 40.0
    k2, f = _mp2a(n, k)
    S = _solver(k2, 0.0)
    _, info = S.solve(to_gpu(f), smoother="jacobi", max_cycles=300, divergence=1e3, raise_on_error=False)
    assert info["status"] == B.MG_E_DIVERGED
    S2 = _solver(k2, 1.0 / k)
    _, info = S2.solve(to_gpu(f), max_cycles=3, raise_on_error=False)
    assert info["status"] == B.MG_NOT_CONVERGED and info["cycles"][0] == 3
    bad = f.copy()
    bad[0, 3, 3] = np.nan
    _, info = S2.solve(to_gpu(bad), raise_on_error=False)
    assert info["status"] == B.MG_E_DIVERGED
    x, info = S2.solve(to_gpu(np.zeros_like(f)))
    assert info["status"] == 0 and info["cycles"][0] == 0 and not to_np(x).any()
    with pytest.raises(B.MGError):
        S2.solve(to_gpu(np.concatenate([f, f])))  # nrhs > max_batch
    with pytest.raises(B.MGError):
        S2.solve(to_gpu(f), precision="fp32_refined")  # no FP32 copies


def test_full_size_against_stored_oracle_runs():
    """n = 1024, k = 200, shift 1/k, GMRES(3): the benchmarked configuration. Cycle counts
    and the relative residual after every cycle match the stored oracle runs."""
    g = json.load(open(os.path.join(GOLDEN, "oracle_full_size.json")))
    n, k = 1024, 200.0
    k2, f = _mp2a(n, k)
    S = _solver(k2, 1.0 / k, precision="fp32_refined")
    A_s = O.helmholtz_matrix(k2, 1.0 / n)
    fs = O.scaled_rhs(f[0]).ravel()
    for name, cyc, prec, hist_tol in [("V11_fp64_shift_1_over_k", "V", "fp64", 1e-8),
                                      ("W11_fp64_shift_1_over_k", "W", "fp64", 1e-8),
                                      ("V11_fp32_refined_shift_1_over_k", "V", "fp32_refined", 5e-2)]:
        ref = g["runs"][name]
        x, info = S.solve(to_gpu(f), tol=g["tol"], cycle=cyc, precision=prec, history=True, max_cycles=300)
        assert info["status"] == 0
        assert abs(info["cycles"][0] - ref["cycles"]) <= 1, (name, info["cycles"], ref["cycles"])
        m = min(len(ref["history"]), info["cycles"][0])
        got = np.array(info["history"][0][:m])
        want = np.array(ref["history"][:m])
        assert np.max(np.abs(got - want) / want) <= hist_tol, (name, np.max(np.abs(got - want) / want))
        r = np.linalg.norm(fs - A_s @ to_np(x)[0].ravel()) / np.linalg.norm(fs)
        assert r <= g["tol"]
