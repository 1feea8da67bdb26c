"""The full-size constant-wavenumber workload (n = 1024, k = 200) under the
smoother, cycle and shift settings of §5.1 (weighted Jacobi, Table 4) and
§5.3.1 (GMRES(3) with nu = 1 ... 5, V and W, Tables 7-8) against the oracle's
stored runs (tests/golden/oracle_config2.json, written by
make_config2_golden.py from oracle/ only): cycle counts within one, the
relative residual after every cycle, the final residual, and at equal cycle
counts the iterate at 4096 sampled nodes (FP64 within 1e-10 of the largest
value at every sampled node); the Jacobi V(1,1)
run that does not converge at this kh ends as diverged within two cycles of
the oracle's stop."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2308_13476_amd import workloads as W
from tests.gpu_common import node_rel, require_gpu, to_gpu, to_np

pytestmark = pytest.mark.gpu
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_config2.json")))
N, K = 1024, 200.0
_SOLVERS = {}


def _solver(shift):
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    if shift not in _SOLVERS:
        _SOLVERS.clear()  # one hierarchy (about 0.6 GB) at a time
        _SOLVERS[shift] = Solver(to_gpu(W.constant_k2(N, K)), 1.0 / N, shift, precision="fp32_refined")
    return _SOLVERS[shift]


@pytest.fixture(scope="module")
def problem():
    k2 = W.constant_k2(N, K)
    f = W.point_source_rhs(N, [W.center_node(N)])
    A_s = O.helmholtz_matrix(k2, 1.0 / N)
    fs = O.scaled_rhs(f[0]).ravel()
    yield f, A_s, fs
    _SOLVERS.clear()


RUNS = sorted(GOLDEN["runs"], key=lambda r: GOLDEN["runs"][r]["shift"])


@pytest.mark.parametrize("name", RUNS)
def test_config2_run_against_stored_oracle_run(name, problem):
    from paper_2308_13476_amd import _binding as B
    f, A_s, fs = problem
    ref = GOLDEN["runs"][name]
    S = _solver(ref["shift"])
    prec = "fp32_refined" if ref["fp32_refined"] else "fp64"
    x, info = S.solve(to_gpu(f), tol=GOLDEN["tol"], cycle="V" if ref["gamma"] == 1 else "W",
                      smoother=ref["smoother"], nu_pre=ref["nu"], nu_post=ref["nu"], omega=4.5,
                      max_cycles=ref["max_cycles"], precision=prec, divergence=GOLDEN["divergence"], history=True,
                      raise_on_error=False)
    got = np.array(info["history"][0])
    want = np.array(ref["history"])
    m = min(len(got), len(want))
    err = np.abs(got[:m] - want[:m]) / want[:m]
    print(f"{name}: GPU {info['cycles'][0]} cycles ({info['status_name']}), oracle {ref['cycles']} "
          f"({ref['status']}); largest relative difference of the residual histories {err.max():.2e}")
    if ref["status"] == "diverged":
        assert info["status"] == B.MG_E_DIVERGED
        assert abs(info["cycles"][0] - ref["cycles"]) <= 2
        # the iteration is linear in the error, so rounding differences stay
        # relative while the residual grows
        assert err.max() <= 1e-6
        return
    assert info["status"] == B.MG_OK
    assert abs(info["cycles"][0] - ref["cycles"]) <= 1
    # A residual history amplifies an iterate difference dx by about
    # ||A|| ||x|| / (||f|| relres); the GPU's Gram-Schmidt variant (classical,
    # with the last Arnoldi norm from the norm identity) differs from the
    # oracle's modified Gram-Schmidt by rounding that cancellation in that
    # identity enlarges when the Krylov space is nearly invariant. Measured
    # worst case 4.6e-8 (W(2,2)); the iterates themselves are compared below.
    assert err.max() <= (5e-2 if ref["fp32_refined"] else 1e-7)
    r = np.linalg.norm(fs - A_s @ to_np(x)[0].ravel()) / np.linalg.norm(fs)
    assert r <= GOLDEN["tol"]
    if info["cycles"][0] == ref["cycles"]:
        idx = np.array(ref["sample_index"])
        want_x = np.array(ref["x_re"]) + 1j * np.array(ref["x_im"])
        got_x = to_np(x)[0].ravel()[idx]
        d = node_rel(got_x, want_x)
        print(f"{name}: iterate after {ref['cycles']} cycles at 4096 sampled nodes, largest difference "
              f"relative to the largest value {d:.2e}")
        # FP64: the parity bar of the method; FP32-refined: both iterates are
        # within the tolerance of the solution, FP32 rounding apart
        assert d <= (1e-5 if ref["fp32_refined"] else 1e-10)
