"""The stop test of a solve (§5: relative residual after each cycle against the
tolerance) is taken on the device while the host keeps a cycle queued ahead.
A solve stopped by its cycle cap and one stopped by its tolerance at the same
cycle hand back the same iterate, bit for bit, in both precisions and at both
parities of the FP64 iterate's ping-pong buffer (the iterate stays where the
stopping cycle left it, also when a further cycle was already queued). The
FP64 iterate equals the oracle's after that many cycles, and the history ends
at the stopping cycle with the reported relative residual."""
import numpy as np
import pytest

import oracle as O
from paper_2308_13476_amd import workloads as W
from tests.gpu_common import require_gpu, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("stop_at", [5, 6])
@pytest.mark.parametrize("precision,smoother,k", [("fp64", "gmres", 30.0), ("fp64", "jacobi", 12.0),
                                                  ("fp32_refined", "gmres", 30.0)])
def test_cap_and_tolerance_stops_agree(precision, smoother, k, stop_at):
    """Jacobi runs at k = 12, where its residual decreases every cycle (at
    k = 30 it stalls after three)."""
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    n = 128
    k2 = W.constant_k2(n, k)
    f = W.point_source_rhs(n, [W.center_node(n)])
    S = Solver(to_gpu(k2), 1.0 / n, 1.0 / k, precision=precision)
    kw = dict(precision=precision, smoother=smoother, history=True)
    xc, ic = S.solve(to_gpu(f), tol=1e-30, max_cycles=stop_at, raise_on_error=False, **kw)
    assert ic["status_name"] == "MG_NOT_CONVERGED" and ic["cycles"] == [stop_at], ic
    h = ic["history"][0]
    assert len(h) == stop_at and np.all(np.isfinite(h))
    assert ic["relres"][0] == h[-1]
    assert h[-1] < min(h[:-1]), h  # a tolerance between the last two residuals stops exactly here
    tol = 0.5 * (h[-1] + min(h[:-1]))
    xt, it = S.solve(to_gpu(f), tol=tol, max_cycles=100, **kw)
    assert it["status"] == 0 and it["cycles"] == [stop_at], it
    assert it["history"][0] == h
    assert torch.equal(xt, xc)
    if precision == "fp64":
        H = O.build_hierarchy(k2, 1.0 / n, 1.0 / k)
        fs = O.scaled_rhs(f[0]).ravel()
        ref = O.solve(H, fs, O.CycleOptions(smoother=smoother), tol=1e-30, max_cycles=stop_at)
        x = to_np(xc)[0].ravel()
        assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_batch_members_stopped_before_the_first_cycle(precision):
    """A batch of a point source, a right-hand side holding a NaN (stopped as
    diverged before the first cycle) and a zero right-hand side (solution
    zero, no cycles): the call reports the divergence, and the point source's
    iterate and cycle count equal its solve alone, bit for bit."""
    require_gpu()
    from paper_2308_13476_amd import _binding as B
    from paper_2308_13476_amd.solver import Solver
    n, k = 128, 30.0
    k2 = W.constant_k2(n, k)
    f0 = W.point_source_rhs(n, [W.center_node(n)])
    bad = W.point_source_rhs(n, [(n // 3, n // 4)])
    bad[0, 5, 7] = np.nan
    batch = np.concatenate([f0, bad, np.zeros_like(f0)])
    S = Solver(to_gpu(k2), 1.0 / n, 1.0 / k, precision=precision, max_batch=3)
    x, info = S.solve(to_gpu(batch), tol=1e-8, precision=precision, raise_on_error=False)
    assert info["status"] == B.MG_E_DIVERGED, info
    assert info["cycles"][1] == 0 and info["cycles"][2] == 0 and info["cycles"][0] > 0, info
    assert not to_np(x[2]).any()
    xs, alone = S.solve(to_gpu(f0), tol=1e-8, precision=precision)
    assert alone["status"] == 0 and alone["cycles"][0] == info["cycles"][0]
    assert torch.equal(x[0:1], xs)


def test_per_cycle_log(monkeypatch, capfd):
    """HELMG_LOG=1 (read at set-up) prints one line per right-hand side and
    cycle as the host reads the stop-test reports: the relative residuals of
    the solve's history, in order, the last one marked converged."""
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    monkeypatch.setenv("HELMG_LOG", "1")
    n, k = 64, 20.0
    S = Solver(to_gpu(W.constant_k2(n, k)), 1.0 / n, 1.0 / k)
    capfd.readouterr()
    x, info = S.solve(to_gpu(W.point_source_rhs(n, [W.center_node(n)])), tol=1e-6, history=True)
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith("helmg: ")]
    assert info["status"] == 0
    assert len(lines) == info["cycles"][0], err[-2000:]
    for c, (ln, r) in enumerate(zip(lines, info["history"][0]), start=1):
        fields = ln.split()
        assert fields[fields.index("cycle") + 1] == str(c)
        assert float(fields[fields.index("relres") + 1]) == pytest.approx(r, rel=1e-6)
    assert lines[-1].endswith("converged") and not any(ln.endswith("converged") for ln in lines[:-1])
