"""Writes tests/golden/oracle_full_size.json from the CPU oracle only.

Full-size workload: MP 2-A (§2) with n = 1024 intervals, k = 200 (kh ~ 0.2),
unit point source 1/h^2 at the centre, GMRES(3) smoothing (§5.3), Bézier
transfers, coarsening to a 4 x 4-interval grid, shift 1/k (§5.3.1). Stores
cycle counts to relative residual 1e-6 and the residual history of every
cycle for V(1,1), W(1,1) and the FP32-refined V(1,1) cycle.

It also stores the FP64 iterate of the V(1,1) run and the exact discrete
solution (sparse LU) at 4096 seeded sample nodes, so that the error of a
GPU result against the FP64 oracle can be stated without re-running it.

Run: python tests/golden/make_oracle_golden.py   (about five minutes, one core)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402
import scipy.sparse.linalg as spla  # noqa: E402

import oracle as O  # noqa: E402
from paper_2308_13476_amd import workloads as W  # noqa: E402


def main():
    n, k, tol = 1024, 200.0, 1e-6
    k2 = W.constant_k2(n, k)
    fs = O.scaled_rhs(W.point_source_rhs(n, [W.center_node(n)])[0]).ravel()
    out = {"workload": "MP 2-A, n=1024, k=200, centre source, GMRES(3), Bezier, coarsest 4x4 intervals",
           "tol": tol, "runs": {}}
    t = time.time()
    H = O.build_hierarchy(k2, 1.0 / n, 1.0 / k)
    out["setup_seconds"] = time.time() - t
    runs = [("V11_fp64_shift_1_over_k", H, 1, False), ("W11_fp64_shift_1_over_k", H, 2, False),
            ("V11_fp32_refined_shift_1_over_k", H, 1, True)]
    for name, hier, gamma, fp32 in runs:
        t = time.time()
        opts = O.CycleOptions(gamma=gamma, smoother="gmres")
        res = (O.solve_refined if fp32 else O.solve)(hier, fs, opts, tol=tol, max_cycles=300)
        out["runs"][name] = {"cycles": res.cycles, "status": res.status, "history": res.history,
                             "seconds": time.time() - t}
        if name == "V11_fp64_shift_1_over_k":
            x_mg = res.x
        print(name, res.cycles, res.status, round(time.time() - t, 1), flush=True)
    exact = spla.splu(H.A[0].tocsc()).solve(fs)
    idx = np.sort(np.random.default_rng(2024).choice(fs.size, size=4096, replace=False))
    out["samples"] = {
        "index": idx.tolist(),
        "fp64_mg_re": x_mg[idx].real.tolist(), "fp64_mg_im": x_mg[idx].imag.tolist(),
        "exact_re": exact[idx].real.tolist(), "exact_im": exact[idx].imag.tolist(),
        "fp64_mg_rel_err_vs_exact_full": float(np.linalg.norm(x_mg - exact) / np.linalg.norm(exact)),
    }
    with open(os.path.join(HERE, "oracle_full_size.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
