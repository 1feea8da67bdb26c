"""Writes tests/golden/mp2b_chi_tables.json: the paper's MP 2-B cycle counts
(§5.2 Tables 5 and 6, weighted Jacobi with shift 0.7; §5.3.2 Table 9,
GMRES(3) with shift 1/k_max) next to the oracle's counts on seeded stand-ins
for the unspecified random profile χ: k = k1 + (k2 - k1) χ with (k1, k2) =
(10, 50) on n = 80 and (10, 75) on n = 120 intervals (max(k) h = 0.625),
coarsened to 5 and 15 intervals, centre point source, Bézier transfers,
nu pre- and nu post-smoothing steps, tol 1e-5, divergence declared when the
relative residual exceeds 1e8 times its initial value (stored as minus the
cycle at which that happened).

  smooth (Table 5): workloads.chi_smooth(n, 5)  Gaussian-filtered noise, width 0.1
  sharp (Tables 6, 9): workloads.chi_sharp(n, 6)  independent uniform values per node

Run: python tests/golden/make_mp2b_golden.py   (about ten minutes, one core)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2308_13476_amd import workloads as W  # noqa: E402

RANGES = [[10, 50], [10, 75]]
SEEDS = {"smooth": 5, "sharp": 6}
COARSEST = {80: 5, 120: 15}
# printed counts, [nu index][range index][gamma index] with gamma = 1 (V), 2 (W)
PAPER = {
    "table5_smooth_jacobi": {"nu": [4, 5, 6, 7, 8], "profile": "smooth", "smoother": "jacobi", "shift": "0.7",
                             "counts": [[[65, 60], [90, 88]], [[62, 59], [86, 86]], [[61, 58], [85, 85]],
                                        [[60, 57], [84, 84]], [[59, 57], [83, 83]]]},
    "table6_sharp_jacobi": {"nu": [4, 5, 6, 7, 8], "profile": "sharp", "smoother": "jacobi", "shift": "0.7",
                            "counts": [[[102, 96], [111, 107]], [[97, 95], [103, 105]], [[95, 95], [101, 104]],
                                       [[94, 94], [102, 104]], [[94, 94], [102, 104]]]},
    "table9_sharp_gmres": {"nu": [1, 2, 3, 4, 5], "profile": "sharp", "smoother": "gmres", "shift": "1/k_max",
                           "counts": [[[28, 12], [31, 12]], [[16, 8], [17, 7]], [[12, 7], [12, 6]],
                                      [[10, 6], [10, 6]], [[9, 6], [9, 6]]]},
}


def main():
    out = {"source": "Dwarka & Vuik, arXiv 2308.13476, Section 5.2 Tables 5 and 6, Section 5.3.2 Table 9",
           "ranges": RANGES, "kh": 0.625, "tol": 1e-5, "seeds": SEEDS, "coarsest": COARSEST,
           "paper": PAPER, "oracle": {}}
    for table, spec in PAPER.items():
        counts = []
        for nu in spec["nu"]:
            row = []
            for k1, k2 in RANGES:
                n = W.mp2b_grid(k2)
                chi = W.chi_smooth(n, SEEDS["smooth"]) if spec["profile"] == "smooth" else W.chi_sharp(n, SEEDS["sharp"])
                k2f = W.k2_from_chi(chi, k1, k2)
                shift = 0.7 if spec["shift"] == "0.7" else 1.0 / k2
                fs = O.scaled_rhs(W.point_source_rhs(n, [W.center_node(n)])[0]).ravel()
                H = O.build_hierarchy(k2f, 1.0 / n, shift, coarsest_n=COARSEST[n])
                pair = []
                for gamma in (1, 2):
                    t = time.time()
                    r = O.solve(H, fs, O.CycleOptions(smoother=spec["smoother"], gamma=gamma, nu1=nu, nu2=nu),
                                tol=1e-5, max_cycles=600)
                    # converged: cycles to tol; diverged: minus the cycle at which it was detected
                    assert r.status in ("converged", "diverged"), r.status
                    pair.append(r.cycles if r.status == "converged" else -r.cycles)
                    print(table, nu, (k1, k2), n, gamma, r.cycles, r.status, round(time.time() - t, 1), flush=True)
                row.append(pair)
            counts.append(row)
        out["oracle"][table] = counts
        with open(os.path.join(HERE, "mp2b_chi_tables.json"), "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
