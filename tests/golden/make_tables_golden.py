"""Writes tests/golden/gmres_tables_kh0625.json: the paper's GMRES(3) cycle
counts of Tables 7 and 8 (§5.3.1; MP 2-A, kh = 0.625, tol 1e-5, Bézier
transfers, nu pre- and nu post-smoothing steps, shift 0.7 in Table 7 and 1/k
in Table 8) next to the oracle's counts for nu = 1 on the grids read as
n = k / 0.625 intervals (80, 160, 240, 320, 400), coarsened to 5, 5, 15, 5 and
25 intervals (the paper's unknown counts N do not fit one grid rule).

Run: python tests/golden/make_tables_golden.py   (about ten minutes, one core)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2308_13476_amd import workloads as W  # noqa: E402

KS = [50, 100, 150, 200, 250]
COARSEST = {80: 5, 160: 5, 240: 15, 320: 5, 400: 25}
# Tables 7 and 8 of §5.3.1 as printed: [nu][k] for V (gamma 1) and W (gamma 2)
PAPER = {
    "table7_shift_0.7": {
        "V": [[37, 68, 99, 132, 162], [29, 53, 78, 104, 128], [24, 45, 67, 89, 112], [22, 40, 59, 78, 98],
              [20, 36, 53, 71, 88]],
        "W": [[36, 67, 98, 131, 161], [29, 53, 78, 104, 128], [24, 45, 67, 89, 112], [22, 40, 59, 78, 98],
              [20, 36, 53, 71, 88]],
    },
    "table8_shift_1_over_k": {
        "V": [[14, 24, 39, 51, 64], [8, 13, 22, 28, 34], [6, 10, 16, 20, 24], [6, 8, 12, 15, 18],
              [5, 7, 11, 13, 15]],
        "W": [[7, 10, 19, 24, 29], [5, 7, 10, 13, 16], [5, 6, 9, 10, 12], [5, 5, 7, 9, 10], [5, 5, 7, 8, 9]],
    },
}


def main():
    out = {"source": "Dwarka & Vuik, arXiv 2308.13476, Section 5.3.1, Tables 7 and 8",
           "k": KS, "kh": 0.625, "tol": 1e-5, "paper": PAPER, "oracle_nu1": {}}
    for table, shift_of in [("table7_shift_0.7", lambda k: 0.7), ("table8_shift_1_over_k", lambda k: 1.0 / k)]:
        res = {"V": [], "W": []}
        for k in KS:
            n = int(round(k / 0.625))
            k2 = W.constant_k2(n, float(k))
            fs = O.scaled_rhs(W.point_source_rhs(n, [W.center_node(n)])[0]).ravel()
            H = O.build_hierarchy(k2, 1.0 / n, shift_of(k), coarsest_n=COARSEST[n])
            for cyc, gamma in [("V", 1), ("W", 2)]:
                t = time.time()
                r = O.solve(H, fs, O.CycleOptions(smoother="gmres", gamma=gamma), tol=1e-5, max_cycles=400)
                res[cyc].append(r.cycles)
                print(table, k, n, cyc, r.cycles, r.status, round(time.time() - t, 1), flush=True)
        out["oracle_nu1"][table] = res
        with open(os.path.join(HERE, "gmres_tables_kh0625.json"), "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
