#!/usr/bin/env python3
"""Benchmark of the MI355X stand-alone Helmholtz multigrid (one GPU).

Workload (MP 2-A of the paper at the benchmarked size): n = 1024 intervals per
side (1,050,625 unknowns), k = 200 (kh ~ 0.2), unit point source 1/h^2 at the
centre, absorbing boundary, Bézier transfers, shift 1/k, GMRES(3) V(1,1)
cycles, coarsening to 4 x 4 intervals, relative residual 1e-6.

One step = rebuild of the Galerkin hierarchy for the k^2 field (setup) + an
FP32-in-FP64-refined solve to tolerance, with all inputs resident in HBM. The
plain FP64 solve of the same problem is timed beside it. `value` is V-cycle
throughput in unknowns x cycles per second over the timed steps.

Prints one JSON line. `--gpus N` with N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to rel.res 1e-6 & V-cycle DOF/s, FP32-refined vs FP64; % HBM peak"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per node (one read of every input, one write of every
# output) of the kernel classes the library can time with HIP events.
# Class 1: the level-0 GMRES(3) pass that orthogonalises the second Arnoldi
# vector and applies the operator to it: reads w_1, z_0, z_1 and k^2, writes
# z_2 (inner products <z_i, w_2>, ||z_2||^2 and ||w_2||^2 ride along) and, in
# the last pre-smoothing step only, w_2 = A z_2 for the residual that the
# update pass forms by recurrence. In the FP32 cycle a vector is 8 B and k^2
# is 4 B: 3*8 + 4 + 8 = 36 B, plus 8 B for w_2 in one of the two launches per
# cycle that the timing covers, 40 B per launch on average.
KERNEL_CLASSES = {
    1: {"name": "level-0 GMRES(3) orthogonalise + apply pass (complex64)", "bytes_per_node": 40.0},
}
# The same pass on complex128 data with an 8-byte k^2: 3*16 + 8 + 16 = 72 B,
# plus 16 B for w_2 in one of the two launches per cycle, 80 B on average.
CLASS1_FP64_BYTES_PER_NODE = 80.0
# In a batch the k^2 plane (4 B per node, complex64 cycle) is one input shared
# by every right-hand side: 36 B per node and right-hand side without it.
CLASS1_FP32_VECTOR_BYTES = 36.0
CLASS1_FP32_K2_BYTES = 4.0

# Traffic of the roofline kernel per launch from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE; profiles/ holds the summaries and the commands),
# each scaled by what the counter reads for a plain copy of known size. These
# counters see the bytes the L2 caches request from and write to the fabric
# (Infinity Cache, then HBM): "L2->fabric" bytes, reported next to the
# algorithmic bytes. Valid only for the kernel sources they were measured on:
# the hash below is of the files in TRAFFIC_SOURCES, and a different hash
# reports traffic as null.
TRAFFIC_SOURCES = ["paper_2308_13476_amd/csrc/hm_level.hip", "paper_2308_13476_amd/csrc/hm_ops.hpp",
                   "paper_2308_13476_amd/csrc/hm_common.hpp", "paper_2308_13476_amd/csrc/hm_kernels.hpp"]
MEASURED_TRAFFIC = {
    "sources_sha256": "732caa4287a4d51b95c76c1481e5ed21ab1a24977b0e2e55076b26ecf54778bf",
    # k_gm_oa<FineOp<float>, float, 2, 4> at n = 1024 (headline workload)
    "mp2a": {"fetch_bytes": 32481573, "write_bytes": 12684816,
             "profile": "profiles/fp32_cycle_level0_n1024_hbm_traffic.md"},
    # k_gm_oa<FineOp<double>, double, 2, 4> at n = 2048 (working set beyond the Infinity Cache)
    "beyond_cache": {"fetch_bytes": 369740140, "write_bytes": 100889850,
                     "profile": "profiles/fp64_level0_n2048_hbm_traffic.md"},
    # k_gm_oa<FineOp<float>, float, 2, 4>, 64 right-hand sides on n = 512
    "batch64": {"fetch_bytes": 908578802, "write_bytes": 198098200,
                "profile": "profiles/batch64_n512_hbm_traffic.md"},
}


def measured_traffic(which):
    """Fetch + write bytes per launch of the roofline kernel of workload
    `which`, or None when the kernel sources changed since the counters were
    taken."""
    if MEASURED_TRAFFIC is None or MEASURED_TRAFFIC["sources_sha256"] != sources_sha256():
        return None
    m = MEASURED_TRAFFIC[which]
    return m["fetch_bytes"] + m["write_bytes"]


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel_path in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel_path), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def class1_roofline(S, run, bytes_of, what):
    """Times every launch of the level-0 orthogonalise + apply pass (kernel
    class 1, start/stop events recorded by its own dispatch) over run();
    bytes_of(nodes_per_launch) gives its algorithmic bytes per launch."""
    import torch
    S.set_timing(1)
    torch.cuda.synchronize()
    run()
    torch.cuda.synchronize()
    launches, kms, knodes = S.get_timing()
    S.set_timing(0)
    if launches == 0:
        return None
    avg_ms = kms / launches
    nbytes = bytes_of(knodes)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": what, "avg_launch_us": avg_ms * 1e3,
            "launches": launches, "algorithmic_bytes_per_launch": nbytes}


def beyond_cache_roofline(steps):
    """The roofline kernel on a working set far beyond the 256 MB Infinity
    Cache: MP 2-A at n = 2048 (4,198,401 unknowns, k = 400, kh ~ 0.2), FP64
    GMRES(3) V(1,1) cycles, where one complex128 plane is ~70 MB and the
    level-0 pass touches six of them."""
    import torch

    from paper_2308_13476_amd import workloads as W
    from paper_2308_13476_amd.solver import Solver

    dev = torch.device("cuda:0")
    n, k = 2048, 400.0
    S = Solver(torch.from_numpy(W.constant_k2(n, k)).to(dev), 1.0 / n, 1.0 / k)
    f = torch.from_numpy(W.point_source_rhs(n, [W.center_node(n)])).to(dev)
    S.solve(f, tol=1e-30, max_cycles=1)  # warm-up: captures nothing while timing is on
    r = class1_roofline(S, lambda: S.solve(f, tol=1e-30, max_cycles=steps),
                        lambda nodes: CLASS1_FP64_BYTES_PER_NODE * nodes,
                        "level-0 GMRES(3) orthogonalise + apply pass (complex128), n=2048")
    del S
    torch.cuda.empty_cache()
    if r is not None:
        r["workload"] = (f"MP 2-A n={n} ({(n + 1) ** 2} unknowns), k={k:g}, FP64 GMRES(3) V(1,1), {steps} cycles; "
                         f"working set beyond the Infinity Cache")
        r["traffic"] = measured_traffic("beyond_cache")
        r["traffic_kind"] = "L2->fabric (HBM here: the working set exceeds the Infinity Cache)"
    return r


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--k", type=float, default=200.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-settings", action="store_true",
                    help="skip the W(1,1) and Jacobi V(4,4) time-to-tolerance measurements")
    ap.add_argument("--no-beyond-cache", action="store_true",
                    help="skip the n=2048 FP64 roofline measurement beyond the Infinity Cache")
    ap.add_argument("--cpu-cycles", type=int, default=36, help="oracle cycles in the CPU sample")
    ap.add_argument("--kernel-class", type=int, default=1)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain elementwise copy of this many MiB (reference for HBM counters)")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner (mg_tune) on the FP32-refined cycle before timing")
    ap.add_argument("--workload", choices=["mp2a", "batch64", "mixed32", "fgmres", "media2048", "mp2b", "roofline2048"],
                    default="mp2a",
                    help="mp2a: the headline n=1024 solve (default); batch64: 64 sources on n=512 in one "
                         "batched solve; mixed32: 32 problems n=128..1024 solved together")
    return ap.parse_args()


def batch_workloads(args):
    """Secondary workloads (batched right-hand sides, mixed-size problems): one
    step is one FP32-refined GMRES(3) V(1,1) solve of the whole batch to 1e-6
    with the hierarchies set up beforehand; value = sum over right-hand sides of
    unknowns x cycles per second. mixed32 also times the same problems solved
    one after another."""
    import numpy as np
    import torch

    from paper_2308_13476_amd import workloads as W
    from paper_2308_13476_amd.solver import Solver

    dev = torch.device("cuda:0")
    kw = dict(tol=1e-6, cycle="V", smoother="gmres", precision="fp32_refined", max_cycles=400)
    if args.workload == "batch64":
        n, k = 512, 100.0
        nodes = W.seeded_interior_nodes(n, 64, 4)
        f = torch.from_numpy(W.point_source_rhs(n, nodes)).to(dev)
        S = Solver(torch.from_numpy(W.constant_k2(n, k)).to(dev), 1.0 / n, 1.0 / k, max_batch=64,
                   precision="fp32_refined")
        run = lambda: [S.solve(f, **kw)[1]]  # noqa: E731
        sizes = [n]
        config = {"workload": "64 point sources at seeded interior nodes, n=512, k=100, shift 1/k, GMRES(3) V(1,1), "
                              "FP32-refined, tol 1e-6, one batched solve", "n": n, "k": k, "batch": 64}
        nb = 64
        def roof():
            r = class1_roofline(
                S, lambda: S.solve(f, tol=1e-30, max_cycles=3, cycle="V", smoother="gmres", precision="fp32_refined"),
                lambda nodes: CLASS1_FP32_VECTOR_BYTES * nodes + CLASS1_FP32_K2_BYTES * nodes / nb,
                "level-0 GMRES(3) orthogonalise + apply pass (complex64), 64 right-hand sides per launch")
            if r is not None:
                r["traffic"] = measured_traffic("batch64")
                r["traffic_kind"] = "L2->fabric"
            return r
    else:
        order = np.random.default_rng(4).permutation(np.repeat([128, 256, 512, 1024], 8))
        solvers, rhs = [], []
        for n in order:
            n = int(n)
            k = 0.3 * n
            solvers.append(Solver(torch.from_numpy(W.constant_k2(n, k)).to(dev), 1.0 / n, 1.0 / k,
                                  precision="fp32_refined"))
            rhs.append(torch.from_numpy(W.point_source_rhs(n, [W.center_node(n)])).to(dev))
        run = lambda: [info for _, info in Solver.solve_multi(solvers, rhs, **kw)]  # noqa: E731
        roof = None
        sizes = [int(n) for n in order]
        config = {"workload": "32 problems, n in {128,256,512,1024} x 8 (seeded order), k=0.3n, centre source, "
                              "shift 1/k, GMRES(3) V(1,1), FP32-refined, tol 1e-6, solved together",
                  "problems": 32}
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    dof = sum((n + 1) ** 2 * sum(info["cycles"]) for n, info in zip(sizes, infos))
    out = {"metric": "batched V-cycle DOF/s (sum over right-hand sides), FP32-refined", "value": dof / dt,
           "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64 cycle in c128 refinement",
           "data": "synthetic", "config": config,
           "cycles": [c for info in infos for c in info["cycles"]], "roofline": roof() if roof else None,
           "cpu_baseline": None}
    if args.workload == "mixed32":
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for S, f in zip(solvers, rhs):
            S.solve(f, **kw)
        torch.cuda.synchronize()
        seq = time.perf_counter() - t0
        out["sequential_ms"] = seq * 1e3
        out["speedup_vs_sequential"] = seq / dt
    print(json.dumps(out))


def cpu_baseline(n, k, cycles):
    """The CPU oracle on a bounded sample of the same workload: FP64 hierarchy
    setup (not counted) and `cycles` GMRES(3) V(1,1) cycles, single thread."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import oracle as O
    from paper_2308_13476_amd import workloads as W

    import contextlib
    with (threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext()):
        k2 = W.constant_k2(n, k)
        fs = O.scaled_rhs(W.point_source_rhs(n, [W.center_node(n)])[0]).ravel()
        H = O.build_hierarchy(k2, 1.0 / n, 1.0 / k)
        opts = O.CycleOptions(smoother="gmres")
        t0 = time.perf_counter()
        O.solve(H, fs, opts, tol=1e-30, max_cycles=cycles)
        dt = time.perf_counter() - t0
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"value": (n + 1) ** 2 * cycles / dt, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "host_cpu_count": os.cpu_count(), "host_cpus_usable": usable,
            "sample": f"{cycles} FP64 GMRES(3) V(1,1) cycles of the same n={n}, k={k:g} problem "
                      f"(oracle setup excluded), {dt:.1f} s on one host thread (SciPy sparse products and "
                      f"the cycle recursion are single-threaded; BLAS pinned to one thread)"}


def fgmres_workload(args):
    """The headline problem solved by FP64 flexible GMRES(20) with one FP32
    GMRES(3) V(1,1) cycle per iteration as preconditioner (multigrid as a
    preconditioner, §1), to relative residual 1e-6, beside the stand-alone
    FP32-refined solve; hierarchy set up beforehand."""
    import torch

    from paper_2308_13476_amd import workloads as W
    from paper_2308_13476_amd.solver import Solver

    dev = torch.device("cuda:0")
    n, k = args.n, args.k
    k2 = torch.from_numpy(W.constant_k2(n, k)).to(dev)
    f = torch.from_numpy(W.point_source_rhs(n, [W.center_node(n)])).to(dev)
    S = Solver(k2, 1.0 / n, 1.0 / k, precision="fp32_refined")

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            info = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps * 1e3, info

    ms_k, info_k = timed(lambda: S.solve_fgmres(f, tol=1e-6, m=20, precision="fp32_refined")[1])
    ms_a, info_a = timed(lambda: S.solve(f, tol=1e-6, precision="fp32_refined")[1])
    out = {"metric": "time to rel.res 1e-6, FGMRES(20) + FP32 V-cycle preconditioner vs stand-alone FP32-refined",
           "value": ms_k, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_k, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "c128 outer, c64 cycle", "data": "synthetic",
           "config": {"workload": f"MP 2-A n={n}, k={k:g}, centre source, shift 1/k, GMRES(3) V(1,1) preconditioner, "
                                  "FGMRES(20) in FP64, tol 1e-6, setup excluded", "n": n, "k": k},
           "fgmres_iterations": info_k["cycles"][0], "fgmres_relres": info_k["relres"][0],
           "standalone_ms": ms_a, "standalone_cycles": info_a["cycles"][0], "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def media_workload(args):
    """n = 2048 (4,198,401 unknowns) in the seeded three-layer wedge and the
    Gaussian random velocity (MP 2-B stand-ins), max kh = 0.3, source near
    the top centre, shift 1/max(k), GMRES(3) V(1,1), tol 1e-6: FP32-refined
    and FP64 solves per medium, hierarchy set up beforehand (timed apart)."""
    import numpy as np
    import torch

    from paper_2308_13476_amd import workloads as W
    from paper_2308_13476_amd.solver import Solver

    dev = torch.device("cuda:0")
    n = 2048
    res = {}
    dof_cycles, secs = 0.0, 0.0
    for medium in ["wedge", "grf"]:
        c = W.wedge_velocity(n, 3) if medium == "wedge" else W.grf_velocity(n, 3)
        k2 = W.k2_from_velocity(c, 0.3)
        kmax = float(np.sqrt(k2.max()))
        f = torch.from_numpy(W.point_source_rhs(n, [(n // 2, int(round(0.9 * n)))])).to(dev)
        k2d = torch.from_numpy(k2).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = Solver(k2d, 1.0 / n, 1.0 / kmax, precision="fp32_refined")
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        row = {"k_max": kmax, "setup_ms": setup_ms}
        for prec in ["fp32_refined", "fp64"]:
            for _ in range(args.warmup):
                S.solve(f, tol=1e-6, precision=prec, max_cycles=800)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, info = S.solve(f, tol=1e-6, precision=prec, max_cycles=800)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            row[prec] = {"ms": dt * 1e3, "cycles": info["cycles"][0], "relres": info["relres"][0],
                         "ms_per_cycle": dt * 1e3 / info["cycles"][0]}
            if prec == "fp32_refined":
                dof_cycles += (n + 1) ** 2 * info["cycles"][0]
                secs += dt
        res[medium] = row
        del S
        torch.cuda.empty_cache()
    out = {"metric": "V-cycle DOF/s to rel.res 1e-6, FP32-refined (both media)", "value": dof_cycles / secs,
           "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": secs * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64 cycle in c128 refinement", "data": "synthetic",
           "config": {"workload": "n=2048 wedge and Gaussian random velocity (seed 3), max kh 0.3, source "
                                  "(n/2, round(0.9n)), shift 1/k_max, GMRES(3) V(1,1), Bezier, coarsest 4x4, "
                                  "tol 1e-6, setup excluded", "n": n},
           "media": res, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def mp2b_workload(args):
    """MP 2-B high variation (§5.3.2, Table 9): k = 10 + 65 χ with the seeded
    node-by-node random χ on n = 120 (max(k) h = 0.625, coarsest 15
    intervals), shift 1/75, GMRES(3) V(nu,nu) and W(nu,nu) for nu = 1..5,
    FP64, tol 1e-5: time to tolerance per solve, hierarchy set up beforehand."""
    import torch

    from paper_2308_13476_amd import workloads as W
    from paper_2308_13476_amd.solver import Solver

    dev = torch.device("cuda:0")
    k1, k2 = 10.0, 75.0
    n = W.mp2b_grid(k2)
    S = Solver(torch.from_numpy(W.k2_from_chi(W.chi_sharp(n, 6), k1, k2)).to(dev), 1.0 / n, 1.0 / k2,
               coarsest_n=15)
    f = torch.from_numpy(W.point_source_rhs(n, [W.center_node(n)])).to(dev)
    rows, total_ms = [], 0.0
    for nu in range(1, 6):
        for cyc in ["V", "W"]:
            kw = dict(tol=1e-5, cycle=cyc, smoother="gmres", nu_pre=nu, nu_post=nu, max_cycles=600)
            for _ in range(args.warmup):
                S.solve(f, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, info = S.solve(f, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            total_ms += ms
            rows.append({"nu": nu, "cycle": cyc, "cycles": info["cycles"][0], "ms": ms})
    out = {"metric": "time to rel.res 1e-5 summed over the Table 9 sweep (10 solves)", "value": total_ms,
           "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
           "config": {"workload": "MP 2-B high variation, k = 10 + 65 chi (chi: seeded independent uniform per node), "
                                  "n=120, coarsest 15, shift 1/75, GMRES(3) V/W(nu,nu) nu=1..5, FP64, tol 1e-5",
                      "n": n},
           "solves": rows, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration_mib > 0:
        # reads and writes exactly copy_calibration_mib MiB per launch: the reference
        # against which FETCH_SIZE / WRITE_SIZE of the solver kernels are scaled
        import torch
        src = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "fgmres":
        fgmres_workload(args)
        return
    if args.workload == "media2048":
        media_workload(args)
        return
    if args.workload == "mp2b":
        mp2b_workload(args)
        return
    if args.workload == "roofline2048":
        # only the beyond-cache roofline measurement (for the HBM counter runs)
        print(json.dumps({"roofline_beyond_cache": beyond_cache_roofline(args.steps)}))
        return
    if args.workload != "mp2a":
        batch_workloads(args)
        return
    import numpy as np
    import torch

    from paper_2308_13476_amd import workloads as W
    from paper_2308_13476_amd.solver import Solver

    dev = torch.device("cuda:0")
    n, k = args.n, args.k
    beta = 1.0 / k
    nodes = (n + 1) ** 2
    k2 = torch.from_numpy(W.constant_k2(n, k)).to(dev)
    f = torch.from_numpy(W.point_source_rhs(n, [W.center_node(n)])).to(dev)
    S = Solver(k2, 1.0 / n, beta, precision="fp32_refined")
    solve_kw = dict(tol=1e-6, cycle="V", smoother="gmres", nu_pre=1, nu_post=1, max_cycles=500)
    tuned = S.tune(f, precision="fp32_refined") if args.tune else None
    print(f"bench: n={n} k={k:g} levels={S.levels} warmup={args.warmup} steps={args.steps}", file=sys.stderr,
          flush=True)

    def step(precision):
        S.update_k2(k2)
        return S.solve(f, precision=precision, **solve_kw)

    def timed(precision, steps, kernel_class=0):
        for _ in range(args.warmup):
            step(precision)
        S.set_timing(kernel_class)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cycles, solve_s, x = 0, 0.0, None
        for _ in range(steps):
            x, info = step(precision)
            assert info["status"] == 0, info
            cycles += info["cycles"][0]
            solve_s += info["seconds"]
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        kt = S.get_timing()
        S.set_timing(0)
        return {"ms_total": ms, "ms_per_step": ms / steps, "cycles_per_solve": cycles / steps,
                "solve_ms_per_step": 1e3 * solve_s / steps, "x": x, "kernel": kt}

    r32 = timed("fp32_refined", args.steps)
    print(f"bench: fp32-refined {r32['ms_per_step']:.2f} ms/step, {r32['cycles_per_solve']:.0f} cycles",
          file=sys.stderr, flush=True)
    # the same steps again, every launch of the roofline kernel recording a
    # start and a stop HIP event with its own dispatch (kernel-by-kernel
    # launches instead of captured graphs)
    rk = timed("fp32_refined", max(1, args.steps // 2), args.kernel_class)
    r64 = timed("fp64", max(2, args.steps // 2))
    print(f"bench: fp64 {r64['ms_per_step']:.2f} ms/step, {r64['cycles_per_solve']:.0f} cycles", file=sys.stderr,
          flush=True)

    # the other cycle / smoother settings of the same workload (§5.1 Table 4:
    # weighted Jacobi V(4,4) with shift 0.7; §5.3.1 Table 8: GMRES(3) W(1,1)),
    # time to tolerance with the hierarchy set up beforehand
    settings = {}
    if not args.no_other_settings:
        def solve_time(solver, precision, reps=2, **kw):
            kw = dict(solve_kw, **kw)
            solver.solve(f, precision=precision, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                _, info = solver.solve(f, precision=precision, **kw)
                assert info["status"] == 0, info
            torch.cuda.synchronize()
            return {"ms": (time.perf_counter() - t0) / reps * 1e3, "cycles": info["cycles"][0]}
        settings["gmres_W11_shift_1_over_k"] = {"fp32_refined": solve_time(S, "fp32_refined", cycle="W"),
                                                "fp64": solve_time(S, "fp64", cycle="W")}
        S07 = Solver(k2, 1.0 / n, 0.7)
        settings["jacobi_V44_shift_0.7"] = {"fp64": solve_time(S07, "fp64", reps=1, smoother="jacobi", nu_pre=4,
                                                               nu_post=4, max_cycles=1000)}
        del S07
        print(f"bench: other settings {settings}", file=sys.stderr, flush=True)

    value = nodes * r32["cycles_per_solve"] * args.steps / (r32["ms_total"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 cycle in c128 refinement",
        "data": "synthetic",
        "config": {"workload": f"MP 2-A, n={n} ({nodes} unknowns), k={k:g}, centre point source, GMRES(3) "
                               f"V(1,1), Bezier transfers, shift 1/k, coarsest 4x4, tol 1e-6, "
                               f"setup + FP32-refined solve per step",
                   "n": n, "k": k, "levels": S.levels},
        "time_to_tol_ms": {"fp32_refined": r32["ms_per_step"], "fp64": r64["ms_per_step"]},
        "solve_only_ms": {"fp32_refined": r32["solve_ms_per_step"], "fp64": r64["solve_ms_per_step"]},
        "cycles": {"fp32_refined": r32["cycles_per_solve"], "fp64": r64["cycles_per_solve"]},
        "vcycle_dof_per_s": {"fp32_refined": value,
                             "fp64": nodes * r64["cycles_per_solve"] / (r64["ms_per_step"] * 1e-3)},
        "fp32_refined_speedup_vs_fp64": r64["ms_per_step"] / r32["ms_per_step"],
        "other_settings_solve_ms": settings or None,
    }
    if tuned is not None:
        out["tuned_settings"] = tuned
    # error of both GPU results against the stored FP64 oracle iterate and exact solution
    gold = os.path.join(ROOT, "tests", "golden", "oracle_full_size.json")
    if n == 1024 and k == 200.0 and os.path.exists(gold):
        g = json.load(open(gold))
        if "samples" in g:
            idx = np.array(g["samples"]["index"])
            mg = np.array(g["samples"]["fp64_mg_re"]) + 1j * np.array(g["samples"]["fp64_mg_im"])
            ex = np.array(g["samples"]["exact_re"]) + 1j * np.array(g["samples"]["exact_im"])
            errs = {}
            for name, r in [("fp32_refined", r32), ("fp64", r64)]:
                xs = r["x"][0].reshape(-1).cpu().numpy()[idx]
                errs[name] = {"vs_fp64_oracle_iterate": float(np.linalg.norm(xs - mg) / np.linalg.norm(mg)),
                              "vs_exact_discrete_solution": float(np.linalg.norm(xs - ex) / np.linalg.norm(ex))}
            out["rel_error_on_4096_sampled_nodes"] = errs
    launches, kms, knodes = rk["kernel"]
    if launches > 0 and args.kernel_class in KERNEL_CLASSES:
        kc = KERNEL_CLASSES[args.kernel_class]
        avg_ms = kms / launches
        achieved = kc["bytes_per_node"] * knodes / (avg_ms * 1e-3) / 1e9
        traffic = measured_traffic("mp2a") if args.kernel_class == 1 else None  # bytes per launch
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_kind": "L2->fabric",
                           "algorithmic_bytes_per_launch": kc["bytes_per_node"] * knodes,
                           "kernel": kc["name"],
                           "avg_launch_us": avg_ms * 1e3, "launches": launches,
                           "timed_in": "repeat of the timed steps; HIP start/stop events recorded by each "
                                       "launch's own dispatch (hipExtLaunchKernelGGL), no graphs"}
    if not args.no_beyond_cache:
        print("bench: roofline kernel beyond the Infinity Cache (n=2048, FP64)", file=sys.stderr, flush=True)
        out["roofline_beyond_cache"] = beyond_cache_roofline(max(2, args.steps // 2))
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(n, k, args.cpu_cycles)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
