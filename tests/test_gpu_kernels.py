"""Kernel-by-kernel parity of the HIP path with the CPU oracle (FP64 and FP32).

Grids span several 64 x 4 thread tiles with ragged tails (65, 97 and 201 nodes
per side); one case has a variable wavenumber and one uses linear transfers.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from paper_2308_13476_amd import workloads as W
from tests.gpu_common import node_rel, rel, require_gpu, stencil_to_csr, to_gpu, to_np

pytestmark = pytest.mark.gpu

# (name, n, k2 builder, shift, transfer, coarsest_n)
CASES = [
    ("const_n64", 64, lambda n: W.constant_k2(n, 20.0), 0.7, "bezier", 4),
    ("varying_n96", 96, lambda n: W.random_k2(n, 3, 10.0, 25.0), 0.05, "bezier", 3),
    ("const_n200", 200, lambda n: W.constant_k2(n, 30.0), 1.0 / 30.0, "bezier", 25),
    ("linear_n64", 64, lambda n: W.constant_k2(n, 10.0), 0.5, "linear", 4),
]

_cache = {}


def _pair(case):
    if case[0] in _cache:
        return _cache[case[0]]
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    name, n, k2f, beta, transfer, nc = case
    k2 = k2f(n)
    H = O.build_hierarchy(k2, 1.0 / n, beta, transfer=transfer, coarsest_n=nc)
    S = Solver(to_gpu(k2), 1.0 / n, beta, levels=H.levels, transfer=transfer, precision="fp32_refined", max_batch=3)
    _cache[case[0]] = (H, S)
    return H, S


def _rand(n_l, nb, seed):
    return W.random_complex((nb, n_l + 1, n_l + 1), seed)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_level_count_and_radius(case):
    H, S = _pair(case)
    assert S.levels == H.levels
    for l in range(H.levels):
        n_l, r = S.level_info(l)
        assert n_l == H.n[l]
        if l == 0:
            assert r == 1
        elif case[4] == "bezier":
            assert r == (2 if l == 1 else 3)
        else:
            assert r == 1


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_galerkin_stencils(case):
    H, S = _pair(case)
    for l in range(1, H.levels):
        got = stencil_to_csr(to_np(S.stencil(l)))
        ref = H.A[l]
        scale = abs(ref).max()
        assert abs(got - ref).max() <= 1e-13 * scale, (l, abs(got - ref).max() / scale)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_operator_apply_and_residual(case):
    H, S = _pair(case)
    for l in range(H.levels):
        x = _rand(H.n[l], 3, 10 + l)
        f = _rand(H.n[l], 3, 20 + l)
        y = to_np(S.apply(l, to_gpu(x)))
        r = to_np(S.residual(l, to_gpu(x), to_gpu(f)))
        for b in range(3):
            yr = H.A[l] @ x[b].ravel()
            assert rel(y[b], yr) <= 1e-13, (l, b)
            assert node_rel(y[b], yr) <= 1e-13, (l, b, node_rel(y[b], yr))
            assert rel(r[b], f[b].ravel() - yr) <= 1e-13
        y32 = to_np(S.apply(l, to_gpu(x.astype(np.complex64)), precision="fp32_refined"))
        assert y32.dtype == np.complex64
        assert rel(y32[0], H.A[l] @ x[0].ravel()) <= 2e-5


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_restriction_and_prolongation(case):
    H, S = _pair(case)
    for l in range(H.levels - 1):
        fine = _rand(H.n[l], 2, 30 + l)
        coarse = _rand(H.n[l + 1], 2, 40 + l)
        rc = to_np(S.restrict(l, to_gpu(fine)))
        pf = to_np(S.prolong_add(l, to_gpu(coarse), to_gpu(fine)))
        for b in range(2):
            assert rel(rc[b], H.R[l] @ fine[b].ravel()) <= 1e-14
            assert node_rel(rc[b], H.R[l] @ fine[b].ravel()) <= 1e-14
            assert rel(pf[b], fine[b].ravel() + H.P[l] @ coarse[b].ravel()) <= 1e-14


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_jacobi_and_gmres_smoothing(case):
    H, S = _pair(case)
    for l in [0, 1, H.levels - 2]:
        u = _rand(H.n[l], 2, 50 + l)
        f = _rand(H.n[l], 2, 60 + l)
        uj = to_np(S.smooth(l, to_gpu(u), to_gpu(f), "jacobi", nsteps=3, omega=4.5))
        ug = to_np(S.smooth(l, to_gpu(u), to_gpu(f), "gmres", nsteps=2))
        for b in range(2):
            ref = u[b].ravel()
            for _ in range(3):
                ref = O.jacobi_step(H.A[l], ref, f[b].ravel(), 4.5)
            assert rel(uj[b], ref) <= 1e-12, (l, b)
            assert node_rel(uj[b], ref) <= 1e-12, (l, b)
            ref = u[b].ravel()
            for _ in range(2):
                ref = O.gmres_step(H.A[l], ref, f[b].ravel())
            assert rel(ug[b], ref) <= 1e-10, (l, b, rel(ug[b], ref))
            assert node_rel(ug[b], ref) <= 1e-10, (l, b, node_rel(ug[b], ref))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp32_smoothing_close_to_fp32_oracle(case):
    H, S = _pair(case)
    l = 0
    u = _rand(H.n[l], 1, 70).astype(np.complex64)
    f = _rand(H.n[l], 1, 71).astype(np.complex64)
    ug = to_np(S.smooth(l, to_gpu(u), to_gpu(f), "gmres", nsteps=1, precision="fp32_refined"))
    ref = O.gmres_step(H.A32[l], u[0].ravel(), f[0].ravel(), breakdown=1e-6)
    assert rel(ug[0], ref) <= 1e-4


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_coarsest_direct_solve(case):
    H, S = _pair(case)
    f = _rand(H.n[-1], 3, 80)
    u = to_np(S.coarse_solve(to_gpu(f)))
    for b in range(3):
        ref = sla.lu_solve(H.lu, f[b].ravel())
        assert rel(u[b], ref) <= 1e-12
    u32 = to_np(S.coarse_solve(to_gpu(f.astype(np.complex64)), precision="fp32_refined"))
    assert rel(u32[0], sla.lu_solve(H.lu, f[0].ravel().astype(np.complex64).astype(complex))) <= 1e-6


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("cyc,smoother", [("V", "jacobi"), ("W", "jacobi"), ("V", "gmres"), ("W", "gmres")])
def test_one_cycle(case, cyc, smoother):
    H, S = _pair(case)
    n = H.n[0]
    u = _rand(n, 2, 90)
    f = _rand(n, 2, 91)
    got = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle=cyc, smoother=smoother))
    opts = O.CycleOptions(gamma=1 if cyc == "V" else 2, smoother=smoother)
    for b in range(2):
        ref = O.cycle(H, 0, u[b].ravel(), f[b].ravel(), opts)
        assert rel(got[b], ref) <= 1e-10, (b, rel(got[b], ref))


def test_full_size_level_operations_on_sampled_rows():
    """n = 1024 (the benchmarked grid), shift 1/k, k = 200: Galerkin rows and level
    applies at sampled nodes against rows of the oracle's matrices."""
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    n, k = 1024, 200.0
    k2 = W.constant_k2(n, k)
    H = O.build_hierarchy(k2, 1.0 / n, 1.0 / k)
    S = Solver(to_gpu(k2), 1.0 / n, 1.0 / k)
    rng = np.random.default_rng(5)
    for l in range(H.levels):
        m = H.n[l] + 1
        x = W.random_complex((1, m, m), 100 + l)
        y = to_np(S.apply(l, to_gpu(x)))[0].ravel()
        rows = np.concatenate([[0, m - 1, m * m - 1, (m // 2) * m + m // 2], rng.integers(0, m * m, size=64)])
        ref = H.A[l][rows] @ x[0].ravel()
        assert rel(y[rows], ref) <= 1e-13, l
        if l >= 1:
            st = stencil_to_csr(to_np(S.stencil(l)))
            diff = abs(st[rows] - H.A[l][rows]).max()
            assert diff <= 1e-13 * abs(H.A[l]).max(), l


@pytest.mark.parametrize("tail_n", ["0", "32"])
@pytest.mark.parametrize("cyc,smoother", [("V", "gmres"), ("W", "gmres"), ("W", "jacobi")])
def test_one_cycle_tail_setting(monkeypatch, tail_n, cyc, smoother):
    """Levels of at most 16 intervals normally run in the single-workgroup LDS
    tail; with the tail off (every level launched kernel by kernel) or starting
    at 32 intervals (FP32 cycles; FP64 planes do not fit LDS there) the cycle
    is the oracle's as well, in FP64 and FP32."""
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    monkeypatch.setenv("HELMG_TAIL_N", tail_n)
    n = 64
    k2 = W.random_k2(n, 9, 8.0, 18.0)
    H = O.build_hierarchy(k2, 1.0 / n, 0.3)
    S = Solver(to_gpu(k2), 1.0 / n, 0.3, max_batch=2, precision="fp32_refined")
    u = _rand(n, 2, 120)
    f = _rand(n, 2, 121)
    got = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle=cyc, smoother=smoother, nu_pre=2, nu_post=1))
    opts = O.CycleOptions(gamma=1 if cyc == "V" else 2, smoother=smoother, nu1=2, nu2=1)
    for b in range(2):
        ref = O.cycle(H, 0, u[b].ravel(), f[b].ravel(), opts)
        assert rel(got[b], ref) <= 1e-10, (b, rel(got[b], ref))
    got32 = to_np(S.cycle(to_gpu(u.astype(np.complex64)), to_gpu(f.astype(np.complex64)), cycle=cyc,
                          smoother=smoother, nu_pre=2, nu_post=1, precision="fp32_refined"))
    ref = O.cycle(H, 0, u[0].ravel(), f[0].ravel(), opts)
    assert rel(got32[0], ref) <= 1e-4, rel(got32[0], ref)


@pytest.mark.parametrize("env", [{"HELMG_MAX_BLOCKS": "64"}, {"HELMG_L1_PRODUCT": "1"},
                                 {"HELMG_L1_PRODUCT": "2", "HELMG_MAX_BLOCKS": "200"},
                                 {"HELMG_FUSE_CORRECTION": "0"}, {"HELMG_FUSE_RESTRICT": "0"}],
                         ids=["block_cap_64", "product_level1_fp32", "product_level1_fp64", "unfused_correction",
                              "unfused_restriction"])
def test_cycle_with_prereduction_and_level1_operators(monkeypatch, env):
    """With a block cap of 64 every GMRES reduction goes through the one-block
    pre-reduction pass; HELMG_L1_PRODUCT=1 makes FP32 cycles apply level 1 as
    the product R C_s P from level-0 data, =2 both precisions (by default both
    apply the stored Galerkin stencil, read as its upper half);
    HELMG_FUSE_CORRECTION=0 runs the coarse grid correction as a pass of its
    own instead of inside the first post-smoothing pass, HELMG_FUSE_RESTRICT=0
    the restriction instead of inside the last pre-smoothing pass. Each
    gives the oracle's level-1 apply and cycle (FP64) and stays close to it in
    FP32."""
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    n = 128
    k2 = W.random_k2(n, 11, 10.0, 30.0)
    H = O.build_hierarchy(k2, 1.0 / n, 0.2)
    S = Solver(to_gpu(k2), 1.0 / n, 0.2, max_batch=2, precision="fp32_refined")
    x = _rand(n // 2, 2, 130)
    y = to_np(S.apply(1, to_gpu(x)))
    for b in range(2):
        assert rel(y[b], H.A[1] @ x[b].ravel()) <= 1e-13
    u = _rand(n, 2, 131)
    f = _rand(n, 2, 132)
    opts = O.CycleOptions(gamma=1, smoother="gmres")
    got = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle="V", smoother="gmres"))
    got32 = to_np(S.cycle(to_gpu(u.astype(np.complex64)), to_gpu(f.astype(np.complex64)), cycle="V",
                          smoother="gmres", precision="fp32_refined"))
    for b in range(2):
        ref = O.cycle(H, 0, u[b].ravel(), f[b].ravel(), opts)
        assert rel(got[b], ref) <= 1e-10, (b, rel(got[b], ref))
        assert rel(got32[b], ref) <= 1e-4, (b, rel(got32[b], ref))


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_tall_tiles_fit_lds(monkeypatch, precision):
    """A block cap of 64 on the 1024-interval grid asks for tiles of 69 rows
    per thread (276 rows per block): every kernel that stages its tile in LDS,
    the FP64 residual passes of the refinement included, lowers its rows per
    thread until the tile fits, and the solve converges as with the default
    cap, to the same cycle count and iterate."""
    require_gpu()
    from paper_2308_13476_amd.solver import Solver
    n, k = 1024, 200.0
    k2 = to_gpu(W.constant_k2(n, k))
    f = to_gpu(W.point_source_rhs(n, [W.center_node(n)]))
    kw = dict(tol=1e-6, max_cycles=200, precision=precision)
    x_ref, ref = Solver(k2, 1.0 / n, 1.0 / k, precision="fp32_refined").solve(f, **kw)
    monkeypatch.setenv("HELMG_MAX_BLOCKS", "64")
    x, info = Solver(k2, 1.0 / n, 1.0 / k, precision="fp32_refined").solve(f, **kw)
    assert info["status"] == 0 and abs(info["cycles"][0] - ref["cycles"][0]) <= 1
    d = rel(to_np(x)[0], to_np(x_ref)[0])
    print(f"{precision}: cycles {info['cycles'][0]} (default cap {ref['cycles'][0]}), iterate difference {d:.2e}")
    if precision == "fp64" and info["cycles"][0] == ref["cycles"][0]:
        assert d <= 1e-10  # the two differ in the order of their reductions only
    else:
        assert d <= 1e-4  # both iterates are within the tolerance of the solution


@pytest.mark.parametrize("transfer", ["bezier", "linear"])
@pytest.mark.parametrize("n,cap", [(128, None), (256, "64"), (96, None)])
def test_fused_restriction_is_bit_identical(monkeypatch, transfer, n, cap):
    """The last pre-smoothing pass that also restricts its residual (staged in
    LDS over the coarse tile's fine region and halo) gives the bits of the
    separate update and restriction passes: V and W cycles, FP64 and FP32,
    both transfers, two right-hand sides, ragged tiles (96 intervals), and
    tall tiles (block cap 64 on 256 intervals)."""
    require_gpu()
    import torch
    from paper_2308_13476_amd.solver import Solver
    if cap:
        monkeypatch.setenv("HELMG_MAX_BLOCKS", cap)
    k2 = to_gpu(W.random_k2(n, 13, 10.0, 30.0))
    u = _rand(n, 2, 140)
    f = _rand(n, 2, 141)
    out = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("HELMG_FUSE_RESTRICT", fuse)
        S = Solver(k2, 1.0 / n, 0.2, transfer=transfer, max_batch=2, precision="fp32_refined",
                   coarsest_n=6 if n == 96 else 4)
        for cyc in ("V", "W"):
            out[fuse, cyc, 64] = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle=cyc, nu_pre=2, nu_post=1))
            out[fuse, cyc, 32] = to_np(S.cycle(to_gpu(u.astype(np.complex64)), to_gpu(f.astype(np.complex64)),
                                            cycle=cyc, nu_pre=1, nu_post=1, precision="fp32_refined"))
        del S
        torch.cuda.synchronize()
    for cyc in ("V", "W"):
        for bits in (64, 32):
            assert np.array_equal(out["1", cyc, bits], out["0", cyc, bits]), (cyc, bits)


@pytest.mark.parametrize("transfer", ["bezier", "linear"])
@pytest.mark.parametrize("n,env", [(128, {}), (256, {"HELMG_MAX_BLOCKS": "64"}), (96, {}),
                                   (128, {"HELMG_FUSE_CORRECTION": "0"}), (128, {"HELMG_TAIL_N": "0"}),
                                   (128, {"HELMG_L1_PRODUCT": "1"})],
                         ids=["n128", "n256_cap64", "n96", "n128_unfused_correction", "n128_no_tail",
                              "n128_product_level1"])
def test_deferred_coarse_update_is_bit_identical(monkeypatch, transfer, n, env):
    """The update pass of a coarse level's last post-smoothing step, formed by
    the next finer level's correction pass at the coarse nodes it reads (or
    launched just before a correction pass that does not fuse), gives the bits
    of the launched update pass: V and W cycles with one and two
    post-smoothing steps, FP64 and FP32 (a level-1 product operator takes no
    pending update, while level 0 takes level 1's), both transfers, ragged
    tiles (96 intervals), pre-reduced partial sums (block cap 64), and a
    hierarchy launched down to its coarsest level (no tail). Handles for one
    right-hand side (those for batches launch every update pass)."""
    require_gpu()
    import torch
    from paper_2308_13476_amd.solver import Solver
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    k2 = to_gpu(W.random_k2(n, 16, 10.0, 30.0))
    u = _rand(n, 1, 170)
    f = _rand(n, 1, 171)
    runs = [("V", 1, 1), ("W", 1, 2), ("V", 2, 2)]
    out = {}
    for defer in ("1", "0"):
        monkeypatch.setenv("HELMG_DEFER_UPDATE", defer)
        S = Solver(k2, 1.0 / n, 0.2, transfer=transfer, max_batch=1, precision="fp32_refined",
                   coarsest_n=6 if n == 96 else 4)
        for cyc, nu1, nu2 in runs:
            out[defer, cyc, nu2, 64] = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle=cyc, nu_pre=nu1, nu_post=nu2))
            out[defer, cyc, nu2, 32] = to_np(S.cycle(to_gpu(u.astype(np.complex64)),
                                                     to_gpu(f.astype(np.complex64)), cycle=cyc, nu_pre=nu1,
                                                     nu_post=nu2, precision="fp32_refined"))
        del S
        torch.cuda.synchronize()
    for cyc, _, nu2 in runs:
        for bits in (64, 32):
            assert np.array_equal(out["1", cyc, nu2, bits], out["0", cyc, nu2, bits]), (cyc, nu2, bits)


@pytest.mark.parametrize("transfer", ["bezier", "linear"])
@pytest.mark.parametrize("n,env,nb", [(128, {}, 1), (96, {}, 1), (256, {"HELMG_MAX_BLOCKS": "64"}, 1), (128, {}, 2),
                                      (128, {"HELMG_DEFER_UPDATE": "0"}, 1)],
                         ids=["n128", "n96", "n256_cap64", "n128_batch2", "n128_no_deferral"])
def test_fused_correction_and_apply(monkeypatch, transfer, n, env, nb):
    """Level 0 of an FP32 cycle: the first post-smoothing pass that also applies
    A to the residual it forms (x staged with a halo of 2, z0 with a halo of 1,
    the ring evaluated as its owning tiles evaluate it) agrees with the
    correction pass followed by the apply pass to FP32 rounding (the same
    expressions, contracted into fused multiply-adds differently by the two
    kernels: within 1e-5 of the largest value at every node after a cycle), and
    both with the oracle's FP64 cycle within 1e-4 (5e-4 on 256 intervals, where
    the separate passes differ from it by 1.4e-4 in FP32): V and W cycles with one and
    two post-smoothing steps, both transfers, ragged tiles (96 intervals),
    pre-reduced partial sums (block cap 64), a batch handle, and without the
    deferred coarse update."""
    require_gpu()
    import torch
    from paper_2308_13476_amd.solver import Solver
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    k2 = W.random_k2(n, 17, 10.0, 30.0)
    cn = 6 if n == 96 else 4
    H = O.build_hierarchy(k2, 1.0 / n, 0.2, transfer=transfer, coarsest_n=cn)
    u = _rand(n, nb, 180).astype(np.complex64)
    f = _rand(n, nb, 181).astype(np.complex64)
    runs = [("V", 1, 1), ("W", 1, 2), ("V", 2, 2)]
    out = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("HELMG_FUSE_R_A0", fuse)
        S = Solver(to_gpu(k2), 1.0 / n, 0.2, transfer=transfer, max_batch=nb, precision="fp32_refined",
                   coarsest_n=cn)
        for cyc, nu1, nu2 in runs:
            out[fuse, cyc, nu2] = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle=cyc, nu_pre=nu1, nu_post=nu2,
                                                precision="fp32_refined"))
        del S
        torch.cuda.synchronize()
    for cyc, nu1, nu2 in runs:
        opts = O.CycleOptions(gamma=1 if cyc == "V" else 2, smoother="gmres", nu1=nu1, nu2=nu2)
        for r in range(nb):
            a, b = out["1", cyc, nu2][r], out["0", cyc, nu2][r]
            d = node_rel(a, b)
            print(f"{cyc}({nu1},{nu2}) rhs {r}: fused vs separate passes, largest node difference {d:.2e}")
            assert d <= 1e-5, (cyc, nu2, r, d)
            ref = O.cycle(H, 0, u[r].astype(np.complex128).ravel(), f[r].astype(np.complex128).ravel(), opts)
            tol = 1e-4 if n <= 128 else 5e-4
            assert rel(a, ref) <= tol and rel(b, ref) <= tol, (cyc, nu2, r, rel(a, ref), rel(b, ref))


@pytest.mark.parametrize("n,env,nb,x0", [(128, {}, 1, False), (96, {}, 1, True), (256, {"HELMG_MAX_BLOCKS": "64"}, 1, False),
                                         (128, {}, 3, True), (64, {"HELMG_DEFER_UPDATE": "0"}, 1, False),
                                         (512, {"HELMG_MAX_BLOCKS": "64"}, 1, False),
                                         (512, {"HELMG_MAX_BLOCKS": "64"}, 2, True)],
                         ids=["n128", "n96_x0", "n256_cap64", "n128_batch3_x0", "n64_no_deferral",
                              "n512_cap64_lowered_rows", "n512_cap64_batch2_lowered_rows"])
def test_fused_refinement_residual_and_apply(monkeypatch, n, env, nb, x0):
    """FP32-refined solves whose FP64 residual pass before each FP32 cycle also
    forms the first product A z_0 of the cycle's first GMRES step (x staged with
    a halo of 2, r32 with a halo of 1 in LDS, the ring evaluated as its owning
    tiles evaluate it) against solves with the separate apply pass: the same
    cycle counts, residual histories within 1e-3 of each other (FP32 cycles,
    FP64 residuals), iterates within 1e-5 of the largest value at every node, and
    both meet the tolerance in the oracle's FP64 residual. V(1,1) (the first
    step is also the one that restricts), W(2,2) and V(2,1); a ragged grid (96
    intervals), pre-reduced partial sums (block cap 64), a batch handle, a
    nonzero start and no deferred coarse update; on 512 intervals with block
    cap 64 the level's tiles are too tall for the pass's LDS stages, which
    then runs with fewer rows per block than the level's other passes."""
    require_gpu()
    import torch
    from paper_2308_13476_amd.solver import Solver
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    k2 = W.random_k2(n, 23, 10.0, 30.0)
    cn = 6 if n == 96 else 4
    A = O.helmholtz_matrix(k2, 1.0 / n)
    f = _rand(n, nb, 190)
    u0 = _rand(n, nb, 191) if x0 else None
    runs = [("V", 1, 1), ("W", 2, 2), ("V", 2, 1)]
    tol = 1e-7
    out = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("HELMG_FUSE_R_A0", fuse)
        S = Solver(to_gpu(k2), 1.0 / n, 0.2, max_batch=nb, precision="fp32_refined", coarsest_n=cn)
        for cyc, nu1, nu2 in runs:
            x, info = S.solve(to_gpu(f), None if u0 is None else to_gpu(u0), tol=tol, cycle=cyc, nu_pre=nu1,
                              nu_post=nu2, precision="fp32_refined", max_cycles=200, history=True)
            out[fuse, cyc, nu1, nu2] = (to_np(x), list(info["cycles"]), info["history"])
        del S
        torch.cuda.synchronize()
    for cyc, nu1, nu2 in runs:
        (xa, ca, ha), (xb, cb, hb) = out["1", cyc, nu1, nu2], out["0", cyc, nu1, nu2]
        assert ca == cb, (cyc, nu1, nu2, ca, cb)
        for r in range(nb):
            d = node_rel(xa[r], xb[r])
            m = ca[r]  # a batch's histories run to its longest solve
            hd = np.max(np.abs(np.array(ha[r][:m]) - np.array(hb[r][:m])) / np.array(hb[r][:m]))
            print(f"{cyc}({nu1},{nu2}) rhs {r}: {ca[r]} cycles; fused vs separate passes, largest node "
                  f"difference {d:.2e}, largest relative history difference {hd:.2e}")
            assert d <= 1e-5 and hd <= 1e-3, (cyc, nu1, nu2, r, d, hd)
            fs = O.scaled_rhs(f[r].astype(np.complex128)).ravel()
            for xx in (xa[r], xb[r]):
                assert np.linalg.norm(fs - A @ xx.ravel()) <= 1.01 * tol * np.linalg.norm(fs)


@pytest.mark.parametrize("n,cap", [(128, None), (96, None), (256, "64")])
def test_paired_jacobi_sweeps(monkeypatch, n, cap):
    """Weighted-Jacobi sweeps on level 0 run two per pass (x staged for the
    tile plus a halo of 2, the first sweep on the tile plus 1 in LDS): V(4,4) and
    W(3,3) cycles, the odd count taking one pass of two and one single sweep,
    match the oracle's cycle (FP64 within 1e-10, FP32 within 1e-4) and the
    one-sweep-per-pass path to rounding; ragged tiles (96 intervals) and tall
    tiles (block cap 64 on 256 intervals, rows lowered until both LDS stages
    fit)."""
    require_gpu()
    import torch
    from paper_2308_13476_amd.solver import Solver
    if cap:
        monkeypatch.setenv("HELMG_MAX_BLOCKS", cap)
    k2 = W.random_k2(n, 14, 8.0, 20.0)
    cn = 6 if n == 96 else 4
    H = O.build_hierarchy(k2, 1.0 / n, 0.7, coarsest_n=cn)
    u = _rand(n, 2, 150)
    f = _rand(n, 2, 151)
    out = {}
    for pairs in ("1", "0"):
        monkeypatch.setenv("HELMG_JACOBI_PAIRS", pairs)
        S = Solver(to_gpu(k2), 1.0 / n, 0.7, max_batch=2, precision="fp32_refined", coarsest_n=cn)
        for cyc, nu in (("V", 4), ("W", 3)):
            out[pairs, cyc, 64] = to_np(S.cycle(to_gpu(u), to_gpu(f), cycle=cyc, smoother="jacobi", nu_pre=nu,
                                                nu_post=nu))
            out[pairs, cyc, 32] = to_np(S.cycle(to_gpu(u.astype(np.complex64)), to_gpu(f.astype(np.complex64)),
                                                cycle=cyc, smoother="jacobi", nu_pre=nu, nu_post=nu,
                                                precision="fp32_refined"))
        del S
        torch.cuda.synchronize()
    for cyc, nu in (("V", 4), ("W", 3)):
        opts = O.CycleOptions(gamma=1 if cyc == "V" else 2, smoother="jacobi", nu1=nu, nu2=nu)
        for b in range(2):
            ref = O.cycle(H, 0, u[b].ravel(), f[b].ravel(), opts)
            assert rel(out["1", cyc, 64][b], ref) <= 1e-10, (cyc, b, rel(out["1", cyc, 64][b], ref))
            assert rel(out["1", cyc, 32][b], ref) <= 1e-4, (cyc, b)
            assert node_rel(out["1", cyc, 64][b], out["0", cyc, 64][b]) <= 1e-12, (cyc, b)
