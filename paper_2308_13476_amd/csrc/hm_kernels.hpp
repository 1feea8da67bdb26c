// Host-side launchers of the HIP kernels (implemented in the .hip files).
// Every launcher enqueues on ctx.stream and never synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include "hm_common.hpp"

namespace hm {

// Per-right-hand-side GMRES(3) state kept on the device between the passes of
// one smoothing step.
struct GmState {
    double beta;          // ||r0||
    double s[4];          // 1 / ||z_j||: the stored Arnoldi vectors are unnormalised
    double hr[4][3];      // Hessenberg matrix, real part
    double hi[4][3];      // Hessenberg matrix, imaginary part
    double yr[3], yi[3];  // least-squares solution times s_i (update weights)
    int k;                // Arnoldi columns in use (0: r0 = 0, nothing to do)
    int arnoldi_done;     // 1 after breakdown or the last column
};

// Per-right-hand-side norms read by the host.
struct RhsNorms {
    double f2;   // ||f_s||^2
    double r2;   // latest ||f_s - A_s x||^2
};

// Stop test of one cycle (§5 stopping criterion), taken on the device by the
// norm pass that ends the cycle, one block per right-hand side: with
// r = sqrt(r2 / f2), a right-hand side stops as diverged when r is not finite
// or exceeds its divergence limit, else as converged when r <= tol. A stopped
// right-hand side has its active flag cleared, so cycles already queued
// behind this one skip it. Every test writes one report into a ring that the
// host reads after the cycle's completion event.
constexpr int kReportRing = 4;

struct RhsReport {
    double f2, r2;  // norms of the test
    int stop;       // 0 running, 1 converged, 2 diverged
    int cycle;      // 1-based count of tests of this right-hand side in the solve
};

struct StopTest {
    RhsReport* ring;       // host-visible [kReportRing][stride]; nullptr: no test
    int* active;           // [nrhs] the solve's active flags (cleared on a stop)
    int* count;            // [nrhs] tests taken so far (zeroed when the solve begins)
    const double* limits;  // [nrhs][2]: tolerance, divergence limit
    int stride;
};

// Shared launch parameters of one batched call.
struct LaunchCtx {
    hipStream_t stream;
    int nrhs;           // batch size (grid z)
    const int* active;  // [nrhs] device flags; 0 skips that right-hand side
    double* partials;   // per-block partial sums: 2 regions x nrhs_cap x kPartStride doubles
    int nrhs_cap;       // right-hand sides the partials were sized for
    int block_cap;      // blocks per right-hand side a level grid aims at (reductions)
    int fuse_correction = 1;  // 0: the coarse grid correction always runs as its own pass
    int fuse_restrict = 1;    // 0: the restriction always runs as its own pass
    int fuse_r_a0 = 1;        // 0: on level 0 (FP32) the first apply pass of a post-smoothing step runs on its own
    StopTest stop{};          // taken by the residual-norm pass when stop.ring is set
    int tall_rows = 4;        // block height of light kernels on grids of >= 256 intervals (4, 8, 16)
    int small_rows = 2;       // block height on grids of <= 128 intervals (2 or 4)
};

// The operator of one level: analytic on level 0 (from k^2), stored Galerkin
// stencil planes of radius `radius` on coarser levels.
template <typename T>
struct LevelOp {
    int level;
    Grid g;
    int radius;
    const cplx<T>* coef;  // [(2r+1)^2][plane], levels >= 1
    const T* k2;          // padded k^2 plane, level 0
    double h;             // level-0 mesh width
    // Level 1 applied as the product R C_s P from level-0 data (product != 0):
    // level-0 grid, shift beta2 of C_s, transfer (0 Bezier, 1 linear).
    int product;
    Grid g0;
    double shift;
    int transfer;
};

// Vectors of one level in the padded layout: `count` consecutive planes.
template <typename T>
struct Vec {
    cplx<T>* p;
    long long plane;
    __host__ __device__ cplx<T>* rhs(int b) const { return p + b * plane; }
};

template <typename T> void launch_apply(const LaunchCtx&, const LevelOp<T>&, Vec<T> x, Vec<T> y);
// Level 0 (lop.level == 0): x = xs widened to FP64, and y = A_s x, in one pass.
void launch_apply_widened(const LaunchCtx&, const LevelOp<double>& lop, Vec<float> xs, Vec<double> x, Vec<double> y);
template <typename T> void launch_residual(const LaunchCtx&, const LevelOp<T>&, Vec<T> x, Vec<T> f, Vec<T> r);
template <typename T>
void launch_jacobi(const LaunchCtx&, const LevelOp<T>&, Vec<T> x, Vec<T> f, Vec<T> y, double inv_omega);
// Two sweeps from x into y in one pass on level 0; returns false, launching
// nothing, on any other level (or where the two LDS stages do not fit).
template <typename T>
bool launch_jacobi2(const LaunchCtx&, const LevelOp<T>&, Vec<T> x, Vec<T> f, Vec<T> y, double inv_omega);
// fc = R r; when uc.p is not null the coarse iterate uc is zeroed in the same
// pass. When z0.p is not null, fc is also written to the first Arnoldi plane of
// z0 (4 planes per right-hand side) with the partial sums of ||fc||^2 in
// reduction region 0: the residual pass of a GMRES step from uc = 0. Returns
// the number of blocks per right-hand side (the partial-sum count).
template <typename T>
int launch_restrict(const LaunchCtx&, Grid fine, Grid coarse, int transfer, Vec<T> r, Vec<T> fc, Vec<T> uc,
                    Vec<T> z0 = Vec<T>{nullptr, 0});
template <typename T>
void launch_prolong_add(const LaunchCtx&, Grid coarse, Grid fine, int transfer, Vec<T> e, Vec<T> u);

// The update pass of a coarse level's last post-smoothing GMRES step, left to
// the pass that reads its result (the coarse grid correction of the next finer
// level): u = base + sum_i c_i z_i with base = uin (or u where uin.p is null)
// and c_i from the step's state and the partial sums of its last Arnoldi pass,
// as the update pass computes them. Z.p null: nothing is pending.
template <typename T>
struct DeferredUpdate {
    Vec<T> Z{nullptr, 0};    // the step's Arnoldi planes (4 per right-hand side)
    Vec<T> u{nullptr, 0};    // the coarse iterate
    Vec<T> uin{nullptr, 0};  // the iterate the step started from, when not u
    const GmState* st = nullptr;
    const double* part = nullptr;  // partial sums of the last Arnoldi pass
    int nblk = 0;
    double breakdown = 0.0;
};

// A coarse grid correction to fold into the next smoothing step: u += P e with
// e on the coarse grid gc; xt receives u + P e. With du.Z.p set, e is the
// pending update du of the coarse level's last smoothing step, formed on the
// fly (e.p is then the coarse iterate that update would have written).
template <typename T>
struct ProlongIn {
    Grid gc{};
    Vec<T> e{nullptr, 0};
    int transfer = 0;
    Vec<T> xt{nullptr, 0};
    DeferredUpdate<T> du{};
};

// The restriction to fold into the last pass of a pre-smoothing step (§3
// coarse grid correction, §4 transfer): fc = R r' on the coarse grid gc for
// the residual r' of the updated iterate, uc = 0 (uc.p may be null) and, with
// zc.p set, fc into the first coarse Arnoldi plane with partial sums of
// ||fc||^2 in reduction region 0, as launch_restrict does. nblk receives the
// number of blocks per right-hand side of that launch.
template <typename T>
struct RestrictOut {
    Grid gc{};
    int transfer = 0;
    Vec<T> fc{nullptr, 0}, uc{nullptr, 0}, zc{nullptr, 0};
    int nblk = 0;
};

// One GMRES(3) smoothing step (§5.3) on A u = f: five passes (residual; apply;
// two fused orthogonalise + apply passes; last column + least squares + update).
// Z holds 4 planes per right-hand side (Arnoldi vectors), Wa / Wb the
// products A z. timed (may be null): a start and a stop event that the
// dispatch of the second orthogonalise + apply pass records itself
// (hipExtLaunchKernelGGL), so that their interval is that kernel's execution
// (timing hook; eager launches only). With res.p set, the
// last pass updates u in place and writes the residual f - A u of the updated
// iterate to res (which may be Wa), formed by recurrence from the first
// residual and the products A z_i of the Arnoldi passes. pro.e.p set: the
// step begins with the coarse grid correction u += P e (coarse level pro.gc),
// formed on the fly by the first pass, which keeps u + P e in pro.xt; the last
// pass then writes the updated iterate to u (the step never changes the
// roles of u and pro.xt). On level 0 of FP32 cycles (ctx.fuse_r_a0) that first
// pass also applies A to the residual it forms, taking the second pass with
// it. r_ready_nblk > 0
// means u = 0 and the residual pass already ran as part of the restriction
// (z_0 = f in Z, r_ready_nblk partial sums of ||f||^2 in region 0): the step
// starts with the second pass. u_zero: the step starts from u = 0 although u
// does not hold zeros (its update pass then writes sum y_i s_i z_i without
// reading u). rout (with res.p; may be null): the last pass restricts the
// residual itself (unless ctx.fuse_restrict is 0) and res is not written;
// rout->nblk is set to the partial-sum count of the coarse launch, or to 0
// when the caller must restrict res itself. defer (may be null; ignored with
// res.p or u_zero): the update pass is not launched and *defer describes it,
// for the caller to hand to the next finer level's correction (ProlongIn::du);
// the step's Z, state and partial sums must then stay untouched until that
// pass has run. Where the step has no plain update pass, defer->Z.p is null.
// w_ready (level 0 of FP32 cycles, with r_ready_nblk): the refinement residual
// pass also formed w_0 = A z_0 in Wa, with ||z_0||^2 and <z_0, w_0> in region
// 1, and the step starts with its first orthogonalise + apply pass.
template <typename T>
void launch_gmres_step(const LaunchCtx&, const LevelOp<T>&, Vec<T> u, Vec<T> f, Vec<T> Z, Vec<T> Wa, Vec<T> Wb,
                       GmState* st, double breakdown, const hipEvent_t* timed, Vec<T> res = Vec<T>{nullptr, 0},
                       int r_ready_nblk = 0,
                       ProlongIn<T> pro = ProlongIn<T>{}, bool u_zero = false, RestrictOut<T>* rout = nullptr,
                       DeferredUpdate<T>* defer = nullptr, bool w_ready = false);

// ||f - A x||^2 per right-hand side into norms[b].r2 (level-0 operator).
template <typename T>
void launch_resnorm(const LaunchCtx&, const LevelOp<T>&, Vec<T> x, Vec<T> f, RhsNorms* norms);
// ||f||^2 into norms[b].f2.
template <typename T> void launch_norm(const LaunchCtx&, Grid g, Vec<T> f, RhsNorms* norms);

// FP32-in-FP64 refinement: r = f - A_s x in FP64, stored as complex64, norm
// into norms[b].r2. With z0.p set (the level-0 Arnoldi planes of the FP32
// cycle), r also becomes that cycle's first residual z_0 (its iterate starting
// at zero) with the partial sums of ||z_0||^2 in region 0, and the norm's
// partials use region 1. Returns the number of partial sums per right-hand side.
// With w0.p set as well (and refine_apply_fits), the pass also applies the
// cycle's FP32 operator (k^2 in k2_32) to z_0 into w0 and hands the cycle's
// first GMRES step ||z_0||^2 and <z_0, w_0> in region 1 (three per block),
// the norm's partials then using region 0; that step (w_ready) starts with
// its first orthogonalise pass.
int launch_refine_residual(const LaunchCtx&, const LevelOp<double>&, Vec<double> x, Vec<double> f, Vec<float> r32,
                           RhsNorms* norms, Vec<float> z0 = Vec<float>{nullptr, 0}, const float* k2_32 = nullptr,
                           Vec<float> w0 = Vec<float>{nullptr, 0});
// x_out = x_in + e (e complex64), then r = f - A_s x_out as above.
int launch_correct_residual(const LaunchCtx&, const LevelOp<double>&, Vec<double> x_in, Vec<float> e,
                            Vec<double> x_out, Vec<double> f, Vec<float> r32, RhsNorms* norms,
                            Vec<float> z0 = Vec<float>{nullptr, 0}, const float* k2_32 = nullptr,
                            Vec<float> w0 = Vec<float>{nullptr, 0});
// Whether the fused refinement residual + apply pass fits its LDS stages on grid g.
bool refine_apply_fits(const LaunchCtx&, Grid g);

// Layout conversion between the caller's dense [b][n+1][n+1] arrays and the
// padded planes. src_is_f32 / dst_is_f32 select complex64 on the caller side.
// scale_w multiplies by W (rhs -> f_s); conj conjugates.
template <typename T>
void launch_copy_in(const LaunchCtx&, Grid g, const void* src, bool src_is_f32, Vec<T> dst, bool scale_w,
                    bool conj);
template <typename T>
void launch_copy_out(const LaunchCtx&, Grid g, Vec<T> src, void* dst, bool dst_is_f32, bool scale_w, bool conj);
template <typename T> void launch_zero(hipStream_t, cplx<T>* p, long long count);
// Fills `bytes` (a multiple of 4) with a 32-bit pattern.
void launch_fill_words(hipStream_t, void* p, long long bytes, unsigned value);

// Adjoint gradient: g_p = sum_b Re[mu_b,p W_p (1 + i s_p / (h k_p)) u_b,p], mu = conj(lambda).
void launch_grad_k2(const LaunchCtx&, Grid g, double h, const double* k2, Vec<double> u, Vec<double> mu,
                    double* grad_k2_dense);

// Coarse tail: the whole sub-cycle on levels l0 .. L-1 (at most kMaxTailLevels)
// in one launch, one workgroup per right-hand side, every vector of those
// levels in LDS. Level q of the tail (q = 0: level l0) holds tail_planes(q)
// planes of tail_pitch(n_q)^2 values: u and f, plus five scratch planes on
// every level that is smoothed (all but the coarsest). Planes carry a zero
// frame of kTailGhost nodes.
constexpr int kMaxTailLevels = 8;
constexpr int kTailGhost = 3;
constexpr int kTailMaxCoarseNodes = 81;              // coarsest (n_c + 1)^2 solved by the explicit inverse
constexpr long long kTailMaxLdsBytes = 156 * 1024;   // dynamic LDS of one tail workgroup
__host__ __device__ inline int tail_pitch(int n) { return n + 1 + 2 * kTailGhost; }
__host__ __device__ inline int tail_planes(int q, int nlev) { return q + 1 < nlev ? 7 : 2; }
__host__ __device__ inline long long tail_plane_values(int n, int q, int nlev) {
    const long long p = tail_pitch(n);
    return tail_planes(q, nlev) * p * p;
}
template <typename T>
struct TailLevel {
    Grid g;
    int radius;
    const cplx<T>* coef;
};
template <typename T>
struct TailArgs {
    int nlev;
    long long lds_bytes;    // total dynamic LDS: the planes, then the inverse when it is staged
    long long plane_bytes;  // sum of tail_plane_values over the levels, in bytes
    long long inv_off;      // byte offset of the LDS copy of inv, or -1 (read from global memory)
    TailLevel<T> lv[kMaxTailLevels];
    cplx<T>* u_top;         // level l0 iterate (read unless top_zero, then overwritten), right-hand side 0; stride g.plane
    const cplx<T>* f_top;   // level l0 right-hand side
    const cplx<double>* inv;  // explicit inverse of the coarsest operator [N][N] (FP64)
    int gamma, smoother, nu1, nu2;  // smoother: 0 Jacobi, 1 GMRES(3)
    double omega, breakdown;
    int bez;
    int top_zero;  // the level l0 iterate holds zeros (its first visit, entered by restriction)
};
template <typename T> void launch_tail(const LaunchCtx&, const TailArgs<T>&);
// Raises the dynamic-LDS limit of the tail kernels (once per process; call
// before the first launch, outside stream capture).
void tail_init();
// inv = A^{-1} from the LU factor and pivots of launch_dense_lu, N <= kTailMaxCoarseNodes.
void launch_lu_inverse(hipStream_t, int N, const cplx<double>* lu, const int* piv, cplx<double>* inv);

// ---- outer flexible GMRES (level-0 FP64 vectors, [j][b][plane]) ----
constexpr int kMaxRestart = 64;  // longest restart cycle m
// w is orthogonalised against V_0..V_j by classical Gram-Schmidt (all h_i =
// <V_i, w> from the incoming w, then w -= sum h_i V_i); H[b * hstride + i]
// receives column j (i = 0..j) and the subdiagonal ||w|| (i = j + 1);
// V_{j+1} = w / ||w||, and its complex64 copy into v32 when v32 is not null.
// z32 (may be null; 4 planes per right-hand side): the complex64 copy is also
// written to z32's first plane, with its partial sums of ||.||^2 in reduction
// region 0 (as many blocks as launch_kry_first returns), the first residual
// of an FP32 cycle from u = 0 on v32 (cycle's r_ready_nblk and u_zero).
void launch_kry_orthogonalise(const LaunchCtx&, Grid g, cplx<double>* V, long long vstride, int j,
                              cplx<double>* w, cplx<double>* H, int hstride, long long plane, cplx<float>* v32,
                              cplx<float>* z32 = nullptr);
// v = r / ||r|| with ||r||^2 from norms[b].r2 (and its complex64 copy into v32,
// and z32, as above). Returns the partial-sum count of the z32 copies.
int launch_kry_first(const LaunchCtx&, Grid g, const cplx<double>* r, cplx<double>* v, long long plane,
                     const RhsNorms* norms, cplx<float>* v32, cplx<float>* z32 = nullptr);
// x += sum_{i < nz} y[b * ystride + i] Z_i.
void launch_kry_update(const LaunchCtx&, Grid g, const cplx<double>* Z, long long zstride, int nz,
                       const cplx<double>* y, int ystride, cplx<double>* x, long long plane);

// ---- setup ----
// Validity of the caller's dense k^2 array (n+1)^2: flags[0] |= 1 (non-finite),
// 2 (negative), 4 (zero on the boundary); flags[1] = min offending index.
// The caller sets flags to {0, INT_MAX} first.
void launch_check_k2(hipStream_t, int n, const double* k2_dense, int* flags);
// Padded k^2 planes from the caller's dense array (FP64 and optionally FP32).
void launch_k2_in(hipStream_t, Grid g, const double* k2_dense, double* k2_64, float* k2_32);
// Galerkin product of level l (fine) into level l+1 (coarse) in FP64.
// Level 0 uses the shifted Laplacian built from k^2 (shift applied here only).
void launch_galerkin(hipStream_t, int fine_level, Grid fine, int fine_radius, const cplx<double>* fine_coef,
                     const double* k2_64, double h, double shift, int transfer, Grid coarse, int coarse_radius,
                     cplx<double>* coarse_coef);
void launch_cast_coef(hipStream_t, const cplx<double>* src, cplx<float>* dst, long long count);
// Dense coarsest matrix [N][N] (N = (n_c+1)^2) from stencil planes, then LU with partial pivoting.
void launch_dense_lu(hipStream_t, Grid g, int radius, const cplx<double>* coef, cplx<double>* dense, int* piv);
// u = A^{-1} f on the coarsest grid with the stored LU (FP64 arithmetic).
template <typename T>
void launch_coarse_solve(const LaunchCtx&, Grid g, const cplx<double>* lu, const int* piv, Vec<T> f, Vec<T> u);
// Stencil planes -> caller's dense [(2r+1)^2][n_l+1][n_l+1] complex128.
void launch_stencil_out(hipStream_t, Grid g, int radius, const cplx<double>* coef, void* out);

}  // namespace hm
