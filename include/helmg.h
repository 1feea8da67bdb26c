/*
 * helmg.h -- C ABI of the MI355X multigrid solver for the 2D Helmholtz equation.
 *
 * Method: Dwarka & Vuik, "Stand-alone multigrid for Helmholtz revisited:
 * towards convergence using standard components" (arXiv 2308.13476).
 *
 * Problem (§2, MP 2-A / MP 2-B): -Laplace(u) - k(x,y)^2 u = f on the unit
 * square with the absorbing condition du/dn - i k u = 0 on the whole
 * boundary, second-order finite differences on a vertex grid with n
 * intervals per side, h = 1/n, (n+1)^2 unknowns (boundary nodes included;
 * the ghost node of the boundary condition is eliminated by a central
 * difference). Rows are scaled by W = w_i w_j (w = 1/2 on the end nodes of a
 * grid line) so that the operator A_s = W A is complex symmetric; the solver
 * works on A_s u = W f.
 *
 * Method (§3-§5): Galerkin coarse operators A_1 = R C P, A_{l+1} = R A_l P
 * with C the complex shifted Laplacian -Laplace - (1 + i beta2) k^2 (§4,
 * Table 1; beta2 of §5), the higher-order (Bézier) prolongation of §4 or
 * linear interpolation, R = P^T / 4, weighted Jacobi u += (omega D)^{-1} r
 * (§3; damping 1/omega) or GMRES(3) smoothing (§5.3), V- or W-cycles (§5),
 * a direct LU solve on the coarsest grid, and a relative-residual stop test.
 *
 * Conventions for every entry point:
 *  - Pointers marked [dev] are device pointers owned by the caller; the
 *    library never allocates device memory: all of its device state lives in
 *    the caller's workspace (a handle also holds a few small pinned host
 *    arrays and two events, freed by mg_destroy). [host] pointers are
 *    ordinary host memory.
 *  - Grid functions are row-major [batch][n+1][n+1] with x (index i) fastest,
 *    node (i, j) at x = i h, y = j h. Complex values are interleaved
 *    (re, im): complex128 = 2 doubles, complex64 = 2 floats.
 *  - All work is enqueued on the caller's HIP stream (NULL = default stream).
 *    mg_solve / mg_grad take the stop test on the device after every cycle
 *    and synchronise with that stream once per cycle to read its result, with
 *    up to one further cycle already enqueued (it skips right-hand sides that
 *    have stopped). A handle must not be used from two threads at once.
 *  - Functions return an mg_status and never abort; argument checks happen
 *    before any HIP call. The detail of the last error is in mg_last_error().
 */
#ifndef HELMG_H
#define HELMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx* mg_handle;

typedef enum {
    MG_OK = 0,
    MG_NOT_CONVERGED = 1, /* warning: max_cycles reached, outputs valid          */
    MG_E_ARG = -1,        /* invalid argument; nothing was enqueued               */
    MG_E_HIP = -2,        /* HIP runtime error; see mg_last_error                 */
    MG_E_DIVERGED = -3,   /* residual non-finite or grew past the divergence cap */
    MG_E_WORKSPACE = -4,  /* workspace too small or misaligned                    */
    MG_E_STATE = -5       /* handle not set up for the request (e.g. FP32 copies) */
} mg_status;

enum { MG_TRANSFER_BEZIER = 0, MG_TRANSFER_LINEAR = 1 };   /* §4, Table 1            */
enum { MG_V = 1, MG_W = 2 };                              /* cycle index gamma (§5) */
enum { MG_JACOBI = 0, MG_GMRES3 = 1 };                    /* smoothers (§3, §5.3)   */
enum { MG_FP64 = 0, MG_FP32_REFINED = 1 };                /* solve precision        */

typedef struct {
    int precision;   /* MG_FP32_REFINED also builds complex64 copies of the hierarchy */
    int max_batch;   /* largest nrhs / nsrc used with this handle (>= 1)              */
    int coarsest_n;  /* intervals per side of the coarsest grid when levels = 0 (4)   */
    int use_graph;   /* 0 or 1: cycles are captured as HIP graphs and replayed (the
                        default); -1: kernels are launched one by one             */
    const char* tune_cache; /* NULL, or a JSON file of autotuned launch settings:
                        mg_tune takes its settings from a matching entry there
                        instead of timing, and records new ones (the path is
                        copied; the file is rewritten whole, so concurrent
                        writers may lose entries)                                */
} mg_setup_opts;

typedef struct {
    int nu_pre;        /* pre-smoothing steps (>= 0)                                   */
    int nu_post;       /* post-smoothing steps (>= 0)                                  */
    double omega;      /* Jacobi parameter of §3: damping factor is 1/omega (4.5)      */
    int max_cycles;    /* cycle cap (>= 1)                                             */
    int precision;     /* MG_FP64 or MG_FP32_REFINED                                   */
    double divergence; /* stop as diverged when relres > divergence * initial relres  */
} mg_solve_opts;

typedef struct {
    int* cycles;         /* [host] nrhs entries or NULL: cycles run per right-hand side */
    double* relres;      /* [host] nrhs entries or NULL: final relative residuals       */
    double* history;     /* [host] history_len entries or NULL: relres after every
                            cycle, entry [it * nrhs + b] for cycle it + 1 of b       */
    int history_len;     /* entries of history; with history set it must be at least
                            opts->max_cycles * nrhs, else the call returns MG_E_ARG  */
    double seconds;      /* wall time of the call (host clock, stream synchronised)     */
} mg_solve_stats;

/* Bytes of device workspace needed for a grid of n intervals (n = c 2^(L-1)),
 * `levels` levels (0 = coarsen to opts.coarsest_n), opts.max_batch right-hand
 * sides and opts.precision. Returns 0 for invalid arguments. */
size_t mg_workspace_bytes(int n, int levels, int transfer, const mg_setup_opts* opts);

/* Builds the multigrid hierarchy (§3, §4) on the device.
 *  k2        [dev] double, (n+1)^2 values of k(x,y)^2: finite, >= 0, and > 0 on
 *            the boundary nodes (the absorbing condition of §2 uses k there).
 *            The field is checked on the device before anything is built (the
 *            only argument check that needs the GPU): MG_E_ARG, with the first
 *            offending node in mg_last_error, if any value violates this.
 *  n         intervals per side (>= 4, divisible by 2^(levels-1)).
 *  h         mesh width (> 0; 1/n for the unit square).
 *  shift     beta2 >= 0, the complex shift of the coarsening operator (§4, §5).
 *  levels    number of levels (>= 2) or 0 for automatic.
 *  transfer  MG_TRANSFER_BEZIER (§4) or MG_TRANSFER_LINEAR.
 *  opts      may be NULL (FP64 only, max_batch 1, coarsest_n 4).
 *  workspace [dev] at least mg_workspace_bytes(...) bytes, 256-byte aligned; it
 *            must stay allocated and untouched until mg_destroy.
 *  stream    hipStream_t or NULL.
 *  out       [host] receives the handle. The k2 array is copied; it may be
 *            freed after the call returns. */
mg_status mg_setup(const double* k2, int n, double h, double shift, int levels, int transfer,
                   const mg_setup_opts* opts, void* workspace, size_t ws_bytes, void* stream,
                   mg_handle* out);

/* Rebuilds the hierarchy for a new k^2 field on the same grid (same workspace).
 * The field is checked as in mg_setup first; on MG_E_ARG the handle keeps its
 * previous hierarchy. Returns once k2 has been copied (it may then be freed);
 * the rebuild itself is enqueued on stream, ahead of the caller's later work
 * there (work on other streams must wait for this stream). */
mg_status mg_update_k2(mg_handle h, const double* k2, void* stream);

/* Solves A_s x = W rhs for nrhs right-hand sides sharing the operator (§5).
 *  rhs   [dev] complex128 [nrhs][n+1][n+1], the PDE right-hand side f
 *        (e.g. 1/h^2 at a point source).
 *  x     [dev] complex128 [nrhs][n+1][n+1]: initial guess in, solution out.
 *  tol   relative residual target ||W f - A_s x|| / ||W f|| (> 0).
 *  cycle MG_V or MG_W; smoother MG_JACOBI or MG_GMRES3.
 *  opts  may be NULL (nu 1/1, omega 4.5, max_cycles 500, FP64, divergence 1e8).
 *  stats may be NULL.
 * Each right-hand side stops at its own first cycle with relres <= tol (its
 * later cycles are skipped). Returns MG_OK, MG_NOT_CONVERGED (x holds the
 * last iterates), or MG_E_DIVERGED (x holds the last iterates). */
mg_status mg_solve(mg_handle h, const void* rhs, void* x, int nrhs, double tol, int cycle, int smoother,
                   const mg_solve_opts* opts, mg_solve_stats* stats, void* stream);

/* Mixed-size batch: several independent problems, each with its own handle
 * (any n, k^2 field, shift, levels; set up separately with mg_setup), solved
 * together. Every cycle of the problems still running is launched as one
 * HIP graph with one branch per problem, so the level kernels of different
 * problems run concurrently and one stream synchronisation per cycle serves
 * all of them (batching of the cycle in §5 across problems; not in the paper).
 *  handles[p]  distinct handles, p < nprob.
 *  rhs[p], x[p], nrhs[p]  as rhs, x, nrhs of mg_solve for problem p.
 *  stats       NULL or an array of nprob mg_solve_stats, each as in mg_solve.
 *  tol, cycle, smoother, opts as in mg_solve, shared by all problems.
 * Each problem stops like mg_solve; the result is that of mg_solve for each
 * problem alone, bit for bit. Returns the worst status over the problems
 * (an error, else MG_E_DIVERGED, else MG_NOT_CONVERGED, else MG_OK); the
 * detail is in mg_last_error of the first failing handle, or of NULL for an
 * argument error that names no handle. */
mg_status mg_solve_multi(mg_handle* handles, int nprob, const void* const* rhs, void* const* x, const int* nrhs,
                         double tol, int cycle, int smoother, const mg_solve_opts* opts, mg_solve_stats* stats,
                         void* stream);

/* Launch settings chosen by mg_tune. */
typedef struct {
    int block_cap;       /* blocks per right-hand side a level grid aims at     */
    int tail_n;          /* levels of at most this many intervals run in the
                            single-workgroup LDS tail (0: none)                 */
    int level1_product;  /* level 1 as R C_s P: 0 never, 1 in FP32 cycles, 2 both */
    double ms_per_cycle; /* measured time of one cycle with these settings      */
    int candidates;      /* settings timed (0 when taken from the cache)        */
    int tall_rows;       /* tile shape: block height (wavefronts) of light
                            kernels on grids of >= 256 intervals (4 or 8)       */
    int small_rows;      /* block height on grids of <= 128 intervals (2 or 4)  */
    int from_cache;      /* 1 when the settings came from the tuning cache      */
} mg_tune_result;

/* Autotuner (a launch-setting search; the method is unchanged): times three
 * captured cycles of the given problem (rhs [dev] complex128 [nrhs][n+1][n+1]
 * as in mg_solve, zero initial guess) for each combination of block cap
 * ({320, 640, 1280} blocks per right-hand side on handles with max_batch 1,
 * {64, 160, 320, 640} on batch handles), tail size {0, 16, 32}, level-1 operator {stored,
 * product} and tile shape (block heights {4, 8} on grids of >= 256 intervals
 * and {2, 4} on grids of <= 128), keeps the fastest on the handle for later
 * solves and reports it in *out (may be NULL). With a tune_cache file (see
 * mg_setup_opts) a matching entry (same grid, levels, transfer, nrhs, cycle,
 * smoother, nu, precision and GPU architecture) is applied without timing,
 * and a new result is added to the file. Overwrites the handle's iterates;
 * results of later solves are those of the chosen settings (equal to any
 * other setting up to rounding). MG_E_STATE while the timing hook is on;
 * MG_E_ARG if the cache file cannot be written. */
mg_status mg_tune(mg_handle h, const void* rhs, int nrhs, int cycle, int smoother, const mg_solve_opts* opts,
                  mg_tune_result* out, void* stream);

/* Outer Krylov solver with the multigrid cycle as preconditioner (§1: multigrid
 * on the CSL used as a preconditioner for GMRES). Restarted flexible GMRES(m)
 * in FP64 on A_s x = W f with right preconditioning: every direction is
 * z_j = one cycle (cycle, smoother, opts->nu_pre / nu_post / omega) on
 * A_s z = v_j from z = 0, an FP64 cycle, or the FP32 cycle when
 * opts->precision is MG_FP32_REFINED; classical Gram-Schmidt Arnoldi (all
 * inner products of a column from one sweep over A_s z_j, then one update
 * sweep; the oracle's modified Gram-Schmidt gives the same column up to
 * rounding); the
 * least-squares problem by Givens rotations on the host, which reads each
 * Hessenberg column while the next iteration already runs (so a solve that
 * stops inside a restart cycle computes one iteration it does not use). The
 * first call on a handle allocates a small pinned host buffer for the
 * columns (up to 2 * max_batch * 65 complex values), kept until mg_destroy;
 * MG_E_HIP if that fails.
 *  rhs, x, nrhs as in mg_solve; m restart length in [1, 64].
 *  krylov [dev] caller's buffer of at least mg_fgmres_workspace_bytes(h, m)
 *         bytes, 256-byte aligned (basis V, directions Z, x, f, w, H, y);
 *         zeroed and overwritten by every call, no contents need survive.
 *  stats->cycles: iterations (= preconditioner cycles); relres: true
 *         relative residual of the returned x; history[it * nrhs + b]: the
 *         iteration's residual estimate (NaN after a right-hand side stopped).
 * A right-hand side stops when the estimate reaches tol (at the end of that
 * restart cycle's update) or after opts->max_cycles iterations. Returns
 * MG_OK, MG_NOT_CONVERGED (x holds the last iterates), MG_E_WORKSPACE, or
 * the errors of mg_solve. */
size_t mg_fgmres_workspace_bytes(mg_handle h, int m);
mg_status mg_solve_fgmres(mg_handle h, const void* rhs, void* x, int nrhs, double tol, int m, int cycle,
                          int smoother, const mg_solve_opts* opts, void* krylov, size_t krylov_bytes,
                          mg_solve_stats* stats, void* stream);

/* Adjoint-state gradient for a real loss L(u) of solutions u = A_s^{-1} W f.
 *  u       [dev] complex128 [nsrc][n+1][n+1], forward solutions.
 *  grad_u  [dev] complex128 [nsrc][n+1][n+1], dL/du in PyTorch's convention
 *          (the conjugate Wirtinger derivative times two), e.g. S^T (S u - d)
 *          for L = 1/2 ||S u - d||^2.
 *  grad_k2 [dev] double [n+1][n+1], out: dL/dk^2 summed over sources.
 *  grad_rhs [dev] complex128 [nsrc][n+1][n+1] or NULL, out: dL/df = W lambda.
 * lambda solves A_s^H lambda = grad_u with the same multigrid (A_s^H =
 * conj(A_s)), run on conjugated data; then
 * dL/dk^2_p = sum_src Re[conj(lambda_p) W_p (1 + i s_p / (h k_p)) u_p],
 * s_p = number of boundary sides of node p. */
mg_status mg_grad(mg_handle h, const void* u, const void* grad_u, int nsrc, double tol, int cycle,
                  int smoother, const mg_solve_opts* opts, double* grad_k2, void* grad_rhs,
                  mg_solve_stats* stats, void* stream);

/* Releases the host state of the handle (the workspace is the caller's). */
mg_status mg_destroy(mg_handle h);

const char* mg_status_string(mg_status s);
/* Detail of the last error on this handle (or of the last failed mg_setup when h is NULL). */
const char* mg_last_error(mg_handle h);

/* ---- Level operations: single steps of the cycle, for testing and for
 * callers that compose their own iteration (e.g. MG as a preconditioner).
 * Vectors use the layout above on the level's own grid of n_l = n / 2^l
 * intervals; precision MG_FP64 means complex128 data and FP64 operators,
 * MG_FP32_REFINED means complex64 data and the FP32 operator copies. ---- */

/* Level count, and for level l its intervals per side and stencil radius
 * (1 on level 0; 2 or 3 for Galerkin levels with Bézier transfer). */
mg_status mg_level_info(mg_handle h, int level, int* n_l, int* radius, int* levels);

/* Copies the Galerkin stencil of level l >= 1 (§3) to out [dev] complex128
 * [(2r+1)^2][n_l+1][n_l+1]: entry [(dy+r)(2r+1) + (dx+r)][j][i] is the
 * coefficient of A_l coupling node (i,j) to node (i+dx, j+dy). */
mg_status mg_get_stencil(mg_handle h, int level, void* out, void* stream);

/* y = A_l x for nvec vectors (level 0 is the scaled fine operator A_s). */
mg_status mg_apply(mg_handle h, int level, const void* x, void* y, int nvec, int precision, void* stream);

/* r = f - A_l x. */
mg_status mg_residual(mg_handle h, int level, const void* x, const void* f, void* r, int nvec, int precision,
                      void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid allocation): the same r = f - A_l x as
 * mg_residual, bit for bit, but x, f and r are staged through a static device
 * scratch array of the library (64 MiB per GPU, held from the first mg_setup
 * on a device until the process ends) instead of the handle's level buffers,
 * which stay untouched. It calls no allocating routine, copies nothing through
 * the host and does not synchronise: the kernels are enqueued on stream and r
 * is ready when the stream reaches them. 3 * nvec padded planes of the level
 * (about 3 * nvec * 18 MB for complex128 at n = 1024) must fit the 64 MiB,
 * else MG_E_ARG; nvec need not respect max_batch. The handle's device must be
 * current. Every call on one GPU shares its scratch: calls that overlap on
 * that GPU (other streams, other threads, other handles) race and must be
 * ordered by the caller. */
mg_status mg_residual_noalloc(mg_handle h, int level, const void* x, const void* f, void* r, int nvec,
                              int precision, void* stream);

/* nsteps smoothing steps on A_l u = f in place: MG_JACOBI with parameter omega
 * (§3) or MG_GMRES3 (§5.3, omega ignored). */
mg_status mg_smooth(mg_handle h, int level, int smoother, int nsteps, double omega, void* u, const void* f,
                    int nvec, int precision, void* stream);

/* coarse = R fine (level l -> l+1), R = P^T / 4 (§4). */
mg_status mg_restrict(mg_handle h, int level, const void* fine, void* coarse, int nvec, int precision,
                      void* stream);

/* fine += P coarse (level l+1 -> l), the prolongation of §4. */
mg_status mg_prolong_add(mg_handle h, int level, const void* coarse, void* fine, int nvec, int precision,
                         void* stream);

/* u = A_{L-1}^{-1} f on the coarsest level (FP64 LU; complex64 data is widened). */
mg_status mg_coarse_solve(mg_handle h, const void* f, void* u, int nvec, int precision, void* stream);

/* One cycle on level 0 for A_s u = f_s: u [dev] in/out, f_s [dev] the already
 * scaled right-hand side W f, both [nvec][n+1][n+1]. complex128 data and an
 * FP64 cycle, or, when opts->precision is MG_FP32_REFINED, complex64 data and
 * the FP32 cycle that the refined solve runs (MG_E_ARG if the setup holds no
 * FP32 data). */
mg_status mg_cycle(mg_handle h, void* u, const void* f_s, int nvec, int cycle, int smoother,
                   const mg_solve_opts* opts, void* stream);

/* ---- Timing hook: HIP events around every launch of one kernel class on
 * the solve stream, accumulated until read. kernel_class: 0 off, 1 level-0
 * GMRES Arnoldi apply pass, 2 level-0 Jacobi sweep, 3 level-0 residual +
 * restriction, 4 level-1 stencil apply pass. While a class is set, cycles are
 * launched kernel by kernel instead of as captured HIP graphs. ---- */
mg_status mg_set_timing(mg_handle h, int kernel_class);
mg_status mg_get_timing(mg_handle h, int* launches, double* total_ms, double* nodes_per_launch);

#ifdef __cplusplus
}
#endif
#endif /* HELMG_H */
