// Level kernels of the multigrid cycle: operator apply, residual, weighted
// Jacobi, transfers, GMRES(3) passes, norms, FP32 refinement, adjoint gradient.
#include <cstdlib>
#include <type_traits>
#include <utility>

#include <hip/hip_ext.h>

#include "hm_ops.hpp"

namespace hm {
namespace {

constexpr int kThreads = kBX * kBY;

// Block height: 64 x 4 for register-heavy Galerkin stencils; light kernels
// on grids of 256 or more intervals use ctx.tall_rows rows (4, 8 or 16), and
// grids of at most 128 intervals ctx.small_rows (2 or 4): their passes are
// latency-bound, and two wavefronts per block shorten each block's
// reductions and spread a pass over twice the compute units. Tiles keep an
// even first row, which the staging of the coarse grid correction relies on
// (it takes coarse row r0 / 2 as its reference). The handle's settings come
// from the environment at set-up or from the autotuner.
int block_rows(const Grid& g, bool heavy, const LaunchCtx& ctx) {
    if (g.n <= 128) return ctx.small_rows == 4 ? kBY : 2;
    if (heavy || g.n < 256) return kBY;
    return (ctx.tall_rows == 8 || ctx.tall_rows == 16) ? ctx.tall_rows : kBY;
}

// Rows per thread: enough that a level grid has at most `cap` blocks (the
// block cap of the context: every consumer of a reduction reads all partial
// sums of its producer, so more blocks cost more of those reads).
int level_rpt(const Grid& g, int by, int cap) {
    const long long m = g.n + 1;
    const long long bx = (m + kBX - 1) / kBX;
    const long long r = (m * bx + (long long)by * cap - 1) / ((long long)by * cap);
    return int(r < 1 ? 1 : r);
}

// Grid of a level launch. pad8 (handles for batches): the row-block count is
// raised until the tiles of one right-hand side are a multiple of 8, so that
// tile t of every right-hand side is dispatched to the same XCD (workgroups
// go to the eight XCDs round-robin by linear id) and the operator data all
// right-hand sides share (stencil coefficient planes, k^2) is fetched once
// into that XCD's L2 instead of once per right-hand side. The extra tiles lie
// below the grid: their blocks touch no node and write zero partial sums.
dim3 level_grid(const Grid& g, int rpt, int nrhs, int by, bool pad8 = false) {
    const unsigned gx = (g.n + 1 + kBX - 1) / kBX;
    unsigned gy = (g.n + 1 + by * rpt - 1) / (by * rpt);
    if (pad8)
        while ((gx * gy) % 8 != 0) ++gy;
    return dim3(gx, gy, nrhs);
}

struct Geom {
    int by, rpt, nblk;
    dim3 grid, block;
};

Geom geom(const Grid& g, bool heavy, const LaunchCtx& ctx) {
    Geom q;
    q.by = block_rows(g, heavy, ctx);
    q.rpt = level_rpt(g, q.by, ctx.block_cap);
    q.grid = level_grid(g, q.rpt, ctx.nrhs, q.by, ctx.nrhs_cap > 1);
    q.block = dim3(kBX, q.by);
    q.nblk = int(q.grid.x * q.grid.y);
    return q;
}

// Geometry of an operator kernel: the level geometry with rows per thread
// lowered until the block's LDS stages fit kMaxTileBytes.
constexpr size_t kMaxTileBytes = 64 * 1024;
template <typename Op, typename T>
__host__ __device__ size_t tile_bytes(int by, int rpt);
template <typename Op, typename T>
Geom geom_op(const Grid& g, const LaunchCtx& ctx) {
    Geom q = geom(g, Op::kHeavy, ctx);
    if (tile_bytes<Op, T>(q.by, q.rpt) > kMaxTileBytes) {
        while (q.rpt > 1 && tile_bytes<Op, T>(q.by, q.rpt) > kMaxTileBytes) --q.rpt;
        q.grid = level_grid(g, q.rpt, ctx.nrhs, q.by, ctx.nrhs_cap > 1);
        q.nblk = int(q.grid.x * q.grid.y);
    }
    return q;
}

// Calls f(integral_constant<int, BY>) for the runtime block height; kernels
// of register-heavy operators are only instantiated with short blocks.
template <bool kHeavy = false, typename F>
void with_by(int by, F&& f) {
    if (by == 2) {
        f(std::integral_constant<int, 2>{});
        return;
    }
    if constexpr (kHeavy) {
        f(std::integral_constant<int, kBY>{});
    } else {
        if (by == 16) f(std::integral_constant<int, 16>{});
        else if (by == 8) f(std::integral_constant<int, 8>{});
        else f(std::integral_constant<int, kBY>{});
    }
}

// Calls f(op) with the concrete operator type of the level.
template <typename T, typename F>
void with_op(const LevelOp<T>& lop, F&& f) {
    if (lop.level == 0) {
        f(FineOp<T>{lop.g, lop.k2, T(1.0 / (lop.h * lop.h)), T(2.0 / lop.h)});
        return;
    }
    if (lop.level == 1 && lop.product) {
        const FineOp<T> fine{lop.g0, lop.k2, T(1.0 / (lop.h * lop.h)), T(2.0 / lop.h)};
        const int D = 2 * lop.radius + 1;
        const cplx<T>* diagc = lop.coef + (long long)(lop.radius * D + lop.radius) * lop.g.plane;
        if (lop.transfer == 0) f(ProductOp<T, true>{lop.g, fine, T(lop.shift), diagc});
        else f(ProductOp<T, false>{lop.g, fine, T(lop.shift), diagc});
        return;
    }
    switch (lop.radius) {
        case 1: f(StencilOp<T, 1>{lop.g, lop.coef}); break;
        case 2: f(StencilOp<T, 2>{lop.g, lop.coef}); break;
        default: f(StencilOp<T, 3>{lop.g, lop.coef}); break;
    }
}

template <typename T>
__device__ __forceinline__ double dnorm2(cplx<T> z) {
    return double(z.re) * double(z.re) + double(z.im) * double(z.im);
}

// Stages 2-4 of a ProductOp apply, after the coarse tile (halo 3) is in LDS:
// y = P x and v = C_s y on the block's fine region, then the restriction of v
// at each coarse node, handed to f(i, j, p, pget(p), x at p, A_1 x at p).
template <typename T, bool kBez, typename PGet, typename F>
__device__ __forceinline__ void product_stages(const ProductOp<T, kBez>& op, const Tile<3>& tl, cplx<T>* lds,
                                               PGet&& pget, F&& f) {
    using PS = ProductStages<T>;
    if (tl.r0 > op.g.n) return;  // padding tile of a batch grid: no coarse node
    const int rows = tl.rows;
    cplx<T>* y = lds + Tile<3>::TW * (rows + 6);
    cplx<T>* v = y + PS::YW * PS::yrows(rows);
    const int nt = blockDim.x * blockDim.y;
    const int tid = threadIdx.y * kBX + threadIdx.x;
    const int nf = op.fine.g.n;
    const int fx0 = 2 * tl.c0 - 3, fy0 = 2 * tl.r0 - 3;  // fine origin of y
    // y = P x: even fine index 2K takes (1/8, 3/4, 1/8) of K-1, K, K+1 (Bezier)
    // or x_K (linear); odd 2K+1 takes (x_K + x_{K+1}) / 2. Zero off the fine
    // grid. One step forms the 2 x 2 fine nodes 2K + {0, 1}, 2L + {0, 1} from
    // the 3 x 3 coarse values around (K, L), rows first. K = c0 - 2 .. c0 + 64
    // and L = r0 - 2 .. r0 + rows cover y; the fine column and row 2 c0 - 4,
    // 2 r0 - 4 of the first steps lie outside it and are dropped.
    constexpr int PX = kBX + 3;
    const int np = PX * (rows + 3);
    const int ny = PS::yrows(rows);
    auto put = [&](int fi, int fj, cplx<T> val) {
        const int a = fi - fx0, bq = fj - fy0;
        if (a < 0 || bq < 0 || a >= PS::YW || bq >= ny) return;
        const bool in = fi >= 0 && fj >= 0 && fi <= nf && fj <= nf;
        y[bq * PS::YW + a] = in ? val : cplx<T>{T(0), T(0)};
    };
    for (int q = tid; q < np; q += nt) {
        const int K = tl.c0 - 2 + q % PX, L = tl.r0 - 2 + q / PX;
        const int base = tl.at(K - 1, L - 1);
        cplx<T> he[3], ho[3];  // rows L - 1 .. L + 1 at fine columns 2K, 2K + 1
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const cplx<T> xa = lds[base + t * Tile<3>::TW];
            const cplx<T> xb = lds[base + t * Tile<3>::TW + 1];
            const cplx<T> xc = lds[base + t * Tile<3>::TW + 2];
            if (kBez) {
                he[t].re = T(0.125) * xa.re + T(0.75) * xb.re + T(0.125) * xc.re;
                he[t].im = T(0.125) * xa.im + T(0.75) * xb.im + T(0.125) * xc.im;
            } else {
                he[t] = xb;
            }
            ho[t].re = T(0.5) * (xb.re + xc.re);
            ho[t].im = T(0.5) * (xb.im + xc.im);
        }
        cplx<T> e0, o0;  // fine row 2L
        if (kBez) {
            e0.re = T(0.125) * he[0].re + T(0.75) * he[1].re + T(0.125) * he[2].re;
            e0.im = T(0.125) * he[0].im + T(0.75) * he[1].im + T(0.125) * he[2].im;
            o0.re = T(0.125) * ho[0].re + T(0.75) * ho[1].re + T(0.125) * ho[2].re;
            o0.im = T(0.125) * ho[0].im + T(0.75) * ho[1].im + T(0.125) * ho[2].im;
        } else {
            e0 = he[1];
            o0 = ho[1];
        }
        put(2 * K, 2 * L, e0);
        put(2 * K + 1, 2 * L, o0);
        put(2 * K, 2 * L + 1, cplx<T>{T(0.5) * (he[1].re + he[2].re), T(0.5) * (he[1].im + he[2].im)});
        put(2 * K + 1, 2 * L + 1, cplx<T>{T(0.5) * (ho[1].re + ho[2].re), T(0.5) * (ho[1].im + ho[2].im)});
    }
    __syncthreads();
    // v = C_s y = A_s y - i beta2 W k^2 y on fine nodes of the grid, zero
    // elsewhere. One step takes the 2 x 2 fine nodes 2K + {0, 1}, 2L + {0, 1}
    // with their 12 distinct y neighbours, K = c0 - 1 .. c0 + 64 and
    // L = r0 - 1 .. r0 + rows; the last fine column and row of these steps lie
    // outside v and are dropped (their neighbours beyond y are read clamped).
    // k^2 of kVBlocks steps is loaded before their arithmetic (nodes off the
    // fine grid read a clamped in-grid node and give zero).
    constexpr int VX = kBX + 2;
    constexpr int kVBlocks = 2;
    const int nvb = VX * (rows + 2);
    T kk[kVBlocks][4];
    auto yat = [&](int c, int r) { return y[min(r, ny - 1) * PS::YW + min(c, PS::YW - 1)]; };
    auto cs_node = [&](int i, int j, T k2v, cplx<T> c, cplx<T> xw, cplx<T> xe, cplx<T> xs, cplx<T> xn) {
        cplx<T> r{T(0), T(0)};
        if (i >= 0 && j >= 0 && i <= nf && j <= nf) {
            r = op.fine.apply5k(i, j, k2v, c, xw, xe, xs, xn);
            const T sw = op.shift * line_w<T>(i, nf) * line_w<T>(j, nf) * k2v;
            r.re += sw * c.im;
            r.im -= sw * c.re;
        }
        return r;
    };
    // fine regions strictly inside the grid skip the boundary terms (a uniform
    // branch between two versions of the loop)
    const bool interior = 2 * tl.c0 - 2 >= 1 && 2 * tl.c0 + 2 * VX - 3 <= nf - 1 && 2 * tl.r0 - 2 >= 1 &&
                          2 * tl.r0 + 2 * rows + 1 <= nf - 1;
    auto cs_inner = [&](T k2v, cplx<T> c, cplx<T> xw, cplx<T> xe, cplx<T> xs, cplx<T> xn) {
        cplx<T> r = op.fine.apply5k_interior(k2v, c, xw, xe, xs, xn);
        const T sw = op.shift * k2v;
        r.re += sw * c.im;
        r.im -= sw * c.re;
        return r;
    };
    auto vstage = [&](auto inner) {
    for_strided_batched<kVBlocks>(
        nvb,
        [&](int u, int q) {
            const int fi = 2 * (tl.c0 - 1 + q % VX), fj = 2 * (tl.r0 - 1 + q / VX);
            const int i0 = min(max(fi, 0), nf), i1 = min(max(fi + 1, 0), nf);
            const int j0 = min(max(fj, 0), nf), j1 = min(max(fj + 1, 0), nf);
            kk[u][0] = op.fine.k2[op.fine.g.at(i0, j0)];
            kk[u][1] = op.fine.k2[op.fine.g.at(i1, j0)];
            kk[u][2] = op.fine.k2[op.fine.g.at(i0, j1)];
            kk[u][3] = op.fine.k2[op.fine.g.at(i1, j1)];
        },
        [&](int u, int q) {
            const int bx = q % VX, by = q / VX;
            const int fi = 2 * (tl.c0 - 1 + bx), fj = 2 * (tl.r0 - 1 + by);
            const int c = 2 * bx + 1, r = 2 * by + 1;  // y column and row of (fi, fj)
            const cplx<T> s0 = yat(c, r - 1), s1 = yat(c + 1, r - 1);
            const cplx<T> w0 = yat(c - 1, r), c00 = yat(c, r), c10 = yat(c + 1, r), e0 = yat(c + 2, r);
            const cplx<T> w1 = yat(c - 1, r + 1), c01 = yat(c, r + 1), c11 = yat(c + 1, r + 1), e1 = yat(c + 2, r + 1);
            const cplx<T> n0 = yat(c, r + 2), n1 = yat(c + 1, r + 2);
            const int vi = 2 * by * PS::VW + 2 * bx;
            const bool east = bx < VX - 1, north = by < rows + 1;
            if constexpr (decltype(inner)::value) {
                v[vi] = cs_inner(kk[u][0], c00, w0, c10, s0, c01);
                if (east) v[vi + 1] = cs_inner(kk[u][1], c10, c00, e0, s1, c11);
                if (north) {
                    v[vi + PS::VW] = cs_inner(kk[u][2], c01, w1, c11, c00, n0);
                    if (east) v[vi + PS::VW + 1] = cs_inner(kk[u][3], c11, c01, e1, c10, n1);
                }
            } else {
                v[vi] = cs_node(fi, fj, kk[u][0], c00, w0, c10, s0, c01);
                if (east) v[vi + 1] = cs_node(fi + 1, fj, kk[u][1], c10, c00, e0, s1, c11);
                if (north) {
                    v[vi + PS::VW] = cs_node(fi, fj + 1, kk[u][2], c01, w1, c11, c00, n0);
                    if (east) v[vi + PS::VW + 1] = cs_node(fi + 1, fj + 1, kk[u][3], c11, c01, e1, c10, n1);
                }
            }
        });
    };
    if (interior) vstage(std::true_type{});
    else vstage(std::false_type{});
    __syncthreads();
    // (R v)_I = (1/4) sum of the prolongation weights of I times v
    const T m5[5] = {T(1), T(4), T(6), T(4), T(1)};
    const T m3[5] = {T(0), T(1), T(2), T(1), T(0)};
    const T scale = kBez ? T(1.0 / 256.0) : T(1.0 / 16.0);
    constexpr int NB = 2;
    decltype(pget(0LL)) pv[NB];
    for_nodes_batched<NB>(op.g, (rows + blockDim.y - 1) / blockDim.y, [&](int u, long long p) { pv[u] = pget(p); },
                          [&](int u, int i, int j, long long p) {
        const int vc = (2 * (j - tl.r0) + 2) * PS::VW + 2 * (i - tl.c0) + 2;
        cplx<T> acc{T(0), T(0)};
#pragma unroll
        for (int dy = -2; dy <= 2; ++dy) {
            cplx<T> row{T(0), T(0)};
#pragma unroll
            for (int dx = -2; dx <= 2; ++dx) {
                const T w = kBez ? m5[dx + 2] : m3[dx + 2];
                const cplx<T> vv = v[vc + dy * PS::VW + dx];
                row.re += w * vv.re;
                row.im += w * vv.im;
            }
            const T w = kBez ? m5[dy + 2] : m3[dy + 2];
            acc.re += w * row.re;
            acc.im += w * row.im;
        }
        f(i, j, p, pv[u], lds[tl.at(i, j)], scale * acc);
    });
}

template <typename Op, typename T, bool kXcd = false, typename PGet, typename F>
__device__ __forceinline__ void apply_from_tile(const Op& op, int rpt, const Tile<op_radius<Op>::value>& tl,
                                                cplx<T>* lds, PGet&& pget, F&& f);

// Runs f(i, j, p, pget(p), x at p, A x at p) over the thread's nodes, where
// x = xmake(xload(p)) (xload only loads): x for the block tile plus halo is
// staged in LDS first (one evaluation per tile node instead of one per
// stencil entry), then the operator reads LDS only. pget loads the caller's
// per-node operands; they and the operator's own (k^2 on level 0) are
// loaded for a batch of rows before the batch's arithmetic.
template <typename Op, typename T, typename XLoad, typename XMake, typename PGet, typename F>
__device__ __forceinline__ void for_nodes_applied_pre(const Op& op, int rpt, XLoad&& xload, XMake&& xmake,
                                                      PGet&& pget, F&& f) {
    constexpr int R = op_radius<Op>::value;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    const Tile<R> tl = block_tile<R>(rpt);
    fill_tile<T, R>(lds, tl, op.g, xload, xmake);
    apply_from_tile<Op, T>(op, rpt, tl, lds, pget, f);
}

// The second half of for_nodes_applied_pre: x of the block tile plus halo is
// in LDS (after a barrier); runs f(i, j, p, pget(p), x at p, A x at p).
template <typename Op, typename T, bool kXcd, typename PGet, typename F>
__device__ __forceinline__ void apply_from_tile(const Op& op, int rpt, const Tile<op_radius<Op>::value>& tl,
                                                cplx<T>* lds, PGet&& pget, F&& f) {
    if constexpr (is_product<Op>::value) {
        static_assert(!kXcd, "the XCD tile map is used by level-0 passes only");
        product_stages(op, tl, lds, pget, f);
    } else if constexpr (std::is_same<Op, FineOp<T>>::value) {
        // tiles whose nodes all lie strictly inside the grid skip the boundary
        // terms (a uniform branch between two versions of the row loop)
        const int n = op.g.n;
        const bool interior = tl.c0 >= 1 && tl.c0 + kBX <= n && tl.r0 >= 1 && tl.r0 + tl.rows <= n;
        constexpr int NB = sizeof(T) == 4 ? 8 : 4;
        constexpr int TW = Tile<1>::TW;
        decltype(pget(0LL)) pv[NB];
        T kk[NB];
        auto rows = [&](auto inner) {
            for_nodes_batched<NB, kXcd>(
                op.g, rpt,
                [&](int u, long long p) {
                    pv[u] = pget(p);
                    kk[u] = op.k2[p];
                },
                [&](int u, int i, int j, long long p) {
                    const int li = tl.at(i, j);
                    const cplx<T> c = lds[li];
                    const cplx<T> ax =
                        decltype(inner)::value
                            ? op.apply5k_interior(kk[u], c, lds[li - 1], lds[li + 1], lds[li - TW], lds[li + TW])
                            : op.apply5k(i, j, kk[u], c, lds[li - 1], lds[li + 1], lds[li - TW], lds[li + TW]);
                    f(i, j, p, pv[u], c, ax);
                });
        };
        if (interior) rows(std::true_type{});
        else rows(std::false_type{});
    } else {
        // rows per batch: stored stencils keep one row per thread on most
        // levels and their FP64 coefficient batches need the registers
        constexpr int NB = is_stencil<Op>::value ? (sizeof(T) == 4 ? 2 : 1) : (sizeof(T) == 4 ? 8 : 4);
        decltype(pget(0LL)) pv[NB];
        typename OpPre<Op>::type ov[NB];
        for_nodes_batched<NB, kXcd>(
            op.g, rpt,
            [&](int u, long long p) {
                pv[u] = pget(p);
                ov[u] = OpPre<Op>::load(op, p);
            },
            [&](int u, int i, int j, long long p) {
                const int li = tl.at(i, j);
                f(i, j, p, pv[u], lds[li], apply_tile_pre(op, lds, li, i, j, p, ov[u]));
            });
    }
}

// for_nodes_applied_pre with x loaded as it is stored (xget(p) = x[p]) and
// no per-node operands of the caller: f(i, j, p, x at p, A x at p).
template <typename Op, typename T, typename XGet, typename F>
__device__ __forceinline__ void for_nodes_applied(const Op& op, int rpt, XGet&& xget, F&& f) {
    for_nodes_applied_pre<Op, T>(op, rpt, xget, Ident{}, [](long long) { return NoVals{}; },
                                 [&](int i, int j, long long p, NoVals, cplx<T> x, cplx<T> ax) { f(i, j, p, x, ax); });
}

// Dynamic LDS bytes of an operator kernel launched with geometry (by, rpt).
template <typename Op, typename T>
__host__ __device__ size_t tile_bytes(int by, int rpt) {
    constexpr int R = op_radius<Op>::value;
    if constexpr (is_product<Op>::value) return ProductStages<T>::values(by * rpt) * sizeof(cplx<T>);
    return size_t(Tile<R>::TW) * size_t(by * rpt + 2 * R) * sizeof(cplx<T>);
}

// ---------------------------------------------------------------- operator
template <typename Op, typename T, int BY>
__global__ __launch_bounds__(kBX * BY) void k_apply(Op op, Vec<T> x, Vec<T> y, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    cplx<T>* yb = y.rhs(b);
    for_nodes_applied<Op, T>(op, rpt, [xb](long long q) { return xb[q]; },
                             [&](int, int, long long p, cplx<T>, cplx<T> ax) {
                                 yb[p] = ax;
                             });
}

// y = A_s x on level 0 with x the complex64 plane xs widened to FP64, which is
// written to x as well (the outer FGMRES keeps the FP32 cycle's result as its
// FP64 vector z_j and applies the operator to it: one pass instead of two).
template <int BY>
__global__ __launch_bounds__(kBX * BY) void k_apply_widened(FineOp<double> op, Vec<float> xs, Vec<double> x,
                                                            Vec<double> y, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<float>* sb = xs.rhs(b);
    cplx<double>* xb = x.rhs(b);
    cplx<double>* yb = y.rhs(b);
    for_nodes_applied_pre<FineOp<double>, double>(
        op, rpt, [sb](long long q) { return sb[q]; }, [](cplx<float> v) { return cast<double>(v); },
        [](long long) { return NoVals{}; },
        [&](int, int, long long p, NoVals, cplx<double> xv, cplx<double> ax) {
            xb[p] = xv;
            yb[p] = ax;
        });
}

template <typename Op, typename T, int BY>
__global__ __launch_bounds__(kBX * BY) void k_residual(Op op, Vec<T> x, Vec<T> f, Vec<T> r, const int* active,
                                                       int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* rb = r.rhs(b);
    for_nodes_applied_pre<Op, T>(op, rpt, [xb](long long q) { return xb[q]; }, Ident{},
                                 [fb](long long q) { return fb[q]; },
                                 [&](int, int, long long p, cplx<T> fp, cplx<T>, cplx<T> ax) {
                                     rb[p] = fp - ax;
                                 });
}

// Weighted Jacobi of §3: y = x + (omega diag(A))^{-1} (f - A x).
template <typename Op, typename T, int BY>
__global__ __launch_bounds__(kBX * BY) void k_jacobi(Op op, Vec<T> x, Vec<T> f, Vec<T> y, T inv_omega,
                                                     const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* yb = y.rhs(b);
    for_nodes_applied_pre<Op, T>(op, rpt, [xb](long long q) { return xb[q]; }, Ident{},
                                 [fb](long long q) { return fb[q]; },
                                 [&](int i, int j, long long p, cplx<T> fp, cplx<T> xp, cplx<T> ax) {
                                 const cplx<T> r = fp - ax;
                                 yb[p] = xp + inv_omega * cdiv(r, op.diag(i, j, p));
                             });
}

// Two weighted-Jacobi sweeps in one pass on level 0 (temporal blocking of the
// smoother of §3): x is staged for the tile plus a halo of 2, the first sweep
// runs on the tile plus a halo of 1 (nodes off the grid hold zero, the ghosts
// the second sweep reads) into a second LDS stage, the second sweep on the
// tile. Per node the arithmetic of k_jacobi (the general form of the
// five-point operator everywhere); f and k^2 of the tile are read by both
// sweeps, the second time from cache, and the loads of each sweep are
// gathered in batches. (On stored-stencil levels the first sweep's halo of R
// nodes, each with its (2R+1)^2 coefficients, cost more than the second pass
// it saves: measured 1.3-2.6x slower, so those levels keep one sweep per pass.)
struct Jacobi2Stage {
    static constexpr int TA = kBX + 4;  // stage A (x): tile plus 2
    static constexpr int TB = kBX + 2;  // stage B (first sweep): tile plus 1
    __host__ __device__ static size_t values(int rows) { return size_t(TA) * (rows + 4) + size_t(TB) * (rows + 2); }
};

template <typename T, int BY>
__global__ __launch_bounds__(kBX * BY) void k_jacobi2(FineOp<T> op, Vec<T> x, Vec<T> f, Vec<T> y, T inv_omega,
                                                      const int* active, int rpt) {
    using JS = Jacobi2Stage;
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* yb = y.rhs(b);
    const Grid& g = op.g;
    const BlockXY bt = block_xy();
    const int rows = BY * rpt;
    const int c0 = bt.x * kBX, r0 = bt.y * rows;
    cplx<T>* sa = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    cplx<T>* sb = sa + JS::TA * (rows + 4);
    constexpr int NB = FillBatch<T>::value;
    if (r0 - 2 <= g.n) {  // padding tiles of batch grids stage nothing
        // stage A: x on the tile plus 2 (zero off the grid)
        cplx<T> v[NB];
        bool ok[NB];
        for_strided_batched<NB>(
            JS::TA * (rows + 4),
            [&](int u, int q) {
                const int i = c0 - 2 + q % JS::TA, j = r0 - 2 + q / JS::TA;
                ok[u] = i >= 0 && i <= g.n && j >= 0 && j <= g.n;
                v[u] = xb[g.at(min(max(i, 0), g.n), min(max(j, 0), g.n))];
            },
            [&](int u, int q) { sa[q] = ok[u] ? v[u] : cplx<T>{T(0), T(0)}; });
        __syncthreads();
        // first sweep on the tile plus 1
        cplx<T> fv[NB];
        T kv[NB];
        for_strided_batched<NB>(
            JS::TB * (rows + 2),
            [&](int u, int q) {
                const int i = c0 - 1 + q % JS::TB, j = r0 - 1 + q / JS::TB;
                ok[u] = i >= 0 && i <= g.n && j >= 0 && j <= g.n;
                const long long p = g.at(min(max(i, 0), g.n), min(max(j, 0), g.n));
                fv[u] = fb[p];
                kv[u] = op.k2[p];
            },
            [&](int u, int q) {
                const int i = c0 - 1 + q % JS::TB, j = r0 - 1 + q / JS::TB;
                cplx<T> out{T(0), T(0)};
                if (ok[u]) {
                    const int la = (j - r0 + 2) * JS::TA + (i - c0 + 2);
                    const cplx<T> r = fv[u] - op.apply5k(i, j, kv[u], sa[la], sa[la - 1], sa[la + 1],
                                                          sa[la - JS::TA], sa[la + JS::TA]);
                    out = sa[la] + inv_omega * cdiv(r, op.diag_k(i, j, kv[u]));
                }
                sb[q] = out;
            });
    }
    __syncthreads();
    // second sweep on the tile
    cplx<T> fv[NB];
    T kv[NB];
    for_nodes_batched<NB>(
        g, rpt,
        [&](int u, long long p) {
            fv[u] = fb[p];
            kv[u] = op.k2[p];
        },
        [&](int u, int i, int j, long long p) {
            const int lb = (j - r0 + 1) * JS::TB + (i - c0 + 1);
            const cplx<T> r = fv[u] - op.apply5k(i, j, kv[u], sb[lb], sb[lb - 1], sb[lb + 1], sb[lb - JS::TB],
                                                  sb[lb + JS::TB]);
            yb[p] = sb[lb] + inv_omega * cdiv(r, op.diag_k(i, j, kv[u]));
        });
}

// ---------------------------------------------------------------- transfers
// Restriction R = P^T / 4 of the §4 prolongation: the 2D row is the outer
// product of [1 4 6 4 1]/16 (Bézier) or [1 2 1]/4 (linear) centred on the
// fine node (2I, 2J); fine ghosts are zero, which truncates at the boundary.
// The coarse iterate that the next cycle starts from (zero) is written in the
// same pass when `uc` is given.
template <typename T, bool kBez, int BY>
__global__ __launch_bounds__(kBX * BY) void k_restrict(Grid gf, Grid gc, Vec<T> r, Vec<T> fc, Vec<T> uc,
                                                       Vec<T> Z, double* pout, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* rb = r.rhs(b);
    cplx<T>* fb = fc.rhs(b);
    cplx<T>* ub = uc.p ? uc.rhs(b) : nullptr;
    cplx<T>* zb = Z.p ? Z.p + (long long)(b * 4) * Z.plane : nullptr;
    double nrm[1] = {0.0};
    auto put = [&](long long pc, cplx<T> v) {
        fb[pc] = v;
        if (zb) {
            zb[pc] = v;
            nrm[0] += dnorm2(v);
        }
    };
    for_nodes(gc, rpt, [&](int I, int J, long long pc) {
        if (ub) ub[pc] = cplx<T>{T(0), T(0)};
        const long long pf = gf.at(2 * I, 2 * J);
        cplx<T> acc{T(0), T(0)};
        if constexpr (kBez) {
            constexpr T w[5] = {T(1), T(4), T(6), T(4), T(1)};
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                cplx<T> row{T(0), T(0)};
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const cplx<T> v = rb[pf + (long long)dy * gf.pitch + dx];
                    row.re += w[dx + 2] * v.re;
                    row.im += w[dx + 2] * v.im;
                }
                acc.re += w[dy + 2] * row.re;
                acc.im += w[dy + 2] * row.im;
            }
            put(pc, T(1.0 / 256.0) * acc);
        } else {
            constexpr T w[3] = {T(1), T(2), T(1)};
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                cplx<T> row{T(0), T(0)};
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const cplx<T> v = rb[pf + (long long)dy * gf.pitch + dx];
                    row.re += w[dx + 1] * v.re;
                    row.im += w[dx + 1] * v.im;
                }
                acc.re += w[dy + 1] * row.re;
                acc.im += w[dy + 1] * row.im;
            }
            put(pc, T(1.0 / 16.0) * acc);
        }
    });
    if (zb) block_partials<1>(nrm, pout + b * kPartStride);
}

// Prolongation of §4 per dimension: fine 2I <- (e[I-1] + 6 e[I] + e[I+1]) / 8,
// fine 2I+1 <- (e[I] + e[I+1]) / 2 (linear transfer: fine 2I <- e[I]);
// coarse ghosts are zero, which drops out-of-range coarse indices.
template <typename T>
__device__ __forceinline__ void taps(int i, bool bez, T (&w)[3]) {
    if (i & 1) {
        w[0] = T(0); w[1] = T(0.5); w[2] = T(0.5);
    } else if (bez) {
        w[0] = T(0.125); w[1] = T(0.75); w[2] = T(0.125);
    } else {
        w[0] = T(0); w[1] = T(1); w[2] = T(0);
    }
}

// The coarse values a block of fine nodes (columns [c0, c0 + 64), rows
// [r0, r0 + rows), c0 and r0 even) reads: coarse columns c0/2 - 1 ..
// c0/2 + 32 and rows r0/2 - 1 .. (r0 + rows - 1)/2 + 1, staged in LDS.
constexpr int kProlongTW = kBX / 2 + 2;
__host__ __device__ inline int prolong_rows(int rows) { return rows / 2 + 3; }

template <typename T, bool kBez, int BY>
__global__ __launch_bounds__(kBX * BY) void k_prolong_add(Grid gc, Grid gf, Vec<T> e, Vec<T> u, const int* active,
                                                          int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* eb = e.rhs(b);
    cplx<T>* ub = u.rhs(b);
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    const BlockXY bt = block_xy();
    const int rows = BY * rpt;
    const int C0 = bt.x * (kBX / 2) - 1, R0 = bt.y * (rows / 2) - 1;  // coarse origin of the LDS tile
    const int ne = kProlongTW * prolong_rows(rows);
    // coarse ghosts (index -1 and nc + 1) hold zero; indices beyond them read
    // a clamped node and store zero
    constexpr int kEBatch = 4;
    cplx<T> ev[kEBatch];
    bool ok[kEBatch];
    for_strided_batched<kEBatch>(
        ne,
        [&](int v, int q) {
            const int I = C0 + q % kProlongTW, J = R0 + q / kProlongTW;
            const int Ic = min(I, gc.n + 1), Jc = min(J, gc.n + 1);
            ok[v] = I == Ic && J == Jc;
            ev[v] = eb[gc.at(Ic, Jc)];
        },
        [&](int v, int q) { lds[q] = ok[v] ? ev[v] : cplx<T>{T(0), T(0)}; });
    __syncthreads();
    constexpr int NB = 8;
    cplx<T> uo[NB];
    for_nodes_batched<NB>(
        gf, rpt, [&](int v, long long pf) { uo[v] = ub[pf]; },
        [&](int v, int i, int j, long long pf) {
            T wx[3], wy[3];
            taps<T>(i, kBez, wx);
            taps<T>(j, kBez, wy);
            const int base = ((j >> 1) - 1 - R0) * kProlongTW + (i >> 1) - 1 - C0;
            cplx<T> acc{T(0), T(0)};
#pragma unroll
            for (int ty = 0; ty < 3; ++ty) {
                cplx<T> row{T(0), T(0)};
#pragma unroll
                for (int tx = 0; tx < 3; ++tx) {
                    const cplx<T> x = lds[base + ty * kProlongTW + tx];
                    row.re += wx[tx] * x.re;
                    row.im += wx[tx] * x.im;
                }
                acc.re += wy[ty] * row.re;
                acc.im += wy[ty] * row.im;
            }
            ub[pf] = uo[v] + acc;
        });
}

// ---------------------------------------------------------------- GMRES(3)
// One smoothing step of §5.3 = one restart cycle of 3 GMRES iterations from
// the current iterate. Arnoldi vectors are stored unnormalised (z_j) with
// s_j = 1/||z_j|| kept in GmState; orthogonalisation is classical
// Gram-Schmidt with the new vector's norm computed directly (two passes per
// Arnoldi step: apply + inner products, orthogonalise + norm).

template <typename T>
__device__ __forceinline__ void acc_dot(double& re, double& im, cplx<T> a, cplx<T> w) {
    // conj(a) * w
    re += double(a.re) * double(w.re) + double(a.im) * double(w.im);
    im += double(a.re) * double(w.im) - double(a.im) * double(w.re);
}

__device__ __forceinline__ bool lead_thread() { return block_linear() == 0 && thread_linear() == 0; }

// Pass 1: z0 = f - A u; partials ||z0||^2.
template <typename Op, typename T, int BY>
__global__ __launch_bounds__(kBX * BY) void k_gm_r(Op op, Vec<T> u, Vec<T> f, Vec<T> Z, double* pout,
                                                   const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* ub = u.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* z0 = Z.p + (long long)(b * 4) * Z.plane;
    double acc[1] = {0.0};
    for_nodes_applied_pre<Op, T>(op, rpt, [ub](long long q) { return ub[q]; }, Ident{},
                                 [fb](long long q) { return fb[q]; },
                                 [&](int, int, long long p, cplx<T> fp, cplx<T>, cplx<T> au) {
                                 const cplx<T> z = fp - au;
                                 z0[p] = z;
                                 acc[0] += dnorm2(z);
                             });
    block_partials<1>(acc, pout + b * kPartStride);
}

// Pass 5 prologue: column 2 of H from pass 4's sums (unless the Arnoldi
// process stopped early), the least-squares problem, and the update weights
// c_i = y_i s_i (k = 0: nothing to add). H[3][2] = ||z_3|| for
// z_3 = s_2 w_2 - sum_i H[i][2] s_i z_i comes from
// ||z_3||^2 = s_2^2 ||w_2||^2 - sum_i |H[i][2]|^2 (the s_i z_i are orthonormal),
// clamped at zero. Every thread reduces the sums and solves the small problem
// in registers.
template <typename T>
__device__ __forceinline__ int gm_update_weights(const GmState* st, int b, double breakdown, const double* pin,
                                                 int nblk_in, cplx<T> (&c)[3]) {
    const GmState S = st[b];
    double t[8];
    reduce_partials<8>(pin + b * kPartStride, nblk_in, t);  // read in any case; used after a full Arnoldi pass
    int k = S.k;
#pragma unroll
    for (int q = 0; q < 3; ++q) c[q] = {T(0), T(0)};
    if (k == 0) return 0;
    double hr[4][3], hi[4][3], s[3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            hr[a][cc] = S.hr[a][cc];
            hi[a][cc] = S.hi[a][cc];
        }
#pragma unroll
    for (int q = 0; q < 3; ++q) s[q] = S.s[q];
    if (!S.arnoldi_done) {
        const double hn = sqrt(t[0]);
        if (!(hn > breakdown * S.beta)) {
            k = 2;
        } else {
            const double s2 = 1.0 / hn;
            s[2] = s2;
            hr[2][1] = hn;
            hi[2][1] = 0.0;
            double sq = s2 * s2 * t[7];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                hr[q][2] = s[q] * s2 * t[1 + 2 * q];
                hi[q][2] = s[q] * s2 * t[2 + 2 * q];
                sq -= hr[q][2] * hr[q][2] + hi[q][2] * hi[q][2];
            }
            hr[3][2] = sqrt(fmax(sq, 0.0));
            hi[3][2] = 0.0;
            k = 3;
        }
    }
    double yr[3], yi[3];
    gm_least_squares_regs(hr, hi, s, S.beta, k, yr, yi);
#pragma unroll
    for (int q = 0; q < 3; ++q) c[q] = {T(yr[q]), T(yi[q])};
    return k;
}

// The coarse values that a fine tile with halo R reads through the §4
// prolongation: coarse columns c0/2 - ceil(R/2) - 1 ... and rows likewise,
// kept in LDS after the operator's own stages.
template <int R>
struct ProlongTile {
    static constexpr int EW = (kBX - 1 + R) / 2 + (R + 1) / 2 + 3;
    __host__ __device__ static int rows(int fine_rows) { return (fine_rows - 1 + R) / 2 + (R + 1) / 2 + 3; }
};

// x = u + P e for the fine tile tl and its halo of R nodes (zero off the grid)
// into X, the coarse values the tile reads staged in E first (coarse grid
// correction of §3 with the §4 prolongation). kDefer: the coarse level's last
// smoothing step left its update pass to this one, and e is formed at the
// coarse nodes the block reads as that pass forms it (same weights, same
// order of operations, so the same bits), e = base + sum_i c_i z_i. Ends with
// a barrier.
template <typename T, bool kBez, int R, bool kDefer>
__device__ __forceinline__ void stage_corrected_tile(const Tile<R>& tl, const Grid& g, const Grid& gc,
                                                     const cplx<T>* eb, const cplx<T>* ub,
                                                     const DeferredUpdate<T>& du, int b, cplx<T>* X, cplx<T>* E) {
    using PT = ProlongTile<R>;
    const int C0 = (tl.c0 >> 1) - (R + 1) / 2 - 1, Q0 = (tl.r0 >> 1) - (R + 1) / 2 - 1;
    const int nc = gc.n, n = g.n;
    constexpr int FB = FillBatch<T>::value;
    cplx<T> uv[FB];
    auto fload = [&](int v, int q) {
        const int i = tl.c0 - R + q % Tile<R>::TW, j = tl.r0 - R + q / Tile<R>::TW;
        uv[v] = ub[g.at(min(max(i, 0), n), min(max(j, 0), n))];
    };
    auto fbody = [&](int v, int q) {
        const int i = tl.c0 - R + q % Tile<R>::TW, j = tl.r0 - R + q / Tile<R>::TW;
        cplx<T> x{T(0), T(0)};
        if (i >= 0 && j >= 0 && i <= n && j <= n) {
            T wx[3], wy[3];
            taps<T>(i, kBez, wx);
            taps<T>(j, kBez, wy);
            const int base = ((j >> 1) - 1 - Q0) * PT::EW + (i >> 1) - 1 - C0;
            x = uv[v];
#pragma unroll
            for (int ty = 0; ty < 3; ++ty) {
                cplx<T> row{T(0), T(0)};
#pragma unroll
                for (int tx = 0; tx < 3; ++tx) {
                    const cplx<T> c = E[base + ty * PT::EW + tx];
                    row.re += wx[tx] * c.re;
                    row.im += wx[tx] * c.im;
                }
                x.re += wy[ty] * row.re;
                x.im += wy[ty] * row.im;
            }
        }
        X[q] = x;
    };
    const int ecount = PT::EW * PT::rows(tl.rows);
    if constexpr (kDefer) {  // coarse e from the pending update; zero off the grid
        cplx<T> c[3];
        const int k = gm_update_weights<T>(du.st, b, du.breakdown, du.part, du.nblk, c);
        const cplx<T>* bb = du.uin.p ? du.uin.rhs(b) : du.u.rhs(b);
        const cplx<T>* zc0 = du.Z.p + (long long)(b * 4) * du.Z.plane;
        const cplx<T>* zc1 = zc0 + du.Z.plane;
        const cplx<T>* zc2 = zc1 + du.Z.plane;
        constexpr int EB = 4;
        cplx<T> xu[EB], x0[EB], x1[EB], x2[EB];
        bool ok[EB];
        for_strided_batched<EB>(
            ecount,
            [&](int v, int q) {
                const int I = C0 + q % PT::EW, J = Q0 + q / PT::EW;
                const int Ic = min(max(I, 0), nc), Jc = min(max(J, 0), nc);
                ok[v] = I == Ic && J == Jc;
                const long long p = gc.at(Ic, Jc);
                xu[v] = bb[p];
                x0[v] = zc0[p];
                x1[v] = zc1[p];
                x2[v] = zc2[p];
            },
            [&](int v, int q) {
                cplx<T> x = xu[v];
                if (k > 0) x = cfma(x, c[0], x0[v]);
                if (k > 1) x = cfma(x, c[1], x1[v]);
                if (k > 2) x = cfma(x, c[2], x2[v]);
                E[q] = ok[v] ? x : cplx<T>{T(0), T(0)};
            });
    } else {  // coarse e: ghosts (index -1, nc + 1) hold zero; beyond them a clamped read gives zero
        constexpr int EB = 8;
        cplx<T> ev[EB];
        bool ok[EB];
        for_strided_batched<EB>(
            ecount,
            [&](int v, int q) {
                const int I = C0 + q % PT::EW, J = Q0 + q / PT::EW;
                const int Ic = min(max(I, -1), nc + 1), Jc = min(max(J, -1), nc + 1);
                ok[v] = I == Ic && J == Jc;
                ev[v] = eb[gc.at(Ic, Jc)];
            },
            [&](int v, int q) { E[q] = ok[v] ? ev[v] : cplx<T>{T(0), T(0)}; });
    }
    __syncthreads();
    for_strided_batched<FB>(tl.count(), fload, fbody);
    __syncthreads();
}

// Pass 1 of the first post-smoothing step fused with the coarse grid
// correction before it: x = u + P e on the block tile and its halo (zero
// off the grid), x to xt (u stays as it was: neighbouring blocks read it),
// z0 = f - A x, partials ||z0||^2. The pass that ends the step reads x from
// xt and writes the updated iterate to u. kDefer: see stage_corrected_tile.
template <typename Op, typename T, bool kBez, int BY, bool kDefer>
__global__ __launch_bounds__(kBX * BY) void k_gm_r_pro(Op op, Grid gc, Vec<T> e, Vec<T> u, Vec<T> f, Vec<T> xt,
                                                       Vec<T> Z, double* pout, const int* active, int rpt,
                                                       DeferredUpdate<T> du) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    constexpr int R = op_radius<Op>::value;
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* xb = xt.rhs(b);
    cplx<T>* z0 = Z.p + (long long)(b * 4) * Z.plane;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    const Tile<R> tl = block_tile<R>(rpt);
    cplx<T>* E = lds + tile_bytes<Op, T>(BY, rpt) / sizeof(cplx<T>);
    stage_corrected_tile<T, kBez, R, kDefer>(tl, op.g, gc, e.rhs(b), u.rhs(b), du, b, lds, E);
    double acc[1] = {0.0};
    apply_from_tile<Op, T>(op, rpt, tl, lds, [fb](long long q) { return fb[q]; },
                           [&](int, int, long long p, cplx<T> fp, cplx<T> x, cplx<T> ax) {
                               const cplx<T> z = fp - ax;
                               xb[p] = x;
                               z0[p] = z;
                               acc[0] += dnorm2(z);
                           });
    block_partials<1>(acc, pout + b * kPartStride);
}

// Level 0: the first post-smoothing pass (k_gm_r_pro) and the apply pass
// after it (k_gm_a0) in one. x = u + P e is staged for the tile and a halo of
// 2, z0 = f - A x for the tile and a halo of 1 (the halo ring evaluated as the
// block owning each ring node evaluates it, with or without the interior form
// of the operator, so that the values equal the ones that block stores), then
// w0 = A z0 on the tile from LDS. The owned nodes are visited in the thread
// order of the two separate passes, so the partial sums ||z0||^2 and
// <z0, w0> (three per block) are those passes' bit for bit; the next pass
// (k_gm_oa<1, kInit>) takes over the state set-up of k_gm_a0.
template <typename T>
struct ResApplyStage {
    static constexpr int kXW = Tile<2>::TW;  // x: tile and a halo of 2
    static constexpr int kZW = Tile<1>::TW;  // z0: tile and a halo of 1
    __host__ __device__ static size_t bytes(int rows) {
        return (size_t(kXW) * (rows + 4) + size_t(kZW) * (rows + 2) +
                size_t(ProlongTile<2>::EW) * ProlongTile<2>::rows(rows)) *
               sizeof(cplx<T>);
    }
};

template <typename T, bool kBez, int BY, bool kDefer>
__global__ __launch_bounds__(kBX * BY) void k_gm_r_pro_a0(FineOp<T> op, Grid gc, Vec<T> e, Vec<T> u, Vec<T> f,
                                                          Vec<T> xt, Vec<T> Z, Vec<T> Wout, double* pout,
                                                          const int* active, int rpt, DeferredUpdate<T> du) {
    using RA = ResApplyStage<T>;
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* xb = xt.rhs(b);
    cplx<T>* z0 = Z.p + (long long)(b * 4) * Z.plane;
    cplx<T>* wb = Wout.rhs(b);
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    const Tile<2> tx = block_tile<2>(rpt);
    const Tile<1> tz{tx.c0, tx.r0, tx.rows};
    cplx<T>* X = lds;
    cplx<T>* ZL = X + RA::kXW * (tx.rows + 4);
    cplx<T>* E = ZL + RA::kZW * (tx.rows + 2);
    stage_corrected_tile<T, kBez, 2, kDefer>(tx, op.g, gc, e.rhs(b), u.rhs(b), du, b, X, E);
    const int n = op.g.n;
    constexpr int XW = RA::kXW, ZW = RA::kZW;
    // operator at fine node (i, j) from X, in the form the tile owning (i, j) uses
    const int trows = int(blockDim.y) * rpt;
    auto owner_interior = [&](int i, int j) {
        const int oc = (i / kBX) * kBX, orow = (j / trows) * trows;
        return oc >= 1 && oc + kBX <= n && orow >= 1 && orow + trows <= n;
    };
    auto ax_at = [&](int i, int j, T kk, bool inner) {
        const int l = tx.at(i, j);
        return inner ? op.apply5k_interior(kk, X[l], X[l - 1], X[l + 1], X[l - XW], X[l + XW])
                     : op.apply5k(i, j, kk, X[l], X[l - 1], X[l + 1], X[l - XW], X[l + XW]);
    };
    // z0 on the halo ring of the tile (top and bottom rows, then the left and
    // right columns): each thread's first ring node has its operands loaded
    // together with those of its tile nodes (one memory round trip), further
    // ones (blocks of two wavefronts) after them
    const int ring = 2 * ZW + 2 * tx.rows;
    auto ring_node = [&](int q, int& i, int& j) {
        if (q < 2 * ZW) {
            i = tx.c0 - 1 + q % ZW;
            j = q < ZW ? tx.r0 - 1 : tx.r0 + tx.rows;
        } else {
            const int m = q - 2 * ZW;
            i = (m & 1) ? tx.c0 + kBX : tx.c0 - 1;
            j = tx.r0 + (m >> 1);
        }
    };
    auto ring_z = [&](int i, int j, T kk, cplx<T> fp) {
        cplx<T> z{T(0), T(0)};
        if (i >= 0 && j >= 0 && i <= n && j <= n) z = fp - ax_at(i, j, kk, owner_interior(i, j));
        ZL[tz.at(i, j)] = z;
    };
    const int tid = thread_linear(), nt = int(blockDim.x * blockDim.y);
    int ri = 0, rj = 0;
    T rk = T(0);
    cplx<T> rf{T(0), T(0)};
    if (tid < ring) {
        ring_node(tid, ri, rj);
        const long long p = op.g.at(min(max(ri, 0), n), min(max(rj, 0), n));
        rk = op.k2[p];
        rf = fb[p];
    }
    // z0 on the tile, in the thread order of the residual pass; each thread
    // first zeroes its own tile positions, so that those off the grid (which
    // the loop skips) read as zero
    for (int rr = 0; rr < rpt; ++rr)
        ZL[tz.at(tx.c0 + int(threadIdx.x), tx.r0 + rr * int(blockDim.y) + int(threadIdx.y))] = cplx<T>{T(0), T(0)};
    const bool interior = tx.c0 >= 1 && tx.c0 + kBX <= n && tx.r0 >= 1 && tx.r0 + tx.rows <= n;
    double acc[3] = {0.0, 0.0, 0.0};
    constexpr int NB = sizeof(T) == 4 ? 8 : 4;
    {
        cplx<T> pv[NB];
        T kk[NB];
        for_nodes_batched<NB>(
            op.g, rpt,
            [&](int v, long long p) {
                pv[v] = fb[p];
                kk[v] = op.k2[p];
            },
            [&](int v, int i, int j, long long p) {
                const cplx<T> z = pv[v] - ax_at(i, j, kk[v], interior);
                xb[p] = X[tx.at(i, j)];
                z0[p] = z;
                ZL[tz.at(i, j)] = z;
                acc[0] += dnorm2(z);
            });
    }
    if (tid < ring) ring_z(ri, rj, rk, rf);
    for (int q = tid + nt; q < ring; q += nt) {
        int i, j;
        ring_node(q, i, j);
        const long long p = op.g.at(min(max(i, 0), n), min(max(j, 0), n));
        ring_z(i, j, op.k2[p], fb[p]);
    }
    __syncthreads();
    {  // w0 = A z0 on the tile from LDS, in the thread order of the apply pass
        T kk[NB];
        for_nodes_batched<NB>(
            op.g, rpt, [&](int v, long long p) { kk[v] = op.k2[p]; },
            [&](int v, int i, int j, long long p) {
                const int l = tz.at(i, j);
                const cplx<T> zp = ZL[l];
                const cplx<T> w =
                    interior ? op.apply5k_interior(kk[v], zp, ZL[l - 1], ZL[l + 1], ZL[l - ZW], ZL[l + ZW])
                             : op.apply5k(i, j, kk[v], zp, ZL[l - 1], ZL[l + 1], ZL[l - ZW], ZL[l + ZW]);
                wb[p] = w;
                acc_dot(acc[1], acc[2], zp, w);
            });
    }
    block_partials<3>(acc, pout + b * kPartStride);
}

// Pass 2: beta = ||z0|| from pass 1; w0 = A z0 (unnormalised); partials <z0, w0>.
// The loads of pass 1's partial sums and of the first batch of the z0 tile
// are in flight together; the reduction runs while the tile loads return.
template <typename Op, typename T, int BY, bool kOv>
__global__ __launch_bounds__(kBX * BY) void k_gm_a0(Op op, Vec<T> Z, Vec<T> Wout, GmState* st, const double* pin,
                                                    int nblk_in, double* pout, const int* active, int rpt) {
    const int b = blockIdx.z;
    const bool act = rhs_active(active, b);
    const cplx<T>* z0 = Z.p + (long long)(b * 4) * Z.plane;
    cplx<T>* wb = Wout.rhs(b);
    // the block leaves after the reduction if its right-hand side is inactive
    // or has a zero (or non-finite) residual (uniform in the block)
    auto mid = [&](const double (&t)[1]) -> bool {
        if (!act) return false;
        const double beta = sqrt(t[0]);
        const bool go = beta > 0.0;
        if (lead_thread()) {
            GmState& S = st[b];
            S.beta = beta;
            S.s[0] = go ? 1.0 / beta : 0.0;
            S.k = go ? 3 : 0;
            S.arnoldi_done = go ? 0 : 1;
        }
        return go;
    };
    constexpr int R = op_radius<Op>::value;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    const Tile<R> tl = block_tile<R>(rpt);
    if (!reduce_and_fill<1, kOv, T, R>(pin + b * kPartStride, nblk_in, lds, tl, op.g,
                                        [z0](long long q) { return z0[q]; }, Ident{}, mid))
        return;
    double acc[2] = {0.0, 0.0};
    apply_from_tile<Op, T>(op, rpt, tl, lds, [](long long) { return NoVals{}; },
                           [&](int, int, long long p, NoVals, cplx<T> zp, cplx<T> w) {
                               wb[p] = w;
                               acc_dot(acc[0], acc[1], zp, w);
                           });
    block_partials<2>(acc, pout + b * kPartStride);
}

// Passes 3 and 4 (J = 1, 2): finish Arnoldi column J-1 from the previous
// pass's sums, then build z_J = s_{J-1} w_{J-1} - sum_i H[i][J-1] s_i z_i,
// w_J = A z_J (z_J recomputed at the stencil neighbours), partials
// ||z_J||^2 and <z_i, w_J> for i <= J, and for J = 2 also ||w_2||^2 (the last
// Arnoldi norm then follows without another pass over the vectors). w_1 goes
// to Wout for pass 4; w_2 only where Wout.p is set (the update pass of the
// last pre-smoothing step forms its residual from it). The raw tile values
// (w_{J-1}, z_0 .. z_{J-1}) of the first batch are loaded together with the
// previous pass's partial sums and combined once the reduction has given the
// coefficients. kInit (J = 1): the previous pass was k_gm_r_pro_a0, whose
// partial sums start with ||z_0||^2, and this pass sets up the step's state
// (beta, s_0, k) as k_gm_a0 does.
template <typename Op, typename T, int J, int BY, bool kOv, bool kInit = false>
__global__ __launch_bounds__(kBX * BY) void k_gm_oa(Op op, Vec<T> Z, Vec<T> Win, Vec<T> Wout, GmState* st,
                                                    double breakdown, const double* pin, int nblk_in, double* pout,
                                                    const int* active, int rpt) {
    static_assert(!kInit || J == 1, "the state set-up belongs to the first orthogonalise pass");
    const int b = blockIdx.z;
    const bool act = rhs_active(active, b);
    const int done = kInit ? 0 : st[b].arnoldi_done;
    double s0 = kInit ? 0.0 : st[b].s[0], beta0 = kInit ? 0.0 : st[b].beta;
    // previous pass: [||z_{J-1}||^2 (J > 1, or kInit)], <z_i, w_{J-1}>
    constexpr int KIN = kInit ? 3 : (J == 1) ? 2 : 5;
    const cplx<T>* z[J];
#pragma unroll
    for (int q = 0; q < J; ++q) z[q] = Z.p + (long long)(b * 4 + q) * Z.plane;
    cplx<T>* zJ = Z.p + (long long)(b * 4 + J) * Z.plane;
    const cplx<T>* wi = Win.rhs(b);
    cplx<T>* wo = Wout.p ? Wout.rhs(b) : nullptr;  // w_2 is stored only for a residual by recurrence
    // z_J = s_{J-1} w_{J-1} - sum_q c_q z_q with c_q = H[q][J-1] s_q, set by mid()
    T sJ1 = T(0);
    cplx<T> c[J];
    // the block leaves after the reduction if there is nothing to do (uniform in the block)
    auto mid = [&](const double (&t)[KIN]) -> bool {
        if (!act) return false;
        if constexpr (kInit) {  // as k_gm_a0: beta = ||z_0||, nothing to do for a zero residual
            beta0 = sqrt(t[0]);
            const bool go = beta0 > 0.0;
            s0 = go ? 1.0 / beta0 : 0.0;
            if (lead_thread()) {
                GmState& S = st[b];
                S.beta = beta0;
                S.s[0] = s0;
                S.k = go ? 3 : 0;
                S.arnoldi_done = go ? 0 : 1;
            }
            if (!go) return false;
        }
        if (done) return false;
        double sv[J];  // s_0 .. s_{J-1}
        sv[0] = s0;
        double hn = 0.0;
        bool broke = false;
        if (J > 1) {
            hn = sqrt(t[0]);
            broke = !(hn > breakdown * beta0);
            sv[J - 1] = broke ? 0.0 : 1.0 / hn;
        }
        constexpr int D0 = (J > 1 || kInit) ? 1 : 0;  // offset of the inner products in t
        double hr[J], hi[J];
#pragma unroll
        for (int q = 0; q < J; ++q) {
            hr[q] = sv[q] * sv[J - 1] * t[D0 + 2 * q];
            hi[q] = sv[q] * sv[J - 1] * t[D0 + 2 * q + 1];
        }
        if (lead_thread()) {
            GmState& S = st[b];
            if (J > 1) {
                S.hr[J - 1][J - 2] = hn;
                S.hi[J - 1][J - 2] = 0.0;
                if (broke) {
                    S.k = J - 1;
                    S.arnoldi_done = 1;
                } else {
                    S.s[J - 1] = sv[J - 1];
                }
            }
            if (!broke)
#pragma unroll
                for (int q = 0; q < J; ++q) {
                    S.hr[q][J - 1] = hr[q];
                    S.hi[q][J - 1] = hi[q];
                }
        }
        if (broke) return false;
        sJ1 = T(sv[J - 1]);
#pragma unroll
        for (int q = 0; q < J; ++q) c[q] = {T(hr[q] * sv[q]), T(hi[q] * sv[q])};
        return true;
    };
    // z_J at a tile node from w_{J-1} (v[0]) and z_0 .. z_{J-1} (v[1..J])
    auto zload = [&](long long q) {
        Vals<T, J + 1> o;
        o.v[0] = wi[q];
#pragma unroll
        for (int a = 0; a < J; ++a) o.v[1 + a] = z[a][q];
        return o;
    };
    auto zmake = [&](const Vals<T, J + 1>& o) {
        cplx<T> v = sJ1 * o.v[0];
#pragma unroll
        for (int a = 0; a < J; ++a) {
            const cplx<T> zq = o.v[1 + a];
            v.re -= c[a].re * zq.re - c[a].im * zq.im;
            v.im -= c[a].re * zq.im + c[a].im * zq.re;
        }
        return v;
    };
    constexpr int R = op_radius<Op>::value;
    // level 0, second pass of a single right-hand side: tiles in contiguous
    // runs per XCD (halo lines of its three tile arrays shared in one L2)
    constexpr bool kX = kOv && J == 2 && std::is_same<Op, FineOp<T>>::value;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    const Tile<R> tl = block_tile<R, kX>(rpt);
    if (!reduce_and_fill<KIN, kOv, T, R>(pin + b * kPartStride, nblk_in, lds, tl, op.g, zload, zmake, mid)) return;
    constexpr int KOUT = 1 + 2 * (J + 1) + (J == 2 ? 1 : 0);
    double acc[KOUT];
#pragma unroll
    for (int q = 0; q < KOUT; ++q) acc[q] = 0.0;
    auto zold = [&](long long q) {
        Vals<T, J> o;
#pragma unroll
        for (int a = 0; a < J; ++a) o.v[a] = z[a][q];
        return o;
    };
    apply_from_tile<Op, T, kX>(op, rpt, tl, lds, zold, [&](int, int, long long p, const Vals<T, J>& zo, cplx<T> zp,
                                                          cplx<T> w) {
        zJ[p] = zp;
        if (J == 1 || wo) wo[p] = w;
        acc[0] += dnorm2(zp);
#pragma unroll
        for (int q = 0; q < J; ++q) acc_dot(acc[1 + 2 * q], acc[2 + 2 * q], zo.v[q], w);
        acc_dot(acc[1 + 2 * J], acc[2 + 2 * J], zp, w);
        if constexpr (J == 2) acc[KOUT - 1] += dnorm2(w);
    });
    block_partials<KOUT, kX>(acc, pout + b * kPartStride);
}

// Pass 5: u += sum y_i s_i z_i.
template <typename T, int BY, bool kFromZero = false>
__global__ __launch_bounds__(kBX * BY) void k_gm_u(Grid g, Vec<T> Z, Vec<T> u, Vec<T> uin, const GmState* st,
                                                   double breakdown, const double* pin, int nblk_in, const int* active,
                                                   int rpt) {
    const int b = blockIdx.z;
    const bool act = rhs_active(active, b);
    cplx<T> c[3];
    const int k = gm_update_weights<T>(st, b, breakdown, pin, nblk_in, c);
    // in place (uin.p null) nothing changes for k = 0; from a separate uin or
    // from zero (kFromZero: the step began at u = 0, which u does not hold)
    // the iterate is always written
    if (!act || (k == 0 && !uin.p && !kFromZero)) return;
    const cplx<T>* z0 = Z.p + (long long)(b * 4) * Z.plane;
    const cplx<T>* z1 = z0 + Z.plane;
    const cplx<T>* z2 = z1 + Z.plane;
    cplx<T>* ub = u.rhs(b);
    const cplx<T>* ib = uin.p ? uin.rhs(b) : ub;
    constexpr int NB = sizeof(T) == 4 ? 8 : 4;
    cplx<T> xu[NB], x0[NB], x1[NB], x2[NB];
    for_nodes_batched<NB>(
        g, rpt,
        [&](int v, long long p) {
            if constexpr (kFromZero) xu[v] = {T(0), T(0)};
            else xu[v] = ib[p];
            x0[v] = z0[p];
            x1[v] = z1[p];
            x2[v] = z2[p];
        },
        [&](int v, int, int, long long p) {
            cplx<T> x = xu[v];
            if (k > 0) x = cfma(x, c[0], x0[v]);
            if (k > 1) x = cfma(x, c[1], x1[v]);
            if (k > 2) x = cfma(x, c[2], x2[v]);
            ub[p] = x;
        });
}

// Pass 5 of the last pre-smoothing step together with the residual that the
// restriction needs: u' = u + sum_i c_i z_i (in place; from u = 0 with
// kFromZero) and r' = z_0 - sum_i c_i w_i, with w_i = A z_i from the Arnoldi
// passes (w_0 in Wa, w_1 in Wb, w_2 in the fourth Arnoldi plane). As
// z_0 = f - A u, this is f - A u' exactly; the pass is pointwise (no stencil,
// no tile), so u' and r' may overwrite u and w_0 in place. Only the k terms of
// the Arnoldi columns in use enter.
template <typename T, int BY, bool kFromZero>
__global__ __launch_bounds__(kBX * BY) void k_gm_u_rr(Grid g, Vec<T> Z, Vec<T> u, Vec<T> Wa, Vec<T> Wb, Vec<T> r,
                                                      const GmState* st, double breakdown, const double* pin,
                                                      int nblk_in, const int* active, int rpt) {
    const int b = blockIdx.z;
    const bool act = rhs_active(active, b);
    cplx<T> c[3];
    const int k = gm_update_weights<T>(st, b, breakdown, pin, nblk_in, c);
    if (!act) return;
    const cplx<T>* z0 = Z.p + (long long)(b * 4) * Z.plane;
    const cplx<T>* z1 = z0 + Z.plane;
    const cplx<T>* z2 = z1 + Z.plane;
    const cplx<T>* w2 = z2 + Z.plane;
    const cplx<T>* w0 = Wa.rhs(b);
    const cplx<T>* w1 = Wb.rhs(b);
    cplx<T>* ub = u.rhs(b);
    cplx<T>* rb = r.rhs(b);
    cplx<T> mc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) mc[q] = {-c[q].re, -c[q].im};
    constexpr int NB = sizeof(T) == 4 ? 4 : 2;
    cplx<T> xu[NB], x0[NB], x1[NB], x2[NB], y0[NB], y1[NB], y2[NB];
    for_nodes_batched<NB>(
        g, rpt,
        [&](int v, long long p) {
            if constexpr (kFromZero) xu[v] = {T(0), T(0)};
            else xu[v] = ub[p];
            x0[v] = z0[p];
            x1[v] = z1[p];
            x2[v] = z2[p];
            y0[v] = w0[p];
            y1[v] = w1[p];
            y2[v] = w2[p];
        },
        [&](int v, int, int, long long p) {
            cplx<T> x = xu[v], rr = x0[v];
            if (k > 0) {
                x = cfma(x, c[0], x0[v]);
                rr = cfma(rr, mc[0], y0[v]);
            }
            if (k > 1) {
                x = cfma(x, c[1], x1[v]);
                rr = cfma(rr, mc[1], y1[v]);
            }
            if (k > 2) {
                x = cfma(x, c[2], x2[v]);
                rr = cfma(rr, mc[2], y2[v]);
            }
            ub[p] = x;
            rb[p] = rr;
        });
}

// Pass 5 of the last pre-smoothing step fused with the restriction of §4
// (one pass instead of k_gm_u_rr + k_restrict): this block owns the coarse
// tile of the coarse-grid geometry and the fine nodes 2I, 2I + 1 (both
// directions) of its coarse nodes I. Over the fine region the tile's
// restriction reads (the owned nodes and a halo of kH fine nodes), the
// residual r' = z_0 - sum_i c_i w_i of the updated iterate is formed by the
// recurrence of k_gm_u_rr and staged in LDS (zero off the grid, as the fine
// ghosts the separate restriction reads); the owned fine nodes also get
// u' = u + sum_i c_i z_i. Then fc = R r' from LDS, in k_restrict's order of
// operations (so both paths give the same bits), with uc = 0, and with zc
// set fc into the first coarse Arnoldi plane and partial sums of ||fc||^2.
template <bool kBez>
struct RestrictStage {
    static constexpr int kH = kBez ? 2 : 1;          // fine halo of the restriction
    static constexpr int TW = 2 * kBX - 1 + 2 * kH;  // staged fine columns
    __host__ __device__ static int rows(int coarse_rows) { return 2 * coarse_rows - 1 + 2 * kH; }
};

template <typename T, int BY, bool kFromZero, bool kBez>
__global__ __launch_bounds__(kBX * BY) void k_gm_u_restrict(Grid gf, Grid gc, Vec<T> Z, Vec<T> u, Vec<T> Wa,
                                                            Vec<T> Wb, const GmState* st, double breakdown,
                                                            const double* pin, int nblk_in, Vec<T> fc, Vec<T> uc,
                                                            Vec<T> Zc, double* pout, const int* active, int rpt) {
    using RS = RestrictStage<kBez>;
    constexpr int H = RS::kH;
    const int b = blockIdx.z;
    const bool act = rhs_active(active, b);
    cplx<T> c[3];
    const int k = gm_update_weights<T>(st, b, breakdown, pin, nblk_in, c);
    if (!act) return;
    const cplx<T>* z0 = Z.p + (long long)(b * 4) * Z.plane;
    const cplx<T>* z1 = z0 + Z.plane;
    const cplx<T>* z2 = z1 + Z.plane;
    const cplx<T>* w2 = z2 + Z.plane;
    const cplx<T>* w0 = Wa.rhs(b);
    const cplx<T>* w1 = Wb.rhs(b);
    cplx<T>* ub = u.rhs(b);
    cplx<T> mc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) mc[q] = {-c[q].re, -c[q].im};
    const BlockXY bt = block_xy();
    const int c0 = bt.x * kBX, r0 = bt.y * BY * rpt;
    const int fi0 = 2 * c0 - H, fj0 = 2 * r0 - H;  // fine node of LDS entry 0
    const int frows = RS::rows(BY * rpt);
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    constexpr int NB = sizeof(T) == 4 ? 8 : 4;  // measured: FP32 4, 12 and FP64 2 slower
    cplx<T> xu[NB], x0[NB], x1[NB], x2[NB], y0[NB], y1[NB], y2[NB];
    bool in[NB], own[NB];
    long long pp[NB];
    for_strided_batched<NB>(
        RS::TW * frows,
        [&](int v, int q) {
            const int di = q % RS::TW, dj = q / RS::TW;
            const int i = fi0 + di, j = fj0 + dj;
            in[v] = i >= 0 && i <= gf.n && j >= 0 && j <= gf.n;
            own[v] = in[v] && di >= H && di < H + 2 * kBX && dj >= H && dj < H + 2 * BY * rpt;
            pp[v] = gf.at(min(max(i, 0), gf.n), min(max(j, 0), gf.n));
            if (in[v]) {
                x0[v] = z0[pp[v]];
                y0[v] = w0[pp[v]];
                y1[v] = w1[pp[v]];
                y2[v] = w2[pp[v]];
            }
            if (own[v]) {
                if constexpr (kFromZero) xu[v] = {T(0), T(0)};
                else xu[v] = ub[pp[v]];
                x1[v] = z1[pp[v]];
                x2[v] = z2[pp[v]];
            }
        },
        [&](int v, int q) {
            cplx<T> rr{T(0), T(0)};
            if (in[v]) {
                rr = x0[v];
                if (k > 0) rr = cfma(rr, mc[0], y0[v]);
                if (k > 1) rr = cfma(rr, mc[1], y1[v]);
                if (k > 2) rr = cfma(rr, mc[2], y2[v]);
            }
            lds[q] = rr;
            if (own[v]) {
                cplx<T> x = xu[v];
                if (k > 0) x = cfma(x, c[0], x0[v]);
                if (k > 1) x = cfma(x, c[1], x1[v]);
                if (k > 2) x = cfma(x, c[2], x2[v]);
                ub[pp[v]] = x;
            }
        });
    __syncthreads();
    cplx<T>* fb = fc.rhs(b);
    cplx<T>* ucb = uc.p ? uc.rhs(b) : nullptr;
    cplx<T>* zb = Zc.p ? Zc.p + (long long)(b * 4) * Zc.plane : nullptr;
    double nrm[1] = {0.0};
    for_nodes(gc, rpt, [&](int I, int J, long long pc) {
        if (ucb) ucb[pc] = cplx<T>{T(0), T(0)};
        const int l = (2 * J - fj0) * RS::TW + (2 * I - fi0);
        cplx<T> acc{T(0), T(0)};
        cplx<T> v;
        if constexpr (kBez) {
            constexpr T w[5] = {T(1), T(4), T(6), T(4), T(1)};
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                cplx<T> row{T(0), T(0)};
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const cplx<T> x = lds[l + dy * RS::TW + dx];
                    row.re += w[dx + 2] * x.re;
                    row.im += w[dx + 2] * x.im;
                }
                acc.re += w[dy + 2] * row.re;
                acc.im += w[dy + 2] * row.im;
            }
            v = T(1.0 / 256.0) * acc;
        } else {
            constexpr T w[3] = {T(1), T(2), T(1)};
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                cplx<T> row{T(0), T(0)};
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const cplx<T> x = lds[l + dy * RS::TW + dx];
                    row.re += w[dx + 1] * x.re;
                    row.im += w[dx + 1] * x.im;
                }
                acc.re += w[dy + 1] * row.re;
                acc.im += w[dy + 1] * row.im;
            }
            v = T(1.0 / 16.0) * acc;
        }
        fb[pc] = v;
        if (zb) {
            zb[pc] = v;
            nrm[0] += dnorm2(v);
        }
    });
    if (zb) block_partials<1>(nrm, pout + b * kPartStride);
}

// Sums the nblk partial rows of a region into row 0 (same thread count and
// order as a consumer-side reduction, hence the same totals), so that the
// consumers of a large producer grid read one row.
template <int K>
__global__ __launch_bounds__(kThreads) void k_prereduce(double* part, int nblk, const int* active) {
    const int b = blockIdx.x;
    const bool act = rhs_active(active, b);
    double t[K];
    reduce_partials<K>(part + b * kPartStride, nblk, t);  // ends with barriers after every read
    if (act && thread_linear() == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) part[b * kPartStride + k] = t[k];
}

// ---------------------------------------------------------------- norms
template <typename Op, typename T, int BY>
__global__ __launch_bounds__(kBX * BY) void k_resnorm(Op op, Vec<T> x, Vec<T> f, double* pout, const int* active,
                                                      int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    double acc[1] = {0.0};
    for_nodes_applied_pre<Op, T>(op, rpt, [xb](long long q) { return xb[q]; }, Ident{},
                                 [fb](long long q) { return fb[q]; },
                                 [&](int, int, long long p, cplx<T> fp, cplx<T>, cplx<T> ax) {
                                     acc[0] += dnorm2(fp - ax);
                                 });
    block_partials<1>(acc, pout + b * kPartStride);
}

template <typename T, int BY>
__global__ __launch_bounds__(kBX * BY) void k_norm(Grid g, Vec<T> f, double* pout, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* fb = f.rhs(b);
    double acc[1] = {0.0};
    for_nodes(g, rpt, [&](int, int, long long p) { acc[0] += dnorm2(fb[p]); });
    block_partials<1>(acc, pout + b * kPartStride);
}

// One block per right-hand side: sum the partials of a norm kernel into
// norms[b].f2 (which = 0) or norms[b].r2 (which = 1), and take the stop test
// of a solve cycle on the latter when st.ring is set.
__global__ __launch_bounds__(kThreads) void k_sum_norms(const double* pin, int nblk_in, RhsNorms* norms, int which,
                                                        const int* active, StopTest st) {
    const int b = blockIdx.x;
    const bool act = rhs_active(active, b);
    double t[1];
    reduce_partials<1>(pin + b * kPartStride, nblk_in, t);
    if (act && thread_linear() == 0) {
        if (which == 0) {
            norms[b].f2 = t[0];
        } else {
            norms[b].r2 = t[0];
            if (st.ring) {
                const double f2 = norms[b].f2;
                const double r = sqrt(t[0] / f2);
                const double* lim = st.limits + 2 * b;
                const int stop = (!isfinite(r) || r > lim[1]) ? 2 : (r <= lim[0] ? 1 : 0);
                const int c = st.count[b] + 1;
                st.ring[((c - 1) % kReportRing) * st.stride + b] = RhsReport{f2, t[0], stop, c};
                st.count[b] = c;
                if (stop) st.active[b] = 0;
            }
        }
    }
}

// ---------------------------------------------------------------- refinement
// r32 = f - A_s x (complex64), partial sums of ||f - A_s x||^2 to pout. With
// Z.p set, r32 also goes to the first Arnoldi plane of the FP32 cycle that
// follows (z_0 = r32 - A 0) and the partial sums of ||z_0||^2 to pz, so that
// the cycle's first GMRES step starts with its second pass.
template <int BY>
__global__ __launch_bounds__(kBX * BY) void k_refine_residual(FineOp<double> op, Vec<double> x, Vec<double> f,
                                                              Vec<float> r32, Vec<float> Z, double* pout, double* pz,
                                                              const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* xb = x.rhs(b);
    const cplx<double>* fb = f.rhs(b);
    cplx<float>* rb = r32.rhs(b);
    cplx<float>* zb = Z.p ? Z.p + (long long)(b * 4) * Z.plane : nullptr;
    double acc[1] = {0.0}, accz[1] = {0.0};
    for_nodes_applied_pre<FineOp<double>, double>(op, rpt, [xb](long long q) { return xb[q]; }, Ident{},
                                                  [fb](long long q) { return fb[q]; },
                                                  [&](int, int, long long p, cplx<double> fp, cplx<double>,
                                                      cplx<double> ax) {
                                                  const cplx<double> r = fp - ax;
                                                  const cplx<float> r1 = cast<float>(r);
                                                  rb[p] = r1;
                                                  acc[0] += dnorm2(r);
                                                  if (zb) {
                                                      zb[p] = r1;
                                                      accz[0] += dnorm2(r1);
                                                  }
                                              });
    block_partials<1>(acc, pout + b * kPartStride);
    if (zb) block_partials<1>(accz, pz + b * kPartStride);
}

template <int BY>
__global__ __launch_bounds__(kBX * BY) void k_correct_residual(FineOp<double> op, Vec<double> x_in, Vec<float> e,
                                                               Vec<double> x_out, Vec<double> f, Vec<float> r32,
                                                               Vec<float> Z, double* pout, double* pz,
                                                               const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* xb = x_in.rhs(b);
    const cplx<float>* eb = e.rhs(b);
    cplx<double>* ob = x_out.rhs(b);
    const cplx<double>* fb = f.rhs(b);
    cplx<float>* rb = r32.rhs(b);
    cplx<float>* zb = Z.p ? Z.p + (long long)(b * 4) * Z.plane : nullptr;
    double acc[1] = {0.0}, accz[1] = {0.0};
    struct XE {
        cplx<double> x;
        cplx<float> e;
    };
    auto xload = [xb, eb](long long q) { return XE{xb[q], eb[q]}; };
    auto xmake = [](const XE& v) { return v.x + cast<double>(v.e); };
    for_nodes_applied_pre<FineOp<double>, double>(op, rpt, xload, xmake, [fb](long long q) { return fb[q]; },
                                                  [&](int, int, long long p, cplx<double> fp, cplx<double> xp,
                                                      cplx<double> ax) {
                                                  ob[p] = xp;
                                                  const cplx<double> r = fp - ax;
                                                  const cplx<float> r1 = cast<float>(r);
                                                  rb[p] = r1;
                                                  acc[0] += dnorm2(r);
                                                  if (zb) {
                                                      zb[p] = r1;
                                                      accz[0] += dnorm2(r1);
                                                  }
                                              });
    block_partials<1>(acc, pout + b * kPartStride);
    if (zb) block_partials<1>(accz, pz + b * kPartStride);
}

// The refinement residual pass (k_refine_residual, or k_correct_residual with
// kCorrect) together with the first apply pass of the FP32 cycle that follows
// it (k_gm_a0 on z_0 = r32): x (x_in + e with kCorrect) is staged with a halo
// of 2, r = f - A_s x in FP64 for the tile and a halo of 1 (the ring in the
// operator form of its owning tile), r32 = r as complex64 in LDS, then
// w_0 = A r32 with the FP32 operator of the cycle. Partial sums: ||r||^2
// (the stop test) to pout; ||r32||^2 and <r32, w_0> to pz, which the first
// orthogonalise pass of the cycle (kInit) reads in place of k_gm_a0's.
template <typename T>
struct RefineApplyStage {
    __host__ __device__ static size_t bytes(int rows) {
        return size_t(Tile<2>::TW) * (rows + 4) * sizeof(cplx<double>) +
               size_t(Tile<1>::TW) * (rows + 2) * sizeof(cplx<float>);
    }
};

template <int BY, bool kCorrect>
__global__ __launch_bounds__(kBX * BY) void k_residual_apply(FineOp<double> op, FineOp<float> op32, Vec<double> x_in,
                                                             Vec<float> e, Vec<double> x_out, Vec<double> f,
                                                             Vec<float> r32, Vec<float> Z, Vec<float> Wout,
                                                             double* pout, double* pz, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* xb = x_in.rhs(b);
    const cplx<float>* eb = kCorrect ? e.rhs(b) : nullptr;
    cplx<double>* ob = kCorrect ? x_out.rhs(b) : nullptr;
    const cplx<double>* fb = f.rhs(b);
    cplx<float>* rb = r32.rhs(b);
    cplx<float>* zb = Z.p + (long long)(b * 4) * Z.plane;
    cplx<float>* wb = Wout.rhs(b);
    const Tile<2> tx = block_tile<2>(rpt);
    const Tile<1> tz{tx.c0, tx.r0, tx.rows};
    cplx<double>* X = reinterpret_cast<cplx<double>*>(hm_dyn_lds);
    cplx<float>* ZL = reinterpret_cast<cplx<float>*>(X + Tile<2>::TW * (tx.rows + 4));
    struct XE {
        cplx<double> x;
        cplx<float> e;
    };
    fill_tile<double, 2>(
        X, tx, op.g,
        [&](long long q) { return XE{xb[q], kCorrect ? eb[q] : cplx<float>{0.0f, 0.0f}}; },
        [](const XE& v) { return kCorrect ? v.x + cast<double>(v.e) : v.x; });
    const int n = op.g.n;
    constexpr int XW = Tile<2>::TW, ZW = Tile<1>::TW;
    const int trows = int(blockDim.y) * rpt;
    auto owner_interior = [&](int i, int j) {
        const int oc = (i / kBX) * kBX, orow = (j / trows) * trows;
        return oc >= 1 && oc + kBX <= n && orow >= 1 && orow + trows <= n;
    };
    auto ax_at = [&](int i, int j, double kk, bool inner) {
        const int l = tx.at(i, j);
        return inner ? op.apply5k_interior(kk, X[l], X[l - 1], X[l + 1], X[l - XW], X[l + XW])
                     : op.apply5k(i, j, kk, X[l], X[l - 1], X[l + 1], X[l - XW], X[l + XW]);
    };
    // r32 on the halo ring (top and bottom rows, then the left and right
    // columns); each thread's first ring node has its operands loaded with
    // those of its tile nodes, further ones after them
    const int ring = 2 * ZW + 2 * tx.rows;
    auto ring_node = [&](int q, int& i, int& j) {
        if (q < 2 * ZW) {
            i = tx.c0 - 1 + q % ZW;
            j = q < ZW ? tx.r0 - 1 : tx.r0 + tx.rows;
        } else {
            const int m = q - 2 * ZW;
            i = (m & 1) ? tx.c0 + kBX : tx.c0 - 1;
            j = tx.r0 + (m >> 1);
        }
    };
    auto ring_r = [&](int i, int j, double kk, cplx<double> fp) {
        cplx<float> z{0.0f, 0.0f};
        if (i >= 0 && j >= 0 && i <= n && j <= n) z = cast<float>(fp - ax_at(i, j, kk, owner_interior(i, j)));
        ZL[tz.at(i, j)] = z;
    };
    const int tid = thread_linear(), nt = int(blockDim.x * blockDim.y);
    int ri = 0, rj = 0;
    double rk = 0.0;
    cplx<double> rf{0.0, 0.0};
    if (tid < ring) {
        ring_node(tid, ri, rj);
        const long long p = op.g.at(min(max(ri, 0), n), min(max(rj, 0), n));
        rk = op.k2[p];
        rf = fb[p];
    }
    // the tile, in the thread order of the residual pass; each thread first
    // zeroes its own tile positions (those off the grid stay zero)
    for (int rr = 0; rr < rpt; ++rr)
        ZL[tz.at(tx.c0 + int(threadIdx.x), tx.r0 + rr * int(blockDim.y) + int(threadIdx.y))] = cplx<float>{0.0f, 0.0f};
    const bool interior = tx.c0 >= 1 && tx.c0 + kBX <= n && tx.r0 >= 1 && tx.r0 + tx.rows <= n;
    double acc[1] = {0.0}, acz[3] = {0.0, 0.0, 0.0};
    {
        constexpr int NB = 4;
        cplx<double> pv[NB];
        double kk[NB];
        for_nodes_batched<NB>(
            op.g, rpt,
            [&](int v, long long p) {
                pv[v] = fb[p];
                kk[v] = op.k2[p];
            },
            [&](int v, int i, int j, long long p) {
                const cplx<double> r = pv[v] - ax_at(i, j, kk[v], interior);
                if constexpr (kCorrect) ob[p] = X[tx.at(i, j)];
                const cplx<float> r1 = cast<float>(r);
                rb[p] = r1;
                zb[p] = r1;
                ZL[tz.at(i, j)] = r1;
                acc[0] += dnorm2(r);
                acz[0] += dnorm2(r1);
            });
    }
    if (tid < ring) ring_r(ri, rj, rk, rf);
    for (int q = tid + nt; q < ring; q += nt) {
        int i, j;
        ring_node(q, i, j);
        const long long p = op.g.at(min(max(i, 0), n), min(max(j, 0), n));
        ring_r(i, j, op.k2[p], fb[p]);
    }
    __syncthreads();
    {  // w_0 = A r32 with the FP32 operator, in the thread order of the apply pass
        constexpr int NB = 8;
        float kk[NB];
        for_nodes_batched<NB>(
            op32.g, rpt, [&](int v, long long p) { kk[v] = op32.k2[p]; },
            [&](int v, int i, int j, long long p) {
                const int l = tz.at(i, j);
                const cplx<float> zp = ZL[l];
                const cplx<float> w =
                    interior ? op32.apply5k_interior(kk[v], zp, ZL[l - 1], ZL[l + 1], ZL[l - ZW], ZL[l + ZW])
                             : op32.apply5k(i, j, kk[v], zp, ZL[l - 1], ZL[l + 1], ZL[l - ZW], ZL[l + ZW]);
                wb[p] = w;
                acc_dot(acz[1], acz[2], zp, w);
            });
    }
    block_partials<1>(acc, pout + b * kPartStride);
    block_partials<3>(acz, pz + b * kPartStride);
}

// ---------------------------------------------------------------- layout
template <typename T, typename S, int BY>
__global__ __launch_bounds__(kBX * BY) void k_copy_in(Grid g, const cplx<S>* src, Vec<T> dst, int scale_w,
                                                      int conj_, int rpt) {
    const int b = blockIdx.z;
    const long long m = g.n + 1;
    const cplx<S>* sb = src + b * m * m;
    cplx<T>* db = dst.rhs(b);
    for_nodes(g, rpt, [&](int i, int j, long long p) {
        cplx<T> v = cast<T>(sb[(long long)j * m + i]);
        if (scale_w) v = (line_w<T>(i, g.n) * line_w<T>(j, g.n)) * v;
        if (conj_) v.im = -v.im;
        db[p] = v;
    });
}

template <typename T, typename S, int BY>
__global__ __launch_bounds__(kBX * BY) void k_copy_out(Grid g, Vec<T> src, cplx<S>* dst, int scale_w, int conj_,
                                                       int rpt) {
    const int b = blockIdx.z;
    const long long m = g.n + 1;
    const cplx<T>* sb = src.rhs(b);
    cplx<S>* db = dst + b * m * m;
    for_nodes(g, rpt, [&](int i, int j, long long p) {
        cplx<T> v = sb[p];
        if (scale_w) v = (line_w<T>(i, g.n) * line_w<T>(j, g.n)) * v;
        if (conj_) v.im = -v.im;
        db[(long long)j * m + i] = cast<S>(v);
    });
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero(cplx<T>* p, long long count) {
    for (long long q = blockIdx.x * (long long)kThreads + threadIdx.x; q < count; q += (long long)gridDim.x * kThreads)
        p[q] = cplx<T>{T(0), T(0)};
}

__global__ __launch_bounds__(kThreads) void k_fill_words(unsigned* p, long long words, unsigned value) {
    for (long long q = blockIdx.x * (long long)kThreads + threadIdx.x; q < words; q += (long long)gridDim.x * kThreads)
        p[q] = value;
}

// ---------------------------------------------------------------- gradient
// dL/dk^2_p = sum_b Re[ mu_b,p W_p (1 + i s_p / (h k_p)) u_b,p ], mu = conj(lambda).
__global__ __launch_bounds__(kThreads) void k_grad_k2(Grid g, double h, const double* k2, Vec<double> u,
                                                      Vec<double> mu, double* out, int nrhs, int rpt) {
    const long long m = g.n + 1;
    for_nodes(g, rpt, [&](int i, int j, long long p) {
        const int n = g.n;
        const double W = line_w<double>(i, n) * line_w<double>(j, n);
        const int s = (i == 0 || i == n) + (j == 0 || j == n);
        // imaginary part of 1 + i s/(h k); zero where k = 0 (as 1/(h k) -> 0
        // is taken there; setup rejects k = 0 on the boundary anyway)
        const double kk = k2[p];
        const double bi = (s && kk > 0.0) ? double(s) / (h * sqrt(kk)) : 0.0;
        double acc = 0.0;
        for (int b = 0; b < nrhs; ++b) {
            const cplx<double> t = mu.rhs(b)[p] * u.rhs(b)[p];
            acc += W * (t.re - bi * t.im);
        }
        out[(long long)j * m + i] = acc;
    });
}

}  // namespace

// ======================================================================= launchers
#define HM_ACTIVE ctx.active

// Launches KERNEL<..., BY> with the geometry q (BY = q.by).
#define HM_LAUNCH(q, KERNEL_BY, ...)                                                                       \
    with_by((q).by, [&](auto byc) {                                                                        \
        constexpr int BY = decltype(byc)::value;                                                          \
        hipLaunchKernelGGL(KERNEL_BY, (q).grid, (q).block, 0, ctx.stream, __VA_ARGS__);                   \
    })
// Same for kernels templated on an operator type Op (heavy operators: short
// blocks only; Galerkin levels get their LDS tile as dynamic shared memory).
#define HM_LAUNCH_OP(q, KERNEL_BY, ...)                                                                    \
    with_by<Op::kHeavy>((q).by, [&](auto byc) {                                                            \
        constexpr int BY = decltype(byc)::value;                                                          \
        const size_t shm_ = tile_bytes<Op, T>((q).by, (q).rpt);                                           \
        hipLaunchKernelGGL(KERNEL_BY, (q).grid, (q).block, shm_, ctx.stream, __VA_ARGS__);                \
    })

template <typename T>
void launch_apply(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> y) {
    with_op(lop, [&](auto op) {
        using Op = decltype(op);
        const Geom q = geom_op<Op, T>(lop.g, ctx);
        HM_LAUNCH_OP(q, (k_apply<Op, T, BY>), op, x, y, HM_ACTIVE, q.rpt);
    });
}

void launch_apply_widened(const LaunchCtx& ctx, const LevelOp<double>& lop, Vec<float> xs, Vec<double> x,
                          Vec<double> y) {
    using Op = FineOp<double>;
    using T = double;
    const Op op{lop.g, lop.k2, 1.0 / (lop.h * lop.h), 2.0 / lop.h};
    const Geom q = geom_op<Op, T>(lop.g, ctx);
    HM_LAUNCH_OP(q, (k_apply_widened<BY>), op, xs, x, y, HM_ACTIVE, q.rpt);
}

template <typename T>
void launch_residual(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> f, Vec<T> r) {
    with_op(lop, [&](auto op) {
        using Op = decltype(op);
        const Geom q = geom_op<Op, T>(lop.g, ctx);
        HM_LAUNCH_OP(q, (k_residual<Op, T, BY>), op, x, f, r, HM_ACTIVE, q.rpt);
    });
}

template <typename T>
void launch_jacobi(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> f, Vec<T> y, double inv_omega) {
    with_op(lop, [&](auto op) {
        using Op = decltype(op);
        const Geom q = geom_op<Op, T>(lop.g, ctx);
        HM_LAUNCH_OP(q, (k_jacobi<Op, T, BY>), op, x, f, y, T(inv_omega), HM_ACTIVE, q.rpt);
    });
}

template <typename T>
bool launch_jacobi2(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> f, Vec<T> y, double inv_omega) {
    bool done = false;
    with_op(lop, [&](auto op) {
        using Op = decltype(op);
        if constexpr (std::is_same<Op, FineOp<T>>::value) {
            Geom q = geom(lop.g, Op::kHeavy, ctx);
            // rows per thread lowered until both LDS stages fit the tile bound
            auto bytes = [&](int rpt) { return Jacobi2Stage::values(q.by * rpt) * sizeof(cplx<T>); };
            while (q.rpt > 1 && bytes(q.rpt) > kMaxTileBytes) --q.rpt;
            q.grid = level_grid(lop.g, q.rpt, ctx.nrhs, q.by, ctx.nrhs_cap > 1);
            if (bytes(q.rpt) <= kMaxTileBytes) {
                with_by(q.by, [&](auto byc) {
                    constexpr int BY = decltype(byc)::value;
                    hipLaunchKernelGGL((k_jacobi2<T, BY>), q.grid, q.block, bytes(q.rpt), ctx.stream, op, x, f, y,
                                       T(inv_omega), HM_ACTIVE, q.rpt);
                });
                done = true;
            }
        }
    });
    return done;
}

double* region(const LaunchCtx& ctx, int r);

template <typename T>
int launch_restrict(const LaunchCtx& ctx, Grid fine, Grid coarse, int transfer, Vec<T> r, Vec<T> fc, Vec<T> uc,
                    Vec<T> z0) {
    const Geom q = geom(coarse, false, ctx);
    double* pout = z0.p ? region(ctx, 0) : nullptr;
    if (transfer == 0) HM_LAUNCH(q, (k_restrict<T, true, BY>), fine, coarse, r, fc, uc, z0, pout, HM_ACTIVE, q.rpt);
    else HM_LAUNCH(q, (k_restrict<T, false, BY>), fine, coarse, r, fc, uc, z0, pout, HM_ACTIVE, q.rpt);
    return q.nblk;
}

template <typename T>
void launch_prolong_add(const LaunchCtx& ctx, Grid coarse, Grid fine, int transfer, Vec<T> e, Vec<T> u) {
    Geom q = geom(fine, false, ctx);
    // the coarse tile is dynamic shared memory: rows per thread lowered until
    // it fits the same bound as the operator tiles
    auto bytes = [&](int rpt) { return size_t(kProlongTW) * prolong_rows(q.by * rpt) * sizeof(cplx<T>); };
    if (bytes(q.rpt) > kMaxTileBytes) {
        while (q.rpt > 1 && bytes(q.rpt) > kMaxTileBytes) --q.rpt;
        q.grid = level_grid(fine, q.rpt, ctx.nrhs, q.by, ctx.nrhs_cap > 1);
        q.nblk = int(q.grid.x * q.grid.y);
    }
    const size_t shm = bytes(q.rpt);
    with_by(q.by, [&](auto byc) {
        constexpr int BY = decltype(byc)::value;
        if (transfer == 0)
            hipLaunchKernelGGL((k_prolong_add<T, true, BY>), q.grid, q.block, shm, ctx.stream, coarse, fine, e, u,
                               HM_ACTIVE, q.rpt);
        else
            hipLaunchKernelGGL((k_prolong_add<T, false, BY>), q.grid, q.block, shm, ctx.stream, coarse, fine, e, u,
                               HM_ACTIVE, q.rpt);
    });
}

double* region(const LaunchCtx& ctx, int r) { return ctx.partials + (long long)r * ctx.nrhs_cap * kPartStride; }

// On batch handles, partial sums of producers with more blocks than this per
// right-hand side are pre-reduced before their consumers.
constexpr int kBatchPrereduceBlocks = 32;

// The pending update pass of a coarse level's last smoothing step, launched
// on its own (where the correction that would form it on the fly does not fit).
template <typename T>
void launch_deferred_update(const LaunchCtx& ctx, Grid gc, const DeferredUpdate<T>& du) {
    const Geom qv = geom(gc, false, ctx);
    HM_LAUNCH(qv, (k_gm_u<T, BY>), gc, du.Z, du.u, du.uin, du.st, du.breakdown, du.part, du.nblk, HM_ACTIVE, qv.rpt);
}

// Level grids of at most this many blocks per right-hand side are resident
// on the GPU at once when solved alone (256 compute units, several blocks each).
constexpr int kOverlapMaxBlocks = 2048;

template <typename T>
void launch_gmres_step(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> u, Vec<T> f, Vec<T> Z, Vec<T> Wa,
                       Vec<T> Wb, GmState* st, double breakdown, const hipEvent_t* timed,
                       Vec<T> res, int r_ready_nblk, ProlongIn<T> pro, bool u_zero, RestrictOut<T>* rout,
                       DeferredUpdate<T>* defer, bool w_ready) {
    // partial sums: each pass reads the region its producer wrote and writes the
    // other one (blocks of a pass still read while others write)
    double* A = region(ctx, 0);
    double* B = region(ctx, 1);
    if (defer) *defer = DeferredUpdate<T>{};
    const Geom qv = geom(lop.g, false, ctx);  // vector-only passes
    int nb_op = 0;
    Vec<T> uin{nullptr, 0};  // iterate the update pass starts from, when not u itself
    with_op(lop, [&](auto op) {
        using Op = decltype(op);
        const Geom q = geom_op<Op, T>(lop.g, ctx);
        nb_op = q.nblk;
        // consumers read the producer's partials directly, or one pre-reduced row
        // (and on handles for batches: every block of a consumer reads all of
        // its right-hand side's partial sums, which for B right-hand sides of
        // nblk blocks each is B nblk^2 values per pass; one block per
        // right-hand side pre-reduces them instead. Solo solves on such a
        // handle take the same path and keep matching batch members bit for bit.)
        const bool pre = q.nblk > ctx.block_cap || (ctx.nrhs_cap > 1 && q.nblk > kBatchPrereduceBlocks);
        const int nb = pre ? 1 : q.nblk;
        auto prereduce = [&](double* part, auto kc) {
            if (pre)
                hipLaunchKernelGGL((k_prereduce<decltype(kc)::value>), dim3(ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream,
                                   part, q.nblk, HM_ACTIVE);
        };
        int nb_r = nb;
        // fused coarse grid correction: its LDS stage must fit beside the operator's
        constexpr int R = op_radius<Op>::value;
        const size_t pro_bytes = tile_bytes<Op, T>(q.by, q.rpt) +
                                 size_t(ProlongTile<R>::EW) * ProlongTile<R>::rows(q.by * q.rpt) * sizeof(cplx<T>);
        const bool fuse_pro = pro.e.p && ctx.fuse_correction && pro_bytes <= kMaxTileBytes;
        const DeferredUpdate<T>& du = pro.du;
        if (pro.e.p && !fuse_pro) {
            if (du.Z.p) launch_deferred_update<T>(ctx, pro.gc, du);
            launch_prolong_add<T>(ctx, pro.gc, lop.g, pro.transfer, pro.e, u);
        }
        bool r_a0 = false;  // the correction pass also applied A to z_0 (partials: ||z_0||^2, <z_0, w_0>)
        if (fuse_pro) {
            const bool d = du.Z.p != nullptr;
            if constexpr (std::is_same<Op, FineOp<T>>::value && sizeof(T) == 4) {
                const size_t ra_bytes = ResApplyStage<T>::bytes(q.by * q.rpt);
                if (ctx.fuse_r_a0 && !rout && ra_bytes <= kMaxTileBytes) {
                    with_by(q.by, [&](auto byc) {
                        constexpr int BY = decltype(byc)::value;
                        auto go = [&](auto kern) {
                            hipLaunchKernelGGL(kern, q.grid, q.block, ra_bytes, ctx.stream, op, pro.gc, pro.e, u, f,
                                               pro.xt, Z, Wa, A, HM_ACTIVE, q.rpt, du);
                        };
                        if (pro.transfer == 0 && d) go(k_gm_r_pro_a0<T, true, BY, true>);
                        else if (pro.transfer == 0) go(k_gm_r_pro_a0<T, true, BY, false>);
                        else if (d) go(k_gm_r_pro_a0<T, false, BY, true>);
                        else go(k_gm_r_pro_a0<T, false, BY, false>);
                    });
                    prereduce(A, std::integral_constant<int, 3>{});
                    // region 1 may hold the pending coarse update's sums, which the
                    // pass reads, so it wrote region 0; the step's later passes
                    // run with the two regions swapped (its last sums, which the
                    // update pass reads, end in region 0)
                    std::swap(A, B);
                    r_a0 = true;
                }
            }
            if (!r_a0) {
                with_by<Op::kHeavy>(q.by, [&](auto byc) {
                    constexpr int BY = decltype(byc)::value;
                    auto go = [&](auto kern) {
                        hipLaunchKernelGGL(kern, q.grid, q.block, pro_bytes, ctx.stream, op, pro.gc, pro.e, u, f,
                                           pro.xt, Z, A, HM_ACTIVE, q.rpt, du);
                    };
                    if (pro.transfer == 0 && d) go(k_gm_r_pro<Op, T, true, BY, true>);
                    else if (pro.transfer == 0) go(k_gm_r_pro<Op, T, true, BY, false>);
                    else if (d) go(k_gm_r_pro<Op, T, false, BY, true>);
                    else go(k_gm_r_pro<Op, T, false, BY, false>);
                });
                prereduce(A, std::integral_constant<int, 1>{});
            }
            uin = pro.xt;
        } else if (r_ready_nblk > 0) {
            // u = 0: z_0 = f and its partial norms were written by the restriction
            // (or the refinement residual pass; with w_ready that pass also
            // formed w_0 = A z_0, its sums ||z_0||^2 and <z_0, w_0> in region 1)
            nb_r = r_ready_nblk;
            if (r_ready_nblk > ctx.block_cap || (ctx.nrhs_cap > 1 && r_ready_nblk > kBatchPrereduceBlocks)) {
                if (w_ready)
                    hipLaunchKernelGGL((k_prereduce<3>), dim3(ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, B,
                                       r_ready_nblk, HM_ACTIVE);
                else
                    hipLaunchKernelGGL((k_prereduce<1>), dim3(ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, A,
                                       r_ready_nblk, HM_ACTIVE);
                nb_r = 1;
            }
        } else {
            HM_LAUNCH_OP(q, (k_gm_r<Op, T, BY>), op, u, f, Z, A, HM_ACTIVE, q.rpt);
            prereduce(A, std::integral_constant<int, 1>{});
        }
        // handles of a single right-hand side overlap the reduction with the
        // tile loads (see reduce_and_fill) and give the second orthogonalise
        // pass of level 0 the XCD tile map; handles for batches keep the
        // reduce-first order and the plain map, which measured faster once a
        // launch queues several rounds of blocks. The choice follows the
        // handle, not the call, so a batch member runs the same code as a solo
        // solve on the same handle and matches it bit for bit.
        const bool ov = ctx.nrhs_cap == 1 && q.nblk <= kOverlapMaxBlocks;
        const bool w0_made = r_a0 || (w_ready && r_ready_nblk > 0 && !fuse_pro);
        if (w0_made) {  // only the level-0 operator of FP32 cycles takes this branch
            if constexpr (std::is_same<Op, FineOp<T>>::value && sizeof(T) == 4) {
                const int nb_in = r_a0 ? nb : nb_r;
                if (ov) HM_LAUNCH_OP(q, (k_gm_oa<Op, T, 1, BY, true, true>), op, Z, Wa, Wb, st, breakdown, B, nb_in,
                                     A, HM_ACTIVE, q.rpt);
                else HM_LAUNCH_OP(q, (k_gm_oa<Op, T, 1, BY, false, true>), op, Z, Wa, Wb, st, breakdown, B, nb_in,
                                  A, HM_ACTIVE, q.rpt);
            }
        } else {
            if (ov) HM_LAUNCH_OP(q, (k_gm_a0<Op, T, BY, true>), op, Z, Wa, st, A, nb_r, B, HM_ACTIVE, q.rpt);
            else HM_LAUNCH_OP(q, (k_gm_a0<Op, T, BY, false>), op, Z, Wa, st, A, nb_r, B, HM_ACTIVE, q.rpt);
            prereduce(B, std::integral_constant<int, 2>{});
            if (ov) HM_LAUNCH_OP(q, (k_gm_oa<Op, T, 1, BY, true>), op, Z, Wa, Wb, st, breakdown, B, nb, A, HM_ACTIVE,
                                 q.rpt);
            else HM_LAUNCH_OP(q, (k_gm_oa<Op, T, 1, BY, false>), op, Z, Wa, Wb, st, breakdown, B, nb, A, HM_ACTIVE,
                              q.rpt);
        }
        prereduce(A, std::integral_constant<int, 5>{});
        // w_2 is kept (in the fourth Arnoldi plane, w_0 stays in Wa) only for a
        // residual by recurrence
        const Vec<T> w2 = res.p ? Vec<T>{Z.p + 3 * Z.plane, 4 * Z.plane} : Vec<T>{nullptr, 0};
        if (timed) {
            with_by<Op::kHeavy>(q.by, [&](auto byc) {
                constexpr int BY = decltype(byc)::value;
                if (ov)
                    hipExtLaunchKernelGGL((k_gm_oa<Op, T, 2, BY, true>), q.grid, q.block,
                                          uint32_t(tile_bytes<Op, T>(q.by, q.rpt)), ctx.stream, timed[0], timed[1],
                                          0u, op, Z, Wb, w2, st, breakdown, (const double*)A, nb, B,
                                          (const int*)HM_ACTIVE, q.rpt);
                else
                    hipExtLaunchKernelGGL((k_gm_oa<Op, T, 2, BY, false>), q.grid, q.block,
                                          uint32_t(tile_bytes<Op, T>(q.by, q.rpt)), ctx.stream, timed[0], timed[1],
                                          0u, op, Z, Wb, w2, st, breakdown, (const double*)A, nb, B,
                                          (const int*)HM_ACTIVE, q.rpt);
            });
        } else {
            if (ov) HM_LAUNCH_OP(q, (k_gm_oa<Op, T, 2, BY, true>), op, Z, Wb, w2, st, breakdown, A, nb, B, HM_ACTIVE, q.rpt);
            else HM_LAUNCH_OP(q, (k_gm_oa<Op, T, 2, BY, false>), op, Z, Wb, w2, st, breakdown, A, nb, B, HM_ACTIVE, q.rpt);
        }
        prereduce(B, std::integral_constant<int, 8>{});
        nb_op = nb;
    });
    if (rout) rout->nblk = 0;
    if (res.p && rout && ctx.fuse_restrict) {
        // update + restriction in one pass on the coarse grid; rows per thread
        // lowered until the staged fine region fits the tile bound
        Geom qr = geom(rout->gc, false, ctx);
        const bool bez = rout->transfer == 0;
        auto bytes = [&](int rpt) {
            return size_t(bez ? RestrictStage<true>::TW : RestrictStage<false>::TW) *
                   (bez ? RestrictStage<true>::rows(qr.by * rpt) : RestrictStage<false>::rows(qr.by * rpt)) *
                   sizeof(cplx<T>);
        };
        if (bytes(qr.rpt) > kMaxTileBytes) {
            while (qr.rpt > 1 && bytes(qr.rpt) > kMaxTileBytes) --qr.rpt;
            qr.grid = level_grid(rout->gc, qr.rpt, ctx.nrhs, qr.by, ctx.nrhs_cap > 1);
            qr.nblk = int(qr.grid.x * qr.grid.y);
        }
        const size_t shm = bytes(qr.rpt);
        const Grid gf = lop.g, gc = rout->gc;
        const RestrictOut<T>& ro = *rout;
        with_by(qr.by, [&](auto byc) {
            constexpr int BY = decltype(byc)::value;
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, qr.grid, qr.block, shm, ctx.stream, gf, gc, Z, u, Wa, Wb, st, breakdown,
                                   (const double*)B, nb_op, ro.fc, ro.uc, ro.zc, A, HM_ACTIVE, qr.rpt);
            };
            if (u_zero && bez) go(k_gm_u_restrict<T, BY, true, true>);
            else if (u_zero) go(k_gm_u_restrict<T, BY, true, false>);
            else if (bez) go(k_gm_u_restrict<T, BY, false, true>);
            else go(k_gm_u_restrict<T, BY, false, false>);
        });
        rout->nblk = qr.nblk;
    } else if (res.p && u_zero)
        HM_LAUNCH(qv, (k_gm_u_rr<T, BY, true>), lop.g, Z, u, Wa, Wb, res, st, breakdown, B, nb_op, HM_ACTIVE, qv.rpt);
    else if (res.p)
        HM_LAUNCH(qv, (k_gm_u_rr<T, BY, false>), lop.g, Z, u, Wa, Wb, res, st, breakdown, B, nb_op, HM_ACTIVE,
                  qv.rpt);
    else if (u_zero)
        HM_LAUNCH(qv, (k_gm_u<T, BY, true>), lop.g, Z, u, uin, st, breakdown, B, nb_op, HM_ACTIVE, qv.rpt);
    else if (defer)
        *defer = DeferredUpdate<T>{Z, u, uin, st, B, nb_op, breakdown};
    else
        HM_LAUNCH(qv, (k_gm_u<T, BY>), lop.g, Z, u, uin, st, breakdown, B, nb_op, HM_ACTIVE, qv.rpt);
}

void launch_sum_norms(const LaunchCtx& ctx, int nb, RhsNorms* norms, int which, int reg = 0) {
    // 64 x 4 threads: the block reduction indexes wavefronts by threadIdx.y
    hipLaunchKernelGGL(k_sum_norms, dim3(ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, region(ctx, reg), nb, norms,
                       which, HM_ACTIVE, which == 1 ? ctx.stop : StopTest{});
}

template <typename T>
void launch_resnorm(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> f, RhsNorms* norms) {
    int nb = 0;
    with_op(lop, [&](auto op) {
        using Op = decltype(op);
        const Geom q = geom_op<Op, T>(lop.g, ctx);
        nb = q.nblk;
        HM_LAUNCH_OP(q, (k_resnorm<Op, T, BY>), op, x, f, region(ctx, 0), HM_ACTIVE, q.rpt);
    });
    launch_sum_norms(ctx, nb, norms, 1);
}

template <typename T>
void launch_norm(const LaunchCtx& ctx, Grid g, Vec<T> f, RhsNorms* norms) {
    const Geom q = geom(g, false, ctx);
    HM_LAUNCH(q, (k_norm<T, BY>), g, f, region(ctx, 0), HM_ACTIVE, q.rpt);
    launch_sum_norms(ctx, q.nblk, norms, 0);
}

namespace {
// The fused refinement residual + apply pass takes the level's operator
// geometry with the rows per thread lowered until its two LDS stages fit (the
// taller tiles of batch handles do not): it hands its partial sums to the
// next pass with their own block count.
Geom refine_apply_geom(const LaunchCtx& ctx, Grid g) {
    Geom q = geom_op<FineOp<double>, double>(g, ctx);
    if (RefineApplyStage<double>::bytes(q.by * q.rpt) > kMaxTileBytes) {
        while (q.rpt > 1 && RefineApplyStage<double>::bytes(q.by * q.rpt) > kMaxTileBytes) --q.rpt;
        q.grid = level_grid(g, q.rpt, ctx.nrhs, q.by, ctx.nrhs_cap > 1);
        q.nblk = int(q.grid.x * q.grid.y);
    }
    return q;
}
}  // namespace

bool refine_apply_fits(const LaunchCtx& ctx, Grid g) {
    const Geom q = refine_apply_geom(ctx, g);
    return RefineApplyStage<double>::bytes(q.by * q.rpt) <= kMaxTileBytes && q.nblk <= kMaxPartialBlocks;
}

namespace {
// The fused refinement residual + apply pass (w0.p set): residual norms to
// region 0, z_0's sums (||z_0||^2, <z_0, w_0>) to region 1.
template <bool kCorrect>
int launch_residual_apply(const LaunchCtx& ctx, const LevelOp<double>& lop, const float* k2_32, Vec<double> x_in,
                          Vec<float> e, Vec<double> x_out, Vec<double> f, Vec<float> r32, RhsNorms* norms,
                          Vec<float> z0, Vec<float> w0) {
    const Geom q = refine_apply_geom(ctx, lop.g);
    const FineOp<double> op{lop.g, lop.k2, 1.0 / (lop.h * lop.h), 2.0 / lop.h};
    const FineOp<float> op32{lop.g, k2_32, float(1.0 / (lop.h * lop.h)), float(2.0 / lop.h)};
    const size_t shm = RefineApplyStage<double>::bytes(q.by * q.rpt);
    with_by(q.by, [&](auto byc) {
        constexpr int BY = decltype(byc)::value;
        hipLaunchKernelGGL((k_residual_apply<BY, kCorrect>), q.grid, q.block, shm, ctx.stream, op, op32, x_in, e,
                           x_out, f, r32, z0, w0, region(ctx, 0), region(ctx, 1), HM_ACTIVE, q.rpt);
    });
    launch_sum_norms(ctx, q.nblk, norms, 1, 0);
    return q.nblk;
}
}  // namespace

// With z0.p set the residual norms use region 1 and z_0's region 0 (where the
// first GMRES step of the next FP32 cycle reads them); with w0.p set as well
// (refine_apply_fits) the pass also forms w_0 = A z_0, the norms use region 0
// and z_0's sums region 1 (see k_residual_apply).
int launch_refine_residual(const LaunchCtx& ctx, const LevelOp<double>& lop, Vec<double> x, Vec<double> f,
                           Vec<float> r32, RhsNorms* norms, Vec<float> z0, const float* k2_32, Vec<float> w0) {
    if (z0.p && w0.p)
        return launch_residual_apply<false>(ctx, lop, k2_32, x, Vec<float>{nullptr, 0}, Vec<double>{nullptr, 0}, f,
                                            r32, norms, z0, w0);
    using Op = FineOp<double>;
    using T = double;
    const Geom q = geom_op<Op, T>(lop.g, ctx);
    FineOp<double> op{lop.g, lop.k2, 1.0 / (lop.h * lop.h), 2.0 / lop.h};
    const int rn = z0.p ? 1 : 0;
    HM_LAUNCH_OP(q, (k_refine_residual<BY>), op, x, f, r32, z0, region(ctx, rn), region(ctx, 0), HM_ACTIVE, q.rpt);
    launch_sum_norms(ctx, q.nblk, norms, 1, rn);
    return q.nblk;
}

int launch_correct_residual(const LaunchCtx& ctx, const LevelOp<double>& lop, Vec<double> x_in, Vec<float> e,
                            Vec<double> x_out, Vec<double> f, Vec<float> r32, RhsNorms* norms, Vec<float> z0,
                            const float* k2_32, Vec<float> w0) {
    if (z0.p && w0.p)
        return launch_residual_apply<true>(ctx, lop, k2_32, x_in, e, x_out, f, r32, norms, z0, w0);
    using Op = FineOp<double>;
    using T = double;
    const Geom q = geom_op<Op, T>(lop.g, ctx);
    FineOp<double> op{lop.g, lop.k2, 1.0 / (lop.h * lop.h), 2.0 / lop.h};
    const int rn = z0.p ? 1 : 0;
    HM_LAUNCH_OP(q, (k_correct_residual<BY>), op, x_in, e, x_out, f, r32, z0, region(ctx, rn), region(ctx, 0),
                 HM_ACTIVE, q.rpt);
    launch_sum_norms(ctx, q.nblk, norms, 1, rn);
    return q.nblk;
}

template <typename T>
void launch_copy_in(const LaunchCtx& ctx, Grid g, const void* src, bool src_is_f32, Vec<T> dst, bool scale_w,
                    bool conj) {
    const Geom q = geom(g, false, ctx);
    if (src_is_f32)
        HM_LAUNCH(q, (k_copy_in<T, float, BY>), g, static_cast<const cplx<float>*>(src), dst, int(scale_w),
                  int(conj), q.rpt);
    else
        HM_LAUNCH(q, (k_copy_in<T, double, BY>), g, static_cast<const cplx<double>*>(src), dst, int(scale_w),
                  int(conj), q.rpt);
}

template <typename T>
void launch_copy_out(const LaunchCtx& ctx, Grid g, Vec<T> src, void* dst, bool dst_is_f32, bool scale_w, bool conj) {
    const Geom q = geom(g, false, ctx);
    if (dst_is_f32)
        HM_LAUNCH(q, (k_copy_out<T, float, BY>), g, src, static_cast<cplx<float>*>(dst), int(scale_w), int(conj),
                  q.rpt);
    else
        HM_LAUNCH(q, (k_copy_out<T, double, BY>), g, src, static_cast<cplx<double>*>(dst), int(scale_w), int(conj),
                  q.rpt);
}

template <typename T>
void launch_zero(hipStream_t s, cplx<T>* p, long long count) {
    if (count <= 0) return;
    long long blocks = (count + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_zero<T>), dim3((unsigned)blocks), dim3(kThreads), 0, s, p, count);
}

void launch_fill_words(hipStream_t s, void* p, long long bytes, unsigned value) {
    const long long words = bytes / 4;
    if (words <= 0) return;
    long long blocks = (words + kThreads - 1) / kThreads;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_words, dim3((unsigned)blocks), dim3(kThreads), 0, s, static_cast<unsigned*>(p), words,
                       value);
}

void launch_grad_k2(const LaunchCtx& ctx, Grid g, double h, const double* k2, Vec<double> u, Vec<double> mu,
                    double* grad_k2_dense) {
    const int rpt = level_rpt(g, kBY, ctx.block_cap);
    hipLaunchKernelGGL(k_grad_k2, level_grid(g, rpt, 1, kBY), dim3(kBX, kBY), 0, ctx.stream, g, h, k2, u, mu,
                       grad_k2_dense, ctx.nrhs, rpt);
}

#define HM_INST(T)                                                                                              \
    template void launch_apply<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>);                         \
    template void launch_residual<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, Vec<T>);              \
    template void launch_jacobi<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, Vec<T>, double);        \
    template bool launch_jacobi2<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, Vec<T>, double);       \
    template int launch_restrict<T>(const LaunchCtx&, Grid, Grid, int, Vec<T>, Vec<T>, Vec<T>, Vec<T>);         \
    template void launch_prolong_add<T>(const LaunchCtx&, Grid, Grid, int, Vec<T>, Vec<T>);                     \
    template void launch_gmres_step<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, Vec<T>, Vec<T>,     \
                                       Vec<T>, GmState*, double, const hipEvent_t*, Vec<T>,                     \
                                       int, ProlongIn<T>, bool, RestrictOut<T>*, DeferredUpdate<T>*, bool);     \
    template void launch_resnorm<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, RhsNorms*);            \
    template void launch_norm<T>(const LaunchCtx&, Grid, Vec<T>, RhsNorms*);                                    \
    template void launch_copy_in<T>(const LaunchCtx&, Grid, const void*, bool, Vec<T>, bool, bool);             \
    template void launch_copy_out<T>(const LaunchCtx&, Grid, Vec<T>, void*, bool, bool, bool);                  \
    template void launch_zero<T>(hipStream_t, cplx<T>*, long long);

HM_INST(double)
HM_INST(float)

}  // namespace hm
