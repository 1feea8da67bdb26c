// Device operators of one level and the deterministic block reduction used
// by every kernel that produces norms or inner products.
#pragma once
#include "hm_common.hpp"
#include "hm_kernels.hpp"

namespace hm {

// Level 0: the scaled discrete operator A_s = W A of MP 2-A/2-B (§2),
// evaluated from k^2 on the fly. With edge weights w_e (1/2 for an edge that
// lies on the boundary, 1 otherwise) it reads
//   (A_s x)_p = W_p (4/h^2 - k_p^2 - 2 i k_p s_p / h) x_p
//               - (1/h^2) [ w_j (x_W + x_E) + w_i (x_S + x_N) ],
// where s_p counts the boundary sides of p; ghost nodes hold zero, which
// drops the couplings that the ghost elimination of the absorbing condition
// folded into the interior-normal neighbour (their weight 2 times W_p = 1/2
// is the edge weight 1).
template <typename T>
struct FineOp {
    static constexpr bool kHeavy = false;  // few registers: tall blocks
    Grid g;
    const T* k2;
    T ih2;    // 1 / h^2
    T two_h;  // 2 / h
    // diagonal at node (i, j) with k^2 = kk there
    __device__ __forceinline__ cplx<T> diag_k(int i, int j, T kk) const {
        const int n = g.n;
        const T W = line_w<T>(i, n) * line_w<T>(j, n);
        const int s = (i == 0 || i == n) + (j == 0 || j == n);
        T im = T(0);
        if (s) im = -two_h * T(s) * sqrt(kk);
        return {W * (T(4) * ih2 - kk), W * im};
    }
    __device__ __forceinline__ cplx<T> diag(int i, int j, long long p) const { return diag_k(i, j, k2[p]); }
    // (A_s x)_p from k^2 at p, the centre value and the west, east, south,
    // north neighbours
    __device__ __forceinline__ cplx<T> apply5k(int i, int j, T kk, cplx<T> c, cplx<T> xw, cplx<T> xe, cplx<T> xs,
                                               cplx<T> xn) const {
        const int n = g.n;
        const cplx<T> d = diag_k(i, j, kk);
        const T cx = ih2 * line_w<T>(j, n), cy = ih2 * line_w<T>(i, n);
        cplx<T> y = d * c;
        y.re -= cx * (xw.re + xe.re) + cy * (xs.re + xn.re);
        y.im -= cx * (xw.im + xe.im) + cy * (xs.im + xn.im);
        return y;
    }
    // the same at a node strictly inside the grid (W = 1, no Sommerfeld term):
    // equal to apply5k there, without the boundary arithmetic
    __device__ __forceinline__ cplx<T> apply5k_interior(T kk, cplx<T> c, cplx<T> xw, cplx<T> xe, cplx<T> xs,
                                                        cplx<T> xn) const {
        const T d = T(4) * ih2 - kk;
        cplx<T> y{d * c.re, d * c.im};
        y.re -= ih2 * (xw.re + xe.re) + ih2 * (xs.re + xn.re);
        y.im -= ih2 * (xw.im + xe.im) + ih2 * (xs.im + xn.im);
        return y;
    }
    __device__ __forceinline__ cplx<T> apply5(int i, int j, long long p, cplx<T> c, cplx<T> xw, cplx<T> xe,
                                              cplx<T> xs, cplx<T> xn) const {
        return apply5k(i, j, k2[p], c, xw, xe, xs, xn);
    }
    template <typename X>
    __device__ __forceinline__ cplx<T> apply_at(const X& x, int i, int j, long long p) const {
        return apply5(i, j, p, x(p), x(p - 1), x(p + 1), x(p - g.pitch), x(p + g.pitch));
    }
    __device__ __forceinline__ cplx<T> apply(const cplx<T>* __restrict__ x, int i, int j, long long p) const {
        return apply_at([x](long long q) { return x[q]; }, i, j, p);
    }
};

// Levels >= 1: stored Galerkin stencil (§3) of radius R, one complex plane per
// offset; ghost coefficients are zero. A Galerkin operator R C P with
// R = P^T / 4 (§4) and a complex symmetric C (the scaled operator W A and its
// shifted form differ from their transposes in no entry) is complex
// symmetric: the coefficient of offset d at node p equals that of offset -d
// at node p + d, up to the rounding of the product that formed them. Passes
// read the offsets of the upper half (dy > 0, or dy = 0 and dx >= 0) at p and
// those of the lower half from the upper-half plane at p + d, so that only
// the upper half of the planes is streamed from memory (the mirrored reads
// are the neighbouring nodes' own coefficients, found in cache); the operator
// applied is then exactly symmetric.
template <typename T, int R>
struct StencilOp {
    static constexpr bool kHeavy = R >= 2;  // 25/49-point stencils: many registers, short blocks
    Grid g;
    const cplx<T>* __restrict__ coef;
    static constexpr int D = 2 * R + 1;
    __device__ __forceinline__ cplx<T> diag(int, int, long long p) const { return coef[(R * D + R) * g.plane + p]; }
    // coefficient of offset (dx, dy) at node p (dx, dy compile-time after unrolling)
    __device__ __forceinline__ cplx<T> at(int dy, int dx, long long p) const {
        const bool lower = dy < 0 || (dy == 0 && dx < 0);
        return lower ? coef[((R - dy) * D + R - dx) * g.plane + p + (long long)dy * g.pitch + dx]
                     : coef[((dy + R) * D + dx + R) * g.plane + p];
    }
    template <typename X>
    __device__ __forceinline__ cplx<T> apply_at(const X& x, int, int, long long p) const {
        cplx<T> y{T(0), T(0)};
#pragma unroll
        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) y = cfma(y, at(dy, dx, p), x(p + (long long)dy * g.pitch + dx));
        return y;
    }
    __device__ __forceinline__ cplx<T> apply(const cplx<T>* __restrict__ x, int i, int j, long long p) const {
        return apply_at([x](long long q) { return x[q]; }, i, j, p);
    }
};

// Level 1 without its stored stencil: A_1 = R C_s P (§3 Galerkin product, §4
// transfers) applied in three steps from level-0 data, y = P x on the fine
// grid, v = C_s y with the shifted Laplacian C_s = A_s - i beta2 W K^2 of
// level 0, then the restriction R = P^T / 4 of v. Equal to the stored
// Galerkin stencil up to rounding; reads x and level-0 k^2 instead of
// (2r+1)^2 complex coefficients per node. The Jacobi diagonal comes from the
// centre plane of the stored stencil.
template <typename T, bool kBez>
struct ProductOp {
    static constexpr bool kHeavy = true;  // short blocks: three LDS stages
    Grid g;                 // level 1
    FineOp<T> fine;         // level-0 operator A_s (grid, k^2, 1/h^2, 2/h)
    T shift;                // beta2
    const cplx<T>* diagc;   // centre plane of the stored level-1 stencil
    __device__ __forceinline__ cplx<T> diag(int, int, long long p) const { return diagc[p]; }
};

// Tile (column block, row block) of this workgroup: blockIdx.x, blockIdx.y.
// (A map that gave each XCD a contiguous run of tiles cut the halo re-reads
// between L2s but made the cycle slower, so tiles follow the block ids.)
struct BlockXY {
    int x, y;
};
// kXcd: the tiles of a grid are dealt out in contiguous runs, one run per
// XCD. Workgroups are dispatched to the eight XCDs round-robin by linear id,
// so the ids of one residue class mod 8 share an XCD (and its L2); giving
// each class a contiguous run of tiles lets horizontally and vertically
// adjacent tiles share their halo lines in one L2 instead of fetching them
// twice. A bijection on the tiles of any grid; used by the pass whose tile
// reads three arrays with a halo (elsewhere the integer division it costs at
// the start of every block outweighed the saving).
template <bool kXcd = false>
__device__ __forceinline__ BlockXY block_xy() {
    if constexpr (kXcd) {
        const int gx = gridDim.x, T = gx * gridDim.y;
        const int t = blockIdx.y * gx + blockIdx.x;
        const int r = t & 7, k = t >> 3, q = T >> 3, rem = T & 7;
        const int tile = r * q + min(r, rem) + k;
        return BlockXY{tile % gx, tile / gx};
    }
    return BlockXY{int(blockIdx.x), int(blockIdx.y)};
}

// Calls f(i, j, p) for the nodes of this thread: column bx * 64 + lane,
// rows interleaved by 4 over rows_per_thread consecutive row groups of row
// block by ((bx, by) = block_xy()).
template <typename F>
__device__ __forceinline__ void for_nodes(const Grid& g, int rpt, F&& f) {
    const BlockXY bt = block_xy();
    const int i = bt.x * kBX + threadIdx.x;
    if (i > g.n) return;
    const int by = blockDim.y;
    for (int rr = 0; rr < rpt; ++rr) {
        const int j = (bt.y * rpt + rr) * by + threadIdx.y;
        if (j > g.n) return;
        f(i, j, g.at(i, j));
    }
}

// Waits until every vector memory operation the wave has issued is done
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt fields at their no-wait maxima).
// Placed after a sweep of loads so that the stores of the following
// arithmetic do not make the compiler wait for them row by row.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The nodes of for_nodes, taken NB rows at a time in two sweeps: load(u, p)
// for the rows of the batch first, then body(u, i, j, p) for the rows that
// exist. The loads of a batch are in flight together: one memory round trip
// per batch instead of one per row. Only the row count decides which loads
// are issued (uniform in the block, so no divergent branch separates them);
// a row below the grid loads its column's last node instead.
template <int NB, bool kXcd = false, typename Load, typename Body>
__device__ __forceinline__ void for_nodes_batched(const Grid& g, int rpt, Load&& load, Body&& body) {
    const BlockXY bt = block_xy<kXcd>();
    const int i = bt.x * kBX + threadIdx.x;
    if (i > g.n) return;
    const int by = blockDim.y;
    const int j0 = bt.y * rpt * by + threadIdx.y;
    if (j0 > g.n) return;
    for (int rr0 = 0; rr0 < rpt; rr0 += NB) {
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (rr0 + u < rpt) load(u, g.at(i, min(j0 + (rr0 + u) * by, g.n)));
        wait_vmem();
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + (rr0 + u) * by;
            if (rr0 + u < rpt && j <= g.n) body(u, i, j, g.at(i, j));
        }
    }
}

// Indices q = tid, tid + nt, ... < count of a block-strided loop, NB at a
// time in two sweeps as in for_nodes_batched: load(u, q) (q clamped to
// count - 1 in the last, partly filled stride; strides beyond it are not
// loaded), then body(u, q) for the indices that exist.
template <int NB, typename Load, typename Body>
__device__ __forceinline__ void for_strided_batched(int count, Load&& load, Body&& body) {
    const int nt = blockDim.x * blockDim.y;
    const int tid = threadIdx.y * kBX + threadIdx.x;
    for (int s0 = 0; s0 < count; s0 += NB * nt) {  // uniform: first index of the round
        const int q0 = s0 + tid;
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (s0 + u * nt < count) load(u, min(q0 + u * nt, count - 1));
        wait_vmem();
#pragma unroll
        for (int u = 0; u < NB; ++u)
            if (q0 + u * nt < count) body(u, q0 + u * nt);
    }
}

// ---------------------------------------------------------------- LDS tiles
// A block of 64 x BY threads with rows_per_thread rpt covers columns
// [c0, c0 + 64) and rows [r0, r0 + BY * rpt) of a level. Its LDS tile adds a
// halo of R nodes on every side so that a radius-R stencil reads LDS only.
extern __shared__ __align__(16) unsigned char hm_dyn_lds[];

template <int R>
struct Tile {
    static constexpr int TW = kBX + 2 * R;
    int c0, r0, rows;
    __device__ __forceinline__ int at(int i, int j) const { return (j - r0 + R) * TW + (i - c0 + R); }
    __device__ __forceinline__ int count() const { return TW * (rows + 2 * R); }
};

template <int R, bool kXcd = false>
__device__ __forceinline__ Tile<R> block_tile(int rpt) {
    const BlockXY bt = block_xy<kXcd>();
    return Tile<R>{bt.x * kBX, bt.y * int(blockDim.y) * rpt, int(blockDim.y) * rpt};
}

// lds[t.at(i, j)] = make(load(g.at(i, j))) for every tile node inside the
// padded frame (ghosts read as stored, zero); nodes beyond it hold zero and
// are never used by an in-domain stencil. load only gathers the values that
// make combines: the loads of FillBatch<T> nodes are issued before any
// combination (a node outside the frame is clamped onto it, R <= kGhost, and
// gives zero), so that they are in flight together.
template <typename T>
struct FillBatch {
    static constexpr int value = sizeof(T) == 4 ? 8 : 4;  // register budget of FP64 tiles
};
struct Ident {
    template <typename X>
    __device__ __forceinline__ X operator()(const X& x) const { return x; }
};
template <typename T, int R>
__device__ __forceinline__ bool tile_below_grid(const Tile<R>& t, const Grid& g) {
    return t.r0 - R > g.n;  // padding tiles of batch grids (uniform in the block)
}
template <typename T, int R, typename Load, typename Make>
__device__ __forceinline__ void fill_tile(cplx<T>* lds, const Tile<R>& t, const Grid& g, Load&& load, Make&& make) {
    static_assert(R <= kGhost, "tile halo beyond the stored ghost layers");
    if (tile_below_grid<T, R>(t, g)) return;  // no node of the tile or its halo exists
    constexpr int FB = FillBatch<T>::value;
    decltype(load(0LL)) v[FB];
    bool ok[FB];
    for_strided_batched<FB>(
        t.count(),
        [&](int u, int q) {
            const int i = t.c0 - R + q % Tile<R>::TW;
            const int j = t.r0 - R + q / Tile<R>::TW;
            const int ic = min(max(i, -R), g.n + R), jc = min(max(j, -R), g.n + R);
            ok[u] = i == ic && j == jc;
            v[u] = load(g.at(ic, jc));
        },
        [&](int u, int q) { lds[q] = ok[u] ? make(v[u]) : cplx<T>{T(0), T(0)}; });
    __syncthreads();
}

// fill_tile with work in the middle: the loads of the first stride batch are
// issued (unconditionally, indices clamped to the tile), then mid() runs
// while they are in flight, then the batch is combined; mid() returning false
// (uniformly in the block) ends the fill before anything is written, and the
// function returns false. make may use what mid() computes.
template <typename T, int R, typename Load, typename Make, typename Mid>
__device__ __forceinline__ bool fill_tile_mid(cplx<T>* lds, const Tile<R>& t, const Grid& g, Load&& load,
                                              Make&& make, Mid&& mid) {
    static_assert(R <= kGhost, "tile halo beyond the stored ghost layers");
    // (no padding-tile test here: only handles for one right-hand side take
    // this path, and their grids have no padding tiles; a second inlined
    // copy of mid() for that test cost the level-0 pass 15 %)
    constexpr int FB = FillBatch<T>::value;
    decltype(load(0LL)) v[FB];
    bool ok[FB];
    const int count = t.count();
    auto ld = [&](int u, int q) {
        const int i = t.c0 - R + q % Tile<R>::TW;
        const int j = t.r0 - R + q / Tile<R>::TW;
        const int ic = min(max(i, -R), g.n + R), jc = min(max(j, -R), g.n + R);
        ok[u] = i == ic && j == jc;
        v[u] = load(g.at(ic, jc));
    };
    const int nt = blockDim.x * blockDim.y;
    const int tid = threadIdx.y * kBX + threadIdx.x;
#pragma unroll
    for (int u = 0; u < FB; ++u) ld(u, min(tid + u * nt, count - 1));
    if (!mid()) return false;
    wait_vmem();
#pragma unroll
    for (int u = 0; u < FB; ++u) {
        const int q = tid + u * nt;
        if (q < count) lds[q] = ok[u] ? make(v[u]) : cplx<T>{T(0), T(0)};
    }
    for (int s0 = FB * nt; s0 < count; s0 += FB * nt) {  // uniform: first index of the round
        const int q0 = s0 + tid;
#pragma unroll
        for (int u = 0; u < FB; ++u)
            if (s0 + u * nt < count) ld(u, min(q0 + u * nt, count - 1));
        wait_vmem();
#pragma unroll
        for (int u = 0; u < FB; ++u)
            if (q0 + u * nt < count) lds[q0 + u * nt] = ok[u] ? make(v[u]) : cplx<T>{T(0), T(0)};
    }
    __syncthreads();
    return true;
}

// Stencil of radius R applied at node p whose tile index is li, values from LDS.
template <typename T, int R>
__device__ __forceinline__ cplx<T> apply_tile(const StencilOp<T, R>& op, const cplx<T>* lds, int li, long long p) {
    constexpr int TW = Tile<R>::TW;
    cplx<T> y{T(0), T(0)};
#pragma unroll
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
        for (int dx = -R; dx <= R; ++dx)
            y = cfma(y, op.at(dy, dx, p), lds[li + dy * TW + dx]);
    return y;
}

// Level-0 operator applied at tile index li from LDS, with k^2 at p given.
template <typename T>
__device__ __forceinline__ cplx<T> apply_tile(const FineOp<T>& op, const cplx<T>* lds, int li, int i, int j, T kk) {
    constexpr int TW = Tile<1>::TW;
    return op.apply5k(i, j, kk, lds[li], lds[li - 1], lds[li + 1], lds[li - TW], lds[li + TW]);
}

// Per-node operand of an operator that a batched sweep loads ahead of the
// arithmetic: k^2 for the level-0 operator; nothing for stored stencils,
// whose coefficient loads stay in the apply (one row per thread there).
struct NoVals {};
template <typename T, int N>
struct Vals {
    cplx<T> v[N];
};
template <typename Op>
struct OpPre {
    using type = NoVals;
    __device__ __forceinline__ static NoVals load(const Op&, long long) { return {}; }
};
template <typename T>
struct OpPre<FineOp<T>> {
    using type = T;
    __device__ __forceinline__ static T load(const FineOp<T>& op, long long p) { return op.k2[p]; }
};
template <typename T, int R>
__device__ __forceinline__ cplx<T> apply_tile_pre(const StencilOp<T, R>& op, const cplx<T>* lds, int li, int,
                                                  int, long long p, NoVals) {
    return apply_tile(op, lds, li, p);
}
template <typename T>
__device__ __forceinline__ cplx<T> apply_tile_pre(const FineOp<T>& op, const cplx<T>* lds, int li, int i, int j,
                                                  long long, T kk) {
    return apply_tile(op, lds, li, i, j, kk);
}

template <typename Op>
struct is_stencil {
    static constexpr bool value = false;
};
template <typename T, int R>
struct is_stencil<StencilOp<T, R>> {
    static constexpr bool value = true;
    static constexpr int radius = R;
};

// Halo width of an operator's LDS tile.
template <typename Op>
struct op_radius {
    static constexpr int value = 1;  // level-0 five-point operator
};
template <typename T, int R>
struct op_radius<StencilOp<T, R>> {
    static constexpr int value = R;
};
template <typename T, bool B>
struct op_radius<ProductOp<T, B>> {
    static constexpr int value = 3;  // coarse halo that the fine stages need
};
template <typename Op>
struct is_product {
    static constexpr bool value = false;
};
template <typename T, bool B>
struct is_product<ProductOp<T, B>> {
    static constexpr bool value = true;
};

// Fine-grid stages of a ProductOp block. The block's coarse tile covers
// columns [c0, c0 + 64) and rows [r0, r0 + rows); the restriction reads fine
// nodes 2I - 2 .. 2I + 2, C_s one more on each side.
template <typename T>
struct ProductStages {
    static constexpr int YW = 2 * kBX + 5;  // fine columns 2 c0 - 3 .. 2 c0 + 129 (y = P x)
    static constexpr int VW = 2 * kBX + 3;  // fine columns 2 c0 - 2 .. 2 c0 + 128 (v = C_s y)
    __host__ __device__ static int yrows(int rows) { return 2 * rows + 5; }
    __host__ __device__ static int vrows(int rows) { return 2 * rows + 3; }
    __host__ __device__ static size_t values(int rows) {
        return size_t(Tile<3>::TW) * (rows + 6) + size_t(YW) * yrows(rows) + size_t(VW) * vrows(rows);
    }
};

__device__ __forceinline__ bool rhs_active(const int* active, int b) { return active == nullptr || active[b] != 0; }

// Grid-wide reductions without atomics. A producer kernel writes one partial
// sum per block (`block_partials`); the kernel launched after it reduces all
// partials itself (`reduce_partials`, identical order in every block, hence
// deterministic), the kernel boundary making the partials visible. The
// partials of right-hand side b and region r live at
// partials + (r * nrhs_cap + b) * kPartStride.

// Row-major index of this block's tile, the slot of its partial sums.
template <bool kXcd = false>
__device__ __forceinline__ int block_linear() {
    const BlockXY bt = block_xy<kXcd>();
    return bt.y * int(gridDim.x) + bt.x;
}
__device__ __forceinline__ int thread_linear() { return threadIdx.y * kBX + threadIdx.x; }

// Sum over the 64 lanes of a wavefront by DPP lane moves (no LDS traffic):
// pairwise within quads, rotations by 4 and 8 within rows of 16, then the
// sums of rows 0 and 2 broadcast into rows 1 and 3 and of rows 0-1 into rows
// 2-3. Lane 63 ends with the total; the order of the additions is fixed, so
// the result is deterministic. Doubles move as two 32-bit halves.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x) {
    const unsigned long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b & 0xffffffffu)), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), CTRL, ROW_MASK, 0xF, true);
    return __longlong_as_double((unsigned long long)unsigned(lo) | ((unsigned long long)unsigned(hi) << 32));
}

// One value summed over the 64 lanes of a wavefront by the moves of
// block_sum; lane 63 ends with the total.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_move<0xb1, 0xF>(x);
    x += dpp_move<0x4e, 0xF>(x);
    x += dpp_move<0x124, 0xF>(x);
    x += dpp_move<0x128, 0xF>(x);
    x += dpp_move<0x142, 0xA>(x);
    x += dpp_move<0x143, 0xC>(x);
    return x;
}

// Block sum for 64 x BY thread blocks, BY <= kMaxBY (wavefront = threadIdx.y):
// each wavefront reduces its K values with DPP moves, lane 63 stores them,
// and every thread adds the wavefront totals in wavefront order.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (&tot)[K]) {
    __shared__ double sh[kMaxBY][K];
    const int lane = threadIdx.x, wave = threadIdx.y;
    __syncthreads();  // sh may still be read from an earlier call
    double w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] = v[k];
    // the K values of one step are independent: their moves overlap
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] += dpp_move<0xb1, 0xF>(w[k]);  // quad_perm [1,0,3,2]
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] += dpp_move<0x4e, 0xF>(w[k]);  // quad_perm [2,3,0,1]
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] += dpp_move<0x124, 0xF>(w[k]);  // row_ror 4
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] += dpp_move<0x128, 0xF>(w[k]);  // row_ror 8
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] += dpp_move<0x142, 0xA>(w[k]);  // row_bcast 15 into rows 1, 3
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] += dpp_move<0x143, 0xC>(w[k]);  // row_bcast 31 into rows 2, 3
    if (lane == kBX - 1)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[wave][k] = w[k];
    __syncthreads();
    // only the block's own wavefronts (a loop over every possible one with a
    // guard per term costs two selects and an add per term and wavefront)
    const int nw = blockDim.y;
#pragma unroll
    for (int k = 0; k < K; ++k) tot[k] = 0.0;
    for (int q = 0; q < nw; ++q)
#pragma unroll
        for (int k = 0; k < K; ++k) tot[k] += sh[q][k];
}

// Writes this block's K sums to out[block * K + k].
template <int K, bool kXcd = false>
__device__ __forceinline__ void block_partials(double (&v)[K], double* out) {
    double tot[K];
    block_sum<K>(v, tot);
    if (thread_linear() == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[block_linear<kXcd>() * K + k] = tot[k];
    }
}

// Sums the K partials of nblk producer blocks; every thread gets the totals.
// Each thread sums partials q = tid, tid + nt, ... in that order; loads are
// gathered kReduceBatch strides at a time so that they are in flight together.
constexpr int kReduceBatch = 4;
template <int K>
__device__ __forceinline__ void reduce_partials(const double* in, int nblk, double (&tot)[K]) {
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int nt = blockDim.x * blockDim.y;
    for (int q0 = thread_linear(); q0 < nblk; q0 += kReduceBatch * nt) {
        double v[kReduceBatch][K];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
            const int q = q0 + u * nt;
#pragma unroll
            for (int k = 0; k < K; ++k) v[u][k] = (q < nblk) ? in[q * K + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += v[u][k];
    }
    block_sum<K>(acc, tot);
}

// reduce_partials in two steps, so that the reduction's loads and the
// caller's next loads are in flight together (one memory round trip instead
// of two on the critical path of a reduction-consuming pass):
// partials_issue loads the first kReduceBatch strides, every index clamped to
// the last partial so that the loads are issued unconditionally and can be
// waited for alone (vector loads complete in order); partials_finish adds
// them, and any further strides, in the order of reduce_partials (the same
// totals) and block-sums.
template <int K>
struct PartialBatch {
    double v[kReduceBatch][K];
};

template <int K>
__device__ __forceinline__ void partials_issue(const double* in, int nblk, PartialBatch<K>& pb) {
    const int nt = blockDim.x * blockDim.y;
    const int last = nblk > 0 ? nblk - 1 : 0;
#pragma unroll
    for (int u = 0; u < kReduceBatch; ++u) {
        const int q = min(thread_linear() + u * nt, last);
#pragma unroll
        for (int k = 0; k < K; ++k) pb.v[u][k] = in[q * K + k];
    }
}

template <int K>
__device__ __forceinline__ void partials_finish(const double* in, int nblk, const PartialBatch<K>& pb,
                                                double (&tot)[K]) {
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int nt = blockDim.x * blockDim.y;
    const int q0 = thread_linear();
#pragma unroll
    for (int u = 0; u < kReduceBatch; ++u) {
        const bool in_range = q0 + u * nt < nblk;
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += in_range ? pb.v[u][k] : 0.0;
    }
    for (int q1 = q0 + kReduceBatch * nt; q1 < nblk; q1 += kReduceBatch * nt) {
        double v[kReduceBatch][K];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
            const int q = q1 + u * nt;
#pragma unroll
            for (int k = 0; k < K; ++k) v[u][k] = (q < nblk) ? in[q * K + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += v[u][k];
    }
    block_sum<K>(acc, tot);
}

// The reduction of the previous pass's K partial sums and the tile fill of a
// reduction-consuming pass, in one of two orders. kOverlap: both sets of
// loads in flight together (the reduction runs while the tile arrives; more
// registers, for launches whose blocks all fit on the GPU at once);
// otherwise the reduction first (fewer registers, hence more resident blocks
// for launches that queue several rounds of blocks). after(totals) returns
// false to end the block (uniformly) before anything is written; make may
// use what it computes.
template <int K, bool kOverlap, typename T, int R, typename Load, typename Make, typename After>
__device__ __forceinline__ bool reduce_and_fill(const double* pin, int nblk, cplx<T>* lds, const Tile<R>& t,
                                                const Grid& g, Load&& load, Make&& make, After&& after) {
    if constexpr (kOverlap) {
        PartialBatch<K> pb;
        partials_issue<K>(pin, nblk, pb);
        return fill_tile_mid<T, R>(lds, t, g, load, make, [&]() -> bool {
            double tot[K];
            partials_finish<K>(pin, nblk, pb, tot);
            return after(tot);
        });
    } else {
        double tot[K];
        reduce_partials<K>(pin, nblk, tot);
        if (!after(tot)) return false;
        fill_tile<T, R>(lds, t, g, load, make);
        return true;
    }
}

// Least-squares min || beta e1 - H y || over the k Arnoldi columns by complex
// Givens rotations, then y_i s_i into st.yr / st.yi. Run by one thread on a
// shared-memory copy of H so that it costs the calling kernel no registers.
struct LsWork {
    double hr[4][3], hi[4][3], gr[4], gi[4], cs[3], sr[3], si[3], yr[3], yi[3];
};

static __device__ __noinline__ void gm_least_squares(GmState& st, LsWork& w) {
    const int k = st.k;
#pragma unroll 1
    for (int a = 0; a < 4; ++a)
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            w.hr[a][c] = st.hr[a][c];
            w.hi[a][c] = st.hi[a][c];
        }
    w.gr[0] = st.beta;
    w.gi[0] = 0.0;
    for (int a = 1; a < 4; ++a) w.gr[a] = w.gi[a] = 0.0;
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
#pragma unroll 1
        for (int i = 0; i < j; ++i) {  // earlier rotations on column j
            const double ar = w.hr[i][j], ai = w.hi[i][j], br = w.hr[i + 1][j], bi = w.hi[i + 1][j];
            const double c = w.cs[i], s_r = w.sr[i], s_i = w.si[i];
            // a' = c a + s b ; b' = -conj(s) a + c b
            w.hr[i][j] = c * ar + (s_r * br - s_i * bi);
            w.hi[i][j] = c * ai + (s_r * bi + s_i * br);
            w.hr[i + 1][j] = -(s_r * ar + s_i * ai) + c * br;
            w.hi[i + 1][j] = -(s_r * ai - s_i * ar) + c * bi;
        }
        const double ar = w.hr[j][j], ai = w.hi[j][j], br = w.hr[j + 1][j], bi = w.hi[j + 1][j];
        const double na = hypot(ar, ai), nb = hypot(br, bi);
        const double rho = hypot(na, nb);
        double c, s_r, s_i;
        if (na == 0.0) {
            c = 0.0;
            s_r = br / nb;
            s_i = -bi / nb;
        } else {
            c = na / rho;
            // s = (a / |a|) conj(b) / rho
            const double ur = ar / na, ui = ai / na;
            s_r = (ur * br + ui * bi) / rho;
            s_i = (ui * br - ur * bi) / rho;
        }
        w.cs[j] = c;
        w.sr[j] = s_r;
        w.si[j] = s_i;
        w.hr[j][j] = c * ar + (s_r * br - s_i * bi);
        w.hi[j][j] = c * ai + (s_r * bi + s_i * br);
        w.hr[j + 1][j] = 0.0;
        w.hi[j + 1][j] = 0.0;
        const double g0r = w.gr[j], g0i = w.gi[j], g1r = w.gr[j + 1], g1i = w.gi[j + 1];
        w.gr[j] = c * g0r + (s_r * g1r - s_i * g1i);
        w.gi[j] = c * g0i + (s_r * g1i + s_i * g1r);
        w.gr[j + 1] = -(s_r * g0r + s_i * g0i) + c * g1r;
        w.gi[j + 1] = -(s_r * g0i - s_i * g0r) + c * g1i;
    }
#pragma unroll 1
    for (int j = k - 1; j >= 0; --j) {
        double tr = w.gr[j], ti = w.gi[j];
#pragma unroll 1
        for (int c = j + 1; c < k; ++c) {
            tr -= w.hr[j][c] * w.yr[c] - w.hi[j][c] * w.yi[c];
            ti -= w.hr[j][c] * w.yi[c] + w.hi[j][c] * w.yr[c];
        }
        const double dr = w.hr[j][j], di = w.hi[j][j];
        const double inv = 1.0 / (dr * dr + di * di);
        w.yr[j] = (tr * dr + ti * di) * inv;
        w.yi[j] = (ti * dr - tr * di) * inv;
    }
#pragma unroll 1
    for (int j = 0; j < 3; ++j) {
        st.yr[j] = (j < k) ? w.yr[j] * st.s[j] : 0.0;
        st.yi[j] = (j < k) ? w.yi[j] * st.s[j] : 0.0;
    }
}

// 1 / sqrt(x) and 1 / x for x > 0 in FP64: the hardware estimates refined by
// two Newton steps each (the estimate's relative error squares per step,
// ending at about one unit in the last place). They stand in for the
// correctly rounded sqrt and division sequences in the short dependent chain
// of the least-squares solve below.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    y = fma(fma(-x, y, 1.0), y, y);
    return y;
}

// The same least-squares solve with every index fixed at compile time, so
// that H, the rotations and y stay in registers: for kernels in which every
// thread holds H. Columns at or beyond k are skipped; y_i s_i for i < k, zero
// beyond.
__device__ __forceinline__ void gm_least_squares_regs(const double (&Hr)[4][3], const double (&Hi)[4][3],
                                                      const double (&s)[3], double beta, int k, double (&yr)[3],
                                                      double (&yi)[3]) {
    double hr[4][3], hi[4][3], gr[4], gi[4], cs[3], sr[3], si[3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bool used = (c < k) && (a <= c + 1);
            hr[a][c] = used ? Hr[a][c] : 0.0;
            hi[a][c] = used ? Hi[a][c] : 0.0;
        }
    gr[0] = beta;
    gi[0] = 0.0;
#pragma unroll
    for (int a = 1; a < 4; ++a) gr[a] = gi[a] = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j < k) {
#pragma unroll
            for (int i = 0; i < j; ++i) {
                const double ar = hr[i][j], ai = hi[i][j], br = hr[i + 1][j], bi = hi[i + 1][j];
                const double c = cs[i], s_r = sr[i], s_i = si[i];
                hr[i][j] = c * ar + (s_r * br - s_i * bi);
                hi[i][j] = c * ai + (s_r * bi + s_i * br);
                hr[i + 1][j] = -(s_r * ar + s_i * ai) + c * br;
                hi[i + 1][j] = -(s_r * ai - s_i * ar) + c * bi;
            }
            // rotation zeroing b under a: c = |a| / rho, s = (a / |a|) conj(b) / rho,
            // rho = sqrt(|a|^2 + |b|^2) (entries of H are bounded by the
            // operator norm, so the squares stay far from overflow)
            const double ar = hr[j][j], ai = hi[j][j], br = hr[j + 1][j], bi = hi[j + 1][j];
            const double a2 = ar * ar + ai * ai;
            const double ir = rsqrt_nr(a2 + (br * br + bi * bi));  // 1 / rho
            double c, s_r, s_i;
            if (a2 == 0.0) {
                c = 0.0;
                s_r = br * ir;
                s_i = -bi * ir;
            } else {
                const double ina = rsqrt_nr(a2);  // 1 / |a|
                const double inr = ir * ina;
                c = a2 * ina * ir;
                s_r = (ar * br + ai * bi) * inr;
                s_i = (ai * br - ar * bi) * inr;
            }
            cs[j] = c;
            sr[j] = s_r;
            si[j] = s_i;
            hr[j][j] = c * ar + (s_r * br - s_i * bi);
            hi[j][j] = c * ai + (s_r * bi + s_i * br);
            hr[j + 1][j] = 0.0;
            hi[j + 1][j] = 0.0;
            const double g0r = gr[j], g0i = gi[j], g1r = gr[j + 1], g1i = gi[j + 1];
            gr[j] = c * g0r + (s_r * g1r - s_i * g1i);
            gi[j] = c * g0i + (s_r * g1i + s_i * g1r);
            gr[j + 1] = -(s_r * g0r + s_i * g0i) + c * g1r;
            gi[j + 1] = -(s_r * g0i - s_i * g0r) + c * g1i;
        }
    }
    double wr[3] = {0.0, 0.0, 0.0}, wi[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 2; j >= 0; --j) {
        if (j < k) {
            double tr = gr[j], ti = gi[j];
#pragma unroll
            for (int c = j + 1; c < 3; ++c) {
                if (c < k) {
                    tr -= hr[j][c] * wr[c] - hi[j][c] * wi[c];
                    ti -= hr[j][c] * wi[c] + hi[j][c] * wr[c];
                }
            }
            const double dr = hr[j][j], di = hi[j][j];
            const double inv = rcp_nr(dr * dr + di * di);
            wr[j] = (tr * dr + ti * di) * inv;
            wi[j] = (ti * dr - tr * di) * inv;
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        yr[j] = (j < k) ? wr[j] * s[j] : 0.0;
        yi[j] = (j < k) ? wi[j] * s[j] : 0.0;
    }
}

// Forward and back substitution with a row-major LU factor (unit lower L,
// upper U, row swaps piv[k] <-> k applied in order) for one right-hand side x
// held in LDS; all nthreads threads of the block take part.
__device__ __forceinline__ void lu_substitute(const cplx<double>* LU, const int* piv, cplx<double>* x, int N, int tid,
                                              int nthreads) {
    if (tid == 0)
        for (int k = 0; k < N; ++k) {
            const int p = piv[k];
            if (p != k) {
                const cplx<double> t = x[k];
                x[k] = x[p];
                x[p] = t;
            }
        }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        const cplx<double> xk = x[k];
        for (int i = k + 1 + tid; i < N; i += nthreads) x[i] = x[i] - LU[i * N + k] * xk;
        __syncthreads();
    }
    for (int k = N - 1; k >= 0; --k) {
        if (tid == 0) x[k] = cdiv(x[k], LU[k * N + k]);
        __syncthreads();
        const cplx<double> xk = x[k];
        for (int i = tid; i < k; i += nthreads) x[i] = x[i] - LU[i * N + k] * xk;
        __syncthreads();
    }
}

}  // namespace hm
