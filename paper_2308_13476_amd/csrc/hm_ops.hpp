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
    Grid g;
    const T* k2;
    T ih2;    // 1 / h^2
    T two_h;  // 2 / h
    __device__ __forceinline__ cplx<T> diag(int i, int j, long long p) const {
        const int n = g.n;
        const T W = line_w<T>(i, n) * line_w<T>(j, n);
        const int s = (i == 0 || i == n) + (j == 0 || j == n);
        const T kk = k2[p];
        T im = T(0);
        if (s) im = -two_h * T(s) * sqrt(kk);
        return {W * (T(4) * ih2 - kk), W * im};
    }
    template <typename X>
    __device__ __forceinline__ cplx<T> apply_at(const X& x, int i, int j, long long p) const {
        const int n = g.n;
        const cplx<T> d = diag(i, j, p);
        const cplx<T> c = x(p);
        const cplx<T> xw = x(p - 1), xe = x(p + 1), xs = x(p - g.pitch), xn = x(p + g.pitch);
        const T cx = ih2 * line_w<T>(j, n), cy = ih2 * line_w<T>(i, n);
        cplx<T> y = d * c;
        y.re -= cx * (xw.re + xe.re) + cy * (xs.re + xn.re);
        y.im -= cx * (xw.im + xe.im) + cy * (xs.im + xn.im);
        return y;
    }
    __device__ __forceinline__ cplx<T> apply(const cplx<T>* __restrict__ x, int i, int j, long long p) const {
        return apply_at([x](long long q) { return x[q]; }, i, j, p);
    }
};

// Levels >= 1: stored Galerkin stencil (§3) of radius R, one complex plane per
// offset; ghost coefficients are zero.
template <typename T, int R>
struct StencilOp {
    Grid g;
    const cplx<T>* __restrict__ coef;
    static constexpr int D = 2 * R + 1;
    __device__ __forceinline__ cplx<T> diag(int, int, long long p) const { return coef[(R * D + R) * g.plane + p]; }
    template <typename X>
    __device__ __forceinline__ cplx<T> apply_at(const X& x, int, int, long long p) const {
        cplx<T> y{T(0), T(0)};
#pragma unroll
        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
            for (int dx = -R; dx <= R; ++dx)
                y = cfma(y, coef[((dy + R) * D + dx + R) * g.plane + p], x(p + (long long)dy * g.pitch + dx));
        return y;
    }
    __device__ __forceinline__ cplx<T> apply(const cplx<T>* __restrict__ x, int i, int j, long long p) const {
        return apply_at([x](long long q) { return x[q]; }, i, j, p);
    }
};

// Calls f(i, j, p) for the nodes of this thread: column blockIdx.x * 64 + lane,
// rows interleaved by 4 over rows_per_thread consecutive row groups.
template <typename F>
__device__ __forceinline__ void for_nodes(const Grid& g, int rpt, F&& f) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    if (i > g.n) return;
    for (int rr = 0; rr < rpt; ++rr) {
        const int j = (blockIdx.y * rpt + rr) * kBY + threadIdx.y;
        if (j > g.n) return;
        f(i, j, g.at(i, j));
    }
}

__device__ __forceinline__ bool rhs_active(const int* active, int b) { return active == nullptr || active[b] != 0; }

// Grid-wide reductions without atomics. A producer kernel writes one partial
// sum per block (`block_partials`); the kernel launched after it reduces all
// partials itself (`reduce_partials`, identical order in every block, hence
// deterministic), the kernel boundary making the partials visible. The
// partials of right-hand side b and region r live at
// partials + (r * nrhs_cap + b) * kPartStride.

__device__ __forceinline__ int block_linear() { return blockIdx.y * gridDim.x + blockIdx.x; }
__device__ __forceinline__ int thread_linear() { return threadIdx.y * kBX + threadIdx.x; }

// Block sum for 64 x 4 thread blocks (wavefront = threadIdx.y).
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (&tot)[K]) {
    __shared__ double sh[K][kBY];
    const int lane = threadIdx.x, wave = threadIdx.y;
    __syncthreads();  // sh may still be read from an earlier call
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) sh[k][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBY; ++w) s += sh[k][w];
        tot[k] = s;
    }
}

// Writes this block's K sums to out[block * K + k].
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double* out) {
    double tot[K];
    block_sum<K>(v, tot);
    if (thread_linear() == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[block_linear() * K + k] = tot[k];
    }
}

// Sums the K partials of nblk producer blocks; every thread gets the totals.
template <int K>
__device__ __forceinline__ void reduce_partials(const double* in, int nblk, double (&tot)[K]) {
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int q = thread_linear(); q < nblk; q += kBX * kBY) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += in[q * K + k];
    }
    block_sum<K>(acc, tot);
}

}  // namespace hm
