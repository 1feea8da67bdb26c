// Level-0 vector kernels of the outer flexible GMRES(m) (§1: multigrid on the
// CSL as a preconditioner for GMRES): classical Gram-Schmidt in two sweeps
// (all inner products <v_i, w> in one pass over w, then w -= sum h_i v_i),
// normalisation, the update x += Z y and the first basis vector r / ||r||
// (the complex64 copies of the basis vectors for FP32 preconditioner cycles
// included). FP64 data, [b][plane] per vector, the Krylov vectors
// [j][b][plane].
#include "hm_ops.hpp"

namespace hm {
namespace {

__device__ __forceinline__ int kry_lead() { return blockIdx.x == 0 && blockIdx.y == 0 && thread_linear() == 0; }

// Inner products <v_i, w> for i = i0 .. i0 + cnt - 1 (cnt <= kCgsChunk) in
// one sweep over w: block partial sums, 2 kCgsChunk per block (re, im per
// vector; unused slots zero) at pout + b * kPartStride.
constexpr int kCgsChunk = 16;
__global__ __launch_bounds__(kBX * kBY) void k_kry_cdots(Grid g, const cplx<double>* V, long long vstride, int i0,
                                                        int cnt, const cplx<double>* w, long long plane,
                                                        double* pout, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* wb = w + b * plane;
    const cplx<double>* vb = V + i0 * vstride + b * plane;
    double acc[2 * kCgsChunk];
#pragma unroll
    for (int k = 0; k < 2 * kCgsChunk; ++k) acc[k] = 0.0;
    for_nodes(g, rpt, [&](int, int, long long p) {
        const cplx<double> c = wb[p];
        cplx<double> a[kCgsChunk];
#pragma unroll
        for (int q = 0; q < kCgsChunk; ++q)
            if (q < cnt) a[q] = vb[q * vstride + p];
#pragma unroll
        for (int q = 0; q < kCgsChunk; ++q)
            if (q < cnt) {
                acc[2 * q] += a[q].re * c.re + a[q].im * c.im;
                acc[2 * q + 1] += a[q].re * c.im - a[q].im * c.re;
            }
    });
    block_partials<2 * kCgsChunk>(acc, pout + b * kPartStride);
}

// h_i = <v_i, w> for i = 0 .. j from the partials of the k_kry_cdots chunks
// (chunk c of nblk blocks at pin + b * kPartStride + c * nblk * 2 kCgsChunk):
// one block per right-hand side, one wavefront per inner product at a time,
// lanes over the blocks in a fixed order (deterministic); H[b][i] = h_i.
__global__ __launch_bounds__(kBX * kBY) void k_kry_hreduce(const double* pin, int nblk, int j, cplx<double>* H,
                                                          int hstride, const int* active) {
    const int b = blockIdx.x;
    if (!rhs_active(active, b)) return;
    const int lane = threadIdx.x;
    for (int i = threadIdx.y; i <= j; i += blockDim.y) {
        const int c = i / kCgsChunk, k = i % kCgsChunk;
        const double* src = pin + b * kPartStride + (long long)c * nblk * 2 * kCgsChunk + 2 * k;
        double re = 0.0, im = 0.0;
        for (int q = lane; q < nblk; q += kBX) {
            re += src[q * 2 * kCgsChunk];
            im += src[q * 2 * kCgsChunk + 1];
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == kBX - 1) H[b * hstride + i] = cplx<double>{re, im};
    }
}

// w -= sum_{i <= j} h_i v_i (h_i from H[b][i], in order of i); partials of
// ||w||^2 (two per block, the second zero: the layout k_kry_normalize reads).
__global__ __launch_bounds__(kBX * kBY) void k_kry_cgs_update(Grid g, const cplx<double>* V, long long vstride, int j,
                                                             cplx<double>* w, long long plane, const cplx<double>* H,
                                                             int hstride, double* pout, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    __shared__ cplx<double> hs[kMaxRestart];
    for (int i = thread_linear(); i <= j; i += kBX * kBY) hs[i] = H[b * hstride + i];
    __syncthreads();
    cplx<double>* wb = w + b * plane;
    const cplx<double>* vb = V + b * plane;
    double acc[2] = {0.0, 0.0};
    for_nodes(g, rpt, [&](int, int, long long p) {
        cplx<double> x = wb[p];
        for (int i0 = 0; i0 <= j; i0 += 8) {
            cplx<double> a[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (i0 + q <= j) a[q] = vb[(i0 + q) * vstride + p];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (i0 + q <= j) {
                    const cplx<double> h = hs[i0 + q];
                    x.re -= h.re * a[q].re - h.im * a[q].im;
                    x.im -= h.re * a[q].im + h.im * a[q].re;
                }
        }
        wb[p] = x;
        acc[0] += x.re * x.re + x.im * x.im;
    });
    block_partials<2>(acc, pout + b * kPartStride);
}

// The complex64 copy of a new basis vector is also the right-hand side of the
// FP32 cycle that preconditions it; with z32 set it is written a second time,
// as the first Arnoldi vector of that cycle's first GMRES step (z32 holds 4
// planes per right-hand side), with its block partial sums of ||v32||^2 at
// pz + b * kPartStride, so that step starts from u = 0 without a residual pass.
__device__ __forceinline__ void kry_out32(cplx<float>* fb, cplx<float>* zb, long long p, cplx<double> v,
                                          double& acc) {
    const cplx<float> v1 = cast<float>(v);
    if (fb) fb[p] = v1;
    if (zb) {
        zb[p] = v1;
        acc += double(v1.re) * double(v1.re) + double(v1.im) * double(v1.im);
    }
}

// ||w|| from the previous pass; H[b][0] = ||w|| (entry j+1 of the column);
// v_out = w / ||w|| (zero when ||w|| = 0).
__global__ __launch_bounds__(kBX * kBY) void k_kry_normalize(Grid g, const cplx<double>* w, cplx<double>* vout,
                                                            long long plane, cplx<double>* Hsub, int hstride,
                                                            const double* pin, int nblk_in, cplx<float>* v32,
                                                            cplx<float>* z32, double* pz, const int* active,
                                                            int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    double t[2];
    reduce_partials<2>(pin + b * kPartStride, nblk_in, t);
    const double hn = sqrt(t[0]);
    if (kry_lead()) Hsub[b * hstride] = cplx<double>{hn, 0.0};
    const double s = hn > 0.0 ? 1.0 / hn : 0.0;
    const cplx<double>* wb = w + b * plane;
    cplx<double>* ob = vout + b * plane;
    cplx<float>* fb = v32 ? v32 + b * plane : nullptr;
    cplx<float>* zb = z32 ? z32 + b * 4 * plane : nullptr;
    double acc[1] = {0.0};
    for_nodes(g, rpt, [&](int, int, long long p) {
        const cplx<double> v = s * wb[p];
        ob[p] = v;
        kry_out32(fb, zb, p, v, acc[0]);
    });
    if (zb) block_partials<1>(acc, pz + b * kPartStride);
}

// v = r / ||r|| with ||r||^2 from norms[b].r2
__global__ __launch_bounds__(kBX * kBY) void k_kry_first(Grid g, const cplx<double>* r, cplx<double>* v,
                                                        long long plane, const RhsNorms* norms, cplx<float>* v32,
                                                        cplx<float>* z32, double* pz, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const double nr = sqrt(norms[b].r2);
    const double s = nr > 0.0 ? 1.0 / nr : 0.0;
    const cplx<double>* rb = r + b * plane;
    cplx<double>* vb = v + b * plane;
    cplx<float>* fb = v32 ? v32 + b * plane : nullptr;
    cplx<float>* zb = z32 ? z32 + b * 4 * plane : nullptr;
    double acc[1] = {0.0};
    for_nodes(g, rpt, [&](int, int, long long p) {
        const cplx<double> x = s * rb[p];
        vb[p] = x;
        kry_out32(fb, zb, p, x, acc[0]);
    });
    if (zb) block_partials<1>(acc, pz + b * kPartStride);
}

// x += sum_i y[b][i] z_i for i < nz (y complex, [b][ystride])
__global__ __launch_bounds__(kBX * kBY) void k_kry_update(Grid g, const cplx<double>* Z, long long zstride, int nz,
                                                         const cplx<double>* y, int ystride, cplx<double>* x,
                                                         long long plane, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* yb = y + b * ystride;
    cplx<double>* xb = x + b * plane;
    for_nodes(g, rpt, [&](int, int, long long p) {
        cplx<double> acc = xb[p];
        for (int i = 0; i < nz; ++i) acc = cfma(acc, yb[i], Z[i * zstride + b * plane + p]);
        xb[p] = acc;
    });
}

struct KGeom {
    dim3 grid, block;
    int rpt, nblk;
};

KGeom kgeom(const LaunchCtx& ctx, const Grid& g, long long cap_limit = 1LL << 30) {
    const long long m = g.n + 1;
    const long long bx = (m + kBX - 1) / kBX;
    const long long cap = std::max(1LL, std::min<long long>(ctx.block_cap, cap_limit - bx));
    long long rpt = (m * bx + (long long)kBY * cap - 1) / ((long long)kBY * cap);
    if (rpt < 1) rpt = 1;
    KGeom q;
    q.rpt = int(rpt);
    q.grid = dim3(unsigned(bx), unsigned((m + kBY * rpt - 1) / (kBY * rpt)), unsigned(ctx.nrhs));
    q.block = dim3(kBX, kBY);
    q.nblk = int(q.grid.x * q.grid.y);
    return q;
}

double* kregion(const LaunchCtx& ctx, int r) { return ctx.partials + (long long)r * ctx.nrhs_cap * kPartStride; }

// the inner-product pass keeps the partials of every chunk in one reduction
// region; the passes that write a basis vector use the same block grid, so
// that the z_0 partial sums of k_kry_first and k_kry_normalize always count
// the same number of blocks
constexpr int kKryChunks = (kMaxRestart + kCgsChunk - 1) / kCgsChunk;
KGeom kry_geom(const LaunchCtx& ctx, const Grid& g) { return kgeom(ctx, g, kPartStride / (2 * kCgsChunk * kKryChunks)); }

}  // namespace

void launch_kry_orthogonalise(const LaunchCtx& ctx, Grid g, cplx<double>* V, long long vstride, int j,
                              cplx<double>* w, cplx<double>* H, int hstride, long long plane, cplx<float>* v32,
                              cplx<float>* z32) {
    const KGeom q = kry_geom(ctx, g);
    double* A = kregion(ctx, 0);
    double* B = kregion(ctx, 1);
    for (int i0 = 0; i0 <= j; i0 += kCgsChunk)
        hipLaunchKernelGGL(k_kry_cdots, q.grid, q.block, 0, ctx.stream, g, V, vstride, i0,
                           std::min(kCgsChunk, j + 1 - i0), w, plane,
                           A + (long long)(i0 / kCgsChunk) * q.nblk * 2 * kCgsChunk, ctx.active, q.rpt);
    hipLaunchKernelGGL(k_kry_hreduce, dim3(ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, A, q.nblk, j, H, hstride,
                       ctx.active);
    hipLaunchKernelGGL(k_kry_cgs_update, q.grid, q.block, 0, ctx.stream, g, V, vstride, j, w, plane, H, hstride, B,
                       ctx.active, q.rpt);
    hipLaunchKernelGGL(k_kry_normalize, q.grid, q.block, 0, ctx.stream, g, w, V + (j + 1) * vstride, plane,
                       H + j + 1, hstride, B, q.nblk, v32, z32, A, ctx.active, q.rpt);
}

int launch_kry_first(const LaunchCtx& ctx, Grid g, const cplx<double>* r, cplx<double>* v, long long plane,
                     const RhsNorms* norms, cplx<float>* v32, cplx<float>* z32) {
    const KGeom q = kry_geom(ctx, g);
    hipLaunchKernelGGL(k_kry_first, q.grid, q.block, 0, ctx.stream, g, r, v, plane, norms, v32, z32,
                       kregion(ctx, 0), ctx.active, q.rpt);
    return q.nblk;
}

void launch_kry_update(const LaunchCtx& ctx, Grid g, const cplx<double>* Z, long long zstride, int nz,
                       const cplx<double>* y, int ystride, cplx<double>* x, long long plane) {
    const KGeom q = kgeom(ctx, g);
    hipLaunchKernelGGL(k_kry_update, q.grid, q.block, 0, ctx.stream, g, Z, zstride, nz, y, ystride, x, plane,
                       ctx.active, q.rpt);
}

}  // namespace hm
