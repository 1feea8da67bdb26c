// Level-0 vector kernels of the outer flexible GMRES(m) (§1: multigrid on the
// CSL as a preconditioner for GMRES): modified Gram-Schmidt passes with
// consumer-side reductions, normalisation, the update x += Z y, precision
// casts of whole planes and the first basis vector r / ||r||. FP64 data,
// [b][plane] per vector, the Krylov vectors [j][b][plane].
#include "hm_ops.hpp"

namespace hm {
namespace {

__device__ __forceinline__ int kry_lead() { return blockIdx.x == 0 && blockIdx.y == 0 && thread_linear() == 0; }

// partials of <v, w>
__global__ __launch_bounds__(kBX * kBY) void k_kry_dot(Grid g, const cplx<double>* v, const cplx<double>* w,
                                                      long long plane, double* pout, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* vb = v + b * plane;
    const cplx<double>* wb = w + b * plane;
    double acc[2] = {0.0, 0.0};
    for_nodes(g, rpt, [&](int, int, long long p) {
        const cplx<double> a = vb[p], c = wb[p];
        acc[0] += a.re * c.re + a.im * c.im;
        acc[1] += a.re * c.im - a.im * c.re;
    });
    block_partials<2>(acc, pout + b * kPartStride);
}

// h = <v_i, w> from the previous pass's partials; H[b][i] = h; w -= h v_i;
// then partials of <v_next, w> (v_next != null) or of ||w||^2.
__global__ __launch_bounds__(kBX * kBY) void k_kry_mgs(Grid g, const cplx<double>* vi, const cplx<double>* vnext,
                                                      cplx<double>* w, long long plane, cplx<double>* Hcol,
                                                      int hstride, const double* pin, int nblk_in, double* pout,
                                                      const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    double t[2];
    reduce_partials<2>(pin + b * kPartStride, nblk_in, t);
    const cplx<double> h{t[0], t[1]};
    if (kry_lead()) Hcol[b * hstride] = h;
    const cplx<double>* vb = vi + b * plane;
    const cplx<double>* nb = vnext ? vnext + b * plane : nullptr;
    cplx<double>* wb = w + b * plane;
    double acc[2] = {0.0, 0.0};
    for_nodes(g, rpt, [&](int, int, long long p) {
        cplx<double> x = wb[p];
        const cplx<double> a = vb[p];
        x.re -= h.re * a.re - h.im * a.im;
        x.im -= h.re * a.im + h.im * a.re;
        wb[p] = x;
        if (nb) {
            const cplx<double> c = nb[p];
            acc[0] += c.re * x.re + c.im * x.im;
            acc[1] += c.re * x.im - c.im * x.re;
        } else {
            acc[0] += x.re * x.re + x.im * x.im;
        }
    });
    block_partials<2>(acc, pout + b * kPartStride);
}

// ||w|| from the previous pass; H[b][0] = ||w|| (entry j+1 of the column);
// v_out = w / ||w|| (zero when ||w|| = 0).
__global__ __launch_bounds__(kBX * kBY) void k_kry_normalize(Grid g, const cplx<double>* w, cplx<double>* vout,
                                                            long long plane, cplx<double>* Hsub, int hstride,
                                                            const double* pin, int nblk_in, const int* active,
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
    for_nodes(g, rpt, [&](int, int, long long p) { ob[p] = s * wb[p]; });
}

// v = r / ||r|| with ||r||^2 from norms[b].r2
__global__ __launch_bounds__(kBX * kBY) void k_kry_first(Grid g, const cplx<double>* r, cplx<double>* v,
                                                        long long plane, const RhsNorms* norms, const int* active,
                                                        int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const double nr = sqrt(norms[b].r2);
    const double s = nr > 0.0 ? 1.0 / nr : 0.0;
    const cplx<double>* rb = r + b * plane;
    cplx<double>* vb = v + b * plane;
    for_nodes(g, rpt, [&](int, int, long long p) { vb[p] = s * rb[p]; });
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

template <typename S, typename D>
__global__ __launch_bounds__(kBX * kBY) void k_kry_cast(Grid g, const cplx<S>* src, cplx<D>* dst, long long plane,
                                                       const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<S>* sb = src + b * plane;
    cplx<D>* db = dst + b * plane;
    for_nodes(g, rpt, [&](int, int, long long p) { db[p] = cast<D>(sb[p]); });
}

struct KGeom {
    dim3 grid, block;
    int rpt, nblk;
};

KGeom kgeom(const LaunchCtx& ctx, const Grid& g) {
    const long long m = g.n + 1;
    const long long bx = (m + kBX - 1) / kBX;
    const long long cap = ctx.block_cap;
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

}  // namespace

void launch_kry_orthogonalise(const LaunchCtx& ctx, Grid g, cplx<double>* V, long long vstride, int j,
                              cplx<double>* w, cplx<double>* H, int hstride, long long plane) {
    const KGeom q = kgeom(ctx, g);
    double* A = kregion(ctx, 0);
    double* B = kregion(ctx, 1);
    hipLaunchKernelGGL(k_kry_dot, q.grid, q.block, 0, ctx.stream, g, V, w, plane, A, ctx.active, q.rpt);
    double* in = A;
    double* out = B;
    for (int i = 0; i <= j; ++i) {
        const cplx<double>* vnext = (i < j) ? V + (i + 1) * vstride : nullptr;
        hipLaunchKernelGGL(k_kry_mgs, q.grid, q.block, 0, ctx.stream, g, V + i * vstride, vnext, w, plane, H + i,
                           hstride, in, q.nblk, out, ctx.active, q.rpt);
        double* t = in;
        in = out;
        out = t;
    }
    hipLaunchKernelGGL(k_kry_normalize, q.grid, q.block, 0, ctx.stream, g, w, V + (j + 1) * vstride, plane,
                       H + j + 1, hstride, in, q.nblk, ctx.active, q.rpt);
}

void launch_kry_first(const LaunchCtx& ctx, Grid g, const cplx<double>* r, cplx<double>* v, long long plane,
                      const RhsNorms* norms) {
    const KGeom q = kgeom(ctx, g);
    hipLaunchKernelGGL(k_kry_first, q.grid, q.block, 0, ctx.stream, g, r, v, plane, norms, ctx.active, q.rpt);
}

void launch_kry_update(const LaunchCtx& ctx, Grid g, const cplx<double>* Z, long long zstride, int nz,
                       const cplx<double>* y, int ystride, cplx<double>* x, long long plane) {
    const KGeom q = kgeom(ctx, g);
    hipLaunchKernelGGL(k_kry_update, q.grid, q.block, 0, ctx.stream, g, Z, zstride, nz, y, ystride, x, plane,
                       ctx.active, q.rpt);
}

void launch_kry_cast_down(const LaunchCtx& ctx, Grid g, const cplx<double>* src, cplx<float>* dst, long long plane) {
    const KGeom q = kgeom(ctx, g);
    hipLaunchKernelGGL((k_kry_cast<double, float>), q.grid, q.block, 0, ctx.stream, g, src, dst, plane, ctx.active,
                       q.rpt);
}

void launch_kry_cast_up(const LaunchCtx& ctx, Grid g, const cplx<float>* src, cplx<double>* dst, long long plane) {
    const KGeom q = kgeom(ctx, g);
    hipLaunchKernelGGL((k_kry_cast<float, double>), q.grid, q.block, 0, ctx.stream, g, src, dst, plane, ctx.active,
                       q.rpt);
}

}  // namespace hm
