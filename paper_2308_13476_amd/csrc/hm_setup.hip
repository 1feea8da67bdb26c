// Setup kernels: k^2 layout, Galerkin coarse operators on the complex
// shifted Laplacian, FP32 copies, the coarsest dense LU and its solves.
#include <algorithm>

#include "hm_ops.hpp"

namespace hm {
namespace {

constexpr int kThreads = kBX * kBY;
constexpr int kMaxCoarse = 1089;  // coarsest grid of at most 32 x 32 intervals

// 1D prolongation weight of the §4 formula for a fine node at offset d from
// the fine image 2K of coarse node K: Bézier [1 4 6 4 1]/8, linear [1 2 1]/2.
__device__ __forceinline__ double mask1(int d, bool bez) {
    const int a = d < 0 ? -d : d;
    if (bez) return a == 0 ? 0.75 : a == 1 ? 0.5 : a == 2 ? 0.125 : 0.0;
    return a == 0 ? 1.0 : a == 1 ? 0.5 : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_k2_in(Grid g, const double* src, double* k64, float* k32) {
    const long long m = g.n + 1;
    for (long long q = blockIdx.x * (long long)kThreads + threadIdx.x; q < m * m; q += (long long)gridDim.x * kThreads) {
        const int i = int(q % m), j = int(q / m);
        const double v = src[q];
        k64[g.at(i, j)] = v;
        if (k32) k32[g.at(i, j)] = float(v);
    }
}

// Checks the caller's k^2 field against the problem statement of §2 (k > 0
// on the absorbing boundary, whose condition uses k = sqrt(k^2); k^2 >= 0
// inside): flags[0] collects 1 for a non-finite value, 2 for a negative one
// and 4 for a zero on the boundary, flags[1] the smallest offending index
// (flags start as {0, INT_MAX}).
__global__ __launch_bounds__(kThreads) void k_check_k2(int n, const double* src, int* flags) {
    const long long m = n + 1;
    for (long long q = blockIdx.x * (long long)kThreads + threadIdx.x; q < m * m; q += (long long)gridDim.x * kThreads) {
        const int i = int(q % m), j = int(q / m);
        const double v = src[q];
        const bool edge = i == 0 || i == n || j == 0 || j == n;
        const int bits = !isfinite(v) ? 1 : (v < 0.0 ? 2 : ((edge && v == 0.0) ? 4 : 0));
        if (bits) {
            atomicOr(flags, bits);
            atomicMin(flags + 1, int(q));
        }
    }
}

// Coupling A(p, p + e) of the fine operator of a Galerkin product.
// Level 0: the shifted Laplacian C_s = A_s - i beta2 W K^2, i.e. the scaled
// 5-point operator of §2 with k^2 replaced by (1 + i beta2) k^2 (§4, §5).
struct FineCoupling {
    int level;
    Grid g;
    int r;
    const cplx<double>* coef;
    const double* k2;
    double ih2, two_h, shift;
    __device__ cplx<double> operator()(int px, int py, int ex, int ey) const {
        if (level > 0) {
            const int D = 2 * r + 1;
            return coef[(long long)((ey + r) * D + ex + r) * g.plane + g.at(px, py)];
        }
        return level0(px, py, ex, ey, k2[g.at(px, py)]);
    }
    // level 0 with k^2 at p given
    __device__ __forceinline__ cplx<double> level0(int px, int py, int ex, int ey, double kk) const {
        const int n = g.n;
        if (ex == 0 && ey == 0) {
            const double W = line_w<double>(px, n) * line_w<double>(py, n);
            const int s = (px == 0 || px == n) + (py == 0 || py == n);
            const double im = -shift * kk - (s ? two_h * s * sqrt(kk) : 0.0);
            return {W * (4.0 * ih2 - kk), W * im};
        }
        if (ey == 0 && (ex == 1 || ex == -1)) return {-ih2 * line_w<double>(py, n), 0.0};
        if (ex == 0 && (ey == 1 || ey == -1)) return {-ih2 * line_w<double>(px, n), 0.0};
        return {0.0, 0.0};
    }
};

// One coarse coefficient per thread: A_c(I, I + D) = sum_p R(I, p) sum_q A(p, q) P(q, I + D)
// with R = P^T / 4 (§3 Galerkin condition, §4 transfers).
__global__ __launch_bounds__(kThreads) void k_galerkin(FineCoupling A, Grid gc, int rc, int bez, cplx<double>* out) {
    const long long mc = gc.n + 1;
    const int Dc = 2 * rc + 1;
    const long long total = mc * mc * Dc * Dc;
    const int nf = A.g.n;
    const int rf = A.r;
    for (long long t = blockIdx.x * (long long)kThreads + threadIdx.x; t < total; t += (long long)gridDim.x * kThreads) {
        const long long node = t % (mc * mc);
        const int d = int(t / (mc * mc));
        const int Ix = int(node % mc), Iy = int(node / mc);
        const int Dx = d % Dc - rc, Dy = d / Dc - rc;
        const int Kx = Ix + Dx, Ky = Iy + Dy;
        cplx<double> acc{0.0, 0.0};
        if (Kx >= 0 && Kx <= gc.n && Ky >= 0 && Ky <= gc.n) {
            for (int ay = -2; ay <= 2; ++ay) {
                const int py = 2 * Iy + ay;
                if (py < 0 || py > nf) continue;
                for (int ax = -2; ax <= 2; ++ax) {
                    const int px = 2 * Ix + ax;
                    if (px < 0 || px > nf) continue;
                    const double rw = 0.25 * mask1(ax, bez) * mask1(ay, bez);
                    if (rw == 0.0) continue;
                    const int ey0 = max(-rf, 2 * Ky - 2 - py), ey1 = min(rf, 2 * Ky + 2 - py);
                    const int ex0 = max(-rf, 2 * Kx - 2 - px), ex1 = min(rf, 2 * Kx + 2 - px);
                    for (int ey = ey0; ey <= ey1; ++ey) {
                        const int qy = py + ey;
                        if (qy < 0 || qy > nf) continue;
                        const double wy = mask1(qy - 2 * Ky, bez);
                        if (wy == 0.0) continue;
                        for (int ex = ex0; ex <= ex1; ++ex) {
                            const int qx = px + ex;
                            if (qx < 0 || qx > nf) continue;
                            const double w = rw * wy * mask1(qx - 2 * Kx, bez);
                            if (w == 0.0) continue;
                            const cplx<double> a = A(px, py, ex, ey);
                            acc.re += w * a.re;
                            acc.im += w * a.im;
                        }
                    }
                }
            }
        }
        out[(long long)d * gc.plane + gc.at(Ix, Iy)] = acc;
    }
}

// Level 1 from the level-0 couplings, one coarse node per thread with its D^2
// coefficients (D = 5 Bézier, 3 linear) in registers:
//   A_1(I, I + dK) = sum_a sum_e W(a, e, dK) C(2I + a, e),
// a the restriction tap (|a| <= 2 per dimension), e one of the five couplings
// of the fine node p = 2I + a, and W = (1/4) m(a) m(a + e - 2 dK) with the 1D
// masks m per dimension: a compile-time table, so only the couplings C are
// loaded (25 fine nodes per coarse node). Taps and couplings off the grid and
// coarse neighbours off the coarse grid contribute nothing.
template <bool kBez>
__global__ __launch_bounds__(kThreads) void k_galerkin0(FineCoupling A, Grid gc, cplx<double>* out) {
    constexpr int rc = kBez ? 2 : 1;
    constexpr int D = 2 * rc + 1;
    const long long mc = gc.n + 1;
    const int nf = A.g.n, nc = gc.n;
    for (long long node = blockIdx.x * (long long)kThreads + threadIdx.x; node < mc * mc;
         node += (long long)gridDim.x * kThreads) {
        const int Ix = int(node % mc), Iy = int(node / mc);
        cplx<double> acc[D * D];
#pragma unroll
        for (int d = 0; d < D * D; ++d) acc[d] = {0.0, 0.0};
        // k^2 of the 25 taps, loaded before any is used (left to itself the
        // compiler waits for each load in turn)
        double kk[5][5];
#pragma unroll
        for (int ay = -2; ay <= 2; ++ay)
#pragma unroll
            for (int ax = -2; ax <= 2; ++ax)
                kk[ay + 2][ax + 2] = A.k2[A.g.at(min(max(2 * Ix + ax, 0), nf), min(max(2 * Iy + ay, 0), nf))];
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int ay = -2; ay <= 2; ++ay)
#pragma unroll
            for (int ax = -2; ax <= 2; ++ax) {
                const double rw = 0.25 * mask1(ax, kBez) * mask1(ay, kBez);
                if (rw == 0.0) continue;  // compile-time (linear transfer)
                const int px = 2 * Ix + ax, py = 2 * Iy + ay;
                const bool pin = px >= 0 && px <= nf && py >= 0 && py <= nf;
                const int pxc = min(max(px, 0), nf), pyc = min(max(py, 0), nf);
#pragma unroll
                for (int e = 0; e < 5; ++e) {
                    const int ex = e == 1 ? -1 : e == 2 ? 1 : 0;
                    const int ey = e == 3 ? -1 : e == 4 ? 1 : 0;
                    const int qx = px + ex, qy = py + ey;
                    const bool ok = pin && qx >= 0 && qx <= nf && qy >= 0 && qy <= nf;
                    const cplx<double> a =
                        ok ? A.level0(pxc, pyc, ex, ey, kk[ay + 2][ax + 2]) : cplx<double>{0.0, 0.0};
#pragma unroll
                    for (int dy = -rc; dy <= rc; ++dy)
#pragma unroll
                        for (int dx = -rc; dx <= rc; ++dx) {
                            const double w = rw * mask1(ax + ex - 2 * dx, kBez) * mask1(ay + ey - 2 * dy, kBez);
                            if (w == 0.0) continue;  // compile-time
                            acc[(dy + rc) * D + dx + rc].re += w * a.re;
                            acc[(dy + rc) * D + dx + rc].im += w * a.im;
                        }
                }
            }
#pragma unroll
        for (int dy = -rc; dy <= rc; ++dy)
#pragma unroll
            for (int dx = -rc; dx <= rc; ++dx) {
                const int Kx = Ix + dx, Ky = Iy + dy;
                const bool kin = Kx >= 0 && Kx <= nc && Ky >= 0 && Ky <= nc;
                out[(long long)((dy + rc) * D + dx + rc) * gc.plane + gc.at(Ix, Iy)] =
                    kin ? acc[(dy + rc) * D + dx + rc] : cplx<double>{0.0, 0.0};
            }
    }
}

// Levels >= 1 from a stored fine stencil of radius RF, one coarse node per
// thread. With s = a + e the offset of the fine column node q = 2I + s from the
// fine image 2I of coarse node I, the product factors as
//   G(I, s)      = sum_a R(a) A(2I + a, s - a)          (restriction taps a)
//   A_c(I, I+d)  = sum_s G(I, s) m(s_x - 2d_x) m(s_y - 2d_y)
// since P(q, I + d) depends on q - 2(I + d) = s - 2d only. Rows s_y are formed
// one at a time (row of G, then the x mask, then the y mask into the D_c^2
// coefficients), so each fine coupling is loaded once per coarse node and only
// one row of G is live. Loads use clamped indices and are masked afterwards,
// so they carry no branches and overlap.
constexpr int kNodeThreads = 64;

template <bool kBez, int RF>
__global__ __launch_bounds__(kNodeThreads) void k_galerkin_node(Grid gf, const cplx<double>* coef, Grid gc,
                                                                cplx<double>* out) {
    constexpr int RA = kBez ? 2 : 1;  // restriction taps |a| <= RA per dimension
    constexpr int RS = RA + RF;
    constexpr int NS = 2 * RS + 1;
    constexpr int RC = (2 * RA + RF) / 2;  // coarse stencil radius
    constexpr int DC = 2 * RC + 1;
    constexpr int DF = 2 * RF + 1;
    const long long mc = gc.n + 1;
    const int nf = gf.n, nc = gc.n;
    for (long long node = blockIdx.x * (long long)kNodeThreads + threadIdx.x; node < mc * mc;
         node += (long long)gridDim.x * kNodeThreads) {
        const int Ix = int(node % mc), Iy = int(node / mc);
        cplx<double> acc[DC * DC];
#pragma unroll
        for (int d = 0; d < DC * DC; ++d) acc[d] = {0.0, 0.0};
#pragma unroll
        for (int sy = -RS; sy <= RS; ++sy) {
            cplx<double> G[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) G[q] = {0.0, 0.0};
#pragma unroll
            for (int ay = -RA; ay <= RA; ++ay) {
                const int ey = sy - ay;
                if (ey < -RF || ey > RF) continue;  // compile-time
                const int py = 2 * Iy + ay, qy = py + ey;
                const bool yok = py >= 0 && py <= nf && qy >= 0 && qy <= nf;
                const int pyc = min(max(py, 0), nf);
                // the couplings of this tap row are loaded before any is used
                // (left to itself the compiler waits for each load in turn)
                cplx<double> v[2 * RA + 1][DF];
#pragma unroll
                for (int ax = -RA; ax <= RA; ++ax) {
                    const long long at = gf.at(min(max(2 * Ix + ax, 0), nf), pyc);
#pragma unroll
                    for (int ex = -RF; ex <= RF; ++ex)
                        v[ax + RA][ex + RF] = coef[(long long)((ey + RF) * DF + ex + RF) * gf.plane + at];
                }
                __asm__ volatile("" ::: "memory");
#pragma unroll
                for (int ax = -RA; ax <= RA; ++ax) {
                    const double rw = 0.25 * mask1(ax, kBez) * mask1(ay, kBez);
                    if (rw == 0.0) continue;  // compile-time
                    const int px = 2 * Ix + ax;
                    const bool pok = yok && px >= 0 && px <= nf;
#pragma unroll
                    for (int ex = -RF; ex <= RF; ++ex) {
                        const int qx = px + ex;
                        const bool ok = pok && qx >= 0 && qx <= nf;
                        const cplx<double> a = v[ax + RA][ex + RF];
                        G[ax + ex + RS].re += ok ? rw * a.re : 0.0;
                        G[ax + ex + RS].im += ok ? rw * a.im : 0.0;
                    }
                }
            }
#pragma unroll
            for (int dx = -RC; dx <= RC; ++dx) {
                cplx<double> h{0.0, 0.0};
#pragma unroll
                for (int sx = -RS; sx <= RS; ++sx) {
                    const double w = mask1(sx - 2 * dx, kBez);
                    if (w == 0.0) continue;  // compile-time
                    h.re += w * G[sx + RS].re;
                    h.im += w * G[sx + RS].im;
                }
#pragma unroll
                for (int dy = -RC; dy <= RC; ++dy) {
                    const double w = mask1(sy - 2 * dy, kBez);
                    if (w == 0.0) continue;  // compile-time
                    acc[(dy + RC) * DC + dx + RC].re += w * h.re;
                    acc[(dy + RC) * DC + dx + RC].im += w * h.im;
                }
            }
        }
#pragma unroll
        for (int dy = -RC; dy <= RC; ++dy)
#pragma unroll
            for (int dx = -RC; dx <= RC; ++dx) {
                const int Kx = Ix + dx, Ky = Iy + dy;
                const bool kin = Kx >= 0 && Kx <= nc && Ky >= 0 && Ky <= nc;
                out[(long long)((dy + RC) * DC + dx + RC) * gc.plane + gc.at(Ix, Iy)] =
                    kin ? acc[(dy + RC) * DC + dx + RC] : cplx<double>{0.0, 0.0};
            }
    }
}

// The same product on small coarse grids, where a node kernel's long
// per-thread chain of loads sets the time: one thread per coarse node,
// stencil row dy and y-mask tap t. It forms the row s_y = 2 dy + t of G,
// reduces it over s_x and scales it by m(t); the taps of a row are then summed
// in LDS in ascending t (a fixed order). A block holds 64 (node, row) pairs
// times the taps, threadIdx.y being the tap.
constexpr int kSplitLanes = 64;

template <bool kBez, int RF>
__global__ __launch_bounds__(kSplitLanes * (kBez ? 5 : 3)) void k_galerkin_split(Grid gf, const cplx<double>* coef,
                                                                                Grid gc, cplx<double>* out) {
    constexpr int RA = kBez ? 2 : 1;  // restriction taps and nonzero y-mask taps: |t| <= RA
    constexpr int NT = 2 * RA + 1;
    constexpr int RS = RA + RF;
    constexpr int NS = 2 * RS + 1;
    constexpr int RC = (2 * RA + RF) / 2;
    constexpr int DC = 2 * RC + 1;
    constexpr int DF = 2 * RF + 1;
    __shared__ cplx<double> part[NT][DC][kSplitLanes];
    const long long mc = gc.n + 1;
    const int nf = gf.n, nc = gc.n;
    const int lane = threadIdx.x, ti = threadIdx.y, t = ti - RA;
    const long long q = blockIdx.x * (long long)kSplitLanes + lane;  // (node, row) pair; the grid covers them once
    const bool pair_ok = q < mc * mc * DC;
    const long long node = pair_ok ? q % (mc * mc) : 0;
    const int dy = pair_ok ? int(q / (mc * mc)) - RC : 0;
    const int Ix = int(node % mc), Iy = int(node / mc);
    const int sy = 2 * dy + t;
    const bool row_ok = pair_ok && sy >= -RS && sy <= RS;
    cplx<double> G[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) G[s] = {0.0, 0.0};
    if (row_ok) {
#pragma unroll
        for (int ay = -RA; ay <= RA; ++ay) {
            const int ey = sy - ay;
            const bool eok = ey >= -RF && ey <= RF;
            const int eyc = min(max(ey, -RF), RF);
            const int py = 2 * Iy + ay, qy = py + ey;
            const bool yok = eok && py >= 0 && py <= nf && qy >= 0 && qy <= nf;
            const int pyc = min(max(py, 0), nf);
            const cplx<double>* crow = coef + (long long)((eyc + RF) * DF + RF) * gf.plane;
#pragma unroll
            for (int ax = -RA; ax <= RA; ++ax) {
                const double rw = 0.25 * mask1(ax, kBez) * mask1(ay, kBez);
                if (rw == 0.0) continue;  // compile-time
                const int px = 2 * Ix + ax;
                const bool pok = yok && px >= 0 && px <= nf;
                const long long at = gf.at(min(max(px, 0), nf), pyc);
#pragma unroll
                for (int ex = -RF; ex <= RF; ++ex) {
                    const int qx = px + ex;
                    const bool ok = pok && qx >= 0 && qx <= nf;
                    const cplx<double> v = crow[(long long)ex * gf.plane + at];
                    G[ax + ex + RS].re += ok ? rw * v.re : 0.0;
                    G[ax + ex + RS].im += ok ? rw * v.im : 0.0;
                }
            }
        }
    }
    // y weight m(t) of this tap (0 for |t| > RA never occurs: NT covers |t| <= RA)
    const double wy = kBez ? (t == 0 ? 0.75 : (t == 1 || t == -1) ? 0.5 : 0.125) : (t == 0 ? 1.0 : 0.5);
#pragma unroll
    for (int dx = -RC; dx <= RC; ++dx) {
        cplx<double> h{0.0, 0.0};
#pragma unroll
        for (int sx = -RS; sx <= RS; ++sx) {
            const double w = mask1(sx - 2 * dx, kBez);
            if (w == 0.0) continue;  // compile-time
            h.re += w * G[sx + RS].re;
            h.im += w * G[sx + RS].im;
        }
        part[ti][dx + RC][lane] = cplx<double>{wy * h.re, wy * h.im};
    }
    __syncthreads();
    if (ti != 0 || !pair_ok) return;
    const int Ky = Iy + dy;
#pragma unroll
    for (int dx = -RC; dx <= RC; ++dx) {
        cplx<double> acc{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            acc.re += part[k][dx + RC][lane].re;
            acc.im += part[k][dx + RC][lane].im;
        }
        const int Kx = Ix + dx;
        const bool kin = Kx >= 0 && Kx <= nc && Ky >= 0 && Ky <= nc;
        out[(long long)((dy + RC) * DC + dx + RC) * gc.plane + gc.at(Ix, Iy)] = kin ? acc : cplx<double>{0.0, 0.0};
    }
}

__global__ __launch_bounds__(kThreads) void k_cast_coef(const cplx<double>* src, cplx<float>* dst, long long count) {
    for (long long q = blockIdx.x * (long long)kThreads + threadIdx.x; q < count; q += (long long)gridDim.x * kThreads)
        dst[q] = cast<float>(src[q]);
}

// Dense coarsest matrix, row P = J m + I, column Q = P + (Dy m + Dx).
__global__ __launch_bounds__(kThreads) void k_dense(Grid g, int r, const cplx<double>* coef, cplx<double>* dense) {
    const int m = g.n + 1;
    const int N = m * m;
    const int D = 2 * r + 1;
    for (long long t = blockIdx.x * (long long)kThreads + threadIdx.x; t < (long long)N * N;
         t += (long long)gridDim.x * kThreads)
        dense[t] = {0.0, 0.0};
    __syncthreads();
    // single block: the zero fill above and the scatter below are ordered by the barrier
    for (long long t = threadIdx.x; t < (long long)N * D * D; t += kThreads) {
        const int P = int(t % N), d = int(t / N);
        const int I = P % m, J = P / m;
        const int dx = d % D - r, dy = d / D - r;
        const int Kx = I + dx, Ky = J + dy;
        if (Kx < 0 || Kx > g.n || Ky < 0 || Ky > g.n) continue;
        dense[(long long)P * N + Ky * m + Kx] = coef[(long long)d * g.plane + g.at(I, J)];
    }
}

__device__ __forceinline__ double cabs1(cplx<double> a) { return fabs(a.re) + fabs(a.im); }

// In-place LU with partial pivoting (largest |re| + |im| in the column, first
// index on ties), row-major; piv[k] is the row swapped with row k at step k.
__global__ __launch_bounds__(kThreads) void k_lu(int N, cplx<double>* A, int* piv) {
    __shared__ double sv[kThreads];
    __shared__ int si[kThreads];
    const int tid = threadIdx.x;
    for (int k = 0; k < N; ++k) {
        double best = -1.0;
        int bi = N;
        for (int i = k + tid; i < N; i += kThreads) {
            const double v = cabs1(A[(long long)i * N + k]);
            if (v > best) { best = v; bi = i; }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (tid < s) {
                const double v2 = sv[tid + s];
                const int i2 = si[tid + s];
                if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) { sv[tid] = v2; si[tid] = i2; }
            }
            __syncthreads();
        }
        const int p = si[0];
        if (tid == 0) piv[k] = p;
        if (p != k)
            for (int c = tid; c < N; c += kThreads) {
                const cplx<double> t = A[(long long)k * N + c];
                A[(long long)k * N + c] = A[(long long)p * N + c];
                A[(long long)p * N + c] = t;
            }
        __syncthreads();
        const cplx<double> pivot = A[(long long)k * N + k];
        for (int i = k + 1 + tid; i < N; i += kThreads) A[(long long)i * N + k] = cdiv(A[(long long)i * N + k], pivot);
        __syncthreads();
        const int rem = N - k - 1;
        for (long long t = tid; t < (long long)rem * rem; t += kThreads) {
            const int i = k + 1 + int(t / rem), c = k + 1 + int(t % rem);
            const cplx<double> l = A[(long long)i * N + k];
            const cplx<double> uu = A[(long long)k * N + c];
            const cplx<double> a = A[(long long)i * N + c];
            A[(long long)i * N + c] = a - l * uu;
        }
        __syncthreads();
    }
}

// One wavefront per right-hand side: permute, unit-lower forward and upper
// back substitution in FP64 (complex64 data is widened). Small factors are
// staged in LDS so that the N sequential steps read no global memory.
constexpr int kSolveThreads = 64;
constexpr int kMaxLdsLU = 45 * 45;

template <typename T>
__global__ __launch_bounds__(kSolveThreads) void k_coarse_solve(Grid g, const cplx<double>* LU, const int* piv, Vec<T> f,
                                                                Vec<T> u, const int* active) {
    const int b = blockIdx.x;
    if (!rhs_active(active, b)) return;
    __shared__ cplx<double> x[kMaxCoarse];
    __shared__ cplx<double> lu_s[kMaxLdsLU];
    __shared__ int piv_s[kMaxCoarse];
    const int m = g.n + 1;
    const int N = m * m;
    const int tid = threadIdx.x;
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* ub = u.rhs(b);
    const bool staged = N * N <= kMaxLdsLU;
    for (int P = tid; P < N; P += kSolveThreads) {
        x[P] = cast<double>(fb[g.at(P % m, P / m)]);
        piv_s[P] = piv[P];
    }
    if (staged)
        for (int q = tid; q < N * N; q += kSolveThreads) lu_s[q] = LU[q];
    __syncthreads();
    lu_substitute(staged ? lu_s : LU, piv_s, x, N, tid, kSolveThreads);
    for (int P = tid; P < N; P += kSolveThreads) ub[g.at(P % m, P / m)] = cast<T>(x[P]);
}

__global__ __launch_bounds__(kThreads) void k_stencil_out(Grid g, int r, const cplx<double>* coef, cplx<double>* out) {
    const long long m = g.n + 1;
    const int D = 2 * r + 1;
    const long long total = m * m * D * D;
    for (long long t = blockIdx.x * (long long)kThreads + threadIdx.x; t < total; t += (long long)gridDim.x * kThreads) {
        const long long node = t % (m * m);
        const int d = int(t / (m * m));
        out[t] = coef[(long long)d * g.plane + g.at(int(node % m), int(node / m))];
    }
}

unsigned blocks_for(long long work) {
    long long b = (work + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

}  // namespace

void launch_check_k2(hipStream_t s, int n, const double* k2_dense, int* flags) {
    const long long m = n + 1;
    hipLaunchKernelGGL(k_check_k2, dim3(blocks_for(m * m)), dim3(kThreads), 0, s, n, k2_dense, flags);
}

void launch_k2_in(hipStream_t s, Grid g, const double* k2_dense, double* k2_64, float* k2_32) {
    const long long m = g.n + 1;
    hipLaunchKernelGGL(k_k2_in, dim3(blocks_for(m * m)), dim3(kThreads), 0, s, g, k2_dense, k2_64, k2_32);
}

void launch_galerkin(hipStream_t s, int fine_level, Grid fine, int fine_radius, const cplx<double>* fine_coef,
                     const double* k2_64, double h, double shift, int transfer, Grid coarse, int coarse_radius,
                     cplx<double>* coarse_coef) {
    FineCoupling A{fine_level, fine, fine_radius, fine_coef, k2_64, 1.0 / (h * h), 2.0 / h, shift};
    const long long mc = coarse.n + 1;
    if (fine_level == 0 && coarse_radius == (transfer == 0 ? 2 : 1)) {
        if (transfer == 0)
            hipLaunchKernelGGL(k_galerkin0<true>, dim3(blocks_for(mc * mc)), dim3(kThreads), 0, s, A, coarse,
                               coarse_coef);
        else
            hipLaunchKernelGGL(k_galerkin0<false>, dim3(blocks_for(mc * mc)), dim3(kThreads), 0, s, A, coarse,
                               coarse_coef);
        return;
    }
    const unsigned node_blocks = (unsigned)std::min<long long>((mc * mc + kNodeThreads - 1) / kNodeThreads, 65536);
    const bool bez = transfer == 0;
    // coarse grids of at most 128 intervals: one stencil row and y tap per thread
    const bool rows = mc <= 129;
    const long long dc = 2 * coarse_radius + 1;
    auto run = [&](auto node_kernel, auto rows_kernel) {
        if (rows)
            hipLaunchKernelGGL(rows_kernel, dim3(unsigned((mc * mc * dc + kSplitLanes - 1) / kSplitLanes)),
                               dim3(kSplitLanes, bez ? 5 : 3), 0, s, fine, fine_coef, coarse, coarse_coef);
        else
            hipLaunchKernelGGL(node_kernel, dim3(node_blocks), dim3(kNodeThreads), 0, s, fine, fine_coef, coarse,
                               coarse_coef);
    };
    if (fine_level > 0 && coarse_radius == (bez ? (4 + fine_radius) / 2 : (2 + fine_radius) / 2)) {
        if (bez && fine_radius == 2) {
            run(k_galerkin_node<true, 2>, k_galerkin_split<true, 2>);
            return;
        }
        if (bez && fine_radius == 3) {
            run(k_galerkin_node<true, 3>, k_galerkin_split<true, 3>);
            return;
        }
        if (!bez && fine_radius == 1) {
            run(k_galerkin_node<false, 1>, k_galerkin_split<false, 1>);
            return;
        }
    }
    const long long D = 2 * coarse_radius + 1;
    hipLaunchKernelGGL(k_galerkin, dim3(blocks_for(mc * mc * D * D)), dim3(kThreads), 0, s, A, coarse, coarse_radius,
                       int(transfer == 0), coarse_coef);
}

void launch_cast_coef(hipStream_t s, const cplx<double>* src, cplx<float>* dst, long long count) {
    hipLaunchKernelGGL(k_cast_coef, dim3(blocks_for(count)), dim3(kThreads), 0, s, src, dst, count);
}

void launch_dense_lu(hipStream_t s, Grid g, int radius, const cplx<double>* coef, cplx<double>* dense, int* piv) {
    const int m = g.n + 1;
    hipLaunchKernelGGL(k_dense, dim3(1), dim3(kThreads), 0, s, g, radius, coef, dense);
    hipLaunchKernelGGL(k_lu, dim3(1), dim3(kThreads), 0, s, m * m, dense, piv);
}

template <typename T>
void launch_coarse_solve(const LaunchCtx& ctx, Grid g, const cplx<double>* lu, const int* piv, Vec<T> f, Vec<T> u) {
    hipLaunchKernelGGL((k_coarse_solve<T>), dim3(ctx.nrhs), dim3(kSolveThreads), 0, ctx.stream, g, lu, piv, f, u,
                       ctx.active);
}
template void launch_coarse_solve<double>(const LaunchCtx&, Grid, const cplx<double>*, const int*, Vec<double>,
                                          Vec<double>);
template void launch_coarse_solve<float>(const LaunchCtx&, Grid, const cplx<double>*, const int*, Vec<float>,
                                         Vec<float>);

void launch_stencil_out(hipStream_t s, Grid g, int radius, const cplx<double>* coef, void* out) {
    const long long m = g.n + 1;
    const long long D = 2 * radius + 1;
    hipLaunchKernelGGL(k_stencil_out, dim3(blocks_for(m * m * D * D)), dim3(kThreads), 0, s, g, radius, coef,
                       static_cast<cplx<double>*>(out));
}

}  // namespace hm
