// Coarse tail of the cycle: one workgroup per right-hand side runs the whole
// sub-cycle (§3 coarse grid correction, §5 V/W cycles) on the small levels at
// the bottom of the hierarchy, with block-level reductions and barriers in
// place of kernel launches. On these grids (at most 33 x 33 nodes) a launch
// per operation costs far more than the arithmetic.
#include "hm_ops.hpp"

namespace hm {
namespace {

constexpr int kTailBY = 8;
constexpr int kTailThreads = kBX * kTailBY;
constexpr int kTailMaxCoarse = 1089;
constexpr int kTailMaxLdsLU = 45 * 45;

template <typename T>
__device__ __forceinline__ double tn2(cplx<T> z) {
    return double(z.re) * double(z.re) + double(z.im) * double(z.im);
}

template <typename T>
__device__ __forceinline__ void tdot(double& re, double& im, cplx<T> a, cplx<T> w) {
    re += double(a.re) * double(w.re) + double(a.im) * double(w.im);
    im += double(a.re) * double(w.im) - double(a.im) * double(w.re);
}

// All threads of the block visit the nodes of a level.
template <typename F>
__device__ __forceinline__ void blk_nodes(const Grid& g, F&& f) {
    const int m = g.n + 1;
    const int N = m * m;
    for (int q = thread_linear(); q < N; q += kTailThreads) {
        const int i = q % m, j = q / m;
        f(i, j, g.at(i, j));
    }
}

// The level's Galerkin stencil as an operator object.
template <typename T, typename F>
__device__ __forceinline__ void with_stencil(const TailLevel<T>& L, F&& f) {
    if (L.radius == 1) f(StencilOp<T, 1>{L.g, L.coef});
    else if (L.radius == 2) f(StencilOp<T, 2>{L.g, L.coef});
    else f(StencilOp<T, 3>{L.g, L.coef});
}

// Per-right-hand-side pointers of one level, with the Jacobi ping-pong
// (u and t exchange roles after every sweep).
template <typename T>
struct Lv {
    TailLevel<T> d;
    cplx<T>* u;
    cplx<T>* t;
};

template <typename T>
__device__ __forceinline__ Lv<T> level_view(const TailArgs<T>& a, int l, int b, unsigned swapped) {
    Lv<T> v;
    v.d = a.lv[l];
    const long long pl = v.d.g.plane;
    v.d.u += b * pl;
    v.d.f += b * pl;
    v.d.t += b * pl;
    v.d.w += b * pl;
    v.d.Z += 4 * b * pl;
    const bool sw = (swapped >> l) & 1u;
    v.u = sw ? v.d.t : v.d.u;
    v.t = sw ? v.d.u : v.d.t;
    return v;
}

template <typename T>
__device__ void tail_jacobi(const Lv<T>& L, double inv_omega) {
    const T w = T(inv_omega);
    with_stencil(L.d, [&](auto op) {
        blk_nodes(L.d.g, [&](int i, int j, long long p) {
            const cplx<T> r = L.d.f[p] - op.apply(L.u, i, j, p);
            L.t[p] = L.u[p] + w * cdiv(r, op.diag(i, j, p));
        });
    });
    __syncthreads();
}

// One GMRES(3) smoothing step (§5.3): classical Gram-Schmidt Arnoldi with the
// same recurrences as the multi-kernel path, reductions inside the block.
template <typename T>
__device__ void tail_gmres(const Lv<T>& L, double breakdown, GmState& S, LsWork& ls) {
    const Grid& g = L.d.g;
    cplx<T>* z0 = L.d.Z;
    cplx<T>* z1 = z0 + g.plane;
    cplx<T>* z2 = z1 + g.plane;
    cplx<T>* wa = L.d.w;
    cplx<T>* wb = L.t;
    double hr[4][3], hi[4][3], s[3];
    int k = 3;
    double beta;
    with_stencil(L.d, [&](auto op) {
        double a1[1] = {0.0}, t1[1];
        blk_nodes(g, [&](int i, int j, long long p) {
            const cplx<T> z = L.d.f[p] - op.apply(L.u, i, j, p);
            z0[p] = z;
            a1[0] += tn2(z);
        });
        block_sum<1>(a1, t1);
        beta = sqrt(t1[0]);
        if (!(beta > 0.0)) {
            k = 0;
            return;
        }
        s[0] = 1.0 / beta;
        // column 0
        double a2[2] = {0.0, 0.0}, t2[2];
        blk_nodes(g, [&](int i, int j, long long p) {
            const cplx<T> w = op.apply(z0, i, j, p);
            wa[p] = w;
            tdot(a2[0], a2[1], z0[p], w);
        });
        block_sum<2>(a2, t2);
        hr[0][0] = s[0] * s[0] * t2[0];
        hi[0][0] = s[0] * s[0] * t2[1];
        // z1 = s0 w0 - H00 s0 z0
        {
            const cplx<T> c0 = {T(hr[0][0] * s[0]), T(hi[0][0] * s[0])};
            const T sc = T(s[0]);
            blk_nodes(g, [&](int, int, long long p) {
                const cplx<T> zq = z0[p];
                cplx<T> v = sc * wa[p];
                v.re -= c0.re * zq.re - c0.im * zq.im;
                v.im -= c0.re * zq.im + c0.im * zq.re;
                z1[p] = v;
            });
        }
        a1[0] = 0.0;
        blk_nodes(g, [&](int, int, long long p) { a1[0] += tn2(z1[p]); });
        block_sum<1>(a1, t1);
        hr[1][0] = sqrt(t1[0]);
        hi[1][0] = 0.0;
        if (!(hr[1][0] > breakdown * beta)) {
            k = 1;
            return;
        }
        s[1] = 1.0 / hr[1][0];
        // column 1
        double a4[4] = {0.0, 0.0, 0.0, 0.0}, t4[4];
        blk_nodes(g, [&](int i, int j, long long p) {
            const cplx<T> w = op.apply(z1, i, j, p);
            wb[p] = w;
            tdot(a4[0], a4[1], z0[p], w);
            tdot(a4[2], a4[3], z1[p], w);
        });
        block_sum<4>(a4, t4);
        for (int q = 0; q < 2; ++q) {
            hr[q][1] = s[q] * s[1] * t4[2 * q];
            hi[q][1] = s[q] * s[1] * t4[2 * q + 1];
        }
        {
            const cplx<T> c0 = {T(hr[0][1] * s[0]), T(hi[0][1] * s[0])};
            const cplx<T> c1 = {T(hr[1][1] * s[1]), T(hi[1][1] * s[1])};
            const T sc = T(s[1]);
            a1[0] = 0.0;
            blk_nodes(g, [&](int, int, long long p) {
                const cplx<T> q0 = z0[p], q1 = z1[p];
                cplx<T> v = sc * wb[p];
                v.re -= c0.re * q0.re - c0.im * q0.im + c1.re * q1.re - c1.im * q1.im;
                v.im -= c0.re * q0.im + c0.im * q0.re + c1.re * q1.im + c1.im * q1.re;
                z2[p] = v;
                a1[0] += tn2(v);
            });
            block_sum<1>(a1, t1);
        }
        hr[2][1] = sqrt(t1[0]);
        hi[2][1] = 0.0;
        if (!(hr[2][1] > breakdown * beta)) {
            k = 2;
            return;
        }
        s[2] = 1.0 / hr[2][1];
        // column 2
        double a6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, t6[6];
        blk_nodes(g, [&](int i, int j, long long p) {
            const cplx<T> w = op.apply(z2, i, j, p);
            wa[p] = w;
            tdot(a6[0], a6[1], z0[p], w);
            tdot(a6[2], a6[3], z1[p], w);
            tdot(a6[4], a6[5], z2[p], w);
        });
        block_sum<6>(a6, t6);
        for (int q = 0; q < 3; ++q) {
            hr[q][2] = s[q] * s[2] * t6[2 * q];
            hi[q][2] = s[q] * s[2] * t6[2 * q + 1];
        }
        {
            cplx<T> c[3];
            for (int q = 0; q < 3; ++q) c[q] = {T(hr[q][2] * s[q]), T(hi[q][2] * s[q])};
            const T sc = T(s[2]);
            a1[0] = 0.0;
            blk_nodes(g, [&](int, int, long long p) {
                cplx<T> v = sc * wa[p];
                const cplx<T> q0 = z0[p], q1 = z1[p], q2 = z2[p];
                v.re -= c[0].re * q0.re - c[0].im * q0.im + c[1].re * q1.re - c[1].im * q1.im + c[2].re * q2.re -
                        c[2].im * q2.im;
                v.im -= c[0].re * q0.im + c[0].im * q0.re + c[1].re * q1.im + c[1].im * q1.re + c[2].re * q2.im +
                        c[2].im * q2.re;
                a1[0] += tn2(v);
            });
            block_sum<1>(a1, t1);
        }
        hr[3][2] = sqrt(t1[0]);
        hi[3][2] = 0.0;
    });
    if (k == 0) return;
    if (thread_linear() == 0) {
        S.beta = beta;
        S.k = k;
        for (int q = 0; q < 3; ++q) S.s[q] = (q < k) ? s[q] : 0.0;
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) {
                const bool used = (c < k) && (a <= c + 1);
                S.hr[a][c] = used ? hr[a][c] : 0.0;
                S.hi[a][c] = used ? hi[a][c] : 0.0;
            }
        gm_least_squares(S, ls);
    }
    __syncthreads();
    cplx<T> c[3];
    for (int q = 0; q < 3; ++q) c[q] = {T(S.yr[q]), T(S.yi[q])};
    blk_nodes(g, [&](int, int, long long p) {
        cplx<T> x = L.u[p];
        x = cfma(x, c[0], z0[p]);
        if (k > 1) x = cfma(x, c[1], z1[p]);
        if (k > 2) x = cfma(x, c[2], z2[p]);
        L.u[p] = x;
    });
    __syncthreads();
}

// f_c = R (f - A u) (§4 transfers, R = P^T / 4) and u_c = 0.
template <typename T>
__device__ void tail_residual_restrict(const Lv<T>& L, const Lv<T>& C, bool bez) {
    with_stencil(L.d, [&](auto op) {
        blk_nodes(L.d.g, [&](int i, int j, long long p) { L.d.w[p] = L.d.f[p] - op.apply(L.u, i, j, p); });
    });
    __syncthreads();
    const Grid& gf = L.d.g;
    blk_nodes(C.d.g, [&](int I, int J, long long pc) {
        const long long pf = gf.at(2 * I, 2 * J);
        const T w5[5] = {T(1), T(4), T(6), T(4), T(1)};
        const T w3[5] = {T(0), T(1), T(2), T(1), T(0)};
        const T* w = bez ? w5 : w3;
        cplx<T> acc{T(0), T(0)};
        for (int dy = -2; dy <= 2; ++dy) {
            cplx<T> row{T(0), T(0)};
            for (int dx = -2; dx <= 2; ++dx) {
                const cplx<T> v = L.d.w[pf + (long long)dy * gf.pitch + dx];
                row.re += w[dx + 2] * v.re;
                row.im += w[dx + 2] * v.im;
            }
            acc.re += w[dy + 2] * row.re;
            acc.im += w[dy + 2] * row.im;
        }
        C.d.f[pc] = T(bez ? 1.0 / 256.0 : 1.0 / 16.0) * acc;
        C.u[pc] = cplx<T>{T(0), T(0)};
    });
    __syncthreads();
}

// u += P e (§4 prolongation; coarse ghosts are zero, which truncates).
template <typename T>
__device__ void tail_prolong(const Lv<T>& C, const Lv<T>& L, bool bez) {
    const Grid& gc = C.d.g;
    blk_nodes(L.d.g, [&](int i, int j, long long pf) {
        T wx[3], wy[3];
        const bool ox = i & 1, oy = j & 1;
        wx[0] = ox ? T(0) : (bez ? T(0.125) : T(0));
        wx[1] = ox ? T(0.5) : (bez ? T(0.75) : T(1));
        wx[2] = ox ? T(0.5) : (bez ? T(0.125) : T(0));
        wy[0] = oy ? T(0) : (bez ? T(0.125) : T(0));
        wy[1] = oy ? T(0.5) : (bez ? T(0.75) : T(1));
        wy[2] = oy ? T(0.5) : (bez ? T(0.125) : T(0));
        const long long pc = gc.at((i >> 1) - 1, (j >> 1) - 1);
        cplx<T> acc{T(0), T(0)};
        for (int ty = 0; ty < 3; ++ty) {
            cplx<T> row{T(0), T(0)};
            for (int tx = 0; tx < 3; ++tx) {
                const cplx<T> v = C.u[pc + (long long)ty * gc.pitch + tx];
                row.re += wx[tx] * v.re;
                row.im += wx[tx] * v.im;
            }
            acc.re += wy[ty] * row.re;
            acc.im += wy[ty] * row.im;
        }
        L.u[pf] = L.u[pf] + acc;
    });
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T> a, const int* active) {
    const int b = blockIdx.x;
    if (!rhs_active(active, b)) return;
    __shared__ cplx<double> x[kTailMaxCoarse];
    __shared__ cplx<double> lu_s[kTailMaxLdsLU];
    __shared__ int piv_s[kTailMaxCoarse];
    __shared__ GmState S;
    __shared__ LsWork ls;
    const int tid = thread_linear();
    const int last = a.nlev - 1;
    const Grid gcst = a.lv[last].g;
    const int mc = gcst.n + 1;
    const int Nc = mc * mc;
    const bool staged = Nc * Nc <= kTailMaxLdsLU;
    for (int q = tid; q < Nc; q += kTailThreads) piv_s[q] = a.piv[q];
    if (staged)
        for (int q = tid; q < Nc * Nc; q += kTailThreads) lu_s[q] = a.lu[q];
    __syncthreads();
    const cplx<double>* LU = staged ? lu_s : a.lu;
    const double inv_omega = 1.0 / a.omega;
    const bool bez = a.bez != 0;

    unsigned swapped = 0u;  // bit l: level l's iterate lives in its t buffer
    unsigned visits = 0u;   // 2 bits per level: coarse visits left
    auto smooth = [&](int l, int nu) {
        for (int s = 0; s < nu; ++s) {
            const Lv<T> L = level_view(a, l, b, swapped);
            if (a.smoother == 0) {
                tail_jacobi(L, inv_omega);
                swapped ^= 1u << l;
            } else {
                tail_gmres(L, a.breakdown, S, ls);
            }
        }
    };
    int l = 0;
    bool up = false;
    for (;;) {
        if (!up) {
            if (l == last) {
                const Lv<T> L = level_view(a, l, b, swapped);
                for (int P = tid; P < Nc; P += kTailThreads) x[P] = cast<double>(L.d.f[gcst.at(P % mc, P / mc)]);
                __syncthreads();
                lu_substitute(LU, piv_s, x, Nc, tid, kTailThreads);
                for (int P = tid; P < Nc; P += kTailThreads) L.u[gcst.at(P % mc, P / mc)] = cast<T>(x[P]);
                __syncthreads();
                if (l == 0) break;
                l -= 1;
                up = true;
                continue;
            }
            smooth(l, a.nu1);
            swapped &= ~(1u << (l + 1));  // the child starts from zero in its u buffer
            tail_residual_restrict(level_view(a, l, b, swapped), level_view(a, l + 1, b, swapped), bez);
            visits = (visits & ~(3u << (2 * l))) | (unsigned(a.gamma) << (2 * l));
            l += 1;
            continue;
        }
        // back from one visit of level l + 1
        const unsigned left = ((visits >> (2 * l)) & 3u) - 1u;
        visits = (visits & ~(3u << (2 * l))) | (left << (2 * l));
        if (left > 0) {
            l += 1;
            up = false;
            continue;
        }
        tail_prolong(level_view(a, l + 1, b, swapped), level_view(a, l, b, swapped), bez);
        smooth(l, a.nu2);
        if (l == 0) break;
        l -= 1;
    }
    // the caller reads the top level's iterate from its u buffer
    if (swapped & 1u) {
        const Lv<T> L = level_view(a, 0, b, 0u);
        blk_nodes(L.d.g, [&](int, int, long long p) { L.u[p] = L.t[p]; });
        __syncthreads();
    }
}

}  // namespace

template <typename T>
void launch_tail(const LaunchCtx& ctx, const TailArgs<T>& args) {
    hipLaunchKernelGGL((k_tail<T>), dim3(ctx.nrhs), dim3(kBX, kTailBY), 0, ctx.stream, args, ctx.active);
}
template void launch_tail<double>(const LaunchCtx&, const TailArgs<double>&);
template void launch_tail<float>(const LaunchCtx&, const TailArgs<float>&);

}  // namespace hm
