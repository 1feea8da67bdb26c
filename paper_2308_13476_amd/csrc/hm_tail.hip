// Coarse tail of the cycle: one workgroup per right-hand side runs the whole
// sub-cycle (§3 coarse grid correction, §5 V/W cycles) on the small levels at
// the bottom of the hierarchy. Every vector of those levels lives in LDS for
// the whole sub-cycle; only the Galerkin stencil planes are read from global
// memory (they stay in L2 between the passes). Barriers and block reductions
// replace the kernel launches and grid-wide reductions of the level kernels,
// which on grids of at most 33 x 33 nodes cost far more than the arithmetic.
#include "hm_ops.hpp"

namespace hm {
namespace {

// Wavefronts of the tail workgroup: 5 in FP32, the fewest that give each of
// the 289 nodes of a 16-interval level its own thread (fewer wavefronts per
// barrier and block sum; 5 measured faster than 8, and 8 than 4); 4 in FP64,
// whose larger registers spill when a SIMD holds two of its wavefronts.
template <typename T>
constexpr int kTailBY = sizeof(T) == 8 ? 4 : 5;
template <typename T>
constexpr int kTailThreads = kBX * kTailBY<T>;

template <typename T>
__device__ __forceinline__ double tn2(cplx<T> z) {
    return double(z.re) * double(z.re) + double(z.im) * double(z.im);
}

// re + i im += conj(a) w
template <typename T>
__device__ __forceinline__ void tdot(double& re, double& im, cplx<T> a, cplx<T> w) {
    re += double(a.re) * double(w.re) + double(a.im) * double(w.im);
    im += double(a.re) * double(w.im) - double(a.im) * double(w.re);
}

// One level of the tail: its stencil in global memory and its LDS planes.
// LDS planes have a zero frame of kTailGhost nodes: node (i, j) sits at
// (j + kTailGhost) * lp + i + kTailGhost.
template <typename T>
struct TLv {
    Grid g;  // global layout (coefficient planes)
    int radius;
    const cplx<T>* coef;
    int m, lp;
    cplx<T>* pl;  // planes: u, f, then z0, z1, z2, wa, wb on smoothed levels
    __device__ __forceinline__ cplx<T>* u() const { return pl; }
    __device__ __forceinline__ cplx<T>* f() const { return pl + lp * lp; }
    __device__ __forceinline__ cplx<T>* s(int k) const { return pl + (2 + k) * lp * lp; }
    __device__ __forceinline__ int li(int i, int j) const { return (j + kTailGhost) * lp + i + kTailGhost; }
};

template <typename T>
__device__ __forceinline__ TLv<T> tail_level(const TailArgs<T>& a, int q, cplx<T>* lds) {
    TLv<T> v;
    v.g = a.lv[q].g;
    v.radius = a.lv[q].radius;
    v.m = v.g.n + 1;
    v.lp = tail_pitch(v.g.n);
    v.coef = a.lv[q].coef;
    long long off = 0;
    for (int r = 0; r < q; ++r) off += tail_plane_values(a.lv[r].g.n, r, a.nlev);
    v.pl = lds + off;
    return v;
}

// All threads visit the nodes of a level: f(i, j, LDS index, global index).
template <typename T, typename F>
__device__ __forceinline__ void tnodes(const TLv<T>& L, F&& f) {
    const int N = L.m * L.m;
    for (int q = thread_linear(); q < N; q += kTailThreads<T>) {
        const int i = q % L.m, j = q / L.m;
        f(i, j, L.li(i, j), L.g.at(i, j));
    }
}

// Stencil of radius R at one node; x from LDS. The coefficients are loaded
// in batches of stencil rows that are all issued before the first product
// (the empty asm keeps the compiler from interleaving each load with its
// use, which would leave one load in flight per wave).
template <typename T, int R>
__device__ __forceinline__ cplx<T> tapply(const TLv<T>& L, const cplx<T>* x, int li, long long gp) {
    constexpr int D = 2 * R + 1;
    constexpr int RB = sizeof(T) == 4 ? 7 : 4;  // stencil rows per batch
    const cplx<T>* cp = L.coef + gp;
    const long long pl = L.g.plane;
    cplx<T> y{T(0), T(0)};
#pragma unroll
    for (int r0 = 0; r0 < D; r0 += RB) {
        cplx<T> c[RB][D];
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (r0 + r < D)
#pragma unroll
                for (int dx = 0; dx < D; ++dx) c[r][dx] = cp[((r0 + r) * D + dx) * pl];
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (r0 + r < D)
#pragma unroll
                for (int dx = 0; dx < D; ++dx) y = cfma(y, c[r][dx], x[li + (r0 + r - R) * L.lp + dx - R]);
    }
    return y;
}

template <typename T, int R>
__device__ __forceinline__ cplx<T> tdiag(const TLv<T>& L, long long gp) {
    constexpr int D = 2 * R + 1;
    return L.coef[(R * D + R) * L.g.plane + gp];
}

template <typename T, typename F>
__device__ __forceinline__ void with_radius(const TLv<T>& L, F&& f) {
    if (L.radius == 1) f(std::integral_constant<int, 1>{});
    else if (L.radius == 2) f(std::integral_constant<int, 2>{});
    else f(std::integral_constant<int, 3>{});
}

template <typename T>
__device__ void tail_jacobi(const TLv<T>& L, double inv_omega) {
    const T w = T(inv_omega);
    cplx<T>* u = L.u();
    cplx<T>* t = L.s(3);
    with_radius(L, [&](auto Rc) {
        constexpr int R = decltype(Rc)::value;
        tnodes(L, [&](int, int, int li, long long gp) {
            const cplx<T> r = L.f()[li] - tapply<T, R>(L, u, li, gp);
            t[li] = u[li] + w * cdiv(r, tdiag<T, R>(L, gp));
        });
    });
    __syncthreads();
    tnodes(L, [&](int, int, int li, long long) { u[li] = t[li]; });
    __syncthreads();
}

// One GMRES(3) smoothing step (§5.3): classical Gram-Schmidt Arnoldi on
// unnormalised vectors z_j with scale s_j = 1 / ||z_j||, the same recurrences
// as the multi-kernel path, reductions inside the block. u_zero: u holds
// zeros (the level was just entered by restriction), so the first residual
// is f itself and is read in place. res (only with u_zero): the plane of w_0
// receives the residual f - A u' of the updated iterate, formed by recurrence
// as z_0 - sum_i c_i w_i (w_2 is kept in the first scratch plane, which z_0
// does not use); returns whether it was formed.
template <typename T>
__device__ bool tail_gmres(const TLv<T>& L, double breakdown, bool u_zero, cplx<T>* res) {
    cplx<T>* u = L.u();
    const cplx<T>* f = L.f();
    cplx<T>* z0w = L.s(0);
    const cplx<T>* z0 = u_zero ? f : z0w;
    cplx<T>* z1 = L.s(1);
    cplx<T>* z2 = L.s(2);
    cplx<T>* wa = L.s(3);
    cplx<T>* wb = L.s(4);
    double hr[4][3] = {}, hi[4][3] = {}, s[3] = {};
    int k = 3;
    double beta;
    with_radius(L, [&](auto Rc) {
        constexpr int R = decltype(Rc)::value;
        // Each Arnoldi vector's norm is summed in the pass that applies A to
        // it, together with that pass's inner products: one block sum per
        // column (the values, and the order of every sum, are those of
        // separate sums; a breakdown found there discards the apply).
        if (!u_zero) {
            tnodes(L, [&](int, int, int li, long long gp) { z0w[li] = f[li] - tapply<T, R>(L, u, li, gp); });
            __syncthreads();
        }
        // column 0: w = A z0; beta = ||z0||, H00 = s0^2 <z0, w>
        double a3[3] = {0.0, 0.0, 0.0}, t3[3];
        tnodes(L, [&](int, int, int li, long long gp) {
            const cplx<T> w = tapply<T, R>(L, z0, li, gp);
            wa[li] = w;
            a3[0] += tn2(z0[li]);
            tdot(a3[1], a3[2], z0[li], w);
        });
        block_sum<3>(a3, t3);
        beta = sqrt(t3[0]);
        if (!(beta > 0.0)) {
            k = 0;
            return;
        }
        s[0] = 1.0 / beta;
        hr[0][0] = s[0] * s[0] * t3[1];
        hi[0][0] = s[0] * s[0] * t3[2];
        // z1 = s0 w - H00 s0 z0
        {
            const cplx<T> c0 = {T(hr[0][0] * s[0]), T(hi[0][0] * s[0])};
            const T sc = T(s[0]);
            tnodes(L, [&](int, int, int li, long long) {
                const cplx<T> zq = z0[li];
                cplx<T> v = sc * wa[li];
                v.re -= c0.re * zq.re - c0.im * zq.im;
                v.im -= c0.re * zq.im + c0.im * zq.re;
                z1[li] = v;
            });
            __syncthreads();
        }
        // column 1: w1 = A z1; ||z1||, <z0, w1>, <z1, w1>
        double a5[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, t5[5];
        tnodes(L, [&](int, int, int li, long long gp) {
            const cplx<T> w = tapply<T, R>(L, z1, li, gp);
            wb[li] = w;
            a5[0] += tn2(z1[li]);
            tdot(a5[1], a5[2], z0[li], w);
            tdot(a5[3], a5[4], z1[li], w);
        });
        block_sum<5>(a5, t5);
        hr[1][0] = sqrt(t5[0]);
        hi[1][0] = 0.0;
        if (!(hr[1][0] > breakdown * beta)) {
            k = 1;
            return;
        }
        s[1] = 1.0 / hr[1][0];
        for (int q = 0; q < 2; ++q) {
            hr[q][1] = s[q] * s[1] * t5[1 + 2 * q];
            hi[q][1] = s[q] * s[1] * t5[2 + 2 * q];
        }
        {
            const cplx<T> c0 = {T(hr[0][1] * s[0]), T(hi[0][1] * s[0])};
            const cplx<T> c1 = {T(hr[1][1] * s[1]), T(hi[1][1] * s[1])};
            const T sc = T(s[1]);
            tnodes(L, [&](int, int, int li, long long) {
                const cplx<T> q0 = z0[li], q1 = z1[li];
                cplx<T> v = sc * wb[li];
                v.re -= c0.re * q0.re - c0.im * q0.im + c1.re * q1.re - c1.im * q1.im;
                v.im -= c0.re * q0.im + c0.im * q0.re + c1.re * q1.im + c1.im * q1.re;
                z2[li] = v;
            });
            __syncthreads();
        }
        // column 2: w2 = A z2; ||z2||, <z_i, w2>, ||w2||^2, and
        // ||z_3||^2 = s_2^2 ||w2||^2 - sum |H[i][2]|^2 (orthonormal s_i z_i)
        double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, t8[8];
        tnodes(L, [&](int, int, int li, long long gp) {
            const cplx<T> w = tapply<T, R>(L, z2, li, gp);
            if (res) z0w[li] = w;
            a8[0] += tn2(z2[li]);
            tdot(a8[1], a8[2], z0[li], w);
            tdot(a8[3], a8[4], z1[li], w);
            tdot(a8[5], a8[6], z2[li], w);
            a8[7] += tn2(w);
        });
        block_sum<8>(a8, t8);
        hr[2][1] = sqrt(t8[0]);
        hi[2][1] = 0.0;
        if (!(hr[2][1] > breakdown * beta)) {
            k = 2;
            return;
        }
        s[2] = 1.0 / hr[2][1];
        double sq = s[2] * s[2] * t8[7];
        for (int q = 0; q < 3; ++q) {
            hr[q][2] = s[q] * s[2] * t8[1 + 2 * q];
            hi[q][2] = s[q] * s[2] * t8[2 + 2 * q];
            sq -= hr[q][2] * hr[q][2] + hi[q][2] * hi[q][2];
        }
        hr[3][2] = sqrt(fmax(sq, 0.0));
        hi[3][2] = 0.0;
    });
    if (k == 0) return false;
    // every thread holds the same H (block sums are identical in all
    // threads) and solves the least-squares problem in registers
    double yr[3], yi[3];
    gm_least_squares_regs(hr, hi, s, beta, k, yr, yi);
    cplx<T> c[3];
    for (int q = 0; q < 3; ++q) c[q] = {T(yr[q]), T(yi[q])};
    const cplx<T> m0 = {-c[0].re, -c[0].im}, m1 = {-c[1].re, -c[1].im}, m2 = {-c[2].re, -c[2].im};
    const cplx<T>* w2 = z0w;
    tnodes(L, [&](int, int, int li, long long) {
        cplx<T> x = u[li];
        x = cfma(x, c[0], z0[li]);
        if (k > 1) x = cfma(x, c[1], z1[li]);
        if (k > 2) x = cfma(x, c[2], z2[li]);
        u[li] = x;
        if (res) {  // read before the store: res is the plane of w_0
            cplx<T> r = cfma(z0[li], m0, wa[li]);
            if (k > 1) r = cfma(r, m1, wb[li]);
            if (k > 2) r = cfma(r, m2, w2[li]);
            res[li] = r;
        }
    });
    __syncthreads();
    return res != nullptr;
}

// f_c = R (f - A u) (§4 transfers, R = P^T / 4) and u_c = 0. The residual
// goes to scratch plane wa of the fine level (r_ready: the last smoothing
// step already put it there); the LDS frame supplies the zero ghosts that
// truncate the mask at the boundary.
template <typename T>
__device__ void tail_residual_restrict(const TLv<T>& L, const TLv<T>& C, bool bez, bool r_ready) {
    cplx<T>* w = L.s(3);
    if (!r_ready) {
        with_radius(L, [&](auto Rc) {
            constexpr int R = decltype(Rc)::value;
            tnodes(L, [&](int, int, int li, long long gp) { w[li] = L.f()[li] - tapply<T, R>(L, L.u(), li, gp); });
        });
        __syncthreads();
    }
    const T w5[5] = {T(1), T(4), T(6), T(4), T(1)};
    const T w3[5] = {T(0), T(1), T(2), T(1), T(0)};
    const T* mw = bez ? w5 : w3;
    const T scale = T(bez ? 1.0 / 256.0 : 1.0 / 16.0);
    tnodes(C, [&](int I, int J, int lc, long long) {
        const int pf = L.li(2 * I, 2 * J);
        cplx<T> acc{T(0), T(0)};
        for (int dy = -2; dy <= 2; ++dy) {
            cplx<T> row{T(0), T(0)};
            for (int dx = -2; dx <= 2; ++dx) {
                const cplx<T> v = w[pf + dy * L.lp + dx];
                row.re += mw[dx + 2] * v.re;
                row.im += mw[dx + 2] * v.im;
            }
            acc.re += mw[dy + 2] * row.re;
            acc.im += mw[dy + 2] * row.im;
        }
        C.f()[lc] = scale * acc;
        C.u()[lc] = cplx<T>{T(0), T(0)};
    });
    __syncthreads();
}

// u += P e (§4 prolongation; the zero frame of the coarse plane truncates).
template <typename T>
__device__ void tail_prolong(const TLv<T>& C, const TLv<T>& L, bool bez) {
    const cplx<T>* e = C.u();
    tnodes(L, [&](int i, int j, int li, long long) {
        T wx[3], wy[3];
        const bool ox = i & 1, oy = j & 1;
        wx[0] = ox ? T(0) : (bez ? T(0.125) : T(0));
        wx[1] = ox ? T(0.5) : (bez ? T(0.75) : T(1));
        wx[2] = ox ? T(0.5) : (bez ? T(0.125) : T(0));
        wy[0] = oy ? T(0) : (bez ? T(0.125) : T(0));
        wy[1] = oy ? T(0.5) : (bez ? T(0.75) : T(1));
        wy[2] = oy ? T(0.5) : (bez ? T(0.125) : T(0));
        const int pc = C.li((i >> 1) - 1, (j >> 1) - 1);
        cplx<T> acc{T(0), T(0)};
        for (int ty = 0; ty < 3; ++ty) {
            cplx<T> row{T(0), T(0)};
            for (int tx = 0; tx < 3; ++tx) {
                const cplx<T> v = e[pc + ty * C.lp + tx];
                row.re += wx[tx] * v.re;
                row.im += wx[tx] * v.im;
            }
            acc.re += wy[ty] * row.re;
            acc.im += wy[ty] * row.im;
        }
        L.u()[li] = L.u()[li] + acc;
    });
    __syncthreads();
}

// u = A_c^{-1} f on the coarsest level with the explicit FP64 inverse
// (complex64 data is widened): one row per thread.
template <typename T>
__device__ void tail_coarse(const TLv<T>& C, const cplx<double>* inv) {
    const int N = C.m * C.m;
    const cplx<T>* f = C.f();
    for (int r = thread_linear(); r < N; r += kTailThreads<T>) {
        const cplx<double>* row = inv + (long long)r * N;
        cplx<double> acc{0.0, 0.0};
        for (int P = 0; P < N; ++P) acc = cfma(acc, row[P], cast<double>(f[C.li(P % C.m, P / C.m)]));
        C.u()[C.li(r % C.m, r / C.m)] = cast<T>(acc);
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kTailThreads<T>) void k_tail(TailArgs<T> a, const int* active) {
    const int b = blockIdx.x;
    if (!rhs_active(active, b)) return;
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(hm_dyn_lds);
    const int last = a.nlev - 1;
    // zero every plane (the frames must read zero), stage the coarsest
    // inverse in LDS when it fits, then load the top level
    {
        const long long total = a.plane_bytes / (long long)sizeof(cplx<T>);
        for (long long q = thread_linear(); q < total; q += kTailThreads<T>) lds[q] = cplx<T>{T(0), T(0)};
        unsigned char* base = reinterpret_cast<unsigned char*>(lds);
        if (a.inv_off >= 0) {
            const int N = (a.lv[a.nlev - 1].g.n + 1) * (a.lv[a.nlev - 1].g.n + 1);
            cplx<double>* dst = reinterpret_cast<cplx<double>*>(base + a.inv_off);
            constexpr int IB = 4;
            cplx<double> v[IB];
            for_strided_batched<IB>(N * N, [&](int u, int q) { v[u] = a.inv[q]; }, [&](int u, int q) { dst[q] = v[u]; });
        }
        __syncthreads();
        const TLv<T> L = tail_level(a, 0, lds);
        const long long off = (long long)b * L.g.plane;
        const bool load_u = a.top_zero == 0;  // otherwise the zeroed plane is the iterate
        tnodes(L, [&](int i, int j, int li, long long) {
            if (load_u) L.u()[li] = a.u_top[off + L.g.at(i, j)];
            L.f()[li] = a.f_top[off + L.g.at(i, j)];
        });
        __syncthreads();
    }
    const cplx<double>* inv = a.inv_off >= 0
                                  ? reinterpret_cast<const cplx<double>*>(reinterpret_cast<unsigned char*>(lds) + a.inv_off)
                                  : a.inv;
    const double inv_omega = 1.0 / a.omega;
    const bool bez = a.bez != 0;
    // Cycle state machine with a single smoothing site (keeps the GMRES
    // passes inlined once): going down, level q is pre-smoothed and its
    // residual restricted; coming back up after its last coarse visit, the
    // correction is prolongated and q is post-smoothed.
    unsigned visits = 0u;  // 2 bits per level: coarse visits left
    int q = 0;
    bool up = false;
    bool fresh = a.top_zero != 0;  // level q holds u = 0 (entered by restriction, not yet smoothed)
    if (last == 0) {
        tail_coarse(tail_level(a, 0, lds), inv);
    } else {
        for (;;) {
            int nu;
            if (!up) {
                if (q == last) {
                    tail_coarse(tail_level(a, q, lds), inv);
                    q -= 1;
                    up = true;
                    continue;
                }
                nu = a.nu1;
            } else {
                // back from one visit of level q + 1: u now holds a result
                fresh = false;
                const unsigned left = ((visits >> (2 * q)) & 3u) - 1u;
                visits = (visits & ~(3u << (2 * q))) | (left << (2 * q));
                if (left > 0) {
                    q += 1;
                    up = false;
                    continue;
                }
                tail_prolong(tail_level(a, q + 1, lds), tail_level(a, q, lds), bez);
                nu = a.nu2;
            }
            bool r_ready = false;  // the last step left f - A u in the restriction's plane
            {
                const TLv<T> L = tail_level(a, q, lds);
                for (int s = 0; s < nu; ++s) {
                    if (a.smoother == 0) {
                        tail_jacobi(L, inv_omega);
                    } else {
                        // a single pre-smoothing step from u = 0 also forms the residual to restrict
                        const bool zero = fresh && s == 0;
                        r_ready = tail_gmres(L, a.breakdown, zero, zero && !up && s + 1 == nu ? L.s(3) : nullptr);
                    }
                }
            }
            if (!up) {
                tail_residual_restrict(tail_level(a, q, lds), tail_level(a, q + 1, lds), bez, r_ready);
                visits = (visits & ~(3u << (2 * q))) | (unsigned(a.gamma) << (2 * q));
                q += 1;
                fresh = true;
            } else {
                if (q == 0) break;
                q -= 1;
            }
        }
    }
    const TLv<T> L = tail_level(a, 0, lds);
    const long long off = (long long)b * L.g.plane;
    tnodes(L, [&](int i, int j, int li, long long) { a.u_top[off + L.g.at(i, j)] = L.u()[li]; });
}

// X = A^{-1} from the row-major LU factor with row swaps piv (X = U^{-1} L^{-1} P),
// N <= kTailMaxCoarseNodes, X staged in LDS.
constexpr int kInvThreads = 1024;
__global__ __launch_bounds__(kInvThreads) void k_lu_inverse(int N, const cplx<double>* LU, const int* piv,
                                                           cplx<double>* inv) {
    cplx<double>* X = reinterpret_cast<cplx<double>*>(hm_dyn_lds);
    __shared__ int perm[kTailMaxCoarseNodes];
    const int tid = threadIdx.x;
    if (tid == 0) {
        for (int r = 0; r < N; ++r) perm[r] = r;
        for (int k = 0; k < N; ++k) {
            const int p = piv[k];
            const int t = perm[k];
            perm[k] = perm[p];
            perm[p] = t;
        }
    }
    __syncthreads();
    // (P I)[r][c] = 1 where perm[r] == c
    for (int t = tid; t < N * N; t += kInvThreads) X[t] = cplx<double>{perm[t / N] == t % N ? 1.0 : 0.0, 0.0};
    __syncthreads();
    for (int k = 0; k < N; ++k) {  // unit lower
        const int rem = N - k - 1;
        for (int t = tid; t < rem * N; t += kInvThreads) {
            const int r = k + 1 + t / N, c = t % N;
            X[r * N + c] = X[r * N + c] - LU[(long long)r * N + k] * X[k * N + c];
        }
        __syncthreads();
    }
    for (int k = N - 1; k >= 0; --k) {  // upper
        const cplx<double> d = LU[(long long)k * N + k];
        for (int c = tid; c < N; c += kInvThreads) X[k * N + c] = cdiv(X[k * N + c], d);
        __syncthreads();
        for (int t = tid; t < k * N; t += kInvThreads) {
            const int r = t / N, c = t % N;
            X[r * N + c] = X[r * N + c] - LU[(long long)r * N + k] * X[k * N + c];
        }
        __syncthreads();
    }
    for (int t = tid; t < N * N; t += kInvThreads) inv[t] = X[t];
}

}  // namespace

void tail_init() {
    static const bool done = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(kTailMaxLdsBytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(kTailMaxLdsBytes));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lu_inverse),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(kTailMaxCoarseNodes * kTailMaxCoarseNodes * sizeof(cplx<double>)));
        return true;
    }();
    (void)done;
}

template <typename T>
void launch_tail(const LaunchCtx& ctx, const TailArgs<T>& args) {
    hipLaunchKernelGGL((k_tail<T>), dim3(ctx.nrhs), dim3(kBX, kTailBY<T>), size_t(args.lds_bytes), ctx.stream, args,
                       ctx.active);
}
template void launch_tail<double>(const LaunchCtx&, const TailArgs<double>&);
template void launch_tail<float>(const LaunchCtx&, const TailArgs<float>&);

void launch_lu_inverse(hipStream_t s, int N, const cplx<double>* lu, const int* piv, cplx<double>* inv) {
    hipLaunchKernelGGL(k_lu_inverse, dim3(1), dim3(kInvThreads), size_t(N) * N * sizeof(cplx<double>), s, N, lu, piv,
                       inv);
}

}  // namespace hm
