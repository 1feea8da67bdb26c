// Level kernels of the multigrid cycle: operator apply, residual, weighted
// Jacobi, transfers, GMRES(3) passes, norms, FP32 refinement, adjoint gradient.
#include "hm_ops.hpp"

namespace hm {
namespace {

constexpr int kThreads = kBX * kBY;

int level_rpt(const Grid& g, int rpt) { return (g.n + 1) < 256 ? 1 : rpt; }

dim3 level_grid(const Grid& g, int rpt, int nrhs) {
    return dim3((g.n + 1 + kBX - 1) / kBX, (g.n + 1 + kBY * rpt - 1) / (kBY * rpt), nrhs);
}

// Calls f(op) with the concrete operator type of the level.
template <typename T, typename F>
void with_op(const LevelOp<T>& lop, F&& f) {
    if (lop.level == 0) {
        f(FineOp<T>{lop.g, lop.k2, T(1.0 / (lop.h * lop.h)), T(2.0 / lop.h)});
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

// ---------------------------------------------------------------- operator
template <typename Op, typename T>
__global__ __launch_bounds__(kThreads) void k_apply(Op op, Vec<T> x, Vec<T> y, const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    cplx<T>* yb = y.rhs(b);
    for_nodes(op.g, rpt, [&](int i, int j, long long p) { yb[p] = op.apply(xb, i, j, p); });
}

template <typename Op, typename T>
__global__ __launch_bounds__(kThreads) void k_residual(Op op, Vec<T> x, Vec<T> f, Vec<T> r, const int* active,
                                                       int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* rb = r.rhs(b);
    for_nodes(op.g, rpt, [&](int i, int j, long long p) { rb[p] = fb[p] - op.apply(xb, i, j, p); });
}

// Weighted Jacobi of §3: y = x + (omega diag(A))^{-1} (f - A x).
template <typename Op, typename T>
__global__ __launch_bounds__(kThreads) void k_jacobi(Op op, Vec<T> x, Vec<T> f, Vec<T> y, T inv_omega,
                                                     const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* yb = y.rhs(b);
    for_nodes(op.g, rpt, [&](int i, int j, long long p) {
        const cplx<T> r = fb[p] - op.apply(xb, i, j, p);
        yb[p] = xb[p] + inv_omega * cdiv(r, op.diag(i, j, p));
    });
}

// ---------------------------------------------------------------- transfers
// Restriction R = P^T / 4 of the §4 prolongation: the 2D row is the outer
// product of [1 4 6 4 1]/16 (Bézier) or [1 2 1]/4 (linear) centred on the
// fine node (2I, 2J); fine ghosts are zero, which truncates at the boundary.
// The coarse iterate that the next cycle starts from (zero) is written in the
// same pass when `uc` is given.
template <typename T, bool kBez>
__global__ __launch_bounds__(kThreads) void k_restrict(Grid gf, Grid gc, Vec<T> r, Vec<T> fc, Vec<T> uc,
                                                       const int* active, int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* rb = r.rhs(b);
    cplx<T>* fb = fc.rhs(b);
    cplx<T>* ub = uc.p ? uc.rhs(b) : nullptr;
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
            fb[pc] = T(1.0 / 256.0) * acc;
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
            fb[pc] = T(1.0 / 16.0) * acc;
        }
    });
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

template <typename T, bool kBez>
__global__ __launch_bounds__(kThreads) void k_prolong_add(Grid gc, Grid gf, Vec<T> e, Vec<T> u, const int* active,
                                                          int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* eb = e.rhs(b);
    cplx<T>* ub = u.rhs(b);
    for_nodes(gf, rpt, [&](int i, int j, long long pf) {
        T wx[3], wy[3];
        taps<T>(i, kBez, wx);
        taps<T>(j, kBez, wy);
        const long long pc = gc.at((i >> 1) - 1, (j >> 1) - 1);
        cplx<T> acc{T(0), T(0)};
#pragma unroll
        for (int ty = 0; ty < 3; ++ty) {
            cplx<T> row{T(0), T(0)};
#pragma unroll
            for (int tx = 0; tx < 3; ++tx) {
                const cplx<T> v = eb[pc + (long long)ty * gc.pitch + tx];
                row.re += wx[tx] * v.re;
                row.im += wx[tx] * v.im;
            }
            acc.re += wy[ty] * row.re;
            acc.im += wy[ty] * row.im;
        }
        ub[pf] = ub[pf] + acc;
    });
}

// ---------------------------------------------------------------- GMRES(3)
// One smoothing step of §5.3 = one restart cycle of 3 GMRES iterations from
// the current iterate. Arnoldi vectors are stored unnormalised (z_j) with
// s_j = 1/||z_j|| kept in GmState; orthogonalisation is classical
// Gram-Schmidt with the new vector's norm computed directly (two passes per
// Arnoldi step: apply + inner products, orthogonalise + norm).

// Least-squares min || beta e1 - H y || over the k Arnoldi columns by complex
// Givens rotations, then y_i s_i into st.yr / st.yi. Run by one thread on a
// shared-memory copy of H so that it costs the calling kernel no registers.
struct LsWork {
    double hr[4][3], hi[4][3], gr[4], gi[4], cs[3], sr[3], si[3], yr[3], yi[3];
};

__device__ __noinline__ void gm_least_squares(GmState& st, LsWork& w) {
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

template <typename Op, typename T>
__global__ __launch_bounds__(kThreads) void k_gm_residual(Op op, Vec<T> u, Vec<T> f, Vec<T> v0, GmState* st,
                                                          const int* active, int rpt, double* partials,
                                                          long long pstride, unsigned* counters) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* ub = u.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    cplx<T>* vb = v0.p + (long long)(b * 4) * v0.plane;  // Arnoldi block of 4 planes per right-hand side
    double acc[1] = {0.0};
    for_nodes(op.g, rpt, [&](int i, int j, long long p) {
        const cplx<T> z = fb[p] - op.apply(ub, i, j, p);
        vb[p] = z;
        acc[0] += dnorm2(z);
    });
    double tot[1];
    if (reduce_last<1>(acc, partials + b * pstride, counters + b, tot) && threadIdx.x == 0 && threadIdx.y == 0) {
        GmState& s = st[b];
        s.beta = sqrt(tot[0]);
        if (s.beta > 0.0) {
            s.s[0] = 1.0 / s.beta;
            s.k = 3;
            s.arnoldi_done = 0;
        } else {
            s.k = 0;
            s.arnoldi_done = 1;
        }
    }
}

// w = A z_J (unscaled); inner products <z_i, w> for i <= J.
template <typename Op, typename T, int J>
__global__ __launch_bounds__(kThreads) void k_gm_apply(Op op, Vec<T> V, Vec<T> w, GmState* st, const int* active,
                                                       int rpt, double* partials, long long pstride,
                                                       unsigned* counters) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b) || st[b].arnoldi_done) return;
    const cplx<T>* z[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) z[i] = V.p + (long long)(b * 4 + i) * V.plane;
    cplx<T>* wb = w.rhs(b);
    double acc[2 * (J + 1)];
#pragma unroll
    for (int i = 0; i < 2 * (J + 1); ++i) acc[i] = 0.0;
    for_nodes(op.g, rpt, [&](int i, int j, long long p) {
        const cplx<T> a = op.apply(z[J], i, j, p);
        wb[p] = a;
        const double wr = double(a.re), wi = double(a.im);
#pragma unroll
        for (int q = 0; q <= J; ++q) {
            const cplx<T> v = z[q][p];
            const double vr = double(v.re), vi = double(v.im);
            acc[2 * q] += vr * wr + vi * wi;
            acc[2 * q + 1] += vr * wi - vi * wr;
        }
    });
    double tot[2 * (J + 1)];
    if (reduce_last<2 * (J + 1)>(acc, partials + b * pstride, counters + b, tot) && threadIdx.x == 0 &&
        threadIdx.y == 0) {
        GmState& s = st[b];
        // H[i][J] = <v_i, A v_J> = s_i s_J <z_i, A z_J>
        for (int q = 0; q <= J; ++q) {
            const double sc = s.s[q] * s.s[J];
            s.hr[q][J] = sc * tot[2 * q];
            s.hi[q][J] = sc * tot[2 * q + 1];
        }
    }
}

// z_{J+1} = s_J w - sum_i H[i][J] s_i z_i, its norm -> H[J+1][J]; at the end of
// the Arnoldi process (breakdown or J = 2) the least-squares problem is solved.
template <typename T, int J>
__global__ __launch_bounds__(kThreads) void k_gm_orth(Grid g, Vec<T> V, Vec<T> w, GmState* st, double breakdown,
                                                      const int* active, int rpt, double* partials,
                                                      long long pstride, unsigned* counters) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b) || st[b].arnoldi_done) return;
    const GmState& s0 = st[b];
    const T sJ = T(s0.s[J]);
    cplx<T> c[J + 1];
#pragma unroll
    for (int q = 0; q <= J; ++q) c[q] = {T(s0.hr[q][J] * s0.s[q]), T(s0.hi[q][J] * s0.s[q])};
    const cplx<T>* z[J + 1];
#pragma unroll
    for (int q = 0; q <= J; ++q) z[q] = V.p + (long long)(b * 4 + q) * V.plane;
    cplx<T>* znew = V.p + (long long)(b * 4 + J + 1) * V.plane;
    const cplx<T>* wb = w.rhs(b);
    double acc[1] = {0.0};
    for_nodes(g, rpt, [&](int i, int j, long long p) {
        cplx<T> v = sJ * wb[p];
#pragma unroll
        for (int q = 0; q <= J; ++q) {
            const cplx<T> zq = z[q][p];
            v.re -= c[q].re * zq.re - c[q].im * zq.im;
            v.im -= c[q].re * zq.im + c[q].im * zq.re;
        }
        if (J < 2) znew[p] = v;
        acc[0] += dnorm2(v);
    });
    double tot[1];
    __shared__ LsWork ls;
    if (reduce_last<1>(acc, partials + b * pstride, counters + b, tot) && threadIdx.x == 0 && threadIdx.y == 0) {
        GmState& s = st[b];
        const double hn = sqrt(tot[0]);
        s.hr[J + 1][J] = hn;
        s.hi[J + 1][J] = 0.0;
        bool done = false;
        if (hn <= breakdown * s.beta) {
            s.k = J + 1;
            done = true;
        } else {
            s.s[J + 1] = 1.0 / hn;
            if (J == 2) {
                s.k = 3;
                done = true;
            }
        }
        if (done) {
            s.arnoldi_done = 1;
            gm_least_squares(s, ls);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gm_update(Grid g, Vec<T> V, Vec<T> u, GmState* st, const int* active,
                                                        int rpt) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const GmState& s = st[b];
    const int k = s.k;
    if (k == 0) return;
    cplx<T> c[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) c[q] = {T(s.yr[q]), T(s.yi[q])};
    const cplx<T>* z0 = V.p + (long long)(b * 4) * V.plane;
    cplx<T>* ub = u.rhs(b);
    for_nodes(g, rpt, [&](int i, int j, long long p) {
        cplx<T> x = ub[p];
        for (int q = 0; q < k; ++q) x = cfma(x, c[q], z0[p + (long long)q * V.plane]);
        ub[p] = x;
    });
}

// ---------------------------------------------------------------- norms
template <typename Op, typename T>
__global__ __launch_bounds__(kThreads) void k_resnorm(Op op, Vec<T> x, Vec<T> f, RhsNorms* norms, const int* active,
                                                      int rpt, double* partials, long long pstride,
                                                      unsigned* counters) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* xb = x.rhs(b);
    const cplx<T>* fb = f.rhs(b);
    double acc[1] = {0.0};
    for_nodes(op.g, rpt, [&](int i, int j, long long p) { acc[0] += dnorm2(fb[p] - op.apply(xb, i, j, p)); });
    double tot[1];
    if (reduce_last<1>(acc, partials + b * pstride, counters + b, tot) && threadIdx.x == 0 && threadIdx.y == 0)
        norms[b].r2 = tot[0];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_norm(Grid g, Vec<T> f, RhsNorms* norms, const int* active, int rpt,
                                                   double* partials, long long pstride, unsigned* counters) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<T>* fb = f.rhs(b);
    double acc[1] = {0.0};
    for_nodes(g, rpt, [&](int, int, long long p) { acc[0] += dnorm2(fb[p]); });
    double tot[1];
    if (reduce_last<1>(acc, partials + b * pstride, counters + b, tot) && threadIdx.x == 0 && threadIdx.y == 0)
        norms[b].f2 = tot[0];
}

// ---------------------------------------------------------------- refinement
__global__ __launch_bounds__(kThreads) void k_refine_residual(FineOp<double> op, Vec<double> x, Vec<double> f,
                                                              Vec<float> r32, RhsNorms* norms, const int* active,
                                                              int rpt, double* partials, long long pstride,
                                                              unsigned* counters) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* xb = x.rhs(b);
    const cplx<double>* fb = f.rhs(b);
    cplx<float>* rb = r32.rhs(b);
    double acc[1] = {0.0};
    for_nodes(op.g, rpt, [&](int i, int j, long long p) {
        const cplx<double> r = fb[p] - op.apply(xb, i, j, p);
        rb[p] = cast<float>(r);
        acc[0] += dnorm2(r);
    });
    double tot[1];
    if (reduce_last<1>(acc, partials + b * pstride, counters + b, tot) && threadIdx.x == 0 && threadIdx.y == 0)
        norms[b].r2 = tot[0];
}

__global__ __launch_bounds__(kThreads) void k_correct_residual(FineOp<double> op, Vec<double> x_in, Vec<float> e,
                                                               Vec<double> x_out, Vec<double> f, Vec<float> r32,
                                                               RhsNorms* norms, const int* active, int rpt,
                                                               double* partials, long long pstride,
                                                               unsigned* counters) {
    const int b = blockIdx.z;
    if (!rhs_active(active, b)) return;
    const cplx<double>* xb = x_in.rhs(b);
    const cplx<float>* eb = e.rhs(b);
    cplx<double>* ob = x_out.rhs(b);
    const cplx<double>* fb = f.rhs(b);
    cplx<float>* rb = r32.rhs(b);
    double acc[1] = {0.0};
    auto xnew = [xb, eb](long long q) { return xb[q] + cast<double>(eb[q]); };
    for_nodes(op.g, rpt, [&](int i, int j, long long p) {
        ob[p] = xnew(p);
        const cplx<double> r = fb[p] - op.apply_at(xnew, i, j, p);
        rb[p] = cast<float>(r);
        acc[0] += dnorm2(r);
    });
    double tot[1];
    if (reduce_last<1>(acc, partials + b * pstride, counters + b, tot) && threadIdx.x == 0 && threadIdx.y == 0)
        norms[b].r2 = tot[0];
}

// ---------------------------------------------------------------- layout
template <typename T, typename S>
__global__ __launch_bounds__(kThreads) void k_copy_in(Grid g, const cplx<S>* src, Vec<T> dst, int scale_w,
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

template <typename T, typename S>
__global__ __launch_bounds__(kThreads) void k_copy_out(Grid g, Vec<T> src, cplx<S>* dst, int scale_w, int conj_,
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
        const double bi = s ? double(s) / (h * sqrt(k2[p])) : 0.0;  // imaginary part of 1 + i s/(h k)
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
#define HM_RED ctx.partials, ctx.max_blocks * 8, ctx.counters

template <typename T>
void launch_apply(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> y) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    with_op(lop, [&](auto op) {
        hipLaunchKernelGGL((k_apply<decltype(op), T>), level_grid(lop.g, rpt, ctx.nrhs), dim3(kBX, kBY), 0,
                           ctx.stream, op, x, y, HM_ACTIVE, rpt);
    });
}

template <typename T>
void launch_residual(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> f, Vec<T> r) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    with_op(lop, [&](auto op) {
        hipLaunchKernelGGL((k_residual<decltype(op), T>), level_grid(lop.g, rpt, ctx.nrhs), dim3(kBX, kBY), 0,
                           ctx.stream, op, x, f, r, HM_ACTIVE, rpt);
    });
}

template <typename T>
void launch_jacobi(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> f, Vec<T> y, double inv_omega) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    with_op(lop, [&](auto op) {
        hipLaunchKernelGGL((k_jacobi<decltype(op), T>), level_grid(lop.g, rpt, ctx.nrhs), dim3(kBX, kBY), 0,
                           ctx.stream, op, x, f, y, T(inv_omega), HM_ACTIVE, rpt);
    });
}

template <typename T>
void launch_restrict(const LaunchCtx& ctx, Grid fine, Grid coarse, int transfer, Vec<T> r, Vec<T> fc, Vec<T> uc) {
    const int rpt = level_rpt(coarse, ctx.rpt);
    const dim3 grid = level_grid(coarse, rpt, ctx.nrhs);
    if (transfer == 0)
        hipLaunchKernelGGL((k_restrict<T, true>), grid, dim3(kBX, kBY), 0, ctx.stream, fine, coarse, r, fc, uc,
                           HM_ACTIVE, rpt);
    else
        hipLaunchKernelGGL((k_restrict<T, false>), grid, dim3(kBX, kBY), 0, ctx.stream, fine, coarse, r, fc, uc,
                           HM_ACTIVE, rpt);
}

template <typename T>
void launch_prolong_add(const LaunchCtx& ctx, Grid coarse, Grid fine, int transfer, Vec<T> e, Vec<T> u) {
    const int rpt = level_rpt(fine, ctx.rpt);
    const dim3 grid = level_grid(fine, rpt, ctx.nrhs);
    if (transfer == 0)
        hipLaunchKernelGGL((k_prolong_add<T, true>), grid, dim3(kBX, kBY), 0, ctx.stream, coarse, fine, e, u,
                           HM_ACTIVE, rpt);
    else
        hipLaunchKernelGGL((k_prolong_add<T, false>), grid, dim3(kBX, kBY), 0, ctx.stream, coarse, fine, e, u,
                           HM_ACTIVE, rpt);
}

template <typename T>
void launch_gm_residual(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> u, Vec<T> f, Vec<T> v0, GmState* st) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    with_op(lop, [&](auto op) {
        hipLaunchKernelGGL((k_gm_residual<decltype(op), T>), level_grid(lop.g, rpt, ctx.nrhs), dim3(kBX, kBY), 0,
                           ctx.stream, op, u, f, v0, st, HM_ACTIVE, rpt, HM_RED);
    });
}

template <typename T>
void launch_gm_apply(const LaunchCtx& ctx, const LevelOp<T>& lop, int j, Vec<T> V, Vec<T> w, GmState* st) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    with_op(lop, [&](auto op) {
        using Op = decltype(op);
        const dim3 grid = level_grid(lop.g, rpt, ctx.nrhs);
        if (j == 0)
            hipLaunchKernelGGL((k_gm_apply<Op, T, 0>), grid, dim3(kBX, kBY), 0, ctx.stream, op, V, w, st, HM_ACTIVE,
                               rpt, HM_RED);
        else if (j == 1)
            hipLaunchKernelGGL((k_gm_apply<Op, T, 1>), grid, dim3(kBX, kBY), 0, ctx.stream, op, V, w, st, HM_ACTIVE,
                               rpt, HM_RED);
        else
            hipLaunchKernelGGL((k_gm_apply<Op, T, 2>), grid, dim3(kBX, kBY), 0, ctx.stream, op, V, w, st, HM_ACTIVE,
                               rpt, HM_RED);
    });
}

template <typename T>
void launch_gm_orth(const LaunchCtx& ctx, Grid g, int j, Vec<T> V, Vec<T> w, GmState* st, double breakdown) {
    const int rpt = level_rpt(g, ctx.rpt);
    const dim3 grid = level_grid(g, rpt, ctx.nrhs);
    if (j == 0)
        hipLaunchKernelGGL((k_gm_orth<T, 0>), grid, dim3(kBX, kBY), 0, ctx.stream, g, V, w, st, breakdown, HM_ACTIVE,
                           rpt, HM_RED);
    else if (j == 1)
        hipLaunchKernelGGL((k_gm_orth<T, 1>), grid, dim3(kBX, kBY), 0, ctx.stream, g, V, w, st, breakdown, HM_ACTIVE,
                           rpt, HM_RED);
    else
        hipLaunchKernelGGL((k_gm_orth<T, 2>), grid, dim3(kBX, kBY), 0, ctx.stream, g, V, w, st, breakdown, HM_ACTIVE,
                           rpt, HM_RED);
}

template <typename T>
void launch_gm_update(const LaunchCtx& ctx, Grid g, Vec<T> V, Vec<T> u, GmState* st) {
    const int rpt = level_rpt(g, ctx.rpt);
    hipLaunchKernelGGL((k_gm_update<T>), level_grid(g, rpt, ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, g, V, u, st,
                       HM_ACTIVE, rpt);
}

template <typename T>
void launch_resnorm(const LaunchCtx& ctx, const LevelOp<T>& lop, Vec<T> x, Vec<T> f, RhsNorms* norms) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    with_op(lop, [&](auto op) {
        hipLaunchKernelGGL((k_resnorm<decltype(op), T>), level_grid(lop.g, rpt, ctx.nrhs), dim3(kBX, kBY), 0,
                           ctx.stream, op, x, f, norms, HM_ACTIVE, rpt, HM_RED);
    });
}

template <typename T>
void launch_norm(const LaunchCtx& ctx, Grid g, Vec<T> f, RhsNorms* norms) {
    const int rpt = level_rpt(g, ctx.rpt);
    hipLaunchKernelGGL((k_norm<T>), level_grid(g, rpt, ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, g, f, norms,
                       HM_ACTIVE, rpt, HM_RED);
}

void launch_refine_residual(const LaunchCtx& ctx, const LevelOp<double>& lop, Vec<double> x, Vec<double> f,
                            Vec<float> r32, RhsNorms* norms) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    FineOp<double> op{lop.g, lop.k2, 1.0 / (lop.h * lop.h), 2.0 / lop.h};
    hipLaunchKernelGGL(k_refine_residual, level_grid(lop.g, rpt, ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, op, x, f,
                       r32, norms, HM_ACTIVE, rpt, HM_RED);
}

void launch_correct_residual(const LaunchCtx& ctx, const LevelOp<double>& lop, Vec<double> x_in, Vec<float> e,
                             Vec<double> x_out, Vec<double> f, Vec<float> r32, RhsNorms* norms) {
    const int rpt = level_rpt(lop.g, ctx.rpt);
    FineOp<double> op{lop.g, lop.k2, 1.0 / (lop.h * lop.h), 2.0 / lop.h};
    hipLaunchKernelGGL(k_correct_residual, level_grid(lop.g, rpt, ctx.nrhs), dim3(kBX, kBY), 0, ctx.stream, op, x_in,
                       e, x_out, f, r32, norms, HM_ACTIVE, rpt, HM_RED);
}

template <typename T>
void launch_copy_in(const LaunchCtx& ctx, Grid g, const void* src, bool src_is_f32, Vec<T> dst, bool scale_w,
                    bool conj) {
    const int rpt = level_rpt(g, ctx.rpt);
    const dim3 grid = level_grid(g, rpt, ctx.nrhs);
    if (src_is_f32)
        hipLaunchKernelGGL((k_copy_in<T, float>), grid, dim3(kBX, kBY), 0, ctx.stream, g,
                           static_cast<const cplx<float>*>(src), dst, int(scale_w), int(conj), rpt);
    else
        hipLaunchKernelGGL((k_copy_in<T, double>), grid, dim3(kBX, kBY), 0, ctx.stream, g,
                           static_cast<const cplx<double>*>(src), dst, int(scale_w), int(conj), rpt);
}

template <typename T>
void launch_copy_out(const LaunchCtx& ctx, Grid g, Vec<T> src, void* dst, bool dst_is_f32, bool scale_w, bool conj) {
    const int rpt = level_rpt(g, ctx.rpt);
    const dim3 grid = level_grid(g, rpt, ctx.nrhs);
    if (dst_is_f32)
        hipLaunchKernelGGL((k_copy_out<T, float>), grid, dim3(kBX, kBY), 0, ctx.stream, g, src,
                           static_cast<cplx<float>*>(dst), int(scale_w), int(conj), rpt);
    else
        hipLaunchKernelGGL((k_copy_out<T, double>), grid, dim3(kBX, kBY), 0, ctx.stream, g, src,
                           static_cast<cplx<double>*>(dst), int(scale_w), int(conj), rpt);
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
    const int rpt = level_rpt(g, ctx.rpt);
    hipLaunchKernelGGL(k_grad_k2, level_grid(g, rpt, 1), dim3(kBX, kBY), 0, ctx.stream, g, h, k2, u, mu,
                       grad_k2_dense, ctx.nrhs, rpt);
}

#define HM_INST(T)                                                                                              \
    template void launch_apply<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>);                         \
    template void launch_residual<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, Vec<T>);              \
    template void launch_jacobi<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, Vec<T>, double);        \
    template void launch_restrict<T>(const LaunchCtx&, Grid, Grid, int, Vec<T>, Vec<T>, Vec<T>);                \
    template void launch_prolong_add<T>(const LaunchCtx&, Grid, Grid, int, Vec<T>, Vec<T>);                     \
    template void launch_gm_residual<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, Vec<T>, GmState*); \
    template void launch_gm_apply<T>(const LaunchCtx&, const LevelOp<T>&, int, Vec<T>, Vec<T>, GmState*);       \
    template void launch_gm_orth<T>(const LaunchCtx&, Grid, int, Vec<T>, Vec<T>, GmState*, double);             \
    template void launch_gm_update<T>(const LaunchCtx&, Grid, Vec<T>, Vec<T>, GmState*);                        \
    template void launch_resnorm<T>(const LaunchCtx&, const LevelOp<T>&, Vec<T>, Vec<T>, RhsNorms*);            \
    template void launch_norm<T>(const LaunchCtx&, Grid, Vec<T>, RhsNorms*);                                    \
    template void launch_copy_in<T>(const LaunchCtx&, Grid, const void*, bool, Vec<T>, bool, bool);             \
    template void launch_copy_out<T>(const LaunchCtx&, Grid, Vec<T>, void*, bool, bool, bool);                  \
    template void launch_zero<T>(hipStream_t, cplx<T>*, long long);

HM_INST(double)
HM_INST(float)

}  // namespace hm
